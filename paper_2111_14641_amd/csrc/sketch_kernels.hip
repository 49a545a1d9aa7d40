// Sketch kernels: out = Theta X for the Gaussian and sparse-sign operators
// (steps 1 and 5 of Algorithm RBGS), computed as per-row-range FP64 partial
// sums followed by a fixed-order reduction, so results are reproducible bit
// for bit and no floating-point atomics are needed.
#include <type_traits>

#include "rbgs_internal.h"
#include "sketch_device.h"

namespace rbgs {

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__global__ __launch_bounds__(kSpThreads) void sparse_plan_kernel(int64_t n, int64_t row0, int k,
                                                                 int zeta, uint32_t key0,
                                                                 uint32_t key1,
                                                                 uint16_t* __restrict__ plan_off,
                                                                 uint16_t* __restrict__ plan_ent) {
  __shared__ PlanLds lds;
  sparse_plan_tile(n, row0, k, zeta, key0, key1, plan_off, plan_ent, blockIdx.x, lds);
}

// Lock-step batch: flattened tiles of all problems.
__global__ __launch_bounds__(kSpThreads) void sparse_plan_batched_kernel(const BatchItem* items,
                                                                         int nprob, int k,
                                                                         int zeta) {
  const int p = batch_find(nprob, blockIdx.x, [&](int q) { return items[q].plan_tile0; });
  const BatchItem& it = items[p];
  __shared__ PlanLds lds;
  sparse_plan_tile(it.n, 0, k, zeta, it.key0, it.key1, it.plan_off_w, it.plan_ent_w,
                   (int64_t)blockIdx.x - it.plan_tile0, lds);
}

// blockIdx.x = row range g + G * slice.
template <typename T, int TPT, bool MANY>
__global__ __launch_bounds__((SpqShape<T, MANY>::NT)) void sketch_sparse_q_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int ncols, int k, int zeta,
    const uint16_t* __restrict__ plan_off, const uint16_t* __restrict__ plan_ent,
    int64_t tiles_per_wg, double* __restrict__ partial, int G) {
  const int g = (int)(blockIdx.x % (unsigned)G);
  const int cs = (int)(blockIdx.x / (unsigned)G);
  typedef SpqShape<T, MANY> Sh;
  __shared__ SpqLds<T, Sh::NC, Sh::TPB> lds;
  sketch_sparse_q_body<T, TPT, Sh::NT, Sh::NC, Sh::TPB>(X, ldx, n, ncols, k, zeta, plan_off,
                                                        plan_ent, tiles_per_wg, partial, g, cs,
                                                        lds);
}

// Lock-step batch: blockIdx.x -> (problem, row range) over the flattened
// ranges, blockIdx.y = column slice; which = 0 sketches W (columns 0 ..),
// which = 1 Q (columns c0 ..).
template <typename T, int TPT>
__global__ __launch_bounds__(SpqShape<T>::NT) void sketch_sparse_q_batched_kernel(
    const BatchItem* items, int nprob, int which, int64_t c0, int ncols, int k, int zeta) {
  const int p = batch_find(nprob, blockIdx.x, [&](int q) { return items[q].sk_wg0; });
  const BatchItem& it = items[p];
  const T* X = which == 0 ? (const T*)it.W : (const T*)it.Q + c0 * it.ldq;
  const int64_t ldx = which == 0 ? it.ldw : it.ldq;
  typedef SpqShape<T> Sh;
  __shared__ SpqLds<T, Sh::NC, Sh::TPB> lds;
  sketch_sparse_q_body<T, TPT, Sh::NT, Sh::NC, Sh::TPB>(
      X, ldx, it.n, ncols, k, zeta, it.plan_off, it.plan_ent, it.sk_tpw, it.part,
      (int)((int64_t)blockIdx.x - it.sk_wg0), blockIdx.y, lds);
}

template <typename T, bool MANY>
static hipError_t launch_sparse_q(const T* X, int64_t ldx, int64_t n, int64_t ncols, int k,
                                  int zeta, const uint16_t* plan_off, const uint16_t* plan_ent,
                                  int64_t tpw, double* partial, int G, hipStream_t st) {
  constexpr int NT = SpqShape<T, MANY>::NT;
  const unsigned slices = (unsigned)ceil_div(ncols, SpqShape<T, MANY>::NC);
  const int tpt = (int)ceil_div(k, NT);
#define RBGS_SPQ(TPT)                                                                         \
  hipLaunchKernelGGL((sketch_sparse_q_kernel<T, TPT, MANY>), dim3((unsigned)G * slices),      \
                     dim3(NT), 0, st, X, ldx, n, (int)ncols, k, zeta, plan_off, plan_ent, tpw, \
                     partial, G)
  constexpr int kMaxTpt = kSpMaxK / NT;
  if (tpt > kMaxTpt) return hipErrorInvalidValue;
  if (tpt <= 1) {
    RBGS_SPQ(1);
  } else if (tpt <= 2) {
    if constexpr (kMaxTpt >= 2) RBGS_SPQ(2);
  } else if (tpt <= 4) {
    if constexpr (kMaxTpt >= 4) RBGS_SPQ(4);
  } else {
    if constexpr (kMaxTpt >= 8) RBGS_SPQ(8);
  }
#undef RBGS_SPQ
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense sketches (Gaussian, Rademacher): out = Z X on FP64 matrix cores
// (v_mfma_f64_16x16x4f64) with Z regenerated from Philox in every pass.  A wave
// owns 64 targets: in each 4-row step lane l holds the four entries
// Z[4(jb + l%16) + q][r], r = step row + l/16 (Gaussian: one Philox call per
// lane and step; Rademacher: the bits of one call per row, made once per 64
// rows by lane r%64 and fetched by lane exchange), and entry q feeds the A
// operand of accumulator q, so accumulator q holds targets 4(jb + i) + q,
// i = 0..15.  The B operand is the X tile staged in LDS (FP64); the next tile
// is loaded into registers while the current one is summed.  A workgroup
// covers 256 targets and NCG 16-column groups of X over its row range.
// ---------------------------------------------------------------------------
constexpr int kGaThreads = 256;
constexpr int kGaTile = 128;

// NCG column groups of 16 per workgroup share every generated entry of Theta
// (the generator dominates; one call feeds 4 NCG matrix-core instructions).
//
// Two sources (the low-sync step that sketches Q_(i) and W_(i+1) together):
// the ncols columns of X take column slots [0, S0), S0 = ncols rounded up to
// a multiple of 16, and the n1 columns of X2 the slots [S0, S0 + n1); partial
// sums are indexed by slot (NS = S0 + n1 slots).  With n1 == 0 the slots are
// the columns of X (NS = ncols).
template <typename T, int KIND, int NCG>
__global__ __launch_bounds__(kGaThreads) void sketch_gauss_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int ncols, int64_t row0, int k,
    uint32_t key0, uint32_t key1, int64_t rows_per_wg, double* __restrict__ partial,
    const T* __restrict__ X2, int64_t ldx2, int n1) {
  constexpr int NC = kSketchCols * NCG;           // column slots per workgroup
  constexpr int TILE = kGaTile / NCG;             // rows staged per step
  __shared__ double xs[TILE * NC];                // [rr][c]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  const int tbase = blockIdx.y * 256 + wave * 64;
  const int col0 = blockIdx.z * NC;
  const int S0 = n1 > 0 ? (ncols + kSketchCols - 1) / kSketchCols * kSketchCols : ncols;
  const int NS = n1 > 0 ? S0 + n1 : ncols;
  // slot -> (source, column, valid); columns of invalid slots are clamped
  auto slot_src = [&](int slot, bool& ok) -> const T* {
    if (slot < S0 || n1 == 0) {
      ok = slot < ncols;
      return X + (int64_t)(slot < ncols ? slot : ncols - 1) * ldx;
    }
    const int c2 = slot - S0;
    ok = c2 < n1;
    return X2 + (int64_t)(c2 < n1 ? c2 : n1 - 1) * ldx2;
  };
  const int64_t rbeg = (int64_t)g * rows_per_wg;
  const int64_t rend = min(n, rbeg + rows_per_wg);
  const uint32_t j = (uint32_t)(tbase / 4 + (lane & 15));
  const bool jvalid = (int)(4 * j) < k;
  const int kk = lane >> 4;

  double4_t acc[NCG][4];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[cg][q] = (double4_t){0.0, 0.0, 0.0, 0.0};

  // unconditional loads from clamped addresses (rows of the tile only), masked
  // when staged; the next tile is loaded while the current one is summed
  constexpr int NV = TILE * NC / kGaThreads;
  T v[NV];
  bool okc[NV];
  const T* srcp[NV];   // each element's column does not change from tile to tile
#pragma unroll
  for (int i = 0; i < NV; ++i) srcp[i] = slot_src(col0 + (tid + i * kGaThreads) / TILE, okc[i]);
  auto load_tile = [&](int64_t t0) {
    const int tr = (int)min((int64_t)TILE, rend - t0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int rr = (tid + i * kGaThreads) % TILE;
      v[i] = srcp[i][t0 + (rr < tr ? rr : tr - 1)];
    }
  };
  if (rbeg < rend) load_tile(rbeg);
  for (int64_t tile0 = rbeg; tile0 < rend; tile0 += TILE) {
    const int trows = (int)min((int64_t)TILE, rend - tile0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = tid + i * kGaThreads;
      const int c = e / TILE, rr = e % TILE;
      xs[rr * NC + c] = (rr < trows && okc[i]) ? to_f64(v[i]) : 0.0;
    }
    __syncthreads();
    if (tile0 + TILE < rend) load_tile(tile0 + TILE);
    for (int rc = 0; rc < trows; rc += 64) {
      // Rademacher: the 16 lanes of a row read 4 bits each of one Philox call
      // (the wave's 64 targets lie in one 128-target call, in words q0 and
      // q0 + 1), so lane l makes the call of row rc + l once per 64 rows and
      // the steps fetch the two words from that lane
      uint32_t wa = 0u, wb = 0u;
      if constexpr (KIND == kRademacher) {
        const uint64_t r = (uint64_t)(row0 + tile0 + rc + lane);
        const u32x4 x = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), (uint32_t)(tbase / 4) >> 5,
                                      kTagRademacher, key0, key1);
        const bool hi = (((uint32_t)(tbase / 4) >> 3) & 3u) != 0u;   // q0 = 0 or 2
        wa = hi ? x.z : x.x;
        wb = hi ? x.w : x.y;
      }
      const int rcend = min(trows, rc + 64);
      for (int rr = rc; rr < rcend; rr += 4) {
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        const bool zok = jvalid && rr + kk < trows;
        if constexpr (KIND == kRademacher) {
          // every lane takes part in the exchange; invalid entries are zeroed
          const int src = rr - rc + kk;
          const uint32_t a = (uint32_t)__shfl((int)wa, src);
          const uint32_t b = (uint32_t)__shfl((int)wb, src);
          const uint32_t bits = ((lane & 8) ? b : a) >> (4u * (uint32_t)(lane & 7));
#pragma unroll
          for (int i = 0; i < 4; ++i) z[i] = zok ? (((bits >> i) & 1u) ? -1.0f : 1.0f) : 0.f;
        } else {
          if (zok) gauss4((uint64_t)(row0 + tile0 + rr + kk), j, key0, key1, z);
        }
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          const double b = xs[(rr + kk) * NC + cg * kSketchCols + (lane & 15)];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[cg][q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)z[q], b, acc[cg][q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
    const int slot = col0 + cg * kSketchCols + (lane & 15);
    bool ok;
    (void)slot_src(slot, ok);
    if (ok) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // v_mfma_f64_16x16x4f64 output: register v of lane l holds row l/16 + 4v
          const int t = 4 * (tbase / 4 + (lane >> 4) + 4 * v) + q;
          if (t < k) partial[((int64_t)g * NS + slot) * k + t] = acc[cg][q][v];
        }
    }
  }
}

#ifndef RBGS_GA_WGS
#define RBGS_GA_WGS 2048   // workgroups of a dense sketch launch (about 8 waves per SIMD)
#endif
// Column groups of 16 per workgroup of the dense sketch kernel.
static int dense_ncg(int64_t groups) { return groups >= 4 ? 4 : (groups >= 2 ? 2 : 1); }

__global__ __launch_bounds__(kRdWaves * 64) void sketch_reduce_kernel(
    const double* __restrict__ partial, int G, int64_t k, int64_t ncols, double scale,
    double* __restrict__ out, int64_t ldo, int64_t part_cols) {
  sketch_reduce_body(partial, G, k, ncols, scale, out, ldo, (int64_t)blockIdx.x * 64, part_cols);
}

// Lock-step batch: blockIdx.y = problem; which = 0: into P, 1: into S (columns c0 ..).
__global__ __launch_bounds__(kRdWaves * 64) void sketch_reduce_batched_kernel(
    const BatchItem* items, int which, int64_t c0, int64_t k, int64_t ncols, double scale) {
  const BatchItem& it = items[blockIdx.y];
  double* out = which == 0 ? it.P : it.S + c0 * k;
  sketch_reduce_body(it.part, it.sk_G, k, ncols, scale, out, k, (int64_t)blockIdx.x * 64, ncols);
}

template <typename T>
__global__ void sketch_identity_kernel(const T* __restrict__ X, int64_t ldx, int64_t n,
                                       int64_t ncols, double* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t r = idx % n, c = idx / n;
  out[r + c * ldo] = to_f64(X[r + c * ldx]);
}

// ---------------------------------------------------------------------------
// Explicit unscaled Theta (k x n, float) for brute-force checks.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// SRHT (Section 1.3): Theta = P H D / sqrt(k) with H the Sylvester-ordered
// Walsh-Hadamard matrix of size 2^logn >= the global row count.  With the row
// index split as r = 1024 h + t, H = H_hi (x) H_1024, so
//     (H D x)[s] = sum_h (-1)^popcount(s_hi & h) (H_1024 D x_h)[s_lo],
// x_h being chunk h (1024 rows, zero outside [row0, row0 + n)).  A workgroup
// takes a range of chunks; for each it transforms the chunk in LDS (FP64,
// butterflies on 4 + 4 + 2 index bits, each group in registers between LDS
// transposes) and thread j adds row s_lo of the result, with the sign above,
// to its k-row sums.  Sums are FP64 in a fixed order; partials per workgroup.
// ---------------------------------------------------------------------------
constexpr int kHrThreads = 1024;
constexpr int kHrChunk = 1024;
constexpr int kHrLd = kSketchCols + 1;   // LDS row stride in doubles

template <int N>
__device__ __forceinline__ void fwht_reg(double (&a)[N]) {
#pragma unroll
  for (int h = 1; h < N; h <<= 1)
#pragma unroll
    for (int i = 0; i < N; ++i)
      if ((i & h) == 0) {
        const double u = a[i], v = a[i + h];
        a[i] = u + v;
        a[i + h] = u - v;
      }
}

template <typename T, int TPT>
__global__ __launch_bounds__(kHrThreads) void sketch_srht_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int ncols, int64_t row0, int k, int logn,
    uint32_t key0, uint32_t key1, int64_t chunks_per_wg, double* __restrict__ partial) {
  __shared__ double ys[kHrChunk * kHrLd];
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int col0 = blockIdx.y * kSketchCols;
  const int nc = min(kSketchCols, ncols - col0);
  const int64_t h0 = row0 / kHrChunk;
  const int64_t h1 = (row0 + n - 1) / kHrChunk + 1;
  const int64_t hb = h0 + (int64_t)g * chunks_per_wg;
  const int64_t he = min(h1, hb + chunks_per_wg);

  uint32_t slo[TPT];
  uint64_t shi[TPT];
#pragma unroll
  for (int j = 0; j < TPT; ++j) {
    const int t = tid + j * kHrThreads;
    const uint64_t sj = srht_sample((uint32_t)(t < k ? t : 0), logn, key0, key1);
    slo[j] = (uint32_t)(sj & (kHrChunk - 1));
    shi[j] = sj >> 10;
  }
  double acc[TPT][kSketchCols];
#pragma unroll
  for (int j = 0; j < TPT; ++j)
#pragma unroll
    for (int c = 0; c < kSketchCols; ++c) acc[j][c] = 0.0;

  for (int64_t h = hb; h < he; ++h) {
    // row tid of the chunk times its sign (clamped loads; rows outside the
    // call's range count as zero)
    {
      const int64_t gr = h * kHrChunk + tid;
      const int64_t r = gr - row0;
      const int64_t rc = r < 0 ? 0 : (r >= n ? n - 1 : r);
      T v[kSketchCols];
#pragma unroll
      for (int c = 0; c < kSketchCols; ++c) v[c] = X[rc + (int64_t)(col0 + (c < nc ? c : nc - 1)) * ldx];
      const double sg = (r >= 0 && r < n) ? srht_sign((uint64_t)gr, key0, key1) : 0.0;
#pragma unroll
      for (int c = 0; c < kSketchCols; ++c) ys[tid * kHrLd + c] = sg * (double)v[c];
    }
    __syncthreads();
    {  // index bits 0-3: thread holds rows 16 b + i of column c
      const int c = tid & 15, b = tid >> 4;
      double a[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = ys[(16 * b + i) * kHrLd + c];
      fwht_reg<16>(a);
#pragma unroll
      for (int i = 0; i < 16; ++i) ys[(16 * b + i) * kHrLd + c] = a[i];
    }
    __syncthreads();
    {  // bits 4-7: rows lo4 + 16 i + 256 hi2
      const int c = tid & 15, lo4 = (tid >> 4) & 15, hi2 = tid >> 8;
      double a[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = ys[(lo4 + 16 * i + 256 * hi2) * kHrLd + c];
      fwht_reg<16>(a);
#pragma unroll
      for (int i = 0; i < 16; ++i) ys[(lo4 + 16 * i + 256 * hi2) * kHrLd + c] = a[i];
    }
    __syncthreads();
    {  // bits 8-9: rows low8 + 256 i of columns 4 cg .. 4 cg + 3
      const int cg = tid & 3, low8 = tid >> 2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = ys[(low8 + 256 * i) * kHrLd + 4 * cg + q];
        fwht_reg<4>(a);
#pragma unroll
        for (int i = 0; i < 4; ++i) ys[(low8 + 256 * i) * kHrLd + 4 * cg + q] = a[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
      const double sgn = (__popcll(shi[j] & (uint64_t)h) & 1) ? -1.0 : 1.0;
      const double* yr = ys + slo[j] * kHrLd;
#pragma unroll
      for (int c = 0; c < kSketchCols; ++c) acc[j][c] = fma(sgn, yr[c], acc[j][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < TPT; ++j) {
    const int t = tid + j * kHrThreads;
    if (t < k) {
#pragma unroll
      for (int c = 0; c < kSketchCols; ++c)
        if (c < nc) partial[((int64_t)g * ncols + col0 + c) * k + t] = acc[j][c];
    }
  }
}

__global__ void theta_dense_kernel(int kind, int64_t k, int zeta, uint32_t key0, uint32_t key1,
                                   int64_t n, int64_t row0, float* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (kind == kGaussian) {
    const int64_t groups = k / 4;
    if (idx >= groups * n) return;
    const int64_t jj = idx % groups, rl = idx / groups;
    float z[4];
    gauss4((uint64_t)(row0 + rl), (uint32_t)jj, key0, key1, z);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[4 * jj + q + k * rl] = z[q];
  } else if (kind == kRademacher) {
    const int64_t groups = k / 4;
    if (idx >= groups * n) return;
    const int64_t jj = idx % groups, rl = idx / groups;
    float z[4];
    rademacher4((uint64_t)(row0 + rl), (uint32_t)jj, key0, key1, z);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[4 * jj + q + k * rl] = z[q];
  } else if (kind == kSrht) {
    if (idx >= k * n) return;
    const int64_t t = idx % k, rl = idx / k;
    const uint64_t r = (uint64_t)(row0 + rl);
    const uint64_t s = srht_sample((uint32_t)t, zeta, key0, key1);
    const double v = srht_sign(r, key0, key1) * ((__popcll(s & r) & 1) ? -1.0 : 1.0);
    out[t + k * rl] = (float)v;
  } else if (kind == kSparse) {
    if (idx >= n) return;
    float* col = out + k * idx;
    for (int64_t t = 0; t < k; ++t) col[t] = 0.f;
    uint32_t w[8];
    sparse_words((uint64_t)(row0 + idx), key0, key1, w);
    const uint32_t L = (uint32_t)(k / zeta);
    for (int s = 0; s < zeta; ++s) col[sparse_target(w[s], (uint32_t)s, L)] = (w[s] & 1u) ? -1.f : 1.f;
  } else {
    if (idx >= k * n) return;
    const int64_t t = idx % k, rl = idx / k;
    out[idx] = (t == row0 + rl) ? 1.f : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

#ifndef RBGS_SP_WGS
#define RBGS_SP_WGS 256    // sparse sign, one 16-column group: row ranges
#endif
#ifndef RBGS_SP_WGSM
#define RBGS_SP_WGSM 256   // sparse sign, several groups: row ranges x groups
#endif
int sketch_num_partials(const SketchDesc& sk, int64_t n, int64_t ncols, int max_groups) {
  // Sparse sign: one 1024-thread workgroup per CU in total (256 CUs) spread
  // over the column groups.  Dense (Gaussian, Rademacher): about RBGS_GA_WGS
  // workgroups of 256 threads.  Each row range is at least one tile long.
  const int64_t groups = ceil_div(ncols, kSketchCols);
  int64_t G, tile;
  if (sk.kind == kGaussian || sk.kind == kRademacher) {
    G = ceil_div(RBGS_GA_WGS, ceil_div(groups, dense_ncg(groups)) * ceil_div(sk.k, 256));
    tile = kGaTile;
  } else if (sk.kind == kSrht) {
    // one 1024-thread workgroup per CU; a range may start mid-chunk, so it
    // can touch one chunk more than n / 1024
    G = std::min<int64_t>(ceil_div(256, groups), ceil_div(n, kHrChunk) + 1);
    if (max_groups > 0) G = std::min<int64_t>(G, max_groups);
    return (int)std::max<int64_t>(1, G);
  } else {
    // RBGS_SP_WGS: row ranges x 16-column groups (one per CU by default)
    G = ceil_div(groups > 1 ? RBGS_SP_WGSM : RBGS_SP_WGS, groups);
    tile = kSpTile;
  }
  G = std::min<int64_t>(G, ceil_div(n, tile));
  if (max_groups > 0) G = std::min<int64_t>(G, max_groups);
  return (int)std::max<int64_t>(1, G);
}

// The entries start at a 16-byte boundary (they are read 8 at a time).
static int64_t plan_ent_offset(const SketchDesc& sk, int64_t n) {
  return ceil_div(ceil_div(n, kSpTile) * (sk.k + 1), 8) * 8;
}

size_t sparse_plan_bytes(const SketchDesc& sk, int64_t n) {
  const int64_t ntiles = ceil_div(n, kSpTile);
  return (size_t)(plan_ent_offset(sk, n) + ntiles * kSpTile * sk.zeta) * sizeof(uint16_t);
}

hipError_t launch_sparse_plan(const SketchDesc& sk, int64_t n, int64_t row0, uint16_t* plan,
                              hipStream_t st) {
  const int64_t ntiles = ceil_div(n, kSpTile);
  uint16_t* off = plan;
  uint16_t* ent = plan + plan_ent_offset(sk, n);
  hipLaunchKernelGGL(sparse_plan_kernel, dim3((unsigned)ntiles), dim3(kSpThreads), 0, st, n, row0,
                     (int)sk.k, sk.zeta, sk.key0, sk.key1, off, ent);
  return hipGetLastError();
}

hipError_t launch_sketch_partials(const SketchDesc& sk, bool f32, const void* X, int64_t ldx,
                                  int64_t n, int64_t ncols, int64_t row0, double* partial,
                                  const uint16_t* plan, hipStream_t st, int max_groups) {
  const uint16_t* plan_off = plan;
  const uint16_t* plan_ent = plan ? plan + plan_ent_offset(sk, n) : nullptr;
  const int G = sketch_num_partials(sk, n, ncols, max_groups);
  const int64_t groups = ceil_div(ncols, kSketchCols);
  if (sk.kind == kSparse) {
    if (plan_off == nullptr || plan_ent == nullptr) return hipErrorInvalidValue;
    const int64_t ntiles = ceil_div(n, kSpTile);
    const int64_t tpw = ceil_div(ntiles, G);
    if (f32 && ncols > kSketchCols)
      return launch_sparse_q<float, true>((const float*)X, ldx, n, ncols, (int)sk.k, sk.zeta,
                                          plan_off, plan_ent, tpw, partial, G, st);
    if (f32)
      return launch_sparse_q<float, false>((const float*)X, ldx, n, ncols, (int)sk.k, sk.zeta,
                                           plan_off, plan_ent, tpw, partial, G, st);
    if (ncols > kSketchCols)
      return launch_sparse_q<double, true>((const double*)X, ldx, n, ncols, (int)sk.k, sk.zeta,
                                           plan_off, plan_ent, tpw, partial, G, st);
    return launch_sparse_q<double, false>((const double*)X, ldx, n, ncols, (int)sk.k, sk.zeta,
                                          plan_off, plan_ent, tpw, partial, G, st);
  } else if (sk.kind == kSrht) {
    const int64_t nchunks = (row0 + n - 1) / kHrChunk + 1 - row0 / kHrChunk;
    const int64_t cpw = ceil_div(nchunks, G);
    dim3 grid(G, (unsigned)groups);
    if (f32) {
      if (sk.k > kHrThreads)
        hipLaunchKernelGGL((sketch_srht_kernel<float, 2>), grid, dim3(kHrThreads), 0, st,
                           (const float*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.zeta, sk.key0,
                           sk.key1, cpw, partial);
      else
        hipLaunchKernelGGL((sketch_srht_kernel<float, 1>), grid, dim3(kHrThreads), 0, st,
                           (const float*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.zeta, sk.key0,
                           sk.key1, cpw, partial);
    } else {
      if (sk.k > kHrThreads)
        hipLaunchKernelGGL((sketch_srht_kernel<double, 2>), grid, dim3(kHrThreads), 0, st,
                           (const double*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.zeta, sk.key0,
                           sk.key1, cpw, partial);
      else
        hipLaunchKernelGGL((sketch_srht_kernel<double, 1>), grid, dim3(kHrThreads), 0, st,
                           (const double*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.zeta, sk.key0,
                           sk.key1, cpw, partial);
    }
  } else {
    const int ncg = dense_ncg(groups);
    const int64_t rpw = ceil_div(ceil_div(n, G), kGaTile) * kGaTile;
    dim3 grid(G, (unsigned)ceil_div(sk.k, 256), (unsigned)ceil_div(groups, ncg));
#define RBGS_GA(T, KIND, NCG)                                                                   \
  hipLaunchKernelGGL((sketch_gauss_kernel<T, KIND, NCG>), grid, dim3(kGaThreads), 0, st,       \
                     (const T*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.key0, sk.key1, rpw, \
                     partial, (const T*)X, ldx, 0)
#define RBGS_GA_NCG(T, KIND)                                 \
  do {                                                       \
    if (ncg == 4) RBGS_GA(T, KIND, 4);                       \
    else if (ncg == 2) RBGS_GA(T, KIND, 2);                  \
    else RBGS_GA(T, KIND, 1);                                \
  } while (0)
    if (sk.kind == kRademacher) {
      if (f32) RBGS_GA_NCG(float, kRademacher); else RBGS_GA_NCG(double, kRademacher);
    } else {
      if (f32) RBGS_GA_NCG(float, kGaussian); else RBGS_GA_NCG(double, kGaussian);
    }
#undef RBGS_GA_NCG
#undef RBGS_GA
  }
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(const double* partial, int G, int64_t k, int64_t ncols,
                                double scale, double* out, int64_t ldo, hipStream_t st,
                                int64_t part_cols) {
  hipLaunchKernelGGL(sketch_reduce_kernel, dim3((unsigned)ceil_div(k * ncols, 64)),
                     dim3(kRdWaves * 64), 0, st, partial, G, k, ncols, scale, out, ldo,
                     part_cols > 0 ? part_cols : ncols);
  return hipGetLastError();
}

int64_t dense_pair_slots(int64_t n0, int64_t n1) { return ceil_div(n0, kSketchCols) * kSketchCols + n1; }

hipError_t launch_sketch_dense_pair(const SketchDesc& sk, bool f32, const void* X0, int64_t ldx0,
                                    int64_t n0, const void* X1, int64_t ldx1, int64_t n1,
                                    int64_t n, int64_t row0, double* partial, hipStream_t st) {
  if (sk.kind != kGaussian && sk.kind != kRademacher) return hipErrorInvalidValue;
  const int64_t NS = dense_pair_slots(n0, n1);
  const int G = sketch_num_partials(sk, n, NS, 0);
  const int64_t groups = ceil_div(NS, kSketchCols);
  const int ncg = dense_ncg(groups);
  const int64_t rpw = ceil_div(ceil_div(n, G), kGaTile) * kGaTile;
  dim3 grid(G, (unsigned)ceil_div(sk.k, 256), (unsigned)ceil_div(groups, ncg));
#define RBGS_GP(T, KIND, NCG)                                                                    \
  hipLaunchKernelGGL((sketch_gauss_kernel<T, KIND, NCG>), grid, dim3(kGaThreads), 0, st,        \
                     (const T*)X0, ldx0, n, (int)n0, row0, (int)sk.k, sk.key0, sk.key1, rpw,   \
                     partial, (const T*)X1, ldx1, (int)n1)
#define RBGS_GP_NCG(T, KIND)                                 \
  do {                                                       \
    if (ncg == 4) RBGS_GP(T, KIND, 4);                       \
    else if (ncg == 2) RBGS_GP(T, KIND, 2);                  \
    else RBGS_GP(T, KIND, 1);                                \
  } while (0)
  if (sk.kind == kRademacher) {
    if (f32) RBGS_GP_NCG(float, kRademacher); else RBGS_GP_NCG(double, kRademacher);
  } else {
    if (f32) RBGS_GP_NCG(float, kGaussian); else RBGS_GP_NCG(double, kGaussian);
  }
#undef RBGS_GP_NCG
#undef RBGS_GP
  return hipGetLastError();
}

int64_t sparse_plan_tiles(int64_t n) { return ceil_div(n, kSpTile); }
int64_t plan_offsets_len(const SketchDesc& sk, int64_t n) { return plan_ent_offset(sk, n); }

hipError_t launch_plan_batched(const BatchItem* items, int nprob, int64_t total_tiles, int k,
                               int zeta, hipStream_t st) {
  if (k > kSpMaxK || zeta > kSpMaxZeta) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sparse_plan_batched_kernel, dim3((unsigned)total_tiles), dim3(kSpThreads), 0,
                     st, items, nprob, k, zeta);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_sparse_q_batched(const BatchItem* items, int nprob, int64_t total_wgs,
                                          int which, int64_t c0, int64_t ncols, int k, int zeta,
                                          hipStream_t st) {
  constexpr int NT = SpqShape<T>::NT;
  constexpr int kMaxTpt = kSpMaxK / NT;
  const int tpt = (int)ceil_div(k, NT);
  if (tpt > kMaxTpt) return hipErrorInvalidValue;
  dim3 grid((unsigned)total_wgs, (unsigned)ceil_div(ncols, SpqShape<T>::NC));
#define RBGS_SPQB(TPT)                                                                       \
  hipLaunchKernelGGL((sketch_sparse_q_batched_kernel<T, TPT>), grid, dim3(NT), 0, st, items, \
                     nprob, which, c0, (int)ncols, k, zeta)
  if (tpt <= 1) {
    RBGS_SPQB(1);
  } else if (tpt <= 2) {
    if constexpr (kMaxTpt >= 2) RBGS_SPQB(2);
  } else if (tpt <= 4) {
    if constexpr (kMaxTpt >= 4) RBGS_SPQB(4);
  } else {
    if constexpr (kMaxTpt >= 8) RBGS_SPQB(8);
  }
#undef RBGS_SPQB
  return hipGetLastError();
}

hipError_t launch_sketch_batched(bool f32, const BatchItem* items, int nprob, int64_t total_wgs,
                                 int which, int64_t c0, int64_t ncols, int k, int zeta,
                                 double scale, hipStream_t st) {
  if (k > kSpMaxK) return hipErrorInvalidValue;
  const hipError_t e =
      f32 ? launch_sparse_q_batched<float>(items, nprob, total_wgs, which, c0, ncols, k, zeta, st)
          : launch_sparse_q_batched<double>(items, nprob, total_wgs, which, c0, ncols, k, zeta, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sketch_reduce_batched_kernel,
                     dim3((unsigned)ceil_div((int64_t)k * ncols, 64), (unsigned)nprob),
                     dim3(kRdWaves * 64), 0, st, items, which, c0, (int64_t)k, ncols, scale);
  return hipGetLastError();
}

hipError_t launch_sketch_identity(bool f32, const void* X, int64_t ldx, int64_t n, int64_t ncols,
                                  double* out, int64_t ldo, hipStream_t st) {
  const int64_t total = n * ncols;
  if (f32)
    hipLaunchKernelGGL(sketch_identity_kernel<float>, dim3((unsigned)ceil_div(total, 256)),
                       dim3(256), 0, st, (const float*)X, ldx, n, ncols, out, ldo);
  else
    hipLaunchKernelGGL(sketch_identity_kernel<double>, dim3((unsigned)ceil_div(total, 256)),
                       dim3(256), 0, st, (const double*)X, ldx, n, ncols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_theta_dense(const SketchDesc& sk, int64_t n, int64_t row0, float* out,
                              hipStream_t st) {
  int64_t total = (sk.kind == kGaussian || sk.kind == kRademacher) ? (sk.k / 4) * n
                                                                     : (sk.kind == kSparse ? n : sk.k * n);
  if (sk.kind == kSrht && row0 + n > ((int64_t)1 << sk.zeta)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(theta_dense_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st,
                     sk.kind, sk.k, sk.zeta, sk.key0, sk.key1, n, row0, out);
  return hipGetLastError();
}

}  // namespace rbgs
