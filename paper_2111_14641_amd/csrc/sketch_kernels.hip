// Sketch kernels: out = Theta X for the Gaussian and sparse-sign operators
// (steps 1 and 5 of Algorithm RBGS), computed as per-row-range FP64 partial
// sums followed by a fixed-order reduction, so results are reproducible bit
// for bit and no floating-point atomics are needed.
#include "rbgs_internal.h"

namespace rbgs {

typedef double double4_t __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ double to_f64(T x) {
  return (double)x;
}

// ---------------------------------------------------------------------------
// Sparse sign: every row r of X contributes +-X[r, :] to zeta target rows of
// the sketch (one per segment of L = k/zeta rows).  Per tile of rows the
// (row, target) pairs are counting-sorted by target in LDS; each thread owns
// one or two targets, sums the rows of its bucket in increasing row order in
// FP64 registers, and keeps its running sums across tiles.  No thread ever
// updates another thread's sums, so there are no floating-point atomics and
// the summation order is fixed.
// ---------------------------------------------------------------------------
constexpr int kSpThreads = 1024;
constexpr int kSpTile = 256;  // rows per tile
constexpr int kSpMaxK = 2048;
constexpr int kSpTPT = kSpMaxK / kSpThreads;

__device__ __forceinline__ void block_exclusive_scan_2048(int* cnt, int* off, int* cur, int k) {
  // Each thread scans two consecutive counters; wave prefix sums via shuffles;
  // wave totals combined by the first wave.
  __shared__ int wtot[kSpThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = 2 * tid, i1 = 2 * tid + 1;
  const int a = i0 < k ? cnt[i0] : 0;
  const int b = i1 < k ? cnt[i1] : 0;
  int incl = a + b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    int v = lane < kSpThreads / 64 ? wtot[lane] : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(v, d, 64);
      if (lane >= d) v += y;
    }
    if (lane < kSpThreads / 64) wtot[lane] = v;  // inclusive wave totals
  }
  __syncthreads();
  const int base = (wave ? wtot[wave - 1] : 0) + incl - (a + b);
  if (i0 < k) { off[i0] = base; cur[i0] = base; }
  if (i1 < k) { off[i1] = base + a; cur[i1] = base + a; }
}

template <typename T>
__global__ __launch_bounds__(kSpThreads) void sketch_sparse_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int ncols, int64_t row0, int k, int zeta,
    uint32_t key0, uint32_t key1, int64_t rows_per_wg, double* __restrict__ partial) {
  __shared__ T xs[kSketchCols * kSpTile];     // [c][rr]
  __shared__ uint16_t sorted[kSpTile * 8];    // (rr << 1) | sign, bucketed by target
  __shared__ int cnt[kSpMaxK];
  __shared__ int off[kSpMaxK];
  __shared__ int cur[kSpMaxK];

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int col0 = blockIdx.y * kSketchCols;
  const int nc = min(kSketchCols, ncols - col0);
  const int64_t rbeg = (int64_t)g * rows_per_wg;
  const int64_t rend = min(n, rbeg + rows_per_wg);
  const uint32_t L = (uint32_t)(k / zeta);

  double acc[kSpTPT][kSketchCols];
#pragma unroll
  for (int j = 0; j < kSpTPT; ++j)
#pragma unroll
    for (int c = 0; c < kSketchCols; ++c) acc[j][c] = 0.0;

  for (int64_t tile0 = rbeg; tile0 < rend; tile0 += kSpTile) {
    const int trows = (int)min((int64_t)kSpTile, rend - tile0);
    for (int t = tid; t < k; t += kSpThreads) cnt[t] = 0;
    for (int e = tid; e < kSketchCols * kSpTile; e += kSpThreads) {
      const int c = e / kSpTile, rr = e % kSpTile;
      xs[e] = (rr < trows && c < nc) ? X[(tile0 + rr) + (int64_t)(col0 + c) * ldx] : (T)0;
    }
    __syncthreads();
    // (row, target) pairs: thread handles row rr = tid/2, segments 4*(tid&1) .. +3
    uint32_t tgt[4], ent[4];
    int nown = 0;
    if (tid < 2 * kSpTile) {
      const int rr = tid >> 1, half = tid & 1;
      if (rr < trows && 4 * half < zeta) {
        const uint64_t r = (uint64_t)(row0 + tile0 + rr);
        const u32x4 w = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), (uint32_t)half,
                                      kTagSparse, key0, key1);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int s = 4 * half + q;
          if (s < zeta) {
            tgt[q] = sparse_target(ws[q], (uint32_t)s, L);
            ent[q] = ((uint32_t)rr << 1) | (ws[q] & 1u);
            atomicAdd(&cnt[tgt[q]], 1);
            nown = q + 1;
          }
        }
      }
    }
    __syncthreads();
    block_exclusive_scan_2048(cnt, off, cur, k);
    __syncthreads();
    for (int q = 0; q < nown; ++q) {
      const int pos = atomicAdd(&cur[tgt[q]], 1);
      sorted[pos] = (uint16_t)ent[q];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSpTPT; ++j) {
      const int t = tid + j * kSpThreads;
      if (t < k) {
        const int b = off[t], e = b + cnt[t];
        // insertion sort of the bucket by row (each row appears once per target)
        for (int i = b + 1; i < e; ++i) {
          const uint16_t v = sorted[i];
          int p = i - 1;
          while (p >= b && sorted[p] > v) {
            sorted[p + 1] = sorted[p];
            --p;
          }
          sorted[p + 1] = v;
        }
        for (int i = b; i < e; ++i) {
          const uint32_t v = sorted[i];
          const int rr = (int)(v >> 1);
          const bool neg = v & 1u;
#pragma unroll
          for (int c = 0; c < kSketchCols; ++c) {
            const double x = to_f64(xs[c * kSpTile + rr]);
            acc[j][c] += neg ? -x : x;
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kSpTPT; ++j) {
    const int t = tid + j * kSpThreads;
    if (t < k) {
#pragma unroll
      for (int c = 0; c < kSketchCols; ++c)
        if (c < nc) partial[((int64_t)g * ncols + col0 + c) * k + t] = acc[j][c];
    }
  }
}

// ---------------------------------------------------------------------------
// Gaussian: out = Z X on FP64 matrix cores (v_mfma_f64_16x16x4f64) with Z
// regenerated from Philox for every 4-row step.  A wave owns 64 targets: lane
// l generates the four entries Z[4(jb + l%16) + q][r], r = step row + l/16,
// from one Philox call, and entry q feeds the A operand of accumulator q, so
// accumulator q holds targets 4(jb + i) + q, i = 0..15.  The B operand is the
// X tile staged in LDS (FP64).  A workgroup covers 256 targets and one
// 16-column group of X over its row range.
// ---------------------------------------------------------------------------
constexpr int kGaThreads = 256;
constexpr int kGaTile = 128;

template <typename T>
__global__ __launch_bounds__(kGaThreads) void sketch_gauss_kernel(
    const T* __restrict__ X, int64_t ldx, int64_t n, int ncols, int64_t row0, int k,
    uint32_t key0, uint32_t key1, int64_t rows_per_wg, double* __restrict__ partial) {
  __shared__ double xs[kGaTile * kSketchCols];  // [rr][c]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  const int tbase = blockIdx.y * 256 + wave * 64;
  const int col0 = blockIdx.z * kSketchCols;
  const int nc = min(kSketchCols, ncols - col0);
  const int64_t rbeg = (int64_t)g * rows_per_wg;
  const int64_t rend = min(n, rbeg + rows_per_wg);
  const uint32_t j = (uint32_t)(tbase / 4 + (lane & 15));
  const bool jvalid = (int)(4 * j) < k;
  const int kk = lane >> 4;

  double4_t acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = (double4_t){0.0, 0.0, 0.0, 0.0};

  for (int64_t tile0 = rbeg; tile0 < rend; tile0 += kGaTile) {
    const int trows = (int)min((int64_t)kGaTile, rend - tile0);
    for (int e = tid; e < kGaTile * kSketchCols; e += kGaThreads) {
      const int c = e / kGaTile, rr = e % kGaTile;
      xs[rr * kSketchCols + c] =
          (rr < trows && c < nc) ? to_f64(X[(tile0 + rr) + (int64_t)(col0 + c) * ldx]) : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < trows; rr += 4) {
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (jvalid && rr + kk < trows) gauss4((uint64_t)(row0 + tile0 + rr + kk), j, key0, key1, z);
      const double b = xs[(rr + kk) * kSketchCols + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)z[q], b, acc[q], 0, 0, 0);
    }
    __syncthreads();
  }
  const int c = col0 + (lane & 15);
  if ((lane & 15) < nc) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // v_mfma_f64_16x16x4f64 output: register v of lane l holds row l/16 + 4v
        const int t = 4 * (tbase / 4 + (lane >> 4) + 4 * v) + q;
        if (t < k) partial[((int64_t)g * ncols + c) * k + t] = acc[q][v];
      }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the partial sums, scaled once in FP64.
// ---------------------------------------------------------------------------
__global__ void sketch_reduce_kernel(const double* __restrict__ partial, int G, int64_t k,
                                     int64_t ncols, double scale, double* __restrict__ out,
                                     int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * ncols) return;
  const int64_t t = idx % k, c = idx / k;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += partial[((int64_t)g * ncols + c) * k + t];
  out[t + c * ldo] = scale * s;
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
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int sketch_num_partials(const SketchDesc& sk, int64_t n, int64_t ncols) {
  // Aim for about 512 workgroups in the grid (two per CU) while keeping each
  // row range at least one tile long.
  const int64_t groups = ceil_div(ncols, kSketchCols);
  int64_t per = 1;
  int64_t tile = kSpTile;
  if (sk.kind == kGaussian) {
    per = ceil_div(sk.k, 256);
    tile = kGaTile;
  }
  int64_t G = ceil_div(512, groups * per);
  G = std::min<int64_t>(G, ceil_div(n, tile));
  return (int)std::max<int64_t>(1, G);
}

hipError_t launch_sketch_partials(const SketchDesc& sk, bool f32, const void* X, int64_t ldx,
                                  int64_t n, int64_t ncols, int64_t row0, double* partial,
                                  hipStream_t st) {
  const int G = sketch_num_partials(sk, n, ncols);
  const int64_t groups = ceil_div(ncols, kSketchCols);
  if (sk.kind == kSparse) {
    const int64_t rpw = ceil_div(ceil_div(n, G), kSpTile) * kSpTile;
    dim3 grid(G, (unsigned)groups);
    if (f32)
      hipLaunchKernelGGL(sketch_sparse_kernel<float>, grid, dim3(kSpThreads), 0, st,
                         (const float*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.zeta, sk.key0,
                         sk.key1, rpw, partial);
    else
      hipLaunchKernelGGL(sketch_sparse_kernel<double>, grid, dim3(kSpThreads), 0, st,
                         (const double*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.zeta, sk.key0,
                         sk.key1, rpw, partial);
  } else {
    const int64_t rpw = ceil_div(ceil_div(n, G), kGaTile) * kGaTile;
    dim3 grid(G, (unsigned)ceil_div(sk.k, 256), (unsigned)groups);
    if (f32)
      hipLaunchKernelGGL(sketch_gauss_kernel<float>, grid, dim3(kGaThreads), 0, st,
                         (const float*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.key0, sk.key1,
                         rpw, partial);
    else
      hipLaunchKernelGGL(sketch_gauss_kernel<double>, grid, dim3(kGaThreads), 0, st,
                         (const double*)X, ldx, n, (int)ncols, row0, (int)sk.k, sk.key0, sk.key1,
                         rpw, partial);
  }
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(const double* partial, int G, int64_t k, int64_t ncols,
                                double scale, double* out, int64_t ldo, hipStream_t st) {
  const int64_t total = k * ncols;
  hipLaunchKernelGGL(sketch_reduce_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st,
                     partial, G, k, ncols, scale, out, ldo);
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
  int64_t total = sk.kind == kGaussian ? (sk.k / 4) * n : (sk.kind == kSparse ? n : sk.k * n);
  hipLaunchKernelGGL(theta_dense_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st,
                     sk.kind, sk.k, sk.zeta, sk.key0, sk.key1, n, row0, out);
  return hipGetLastError();
}

}  // namespace rbgs
