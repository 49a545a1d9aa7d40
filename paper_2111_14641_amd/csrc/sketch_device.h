// Device-side bodies of the sparse-sign sketch (plan of a tile, partial sums
// of a row range, fixed-order reduction), shared by the sketch kernels and the
// persistent batch kernel.
#ifndef RBGS_SKETCH_DEVICE_H
#define RBGS_SKETCH_DEVICE_H

#include <type_traits>

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
// one or more targets, sums the rows of its buckets in increasing row order
// in FP64 registers, and keeps its running sums across tiles.  No thread ever
// updates another thread's sums, so there are no floating-point atomics and
// the summation order is fixed.
// ---------------------------------------------------------------------------
constexpr int kSpThreads = 1024;  // plan kernels
constexpr int kSpTile = 1024;  // rows per tile (one row per thread)
constexpr int kSpMaxK = 2048;
constexpr int kSpMaxZeta = 8;

__device__ __forceinline__ void block_exclusive_scan_2048(int* cnt, int* off, int* cur, int* wtot,
                                                          int k) {
  // Each thread scans two consecutive counters; wave prefix sums via shuffles;
  // wave totals (kSpThreads / 64 of them) combined by the first wave.
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

// Sketch plan: Theta is the same matrix for every sketch of one factorization,
// so its nonzeros are bucketed once.  For each tile of kSpTile rows the plan
// holds, sorted by target and, within a target, by row, the entries
// (row-in-tile << 1) | sign_bit, and the offsets of every target's bucket.
//   off: [ntiles][k + 1] uint16     ent: [ntiles][kSpTile * zeta] uint16
// The LDS of one workgroup (kSpThreads threads) while it plans a tile:
struct PlanLds {
  uint16_t sorted[kSpTile * kSpMaxZeta];
  int cnt[kSpMaxK];
  int off[kSpMaxK];
  int cur[kSpMaxK];
  int wtot[kSpThreads / 64];
};
__device__ __forceinline__ void sparse_plan_tile(int64_t n, int64_t row0, int k, int zeta,
                                                 uint32_t key0, uint32_t key1,
                                                 uint16_t* __restrict__ plan_off,
                                                 uint16_t* __restrict__ plan_ent, int64_t tile,
                                                 PlanLds& lds) {
  uint16_t* sorted = lds.sorted;
  int* cnt = lds.cnt;
  int* off = lds.off;
  int* cur = lds.cur;
  const int tid = threadIdx.x;
  const int64_t tile0 = tile * kSpTile;
  const int trows = (int)min((int64_t)kSpTile, n - tile0);
  const uint32_t L = (uint32_t)(k / zeta);
  for (int t = tid; t < k; t += kSpThreads) cnt[t] = 0;
  __syncthreads();
  // task = 2 rr + half: row rr, segments 4 half .. 4 half + 3 (one Philox call)
  constexpr int kTasks = 2 * kSpTile / kSpThreads;
  uint32_t tgt[4 * kTasks], ent[4 * kTasks];
  unsigned own = 0;  // bit j: slot j holds an entry
#pragma unroll
  for (int h = 0; h < kTasks; ++h) {
    const int task = tid + h * kSpThreads;
    const int rr = task >> 1, half = task & 1;
    if (rr < trows && 4 * half < zeta) {
      const uint64_t r = (uint64_t)(row0 + tile0 + rr);
      const u32x4 w = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), (uint32_t)half, kTagSparse,
                                    key0, key1);
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int s = 4 * half + q;
        if (s < zeta) {
          tgt[4 * h + q] = sparse_target(ws[q], (uint32_t)s, L);
          ent[4 * h + q] = ((uint32_t)rr << 1) | (ws[q] & 1u);
          atomicAdd(&cnt[tgt[4 * h + q]], 1);
          own |= 1u << (4 * h + q);
        }
      }
    }
  }
  __syncthreads();
  block_exclusive_scan_2048(cnt, off, cur, lds.wtot, k);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4 * kTasks; ++j) {
    if (own & (1u << j)) {
      const int pos = atomicAdd(&cur[tgt[j]], 1);
      sorted[pos] = (uint16_t)ent[j];
    }
  }
  __syncthreads();
  uint16_t* po = plan_off + tile * (k + 1);
  for (int t = tid; t < k; t += kSpThreads) {
    const int b = off[t], e = b + cnt[t];
    // bucket order: increasing row (each row appears once per target)
    for (int i = b + 1; i < e; ++i) {
      const uint16_t v = sorted[i];
      int p = i - 1;
      while (p >= b && sorted[p] > v) {
        sorted[p + 1] = sorted[p];
        --p;
      }
      sorted[p + 1] = v;
    }
    po[t] = (uint16_t)b;
  }
  if (tid == 0) po[k] = (uint16_t)(trows * zeta);
  __syncthreads();
  uint16_t* pe = plan_ent + tile * (int64_t)(kSpTile * zeta);
  for (int i = tid; i < trows * zeta; i += kSpThreads) pe[i] = sorted[i];
}

// Sparse-sign partial sums from a plan.  A workgroup of NT threads owns a
// range of tiles and a slice of NC columns; thread t owns targets t + NT j
// (j < TPT).  Per tile the rows are staged in LDS in the storage precision
// (exact), and each thread sums the rows of its buckets in row order in FP64
// with an exact sign (fma with +-1), keeping its running sums in registers
// across tiles.  The next tile is prefetched into registers while the current
// one is summed; every prefetch load is unconditional (clamped index).  The
// shape is chosen per storage type and width (measured): 1024 threads with 8
// FP32 columns (68 KB of LDS, two workgroups per CU) for a sketch of at most 16
// columns, 16 FP32 columns (100 KB, one per CU, the plan of a tile read once
// for twice the columns) for wider ones, or 4 FP64 columns (1024 threads for a
// 16-column sketch, 512 for wider ones), so several workgroups share a CU and
// hide one another's latency and barriers.  Staging two tiles per barrier (so
// that each barrier waits on the sum of two buckets) measured slower.  The slices of
// one row range are G apart in blockIdx.x (a multiple of 8 when G is), so
// they run on the same XCD and share the plan through its L2.
#ifndef RBGS_SPQ_NT32
#define RBGS_SPQ_NT32 1024   // FP32 storage: threads per workgroup
#endif
#ifndef RBGS_SPQ_NC32
#define RBGS_SPQ_NC32 8      // FP32 storage: columns per workgroup
#endif
#ifndef RBGS_SPQ_NT64
#define RBGS_SPQ_NT64 1024   // FP64 storage
#endif
#ifndef RBGS_SPQ_NC64
#define RBGS_SPQ_NC64 4
#endif
#ifndef RBGS_SPQ_NT32M
#define RBGS_SPQ_NT32M 1024  // FP32 storage, sketches of more than 16 columns
#endif
#ifndef RBGS_SPQ_NC32M
#define RBGS_SPQ_NC32M 16   // measured: 4e6 x 512 sketches 10.2 -> 8.6 ms per QR, 1e6 x 256 unchanged
#endif
#ifndef RBGS_SPQ_NT64M
#define RBGS_SPQ_NT64M 512   // FP64 storage, sketches of more than 16 columns
#endif
#ifndef RBGS_SPQ_NC64M
#define RBGS_SPQ_NC64M 4
#endif
#ifndef RBGS_SPQ_TPB32
#define RBGS_SPQ_TPB32 1     // FP32 storage: tiles staged per barrier
#endif
#ifndef RBGS_SPQ_TPB32M
#define RBGS_SPQ_TPB32M 1
#endif
#ifndef RBGS_SPQ_TPB64
#define RBGS_SPQ_TPB64 1
#endif
#ifndef RBGS_SPQ_TPB64M
#define RBGS_SPQ_TPB64M 1
#endif
// MANY: the sketch has more than one 16-column group (all of W at once)
template <typename T, bool MANY = false>
struct SpqShape {
  static constexpr int NT = sizeof(T) == 4 ? (MANY ? RBGS_SPQ_NT32M : RBGS_SPQ_NT32)
                                           : (MANY ? RBGS_SPQ_NT64M : RBGS_SPQ_NT64);
  static constexpr int NC = sizeof(T) == 4 ? (MANY ? RBGS_SPQ_NC32M : RBGS_SPQ_NC32)
                                           : (MANY ? RBGS_SPQ_NC64M : RBGS_SPQ_NC64);
  static constexpr int TPB = sizeof(T) == 4 ? (MANY ? RBGS_SPQ_TPB32M : RBGS_SPQ_TPB32)
                                            : (MANY ? RBGS_SPQ_TPB64M : RBGS_SPQ_TPB64);
};

// LDS of one workgroup summing NC columns, TB tiles staged per barrier.  Row
// stride: FP32 rows of 8 or more columns are padded by 16 bytes so that rows
// gathered at random start on more distinct banks.
template <typename T, int NC, int TB>
struct SpqLds {
  typedef unsigned short U8 __attribute__((ext_vector_type(8)));
  static constexpr int XC = NC + ((sizeof(T) == 4 && NC >= 8) ? 4 : 0);
  __attribute__((aligned(32))) T xs[TB][kSpTile * XC];  // [tile][rr][c]
  __attribute__((aligned(16))) U8 ent8[TB][kSpTile * kSpMaxZeta / 8];
  uint16_t off[TB][kSpMaxK + 1];
};

// NT threads (thread t owns targets t + NT j, j < TPT), NC columns, TB tiles
// staged per barrier.
template <typename T, int TPT, int NT, int NC, int TB>
__device__ __forceinline__ void sketch_sparse_q_body(
    const T* __restrict__ X, int64_t ldx, int64_t n, int ncols, int k, int zeta,
    const uint16_t* __restrict__ plan_off, const uint16_t* __restrict__ plan_ent,
    int64_t tiles_per_wg, double* __restrict__ partial, int g, int cs, SpqLds<T, NC, TB>& L) {
  static_assert(NC % 4 == 0, "columns per workgroup: a multiple of 4");
  typedef T V4 __attribute__((ext_vector_type(4)));
  typedef typename SpqLds<T, NC, TB>::U8 U8;
  constexpr int RPT = kSpTile / NT;                    // staged rows per thread and tile
  constexpr int EVT = kSpTile * kSpMaxZeta / 8 / NT;   // entry vectors per thread and tile
  constexpr int XC = SpqLds<T, NC, TB>::XC;
  auto& xs = L.xs;
  auto& ent8 = L.ent8;
  auto& off = L.off;

  const int tid = threadIdx.x;
  const int col0 = cs * NC;
  const int nc = min(NC, ncols - col0);
  const int64_t ntiles = (n + kSpTile - 1) / kSpTile;
  const int64_t tbeg = (int64_t)g * tiles_per_wg;
  const int64_t tend = min(ntiles, tbeg + tiles_per_wg);
  const int E = kSpTile * zeta;  // plan entries per tile (a multiple of 8)
  const int nvec = E / 8;

  double acc[TPT][NC];
#pragma unroll
  for (int j = 0; j < TPT; ++j)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[j][c] = 0.0;

  T px[TB][RPT][NC];
  U8 pe[TB][EVT];
  uint16_t po[TB][TPT + 1];
  // group of TB consecutive tiles from `tile` (tiles >= tend are clamped to
  // tend - 1 and never summed)
  auto fetch = [&](int64_t tile0) {
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const int64_t tile = tile0 + b < tend ? tile0 + b : tend - 1;
      const int64_t r0 = tile * kSpTile;
      const int trows = (int)min((int64_t)kSpTile, n - r0);
      // clamped, unmasked loads: no plan entry names a row past the end, and
      // the sums of columns past nc are never stored
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int rr = tid + NT * q;
        const int64_t r = r0 + (rr < trows ? rr : trows - 1);
#pragma unroll
        for (int c = 0; c < NC; ++c)
          px[b][q][c] = X[r + (int64_t)(col0 + (c < nc ? c : nc - 1)) * ldx];
      }
      const U8* pv = (const U8*)(plan_ent + tile * (int64_t)E);
#pragma unroll
      for (int q = 0; q < EVT; ++q) {
        const int v = tid + NT * q;
        pe[b][q] = pv[v < nvec ? v : nvec - 1];
      }
      const uint16_t* so = plan_off + tile * (int64_t)(k + 1);
#pragma unroll
      for (int i = 0; i <= TPT; ++i) {
        const int t = tid + i * NT;
        po[b][i] = so[t <= k ? t : k];
      }
    }
  };
  if (tbeg < tend) fetch(tbeg);
  for (int64_t tile = tbeg; tile < tend; tile += TB) {
#pragma unroll
    for (int b = 0; b < TB; ++b) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        V4* xw = (V4*)(xs[b] + (tid + NT * q) * XC);
#pragma unroll
        for (int w = 0; w < NC / 4; ++w)
          xw[w] = (V4){px[b][q][4 * w], px[b][q][4 * w + 1], px[b][q][4 * w + 2], px[b][q][4 * w + 3]};
      }
#pragma unroll
      for (int q = 0; q < EVT; ++q) {
        const int v = tid + NT * q;
        if (v < nvec) ent8[b][v] = pe[b][q];
      }
#pragma unroll
      for (int i = 0; i <= TPT; ++i) {
        const int t = tid + i * NT;
        if (t <= k) off[b][t] = po[b][i];
      }
    }
    if (tile + TB < tend) fetch(tile + TB);   // in flight while these tiles are summed
    __syncthreads();
    const int nb = (int)min((int64_t)TB, tend - tile);
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
      const int t = tid + j * NT;
      if (t < k) {
        // the staged tiles in order; in each, one entry per pass, the next
        // entry read while this one is summed
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          if (b < nb) {
            const uint16_t* ent = (const uint16_t*)ent8[b];
            const int bb = off[b][t], e = off[b][t + 1];
            uint32_t vn = ent[bb < e ? bb : 0];
            for (int i = bb; i < e; ++i) {
              const uint32_t v = vn;
              vn = ent[i + 1 < e ? i + 1 : i];
              const V4* xr = (const V4*)(xs[b] + (v >> 1) * XC);
              const double sg = (v & 1u) ? -1.0 : 1.0;
#pragma unroll
              for (int w = 0; w < NC / 4; ++w) {
                const V4 x = xr[w];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[j][4 * w + u] = fma(sg, (double)x[u], acc[j][4 * w + u]);
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < TPT; ++j) {
    const int t = tid + j * NT;
    if (t < k) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < nc) partial[((int64_t)g * ncols + col0 + c) * k + t] = acc[j][c];
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the partial sums, scaled once in FP64.
// ---------------------------------------------------------------------------
// A workgroup of kRdWaves waves owns 64 consecutive outputs (consecutive
// sketch rows t of one column, so every load of a wave is one contiguous
// 512-byte segment); wave w sums the partials g = w, w + kRdWaves, ... in
// order, and the wave sums are added in the order w = 0, 1, .. through LDS.
constexpr int kRdWaves = 16;
__device__ __forceinline__ void sketch_reduce_body(const double* __restrict__ partial, int G,
                                                   int64_t k, int64_t ncols, double scale,
                                                   double* __restrict__ out, int64_t ldo,
                                                   int64_t idx0, int64_t part_cols) {
  __shared__ double red[kRdWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t idx = idx0 + lane;
  const bool ok = idx < k * ncols;
  const int64_t ic = ok ? idx : 0;
  const int64_t t = ic % k, c = ic / k;
  const double* p = partial + c * k + t;
  const int64_t stride = part_cols * k;
  double s = 0.0;
#pragma unroll 4
  for (int g = wave; g < G; g += kRdWaves) s += p[(int64_t)g * stride];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0) {
    double tot = red[0][lane];
#pragma unroll
    for (int w = 1; w < kRdWaves; ++w) tot += red[w][lane];
    if (ok) out[t + c * ldo] = scale * tot;
  }
}

}  // namespace rbgs

#endif  // RBGS_SKETCH_DEVICE_H
