// Device-side bodies of the persistent update form (FP64 arithmetic, the
// substitution fused), shared by the update kernel and the persistent batch
// kernel, and the matrix-core and vector helpers of every update form.
#ifndef RBGS_UPDATE_DEVICE_H
#define RBGS_UPDATE_DEVICE_H

#include <type_traits>

#include "rbgs_internal.h"

namespace rbgs {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Matrix-core operations by compute type.  Output layout of the 16x16x4
// instructions (lane l, accumulator register e, column l % 16):
//   f32: row 4 (l / 16) + e        f64: row l / 16 + 4 e
template <typename C>
struct Mfma;

template <>
struct Mfma<float> {
  typedef float4_t acc_t;
  __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int kk, int e) { return 4 * kk + e; }
};

template <>
struct Mfma<double> {
  typedef double4_t acc_t;
  __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int kk, int e) { return kk + 4 * e; }
};

template <typename T>
struct Vec16;  // 16-byte vector of storage elements
template <>
struct Vec16<float> {
  static constexpr int N = 4;
  typedef f32x4 t;
};
template <>
struct Vec16<double> {
  static constexpr int N = 2;
  typedef f64x2 t;
};

// Streaming accesses of the persistent update (NT = true): for a single large
// factorization Q_(1:i-1) and W_(i) are read once per launch and Q_(i)
// written once, all far larger than the caches, so they carry the nontemporal
// hint (measured on the 1e6 x 256 workload, loads: 242 -> 225 us per launch
// at K = 240, 119 -> 109 us at K = 96, the QR 3.91 -> 3.70 ms; stores: the
// update a further 2 % faster, the sketch of Q_(i) that reads it back
// unchanged).  The persistent batch, whose problems stay in the caches
// between stages, uses plain accesses (with the hint its 512-problem batch
// went from 81 to 89 ms).
template <bool NT, typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ void st_result(V v, V* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ---------------------------------------------------------------------------
// Persistent form for FP64 arithmetic, bw <= 16 NB and K <= UpPShape::MAXK
// (NB = 1: one 16-column group, four 256-thread workgroups per CU; NB = 2: two
// groups for blocks of 17..32 columns, one 512-thread workgroup per CU, whose
// R_(1:i-1,i) fills most of the CU's LDS): each workgroup stages
// R_(1:i-1,i) in LDS once and walks tiles blockIdx.x, blockIdx.x + gridDim.x,
// ... without further barriers.  The product is formed transposed,
// (Q R)^T = R^T Q^T (the R entry is the A operand, the Q element the B
// operand), so lane (kk, li) ends with rows VEC li + v of the wave's strip and
// columns 16 nb + kk + 4 e: each row is spread over the four lanes
// (0..3, li).  The forward substitution of steps 4-5 runs on those registers
// column by column, the solved entry handed across the four lanes by a lane
// shuffle, so W, the result and the stores stay in registers: no LDS round
// trip, no epilogue barrier.
// ---------------------------------------------------------------------------
constexpr int kUpPMaxK = 512;   // NB = 1: rows of R_(1:i-1,i) held in LDS (64 KB)
constexpr int kUpP2MaxK = 480;  // NB = 2: 480 x 32 FP64 (120 KB)
#ifndef RBGS_UP_PUNROLL32
#define RBGS_UP_PUNROLL32 2
#endif
#ifndef RBGS_UP_PUNROLL64
#define RBGS_UP_PUNROLL64 2
#endif
#ifndef RBGS_UP_P2UNROLL
#define RBGS_UP_P2UNROLL 4      // NB = 2: K-steps of loads issued together
#endif
// K-steps of loads issued together (measured for NB = 1)
template <typename T, int NB = 1>
struct UpPUnroll {
  static constexpr int N =
      NB == 2 ? RBGS_UP_P2UNROLL : (sizeof(T) == 4 ? RBGS_UP_PUNROLL32 : RBGS_UP_PUNROLL64);
};
// WV: waves per workgroup (the update kernels: 8; the persistent batch
// kernel: 16).  VE: rows per lane, read as one vector of VE
// elements (the update kernel: 16 bytes; the persistent batch kernel halves it
// for NB = 2, to fit its register budget).
template <typename T, int NB, int WV = 8, int VE = Vec16<T>::N>
struct UpPShape {
  static constexpr int VEC = VE;
  static constexpr int WAVES = WV;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int TILE = WAVES * 16 * VEC;           // rows per tile
  static constexpr int NCOL = 16 * NB;
  static constexpr int MAXK = NB == 1 ? kUpPMaxK : kUpP2MaxK;
  static constexpr int MINW = NB == 1 ? 4 : 2;            // waves per SIMD asked of the compiler
  static constexpr int GS = 4 * UpPUnroll<T, NB>::N;      // K-steps of one load group
  static_assert(up_p_kalign(NB) % (2 * GS) == 0, "staged rows: whole pairs of load groups");
  static_assert(MAXK % up_p_kalign(NB) == 0, "largest K: whole pairs of load groups");
};

// Forward substitution of steps 4-5 on the transposed-layout registers
// acc[v][nb][e] (row VEC li + v, column 16 nb + kk + 4 e), FP64:
// x_c = q'_c / R_cc (as q'_c (1 / R_cc)), then q'_c' -= x_c R_cc' for c' > c.
// Column c of this lane's rows sits in lane (c % 4, li), group c / 16,
// element (c % 16) / 4; it is handed to the lanes holding the other columns of
// the same rows by a lane shuffle.  Ru holds the strictly upper part of
// R_(i,i) (row-major, 16 NB per row; zero elsewhere and past bw), so the
// update needs no mask.  (The 16-column forms with four rows per lane use
// rows_substitute instead: same operations, in the same order.)
template <int VEC, int NB>
__device__ __forceinline__ void p_substitute(double4_t (&acc)[VEC][NB], const double* Ru,
                                             const double* Rinv, int bw, int kk, int li) {
  constexpr int NCOL = 16 * NB;
#pragma unroll
  for (int c = 0; c < NCOL; ++c) {
    if (c < bw) {
      const int nbc = c >> 4, kc = c & 3, ec = (c & 15) >> 2;
      const double rinv = Rinv[c];
      double xb[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) xb[v] = __shfl(acc[v][nbc][ec] * rinv, 16 * kc + li, 64);
      if (kk == kc) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v][nbc][ec] = xb[v];
      }
      // columns below c in every lane (earlier groups, e < ec) need nothing
#pragma unroll
      for (int nb = nbc; nb < NB; ++nb) {
        double ru[4];
#pragma unroll
        for (int e = (nb == nbc ? ec : 0); e < 4; ++e) ru[e] = Ru[c * NCOL + 16 * nb + kk + 4 * e];
#pragma unroll
        for (int v = 0; v < VEC; ++v)
#pragma unroll
          for (int e = (nb == nbc ? ec : 0); e < 4; ++e) acc[v][nb][e] = fma(-xb[v], ru[e], acc[v][nb][e]);
      }
    }
  }
}

// 4 x 4 transpose across the four 16-lane rows of a wave, on doubles: after
// it, register s of lane (row r, li) holds what register r of lane (row s, li)
// held.  Two rounds of gfx950 lane swaps on each 32-bit half: rows 2-3 of x[s]
// with rows 0-1 of x[s + 2], then rows 1 and 3 of x[s] with rows 0 and 2 of
// x[s + 1].
__device__ __forceinline__ void rows_transpose4(double (&x)[4]) {
  unsigned h[2][4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x[s]);
    h[0][s] = (unsigned)b;
    h[1][s] = (unsigned)(b >> 32);
  }
#pragma unroll
  for (int w = 0; w < 2; ++w) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const auto t = __builtin_amdgcn_permlane32_swap(h[w][s], h[w][s + 2], false, false);
      h[w][s] = t[0];
      h[w][s + 2] = t[1];
    }
#pragma unroll
    for (int s = 0; s < 4; s += 2) {
      const auto t = __builtin_amdgcn_permlane16_swap(h[w][s], h[w][s + 1], false, false);
      h[w][s] = t[0];
      h[w][s + 1] = t[1];
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
    x[s] = __longlong_as_double((long long)(((unsigned long long)h[1][s] << 32) | h[0][s]));
}

// Forward substitution of steps 4-5 on one row held by this lane, y[c] =
// column c (NCOL = 16 NB): x_c = q'_c (1 / R_cc), then q'_c' -= x_c R_cc' for
// c' > c, column after column (Ru row-major as in p_substitute; rows of R are
// read as LDS broadcasts).
template <int NCOL>
__device__ __forceinline__ void rows_substitute(double (&y)[NCOL], const double* Ru,
                                                const double* Rinv, int bw) {
#pragma unroll
  for (int c = 0; c < NCOL; ++c) {
    if (c < bw) {
      y[c] = y[c] * Rinv[c];
#pragma unroll
      for (int c2 = c + 1; c2 < NCOL; ++c2) y[c2] = fma(-y[c], Ru[c * NCOL + c2], y[c2]);
    }
  }
}

// One tile with guarded element loads and stores (rows >= n are neither read
// nor written; any alignment).  Same arithmetic as update_p_full_tiles.
template <typename T, int NB, int WV = 8, int VE = Vec16<T>::N>
__device__ __forceinline__ void update_p_guarded_tile(const T* W, int64_t ldw,
                                                      const T* __restrict__ Q, int64_t ldq,
                                                      T* Qout, int64_t ldqo, const double* Rs,
                                                      const double* Ru, const double* Rinv,
                                                      bool subst, int64_t tile0, int64_t n,
                                                      int K, int bw) {
  typedef Mfma<double> M;
  typedef UpPShape<T, NB, WV, VE> Sh;
  constexpr int VEC = Sh::VEC;
  constexpr int WROWS = 16 * VEC;
  constexpr int NCOL = Sh::NCOL;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, li = lane & 15;
  const int64_t arow = tile0 + (int64_t)wave * WROWS + (int64_t)VEC * li;  // this lane's rows
  const int bwc = bw - 1;

  // The accumulators start at -W_(i) (transposed layout: acc[v][nb][e] holds
  // row arow + v, column 16 nb + kk + 4 e), so W is not held through the
  // product; its loads are issued together with the first group of Q.
  constexpr int kUnroll = UpPUnroll<T, NB>::N;
  constexpr int GS = 4 * kUnroll;
  auto load_group = [&](T (&a)[kUnroll][VEC], int ks0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      int col = ks0 + 4 * u + kk;
      col = col < K ? col : K - 1;  // padded steps are skipped
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const bool in = arow + v < n;
        const T x = Q[(in ? arow + v : n - 1) + (int64_t)col * ldq];
        a[u][v] = in ? x : (T)0;
      }
    }
  };
  M::acc_t acc[VEC][NB];
  auto mma_group = [&](const T (&a)[kUnroll][VEC], int ks0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (ks0 + 4 * u < K) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          // R[ks + kk][16 nb + li] = R^T[li][ks + kk]
          const double b = Rs[(ks0 + 4 * u + kk) * NCOL + 16 * nb + li];
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v][nb] = M::mma(b, (double)a[u][v], acc[v][nb]);
        }
      }
    }
  };
  T a0[kUnroll][VEC], a1[kUnroll][VEC];
  {
    T w[NB][4][VEC];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * nb + kk + 4 * e < bw ? 16 * nb + kk + 4 * e : bwc;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool in = arow + v < n;
          const T x = W[(in ? arow + v : n - 1) + (int64_t)c * ldw];
          w[nb][e][v] = in ? x : (T)0;
        }
      }
    if (K > 0) load_group(a0, 0);
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[v][nb] = (M::acc_t){-(double)w[nb][0][v], -(double)w[nb][1][v], -(double)w[nb][2][v],
                                -(double)w[nb][3][v]};
  }
  for (int ks0 = 0; ks0 < K; ks0 += 2 * GS) {
    if (ks0 + GS < K) load_group(a1, ks0 + GS);
    mma_group(a0, ks0);
    if (ks0 + GS < K) {
      if (ks0 + 2 * GS < K) load_group(a0, ks0 + 2 * GS);
      mma_group(a1, ks0 + GS);
    }
  }
  // step 3: acc = Q R - W = -Q'_(i) (FP64)
#pragma unroll
  for (int v = 0; v < VEC; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[v][nb] = -acc[v][nb];
  if (subst) p_substitute<VEC, NB>(acc, Ru, Rinv, bw, kk, li);
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = 16 * nb + kk + 4 * e;
      if (c < bw) {
        T* dst = Qout + arow + (int64_t)c * ldqo;
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          if (arow + v < n) dst[v] = (T)acc[v][nb][e];
      }
    }
}

// The full tiles of one workgroup (tile = first, first + stride, .. < nfull),
// software-pipelined as a ring of two load groups (GS K-steps each): group
// g + 2 is loaded into the registers of group g right after g's products, so
// every load has a whole group of products to arrive in; the ring runs on
// across tiles (the last pair of a tile loads the next tile's groups 0 and 1),
// and the next tile's W is loaded as soon as the current tile's W has been
// taken into the accumulators.  No load is issued under a branch: loads and
// stores share one in-order counter on this target, and where paths with
// different numbers of accesses meet the compiler waits for all of them.  So
// R_(1:i-1,i) is staged with Kp = up_p_rows(K, NB) rows (zero past K), a
// K-step at or past Kf = K - K % 4 reads column min(Kf + kk, K - 1) (a
// column of Q_(1:i-1), multiplied by zero rows where it is padding), and a
// workgroup's last tile prefetches that column of its own rows again (cached)
// instead of a next tile.  FULL: bw = 16 NB (every column stored
// unconditionally).  Same arithmetic, in the same order, as
// update_p_guarded_tile, up to products by the zero rows of the padding.
template <typename T, int NB, int WV, int VE, bool FULL, bool NT, bool ROWS, bool HOOKED,
          typename Hook>
__device__ __forceinline__ void update_p_tiles_k(const T* W, int64_t ldw, const T* __restrict__ Q,
                                                 int64_t ldq, T* Qout, int64_t ldqo,
                                                 const double* Rs, const double* Ru,
                                                 const double* Rinv, bool subst, int64_t first,
                                                 int64_t stride, int64_t nfull, int K, int bw,
                                                 Hook& hook) {
  typedef Mfma<double> M;
  typedef UpPShape<T, NB, WV, VE> Sh;
  constexpr int VEC = Sh::VEC;
  constexpr int WROWS = 16 * VEC;
  constexpr int TILE = Sh::TILE;
  constexpr int NCOL = Sh::NCOL;
  typedef T VT __attribute__((ext_vector_type(VE)));
  constexpr int kUnroll = UpPUnroll<T, NB>::N;
  constexpr int GS = Sh::GS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, li = lane & 15;
  const int64_t roff = (int64_t)wave * WROWS + (int64_t)VEC * li;  // row of this lane in a tile
  const int bwc = bw - 1;
  const int ngroups = up_p_rows(K, NB) / GS;  // even, >= 2 (K > 0)
  const int Kf = K & ~3;
  const int64_t kko = (int64_t)kk * ldq;                      // column kk
  const int64_t klo = (int64_t)min(Kf + kk, K - 1) * ldq;     // column of the steps >= Kf

  // column c of W at rows wp.. (clamped past bw); cs = 0 reads one vector
  // 4 NB times (the prefetch without a next tile)
  auto load_w = [&](VT (&wv)[NB][4], const T* wp, int64_t cs) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = FULL ? 16 * nb + kk + 4 * e
                           : (16 * nb + kk + 4 * e < bw ? 16 * nb + kk + 4 * e : bwc);
        wv[nb][e] = ld_stream<NT>(reinterpret_cast<const VT*>(wp + (int64_t)c * cs));
      }
  };
  // group g of Q: step s = g GS + 4 u reads column s + kk from qk (stride cs)
  // below Kf, else the vector at ql
  auto load_group = [&](VT (&a)[kUnroll], const T* qk, const T* ql, int64_t cs, int g) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int s = g * GS + 4 * u;
      a[u] = ld_stream<NT>(reinterpret_cast<const VT*>(s < Kf ? qk + (int64_t)s * cs : ql));
    }
  };
  M::acc_t acc[VEC][NB];
  auto mma_group = [&](const VT (&a)[kUnroll], int g) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const double b = Rs[(g * GS + 4 * u + kk) * NCOL + 16 * nb + li];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v][nb] = M::mma(b, (double)a[u][v], acc[v][nb]);
      }
    }
  };

  int64_t tile = first;
  if (tile >= nfull) return;
  VT wv[NB][4], a0[kUnroll], a1[kUnroll];
  const T* qk = Q + tile * TILE + roff + kko;
  const T* ql = Q + tile * TILE + roff + klo;
  load_w(wv, W + tile * TILE + roff, ldw);
  load_group(a0, qk, ql, ldq, 0);
  load_group(a1, qk, ql, ldq, 1);
  // one tile; the first copy (HOOKED) calls hook() before its substitution
  auto step = [&](auto hooked) -> bool {
    const int64_t arow = tile * TILE + roff;
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[v][nb] = (M::acc_t){-(double)wv[nb][0][v], -(double)wv[nb][1][v],
                                -(double)wv[nb][2][v], -(double)wv[nb][3][v]};
    const int64_t next = tile + stride;
    const bool more = next < nfull;
    const T* hot = ql;  // read by this tile's last group
    load_w(wv, more ? W + next * TILE + roff : hot, more ? ldw : 0);
    int g = 0;
    for (; g + 2 < ngroups; g += 2) {
      mma_group(a0, g);
      load_group(a0, qk, ql, ldq, g + 2);
      mma_group(a1, g + 1);
      load_group(a1, qk, ql, ldq, g + 3);
    }
    const T* qkn = more ? Q + next * TILE + roff + kko : hot;
    const T* qln = more ? Q + next * TILE + roff + klo : hot;
    const int64_t csn = more ? ldq : 0;
    mma_group(a0, g);
    load_group(a0, qkn, qln, csn, 0);
    mma_group(a1, g + 1);
    load_group(a1, qkn, qln, csn, 1);
    if constexpr (ROWS && FULL && VEC == 4 && NB == 1) {
      // rows to lanes: lane (kk, li) takes row 4 li + kk, all 16 columns
      // (measured: 1e6 x 256 QR 3.68 -> 3.63 ms; for 32 columns the shuffle form
      // below stays, the row form measured 1 % slower there)
      double y[NCOL];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double x[4] = {acc[0][nb][e], acc[1][nb][e], acc[2][nb][e], acc[3][nb][e]};
          rows_transpose4(x);
#pragma unroll
          for (int s = 0; s < 4; ++s) y[16 * nb + 4 * e + s] = -x[s];
        }
      if constexpr (decltype(hooked)::value) hook();
      if (subst) rows_substitute<NCOL>(y, Ru, Rinv, FULL ? NCOL : bw);
      // and back (the transpose is its own inverse): 16-byte stores of 4 rows
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double x[4] = {y[4 * e], y[4 * e + 1], y[4 * e + 2], y[4 * e + 3]};
        rows_transpose4(x);
        const int c = kk + 4 * e;
        if (FULL || c < bw) {
          VT vv;
#pragma unroll
          for (int v = 0; v < VEC; ++v) vv[v] = (T)x[v];
          st_result<NT>(vv, reinterpret_cast<VT*>(Qout + arow + (int64_t)c * ldqo));
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[v][nb] = -acc[v][nb];
      if constexpr (decltype(hooked)::value) hook();
      if (subst) p_substitute<VEC, NB>(acc, Ru, Rinv, bw, kk, li);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 16 * nb + kk + 4 * e;
          if (FULL || c < bw) {
            VT vv;
#pragma unroll
            for (int v = 0; v < VEC; ++v) vv[v] = (T)acc[v][nb][e];
            st_result<NT>(vv, reinterpret_cast<VT*>(Qout + arow + (int64_t)c * ldqo));
          }
        }
    }
    if (more) {
      tile = next;
      qk = qkn;
      ql = qln;
    }
    return more;
  };
  if constexpr (HOOKED) {
    if (!step(std::true_type{})) return;
  }
  while (step(std::false_type{})) {
  }
}

// K = 0 (the first block): W and the substitution only; the next tile's W is
// loaded ahead of the current one's substitution and stores.  With four rows
// per lane and all 16 columns (ROWS, FULL) the substitution runs in row layout
// between two lane-swap transposes, the loads and stores staying 16-byte
// vectors (in row layout, one 4-byte element per lane and instruction, the
// K = 0 launch took 32 us instead of 23 without its substitution); the
// prefetch is skipped on a workgroup's last tile (the loop has no later load
// whose wait it could lengthen).  The other shapes prefetch the current
// tile's W again there.
template <typename T, int NB, int WV, int VE, bool FULL, bool NT, bool ROWS>
__device__ __forceinline__ void update_p_tiles_0(const T* W, int64_t ldw, T* Qout, int64_t ldqo,
                                                 const double* Ru, const double* Rinv, bool subst,
                                                 int64_t first, int64_t stride, int64_t nfull,
                                                 int bw) {
  typedef Mfma<double> M;
  typedef UpPShape<T, NB, WV, VE> Sh;
  constexpr int VEC = Sh::VEC;
  constexpr int WROWS = 16 * VEC;
  constexpr int TILE = Sh::TILE;
  constexpr int NCOL = Sh::NCOL;
  typedef T VT __attribute__((ext_vector_type(VE)));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, li = lane & 15;
  const int bwc = bw - 1;
  int64_t tile = first;
  if (tile >= nfull) return;
  if constexpr (ROWS && FULL && VEC == 4 && NB == 1) {
    // W as 16-byte vectors of 4 rows (lane (kk, li): rows 4 li + v of columns
    // kk + 4 e), into row layout for the substitution and back for the stores
    const int64_t roff = (int64_t)wave * WROWS + (int64_t)VEC * li;
    auto load_w = [&](VT (&wv)[4], const T* wp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = FULL ? kk + 4 * e : (kk + 4 * e < bw ? kk + 4 * e : bwc);
        wv[e] = ld_stream<NT>(reinterpret_cast<const VT*>(wp + (int64_t)c * ldw));
      }
    };
    VT wv[4];
    load_w(wv, W + tile * TILE + roff);
    for (;;) {
      const int64_t arow = tile * TILE + roff;
      double y[NCOL];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double x[4] = {(double)wv[e][0], (double)wv[e][1], (double)wv[e][2], (double)wv[e][3]};
        rows_transpose4(x);
#pragma unroll
        for (int s = 0; s < 4; ++s) y[4 * e + s] = x[s];
      }
      const int64_t next = tile + stride;
      const bool more = next < nfull;
      if (more) load_w(wv, W + next * TILE + roff);
      if (subst) rows_substitute<NCOL>(y, Ru, Rinv, FULL ? NCOL : bw);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double x[4] = {y[4 * e], y[4 * e + 1], y[4 * e + 2], y[4 * e + 3]};
        rows_transpose4(x);
        const int c = kk + 4 * e;
        if (FULL || c < bw) {
          VT vv;
#pragma unroll
          for (int v = 0; v < VEC; ++v) vv[v] = (T)x[v];
          st_result<NT>(vv, reinterpret_cast<VT*>(Qout + arow + (int64_t)c * ldqo));
        }
      }
      if (!more) break;
      tile = next;
    }
  } else {
    const int64_t roff = (int64_t)wave * WROWS + (int64_t)VEC * li;
    auto load_w = [&](VT (&wv)[NB][4], const T* wp) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = FULL ? 16 * nb + kk + 4 * e
                             : (16 * nb + kk + 4 * e < bw ? 16 * nb + kk + 4 * e : bwc);
          wv[nb][e] = ld_stream<NT>(reinterpret_cast<const VT*>(wp + (int64_t)c * ldw));
        }
    };
    VT wv[NB][4];
    M::acc_t acc[VEC][NB];
    load_w(wv, W + tile * TILE + roff);
    for (;;) {
      const int64_t arow = tile * TILE + roff;
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[v][nb] = (M::acc_t){(double)wv[nb][0][v], (double)wv[nb][1][v],
                                  (double)wv[nb][2][v], (double)wv[nb][3][v]};
      const int64_t next = tile + stride;
      const bool more = next < nfull;
      load_w(wv, W + (more ? next : tile) * TILE + roff);
      if (subst) p_substitute<VEC, NB>(acc, Ru, Rinv, bw, kk, li);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 16 * nb + kk + 4 * e;
          if (FULL || c < bw) {
            VT vv;
#pragma unroll
            for (int v = 0; v < VEC; ++v) vv[v] = (T)acc[v][nb][e];
            st_result<NT>(vv, reinterpret_cast<VT*>(Qout + arow + (int64_t)c * ldqo));
          }
        }
      if (!more) break;
      tile = next;
    }
  }
}

// Forms of the full-tile walk: K = 0 or K > 0, and all 16 NB columns of the
// block stored or only bw < 16 NB of them.  Each form is instantiated on its
// own (a kernel, or a function of its own), so that its registers are
// allocated for it alone: with the forms in one function the compiler kept
// values of one live across the other and spilled.
__host__ __device__ inline int up_p_form(int K, int bw, int nb) {
  return (K > 0 ? 2 : 0) + (bw == 16 * nb ? 1 : 0);
}

// The full tiles of one workgroup (tile = first, first + stride, .. < nfull)
// in form FORM = up_p_form(K, bw, NB); with HOOKED (K > 0 forms) hook() runs
// once, in the first tile, after its products and before its substitution
// (it may synchronize the workgroup and stage Ru and Rinv); streaming
// accesses if NT, the epilogue
// of full 16-column blocks with four rows per lane in row layout if ROWS (the
// update kernel; in the persistent batch's stage functions, with their smaller
// register budget, the row layout spilled: 192 -> 1356 bytes of scratch per
// lane; narrower blocks keep the shuffle form, where the masked row form
// spilled too).  Rs holds up_p_rows(K, NB) rows.
template <typename T, int NB, int FORM, bool NT, bool ROWS, int WV, int VE, bool HOOKED,
          typename Hook>
__device__ __forceinline__ void update_p_full_tiles_h(const T* W, int64_t ldw,
                                                      const T* __restrict__ Q, int64_t ldq,
                                                      T* Qout, int64_t ldqo, const double* Rs,
                                                      const double* Ru, const double* Rinv,
                                                      bool subst, int64_t first, int64_t stride,
                                                      int64_t nfull, int K, int bw, Hook& hook) {
  constexpr bool FULL = (FORM & 1) != 0;
  if constexpr (FORM >= 2)
    update_p_tiles_k<T, NB, WV, VE, FULL, NT, ROWS, HOOKED>(W, ldw, Q, ldq, Qout, ldqo, Rs, Ru,
                                                            Rinv, subst, first, stride, nfull, K,
                                                            bw, hook);
  else
    update_p_tiles_0<T, NB, WV, VE, FULL, NT, ROWS>(W, ldw, Qout, ldqo, Ru, Rinv, subst, first, stride,
                                          nfull, bw);
}

// Without a hook (R_(i,i) staged before the walk).
struct NoHook {
  __device__ void operator()() const {}
};
template <typename T, int NB, int FORM, bool NT, bool ROWS, int WV = 8,
          int VE = Vec16<T>::N>
__device__ __forceinline__ void update_p_full_tiles(const T* W, int64_t ldw,
                                                    const T* __restrict__ Q, int64_t ldq,
                                                    T* Qout, int64_t ldqo, const double* Rs,
                                                    const double* Ru, const double* Rinv,
                                                    bool subst, int64_t first, int64_t stride,
                                                    int64_t nfull, int K, int bw) {
  NoHook none;
  update_p_full_tiles_h<T, NB, FORM, NT, ROWS, WV, VE, false>(W, ldw, Q, ldq, Qout, ldqo, Rs, Ru,
                                                              Rinv, subst, first, stride, nfull, K,
                                                              bw, none);
}

// Ru [NCOL][NCOL] (row-major) = the strictly upper part of R_(i,i), zero past
// bw, and Rinv [NCOL] = 1 / R_cc (1 past bw), FP64, by NT threads.  COH: read
// R_(i,i) with device-coherent loads (relaxed atomics at agent scope), for a
// factor written during the same launch by a workgroup on another XCD; this
// replaces an acquire fence, whose cache invalidation in every workgroup was
// measured at about a tenth of the update's time.
template <int NCOL, int NT, bool COH = false>
__device__ __forceinline__ void update_p_stage_rii(const double* __restrict__ Rii, int64_t ldr,
                                                   int bw, double* Ru, double* Rinv) {
  auto ld = [&](int64_t i) -> double {
    if constexpr (COH)
      return __hip_atomic_load(const_cast<double*>(Rii) + i, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    else
      return Rii[i];
  };
  for (int e = threadIdx.x; e < NCOL * NCOL; e += NT) {
    const int r = e / NCOL, c = e % NCOL;
    const bool in = r < c && c < bw;
    const double v = ld((in ? r : 0) + (int64_t)(in ? c : 0) * ldr);
    Ru[e] = in ? v : 0.0;
  }
  if (threadIdx.x < NCOL) {
    const int c = threadIdx.x;
    Rinv[c] = c < bw ? 1.0 / ld(c + (int64_t)c * ldr) : 1.0;
  }
}

// Stages the factors of block i in LDS for the persistent form (NCOL = 16 NB
// columns, NT threads): Rs [Kp][NCOL] = R_(1:i-1,i) (rows >= K and columns >=
// bw zero); with Rii given, Ru [NCOL][NCOL] (row-major) = the strictly upper
// part of R_(i,i), zero past bw, and Rinv [NCOL] = 1 / R_cc (1 past bw).  FP64.
// Every load is unconditional (clamped index).  The caller synchronizes.
template <int NCOL, int NT>
__device__ __forceinline__ void update_p_stage(const double* __restrict__ Rk,
                                               const double* __restrict__ Rii, int64_t ldr, int K,
                                               int Kp, int bw, double* Rs, double* Ru,
                                               double* Rinv) {
  for (int e = threadIdx.x; e < Kp * NCOL; e += NT) {
    const int r = e / NCOL, c = e % NCOL;
    const bool in = r < K && c < bw;
    const double v = Rk[(in ? r : 0) + (int64_t)(in ? c : 0) * ldr];
    Rs[e] = in ? v : 0.0;
  }
  if (Rii != nullptr) update_p_stage_rii<NCOL, NT>(Rii, ldr, bw, Ru, Rinv);
}

}  // namespace rbgs

#endif  // RBGS_UPDATE_DEVICE_H
