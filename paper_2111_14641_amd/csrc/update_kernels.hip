// Tall-skinny update of Algorithm RBGS, step 3:  Q'_(i) = W_(i) - Q_(1:i-1) R_(1:i-1,i),
// optionally followed in the same pass by the substitution of steps 4-5,
// Q_(i) = Q'_(i) R_(i,i)^{-1} (FP64 arithmetic).
//
// Two forms.  The persistent form (update_p_kernel: FP64 arithmetic, bw <= 32,
// K <= kUpPMaxK, kUpP2MaxK for 32 columns, the common case; update_fused_kernel
// adds the QR of the sketch) keeps R_(1:i-1,i) in LDS for the whole launch,
// forms the product on FP64 matrix cores and runs the forward substitution in
// its epilogue; its device bodies are in update_device.h.  The general form
// (update_kernel: any width up to 32, any K, and FP32 arithmetic) is below.
//
// General form.  The product runs on matrix cores, in FP64
// (v_mfma_f64_16x16x4f64; FP32 data are converted exactly) or, on request for
// FP32 storage, in FP32 (v_mfma_f32_16x16x4f32 with FP32 accumulation) or as
// split BF16x3 products (v_mfma_f32_16x16x32_bf16, FP32 accumulation; below).  Each
// lane loads VEC consecutive rows of one column of Q with one 16-byte load;
// element v of that vector feeds the A operand of accumulator v, so
// accumulator v covers rows VEC*i + v of the wave's row strip and one load
// feeds VEC*NB matrix-core instructions.  R is staged in LDS in chunks of kKC
// rows.  The epilogue moves the product through LDS so that each lane owns one
// full row for the substitution and the stores are coalesced column by column.
#include <algorithm>
#include <type_traits>

#include "small_device.h"
#include "update_device.h"

namespace rbgs {

#ifndef RBGS_UP_UNROLL
#define RBGS_UP_UNROLL 4   // FP32 storage; FP64 storage (twice the bytes per load) uses half
#endif
#ifndef RBGS_UP_SLAB
#define RBGS_UP_SLAB 16   // columns of the product per pass through LDS in the epilogue
#endif
#ifndef RBGS_UP_MINW
#define RBGS_UP_MINW 0    // > 0: ask the compiler for this many waves per SIMD
#endif

constexpr int kUpThreads = 256;
constexpr int kKC = 128;                  // rows of R per LDS chunk
// K-steps whose loads are issued together (measured: 4 for FP32, 2 for FP64 storage)
template <typename T>
struct UpUnroll {
  static constexpr int N = sizeof(T) == 4 ? RBGS_UP_UNROLL : (RBGS_UP_UNROLL + 1) / 2;
};
constexpr int kMaxB = 32;

// Compute-type tag of the split BF16x3 product: every FP32 element a of Q is
// split as a_hi = bf16(a), a_lo = bf16(a - a_hi) (round to nearest even; a -
// a_hi is exact in FP32), every FP64 element b of R_(1:i-1,i) as
// b_hi = bf16(fl32(b)), b_lo = bf16(fl32(b - b_hi)), and a b is taken as
// a_hi b_hi + a_hi b_lo + a_lo b_hi (the term a_lo b_lo and the parts of a and b
// beyond the two pieces, each at most about 2^-16 |a b|, are dropped), on the
// bf16 matrix cores with FP32 accumulation.
struct Bf16x3 {};
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Forward substitution of one row: x R = q', R upper triangular (bw x bw,
// bw <= NC) in LDS (column-major, ld NC).  FP64 arithmetic.
template <int NC>
__device__ __forceinline__ void row_substitute(double* x, const double* Rs, int bw) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c < bw) {
      double s = x[c];
#pragma unroll
      for (int l = 0; l < NC; ++l)
        if (l < c) s = fma(-x[l], Rs[l + c * NC], s);
      x[c] = s / Rs[c + c * NC];
    }
  }
}

// T: storage type of W and Q; C: arithmetic of the product (float: FP32
// matrix cores with FP32 accumulation; double: FP64 matrix cores, FP32 data
// converted exactly).  NB: 16-column blocks of R_(1:i-1,i) (1 or 2).
// TAIL = false: every row of the workgroup's 4*WROWS-row tile exists and the
// 16-byte vector loads are aligned; all loads are unconditional (columns past
// K are clamped and meet zero rows of R), so no load waits on a branch.
// TAIL = true: guarded element loads, for the last partial tile or unaligned Q.
template <typename T, typename C, int NB>
struct UpdateShape {
  static constexpr bool BF3 = std::is_same<C, Bf16x3>::value;
  typedef typename std::conditional<BF3, float, C>::type CE;  // element type of the product
  static constexpr int VEC = Vec16<T>::N;
  static constexpr int WROWS = 16 * VEC;  // rows per wave
  static constexpr int TILE = 4 * WROWS;  // rows per workgroup
  static constexpr int NCOL = 16 * NB;
  static constexpr int SLAB = RBGS_UP_SLAB;
  static constexpr int CT_LD = SLAB + 1;  // one slab of the product per pass
  // R chunk: kKC x NCOL as CE, or (BF16x3) hi and lo pieces as bf16
  static constexpr int RS_BYTES = BF3 ? 2 * kKC * NCOL * 2 : kKC * NCOL * (int)sizeof(CE);
  static constexpr int CT_BYTES = 4 * WROWS * CT_LD * sizeof(CE);
  static constexpr int U_BYTES = RS_BYTES > CT_BYTES ? RS_BYTES : CT_BYTES;
};

// BF16x3 product of one wave's row strip: acc[v][nb] += Q_(1:i-1) R_(1:i-1,i)
// for rows arow + v.  A K-step group is 8 loads of 4 columns (32 columns); for
// row element v the lane holds the 8 columns ks + kk + 4 j, j = 0..7, which
// are the 8 consecutive K-slots 8 kk + j of the A operand of
// v_mfma_f32_16x16x32_bf16 (row li).  The R chunk is staged in LDS in the same
// slot order, hi and lo pieces apart: Rb[hl][s][nb][g][n][j] =
// piece hl of R[kc0 + 32 s + g + 4 j][16 nb + n], so lane (g, n) reads its
// 8-slot B operand as one 16-byte vector.  The output layout is that of the
// FP32 16x16 instructions (row 4 (l / 16) + e, column l % 16).
template <int NB, bool TAIL>
__device__ __forceinline__ void product_bf16x3(float4_t (&acc)[4][NB], const float* __restrict__ Q,
                                               int64_t ldq, const double* __restrict__ Rk,
                                               int64_t ldr, int64_t arow, int64_t n, int K, int bw,
                                               unsigned char* ubuf_raw) {
  constexpr int VEC = 4;
  constexpr int NCOL = 16 * NB;
  constexpr int PIECE = kKC * NCOL;  // bf16 entries of one piece of a chunk
  __bf16* Rb = reinterpret_cast<__bf16*>(ubuf_raw);
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, li = lane & 15;
  auto load8 = [&](float (&a)[8][VEC], int kc0, int ks0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      int col = kc0 + ks0 + 4 * j + kk;
      col = col < K ? col : K - 1;  // padded slots meet zero rows of R
      const float* src = Q + arow + (int64_t)col * ldq;
      if (!TAIL) {
        const f32x4 vv = *reinterpret_cast<const f32x4*>(src);
#pragma unroll
        for (int v = 0; v < VEC; ++v) a[j][v] = vv[v];
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool in = arow + v < n;
          const float x = Q[(in ? arow + v : n - 1) + (int64_t)col * ldq];
          a[j][v] = in ? x : 0.f;
        }
      }
    }
  };
  auto mma8 = [&](const float (&a)[8][VEC], int s) {
    bf16x8 bh[NB], bl[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int o = (((s * NB + nb) * 4 + kk) * 16 + li) * 8;
      bh[nb] = *reinterpret_cast<const bf16x8*>(Rb + o);
      bl[nb] = *reinterpret_cast<const bf16x8*>(Rb + PIECE + o);
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      bf16x8 ah, al;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const __bf16 h = (__bf16)a[j][v];
        ah[j] = h;
        al[j] = (__bf16)(a[j][v] - (float)h);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[nb], acc[v][nb], 0, 0, 0);
        acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[nb], acc[v][nb], 0, 0, 0);
        acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[nb], acc[v][nb], 0, 0, 0);
      }
    }
  };
  for (int kc0 = 0; kc0 < K; kc0 += kKC) {
    const int kc = min(kKC, K - kc0);
    __syncthreads();
    for (int e = threadIdx.x; e < PIECE; e += kUpThreads) {
      // e = (((s NB + nb) 4 + g) 16 + nn) 8 + j
      const int j = e & 7, nn = (e >> 3) & 15, g = (e >> 7) & 3, snb = e >> 9;
      const int nb = snb % NB, st = snb / NB;
      const int r = 32 * st + g + 4 * j, c = 16 * nb + nn;
      const bool in = r < kc && c < bw;
      const double b = Rk[(kc0 + (in ? r : 0)) + (int64_t)(in ? c : 0) * ldr];
      const double bv = in ? b : 0.0;
      const __bf16 h = (__bf16)(float)bv;
      Rb[e] = h;
      Rb[PIECE + e] = (__bf16)(float)(bv - (double)(float)h);
    }
    __syncthreads();
    // ping-pong over 32-column steps: the loads of step s+1 are in flight
    // during the products of step s
    float a0[8][VEC], a1[8][VEC];
    load8(a0, kc0, 0);
    for (int ks0 = 0; ks0 < kc; ks0 += 64) {
      if (ks0 + 32 < kc) load8(a1, kc0, ks0 + 32);
      mma8(a0, ks0 >> 5);
      if (ks0 + 32 < kc) {
        if (ks0 + 64 < kc) load8(a0, kc0, ks0 + 64);
        mma8(a1, (ks0 >> 5) + 1);
      }
    }
  }
}

template <typename T, typename C, int NB, bool TAIL>
__device__ __forceinline__ void update_tile(
    const T* W, int64_t ldw, const T* __restrict__ Q, int64_t ldq, T* Qout, int64_t ldqo,
    const double* __restrict__ Rk, const double* __restrict__ Rii, int64_t ldr, int64_t tile_row0,
    int64_t n, int K, int bw, unsigned char* ubuf_raw, double* Rd) {
  typedef UpdateShape<T, C, NB> Sh;
  typedef typename Sh::CE CE;
  typedef Mfma<CE> M;
  constexpr int VEC = Sh::VEC;
  constexpr int WROWS = Sh::WROWS;
  constexpr int NCOL = Sh::NCOL;
  constexpr int CT_LD = Sh::CT_LD;
  CE* ubuf = reinterpret_cast<CE*>(ubuf_raw);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wrow0 = tile_row0 + (int64_t)wave * WROWS;
  const int kk = lane >> 4, li = lane & 15;
  const int64_t arow = wrow0 + (int64_t)VEC * li;   // first row of this lane's A vector
  const int64_t row = wrow0 + lane;                  // row owned in the epilogue (lane < WROWS)
  const bool own = lane < WROWS && (!TAIL || row < n);
  const int bwc = bw - 1;

  // W_(i) row of this lane, loaded first so its latency overlaps the product
  T wrow[NCOL];
  {
    const int64_t rr = TAIL ? (row < n ? row : n - 1) : (lane < WROWS ? row : wrow0);
#pragma unroll
    for (int c = 0; c < NCOL; ++c) wrow[c] = W[rr + (int64_t)(c < bw ? c : bwc) * ldw];
  }
  if (Rii != nullptr) {
    for (int e = threadIdx.x; e < NCOL * NCOL; e += kUpThreads) {
      const int r = e % NCOL, c = e / NCOL;
      const bool in = r < bw && c < bw;
      const double v = Rii[(in ? r : 0) + (int64_t)(in ? c : 0) * ldr];
      Rd[e] = in ? v : (r == c ? 1.0 : 0.0);
    }
  }

  typename M::acc_t acc[VEC][NB];
#pragma unroll
  for (int v = 0; v < VEC; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[v][nb] = (typename M::acc_t){0, 0, 0, 0};

  if constexpr (Sh::BF3) {
    static_assert(std::is_same<T, float>::value, "BF16x3 products need FP32 storage");
    product_bf16x3<NB, TAIL>(acc, Q, ldq, Rk, ldr, arow, n, K, bw, ubuf_raw);
  } else {
  constexpr int kUnroll = UpUnroll<T>::N;
  // A operand group: kUnroll K-steps of 4 columns, one 16-byte load per step.
  auto load_group = [&](T (&a)[kUnroll][VEC], int kc0, int ks0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      int col = kc0 + ks0 + 4 * u + kk;
      col = col < K ? col : K - 1;  // padded steps meet zero rows of R
      const T* src = Q + arow + (int64_t)col * ldq;
      if (!TAIL) {
        typename Vec16<T>::t vv = *reinterpret_cast<const typename Vec16<T>::t*>(src);
#pragma unroll
        for (int v = 0; v < VEC; ++v) a[u][v] = vv[v];
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool in = arow + v < n;
          const T x = Q[(in ? arow + v : n - 1) + (int64_t)col * ldq];
          a[u][v] = in ? x : (T)0;
        }
      }
    }
  };
  auto mma_group = [&](const T (&a)[kUnroll][VEC], int kc, int ks0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (ks0 + 4 * u < kc) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const CE b = ubuf[(ks0 + 4 * u + kk) * NCOL + nb * 16 + li];
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v][nb] = M::mma((CE)a[u][v], b, acc[v][nb]);
        }
      }
    }
  };

  for (int kc0 = 0; kc0 < K; kc0 += kKC) {
    const int kc = min(kKC, K - kc0);
    __syncthreads();
    for (int e = threadIdx.x; e < kKC * NCOL; e += kUpThreads) {
      const int r = e / NCOL, c = e % NCOL;
      const bool in = r < kc && c < bw;
      const double v = Rk[(kc0 + (in ? r : 0)) + (int64_t)(in ? c : 0) * ldr];
      ubuf[e] = in ? (CE)v : (CE)0;
    }
    __syncthreads();
    constexpr int GS = 4 * kUnroll;
    // ping-pong: the loads of group g+1 are in flight during the products of group g
    T a0[kUnroll][VEC], a1[kUnroll][VEC];
    load_group(a0, kc0, 0);
    for (int ks0 = 0; ks0 < kc; ks0 += 2 * GS) {
      if (ks0 + GS < kc) load_group(a1, kc0, ks0 + GS);
      mma_group(a0, kc, ks0);
      if (ks0 + GS < kc) {
        if (ks0 + 2 * GS < kc) load_group(a0, kc0, ks0 + 2 * GS);
        mma_group(a1, kc, ks0 + GS);
      }
    }
  }
  }
  // Epilogue: lane owns row wrow0 + lane (lanes >= WROWS idle); the product is
  // moved through LDS one slab of SLAB columns at a time.
  constexpr int SLAB = Sh::SLAB;
  CE* ct = ubuf + wave * WROWS * CT_LD;
  double x[NCOL];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
    for (int h = 0; h < 16 / SLAB; ++h) {
      __syncthreads();
      if (li / SLAB == h) {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            ct[(VEC * M::row(kk, e) + v) * CT_LD + (li - h * SLAB)] = acc[v][nb][e];
      }
      // the slab region of a wave is written and read by that wave only:
      // wave-level ordering suffices
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int lr = lane < WROWS ? lane : 0;
#pragma unroll
      for (int c = 0; c < SLAB; ++c) {
        // step 3: Q' = W - Q R in the arithmetic C, from storage T
        const int cc = nb * 16 + h * SLAB + c;
        const CE qp = (CE)wrow[cc] - ct[lr * CT_LD + c];
        x[cc] = (double)qp;
      }
    }
  }
  if (own) {
    if (Rii != nullptr) row_substitute<NCOL>(x, Rd, bw);
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
      if (c < bw) Qout[row + (int64_t)c * ldqo] = (T)x[c];
  }
}

// Workgroups [0, nfull) take full tiles on the branch-free path; a last
// workgroup, if n is not a multiple of the tile (or Q is not 16-byte aligned
// along columns, then all workgroups), takes the guarded path.
template <typename T, typename C, int NB>
__global__ __launch_bounds__(kUpThreads, RBGS_UP_MINW) void update_kernel(
    const T* W, int64_t ldw, const T* __restrict__ Q, int64_t ldq, T* Qout, int64_t ldqo,
    const double* __restrict__ Rk, const double* __restrict__ Rii, int64_t ldr, int64_t nfull,
    int64_t n, int K, int bw) {
  typedef UpdateShape<T, C, NB> Sh;
  __shared__ __attribute__((aligned(16))) unsigned char ubuf_raw[Sh::U_BYTES];  // R chunk, then product slab
  __shared__ double Rd[Sh::NCOL * Sh::NCOL];                                      // R_(i,i)
  const int64_t row0 = (int64_t)blockIdx.x * Sh::TILE;
  if ((int64_t)blockIdx.x < nfull)
    update_tile<T, C, NB, false>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, row0, n, K, bw,
                                 ubuf_raw, Rd);
  else
    update_tile<T, C, NB, true>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, row0, n, K, bw,
                                ubuf_raw, Rd);
}

// Lock-step batch (low-sync form): workgroup -> (problem, tile) over the
// flattened tiles; block columns c0 = K .. K + bw of each problem.
template <typename T, typename C, int NB>
__global__ __launch_bounds__(kUpThreads, RBGS_UP_MINW) void update_batched_kernel(
    const BatchItem* items, int nprob, int K, int bw) {
  typedef UpdateShape<T, C, NB> Sh;
  __shared__ __attribute__((aligned(16))) unsigned char ubuf_raw[Sh::U_BYTES];
  __shared__ double Rd[Sh::NCOL * Sh::NCOL];
  const int p = batch_find(nprob, blockIdx.x, [&](int q) { return items[q].up_tile0; });
  const BatchItem& it = items[p];
  const int64_t tile = (int64_t)blockIdx.x - it.up_tile0;
  const T* Wi = (const T*)it.W + (int64_t)K * it.ldw;
  const T* Q = (const T*)it.Q;
  T* Qi = (T*)it.Q + (int64_t)K * it.ldq;
  const double* Rk = it.R + (int64_t)K * it.ldr;
  const double* Rii = it.R + K + (int64_t)K * it.ldr;
  if (tile < it.up_nfull)
    update_tile<T, C, NB, false>(Wi, it.ldw, Q, it.ldq, Qi, it.ldq, Rk, Rii, it.ldr,
                                 tile * Sh::TILE, it.n, K, bw, ubuf_raw, Rd);
  else
    update_tile<T, C, NB, true>(Wi, it.ldw, Q, it.ldq, Qi, it.ldq, Rk, Rii, it.ldr,
                                tile * Sh::TILE, it.n, K, bw, ubuf_raw, Rd);
}

// Persistent workgroups of eight waves (two per CU; measured faster than four
// waves, four per CU, at large K, where R_(1:i-1,i) leaves LDS for two
// workgroups either way) walk the tiles.  LDS: Rs [Kp][16 NB]
// (Kp = up_p_rows(K, NB); rows >= K zero); Ru [16 NB][16 NB] (row-major) =
// strictly upper part of R_(i,i), zero past bw; Rinv [16 NB] = 1 / R_cc (1 past
// bw).  FP64.
template <typename T, int NB, int FORM>
__global__ __launch_bounds__((UpPShape<T, NB>::THREADS), (UpPShape<T, NB>::MINW)) void update_p_kernel(
    const T* W, int64_t ldw, const T* __restrict__ Q, int64_t ldq, T* Qout, int64_t ldqo,
    const double* __restrict__ Rk, const double* __restrict__ Rii, int64_t ldr, int64_t ntiles,
    int64_t nfull, int64_t n, int K, int Kp, int bw) {
  typedef UpPShape<T, NB> Sh;
  constexpr int NCOL = Sh::NCOL;
  extern __shared__ __attribute__((aligned(16))) double up_lds[];
  double* Rs = up_lds;
  double* Ru = up_lds + (int64_t)Kp * NCOL;
  double* Rinv = Ru + NCOL * NCOL;
  constexpr int TILE = Sh::TILE;
  update_p_stage<NCOL, Sh::THREADS>(Rk, Rii, ldr, K, Kp, bw, Rs, Ru, Rinv);
  const bool subst = Rii != nullptr;
  __syncthreads();
  update_p_full_tiles<T, NB, FORM, true, true, Sh::WAVES, Sh::VEC>(
      W, ldw, Q, ldq, Qout, ldqo, Rs, Ru, Rinv, subst, blockIdx.x, gridDim.x, nfull, K, bw);
  // the guarded tiles (a ragged last tile, or every tile when a pointer or
  // leading dimension is not 16-byte aligned) come after the full ones, dealt
  // from the last workgroup backwards: the last workgroups have the fewest
  // full tiles (workgroup b has those b + j gridDim.x < nfull)
  for (int64_t tile = nfull + (gridDim.x - 1 - blockIdx.x); tile < ntiles; tile += gridDim.x)
    update_p_guarded_tile<T, NB, Sh::WAVES, Sh::VEC>(W, ldw, Q, ldq, Qout, ldqo, Rs, Ru, Rinv,
                                                     subst, tile * TILE, n, K, bw);
}

// Low-sync update with the QR of the sketch in the same launch (Section
// 2.2.3: R_(i,i) is needed only by the substitution of each row, after the
// product Q_(1:i-1) R_(1:i-1,i)).  Workgroup 0 factors the residual sketch E
// with its eight waves and releases R_(i,i) (device-scope fence, then the
// ready value); workgroups 1.. walk the tiles of the persistent form with
// R_(1:i-1,i) staged, and in their first tile, between the products and the
// substitution, wait for the ready value (polling with sleeps, bounded by
// `limit` ticks of the device's wall clock; on expiry the block is reported as
// a breakdown), then stage Ru and Rinv with device-coherent loads (no acquire
// fence: its cache invalidation in every workgroup costs more than the QR).
// Workgroup 0 is dispatched first, so it is resident before anyone waits for
// it, and it waits for no one.
__device__ __forceinline__ void wait_ready(unsigned* ready, unsigned target, int64_t* flag,
                                           int64_t col0, uint64_t limit) {
  const uint64_t t0 = wall_clock64();
  while (__hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (wall_clock64() - t0 > limit) {
      atomicCAS((unsigned long long*)flag, (unsigned long long)(-1LL), (unsigned long long)col0);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Eight-wave workgroups (512-row tiles for FP32 storage, two per CU): the QR
// of a 1024 x 16 sketch in four waves would need 64 doubles per lane for the
// matrix alone, more than the update's register budget.
template <typename T>
using UpFShape = UpPShape<T, 1, 8>;

template <typename T, int FORM, int RPT>
__global__ __launch_bounds__((UpFShape<T>::THREADS), (UpFShape<T>::MINW)) void update_fused_kernel(
    const T* W, int64_t ldw, const T* __restrict__ Q, int64_t ldq, T* Qout, int64_t ldqo,
    const double* __restrict__ Rk, double* Rii, int64_t ldr, int64_t ntiles, int64_t nfull,
    int64_t n, int K, int Kp, int bw, const double* __restrict__ E, int64_t k, int64_t* flag,
    int64_t col0, unsigned* ready, uint64_t limit, int subst) {
  typedef UpFShape<T> Sh;
  constexpr int NCOL = Sh::NCOL;
  constexpr int TILE = Sh::TILE;
  extern __shared__ __attribute__((aligned(16))) double up_lds[];
  const unsigned target = (unsigned)(col0 + 1);
  if (blockIdx.x == 0) {
    qr_waven_body<RPT, Sh::WAVES>(E, k, bw, Rii, ldr, flag, col0,
                                  *reinterpret_cast<QwNLds<RPT>*>(up_lds));
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(ready, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  double* Rs = up_lds;
  double* Ru = up_lds + (int64_t)Kp * NCOL;
  double* Rinv = Ru + NCOL * NCOL;
  update_p_stage<NCOL, Sh::THREADS>(Rk, nullptr, ldr, K, Kp, bw, Rs, Ru, Rinv);
  __syncthreads();
  bool staged = false;
  auto hook = [&]() {
    if (threadIdx.x == 0) wait_ready(ready, target, flag, col0, limit);
    __syncthreads();
    update_p_stage_rii<NCOL, Sh::THREADS, true>(Rii, ldr, bw, Ru, Rinv);
    __syncthreads();
    staged = true;
  };
  const int64_t b = blockIdx.x - 1, G = gridDim.x - 1;
  // subst (always 1) is a launch argument on purpose: with a constant the
  // compiler hoists the reads of R_(i,i) out of the tile loop (136 of them, in
  // registers) and spills
  update_p_full_tiles_h<T, 1, FORM, true, true, Sh::WAVES, Sh::VEC, true>(
      W, ldw, Q, ldq, Qout, ldqo, Rs, Ru, Rinv, subst != 0, b, G, nfull, K, bw, hook);
  const int64_t g0 = nfull + (G - 1 - b);
  if (g0 < ntiles && !staged) hook();
  for (int64_t tile = g0; tile < ntiles; tile += G)
    update_p_guarded_tile<T, 1, Sh::WAVES, Sh::VEC>(W, ldw, Q, ldq, Qout, ldqo, Rs, Ru, Rinv,
                                                    subst != 0, tile * TILE, n, K, bw);
}

// Plain variant: in-place substitution Q_(i) = Q'_(i) R_(i,i)^{-1}, one row per thread.
template <typename T>
__global__ __launch_bounds__(256) void trsm_kernel(T* __restrict__ Qb, int64_t ldq,
                                                   const double* __restrict__ Rii, int64_t ldr,
                                                   int64_t n, int bw) {
  __shared__ double Rd[kMaxB * kMaxB];
  for (int e = threadIdx.x; e < kMaxB * kMaxB; e += blockDim.x) {
    const int r = e % kMaxB, c = e / kMaxB;
    Rd[e] = (r < bw && c < bw) ? Rii[r + (int64_t)c * ldr] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double x[kMaxB];
#pragma unroll
  for (int c = 0; c < kMaxB; ++c) {
    const double v = (double)Qb[row + (int64_t)(c < bw ? c : bw - 1) * ldq];  // unconditional load
    x[c] = c < bw ? v : 0.0;
  }
  row_substitute<kMaxB>(x, Rd, bw);
#pragma unroll
  for (int c = 0; c < kMaxB; ++c)
    if (c < bw) Qb[row + (int64_t)c * ldq] = (T)x[c];
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T, typename C, int NB>
static hipError_t launch_update_nb(const void* W, int64_t ldw, const void* Q, int64_t ldq,
                                   void* Qout, int64_t ldqo, const double* Rk, const double* Rii,
                                   int64_t ldr, int64_t n, int64_t K, int bw, hipStream_t st) {
  constexpr int VEC = Vec16<T>::N;
  constexpr int TILE = UpdateShape<T, C, NB>::TILE;
  const bool vec_ok = ((ldq % VEC) == 0) && ((reinterpret_cast<uintptr_t>(Q) % 16) == 0);
  const int64_t nfull = vec_ok ? n / TILE : 0;
  hipLaunchKernelGGL((update_kernel<T, C, NB>), dim3((unsigned)ceil_div(n, TILE)), dim3(kUpThreads),
                     0, st, (const T*)W, ldw, (const T*)Q, ldq, (T*)Qout, ldqo, Rk, Rii, ldr, nfull,
                     n, (int)K, bw);
  return hipGetLastError();
}

#ifndef RBGS_UP_PWGS
#define RBGS_UP_PWGS 512    // workgroups of the persistent form (two of eight waves per CU)
#endif

static bool aligned16(const void* p, int64_t ld, int vec) {
  return (ld % vec) == 0 && (reinterpret_cast<uintptr_t>(p) % 16) == 0;
}

template <typename T, int NB, int FORM>
static hipError_t launch_update_p_form(unsigned grid, size_t lds, const void* W, int64_t ldw,
                                       const void* Q, int64_t ldq, void* Qout, int64_t ldqo,
                                       const double* Rk, const double* Rii, int64_t ldr,
                                       int64_t ntiles, int64_t nfull, int64_t n, int64_t K, int Kp,
                                       int bw, hipStream_t st) {
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&update_p_kernel<T, NB, FORM>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((update_p_kernel<T, NB, FORM>), dim3(grid), dim3(UpPShape<T, NB>::THREADS),
                     lds, st, (const T*)W, ldw, (const T*)Q, ldq, (T*)Qout, ldqo, Rk, Rii, ldr,
                     ntiles, nfull, n, (int)K, Kp, bw);
  return hipGetLastError();
}

template <typename T, int NB>
static hipError_t launch_update_p(const void* W, int64_t ldw, const void* Q, int64_t ldq,
                                  void* Qout, int64_t ldqo, const double* Rk, const double* Rii,
                                  int64_t ldr, int64_t n, int64_t K, int bw, hipStream_t st) {
  typedef UpPShape<T, NB> Sh;
  constexpr int VEC = Sh::VEC;
  constexpr int TILE = Sh::TILE;
  const bool vec_ok = aligned16(W, ldw, VEC) && aligned16(Qout, ldqo, VEC) &&
                      (K == 0 || aligned16(Q, ldq, VEC));
  const int64_t ntiles = ceil_div(n, TILE);
  const int64_t nfull = vec_ok ? n / TILE : 0;
  const int Kp = up_p_rows((int)K, NB);
  const size_t lds = ((size_t)Kp * Sh::NCOL + (size_t)Sh::NCOL * Sh::NCOL + Sh::NCOL) * sizeof(double);
  unsigned grid;
  if (NB == 1) {
    // FP32 storage: as many workgroups as give every one the same number of
    // tiles (no partly empty last round; measured -0.6 % on the step, while
    // FP64 storage, with twice the tiles, is better with all of them)
    const int64_t per = ceil_div(ntiles, RBGS_UP_PWGS);
    grid = sizeof(T) == 4 ? (unsigned)ceil_div(ntiles, per)
                          : (unsigned)std::min<int64_t>(ntiles, RBGS_UP_PWGS);
  } else {
    // one workgroup per CU (its R_(1:i-1,i) fills most of the LDS)
    const int64_t per = ceil_div(ntiles, 256);
    grid = (unsigned)ceil_div(ntiles, per);
  }
  switch (up_p_form((int)K, bw, NB)) {
    case 0:
      return launch_update_p_form<T, NB, 0>(grid, lds, W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr,
                                            ntiles, nfull, n, K, Kp, bw, st);
    case 1:
      return launch_update_p_form<T, NB, 1>(grid, lds, W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr,
                                            ntiles, nfull, n, K, Kp, bw, st);
    case 2:
      return launch_update_p_form<T, NB, 2>(grid, lds, W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr,
                                            ntiles, nfull, n, K, Kp, bw, st);
    default:
      return launch_update_p_form<T, NB, 3>(grid, lds, W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr,
                                            ntiles, nfull, n, K, Kp, bw, st);
  }
}

template <typename T, typename C>
static hipError_t launch_update_t(const void* W, int64_t ldw, const void* Q, int64_t ldq,
                                  void* Qout, int64_t ldqo, const double* Rk, const double* Rii,
                                  int64_t ldr, int64_t n, int64_t K, int bw, hipStream_t st) {
  if (std::is_same<C, double>::value && bw <= 16 && K <= kUpPMaxK)
    return launch_update_p<T, 1>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  if (std::is_same<C, double>::value && bw <= 32 && K <= kUpP2MaxK)
    return launch_update_p<T, 2>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  if (bw <= 16) return launch_update_nb<T, C, 1>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  return launch_update_nb<T, C, 2>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
}

bool update_fused_ok(int math, int64_t K, int bw, int64_t k) {
  return math == kMathF64 && bw == 16 && K >= 48 && K <= kUpPMaxK && k >= bw && k <= 1024;
}

template <typename T, int FORM, int RPT>
static hipError_t launch_update_fused_t(unsigned grid, size_t lds, const void* W, int64_t ldw,
                                        const void* Q, int64_t ldq, void* Qout, int64_t ldqo,
                                        const double* Rk, double* Rii, int64_t ldr,
                                        int64_t ntiles, int64_t nfull, int64_t n, int64_t K, int Kp,
                                        int bw, const double* E, int64_t k, int64_t* flag,
                                        int64_t col0, unsigned* ready, uint64_t limit,
                                        hipStream_t st) {
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&update_fused_kernel<T, FORM, RPT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((update_fused_kernel<T, FORM, RPT>), dim3(grid), dim3(UpFShape<T>::THREADS),
                     lds, st, (const T*)W, ldw, (const T*)Q, ldq, (T*)Qout, ldqo, Rk, Rii, ldr,
                     ntiles, nfull, n, (int)K, Kp, bw, E, k, flag, col0, ready, limit, 1);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_update_fused_s(const void* W, int64_t ldw, const void* Q, int64_t ldq,
                                        void* Qout, int64_t ldqo, const double* Rk, double* Rii,
                                        int64_t ldr, int64_t n, int64_t K, int bw, const double* E,
                                        int64_t k, int64_t* flag, int64_t col0, unsigned* ready,
                                        uint64_t limit, hipStream_t st) {
  typedef UpFShape<T> Sh;
  constexpr int VEC = Sh::VEC;
  constexpr int TILE = Sh::TILE;
  const bool vec_ok = aligned16(W, ldw, VEC) && aligned16(Qout, ldqo, VEC) && aligned16(Q, ldq, VEC);
  const int64_t ntiles = ceil_div(n, TILE);
  const int64_t nfull = vec_ok ? n / TILE : 0;
  const int Kp = up_p_rows((int)K, 1);
  const int RPT = k <= 256 ? 4 : (k <= 512 ? 8 : 16);
  const size_t lds_up = ((size_t)Kp * Sh::NCOL + (size_t)Sh::NCOL * Sh::NCOL + Sh::NCOL) * sizeof(double);
  const size_t lds_qr = (size_t)(2 * 64 * RPT + 2 + 16) * sizeof(double);
  const size_t lds = std::max(lds_up, lds_qr);
  // as the persistent form (two workgroups of eight waves per CU): workgroups
  // with the same number of tiles (FP32 storage) or all 512, plus the first
  // workgroup for the QR
  const int64_t per = ceil_div(ntiles, RBGS_UP_PWGS);
  const unsigned grid = 1 + (sizeof(T) == 4 ? (unsigned)ceil_div(ntiles, per)
                                            : (unsigned)std::min<int64_t>(ntiles, RBGS_UP_PWGS));
  // full 16-column blocks only (form 3; the partial form spilled here)
#define RBGS_UF(R)                                                                                 \
  return launch_update_fused_t<T, 3, R>(grid, lds, W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr,     \
                                        ntiles, nfull, n, K, Kp, bw, E, k, flag, col0, ready,     \
                                        limit, st)
  if (RPT == 4) RBGS_UF(4);
  if (RPT == 8) RBGS_UF(8);
  RBGS_UF(16);
#undef RBGS_UF
}

hipError_t launch_update_fused(bool f32, const void* W, int64_t ldw, const void* Q, int64_t ldq,
                               void* Qout, int64_t ldqo, const double* Rk, double* Rii,
                               int64_t ldr, int64_t n, int64_t K, int bw, const double* E,
                               int64_t k, int64_t* flag, int64_t col0, unsigned* ready,
                               uint64_t limit, hipStream_t st) {
  if (!update_fused_ok(kMathF64, K, bw, k) || limit == 0) return hipErrorInvalidValue;
  if (f32)
    return launch_update_fused_s<float>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, E, k,
                                        flag, col0, ready, limit, st);
  return launch_update_fused_s<double>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, E, k,
                                       flag, col0, ready, limit, st);
}

hipError_t launch_update(bool f32, int math, const void* W, int64_t ldw, const void* Q,
                         int64_t ldq, void* Qout, int64_t ldqo, const double* Rk,
                         const double* Rii, int64_t ldr, int64_t n, int64_t K, int bw,
                         hipStream_t st) {
  if (f32 && math == kMathBf16x3)
    return launch_update_t<float, Bf16x3>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  if (f32 && math == kMathF32)
    return launch_update_t<float, float>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  if (f32)
    return launch_update_t<float, double>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  return launch_update_t<double, double>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
}

int64_t update_tile_rows(bool f32) {
  return f32 ? UpdateShape<float, double, 1>::TILE : UpdateShape<double, double, 1>::TILE;
}

bool update_vec_ok(bool f32, const void* Q, int64_t ldq) {
  const int VEC = f32 ? Vec16<float>::N : Vec16<double>::N;
  return ((ldq % VEC) == 0) && ((reinterpret_cast<uintptr_t>(Q) % 16) == 0);
}

hipError_t launch_update_batched(bool f32, int math, const BatchItem* items, int nprob,
                                 int64_t total_tiles, int64_t K, int bw, hipStream_t st) {
  if (bw > kMaxB) return hipErrorInvalidValue;
  dim3 grid((unsigned)total_tiles);
#define RBGS_UPB(T, C, NB)                                                                      \
  hipLaunchKernelGGL((update_batched_kernel<T, C, NB>), grid, dim3(kUpThreads), 0, st, items, \
                     nprob, (int)K, bw)
  if (bw <= 16) {
    if (f32 && math == kMathBf16x3) RBGS_UPB(float, Bf16x3, 1);
    else if (f32 && math == kMathF32) RBGS_UPB(float, float, 1);
    else if (f32) RBGS_UPB(float, double, 1);
    else RBGS_UPB(double, double, 1);
  } else {
    if (f32 && math == kMathBf16x3) RBGS_UPB(float, Bf16x3, 2);
    else if (f32 && math == kMathF32) RBGS_UPB(float, float, 2);
    else if (f32) RBGS_UPB(float, double, 2);
    else RBGS_UPB(double, double, 2);
  }
#undef RBGS_UPB
  return hipGetLastError();
}

hipError_t launch_trsm(bool f32, void* Q, int64_t ldq, const double* Rii, int64_t ldr, int64_t n,
                       int bw, hipStream_t st) {
  dim3 grid((unsigned)ceil_div(n, 256));
  if (f32)
    hipLaunchKernelGGL(trsm_kernel<float>, grid, dim3(256), 0, st, (float*)Q, ldq, Rii, ldr, n, bw);
  else
    hipLaunchKernelGGL(trsm_kernel<double>, grid, dim3(256), 0, st, (double*)Q, ldq, Rii, ldr, n,
                       bw);
  return hipGetLastError();
}

}  // namespace rbgs
