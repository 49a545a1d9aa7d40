// Tall-skinny update of Algorithm RBGS, step 3:  Q'_(i) = W_(i) - Q_(1:i-1) R_(1:i-1,i),
// optionally followed in the same pass by the substitution of steps 4-5,
// Q_(i) = Q'_(i) R_(i,i)^{-1} (row by row, FP64 arithmetic).
//
// The product runs on matrix cores, in FP64 (v_mfma_f64_16x16x4f64; FP32 data
// are converted exactly) or, on request for FP32 storage, in FP32
// (v_mfma_f32_16x16x4f32 with FP32 accumulation).  Each lane loads VEC
// consecutive rows of one column of Q with one 16-byte load; element v of that
// vector feeds the A operand of accumulator v, so accumulator v covers rows
// VEC*i + v of the wave's row strip and one load feeds VEC*NB matrix-core
// instructions.  R is staged in LDS in chunks of kKC rows.  The epilogue moves
// the product through LDS so that each lane owns one full row for the
// substitution and the stores are coalesced column by column.
#include "rbgs_internal.h"

namespace rbgs {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kUpThreads = 256;
constexpr int kKC = 128;      // rows of R per LDS chunk
constexpr int kUnroll = 8;    // K-steps whose loads are issued together
constexpr int kMaxB = 32;

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
template <typename T, typename C, int NB>
__global__ __launch_bounds__(kUpThreads) void update_kernel(
    const T* W, int64_t ldw, const T* __restrict__ Q, int64_t ldq, T* Qout, int64_t ldqo,
    const double* __restrict__ Rk, const double* __restrict__ Rii, int64_t ldr, int64_t n, int K,
    int bw, int vec_ok) {
  typedef Mfma<C> M;
  constexpr int VEC = Vec16<T>::N;
  constexpr int WROWS = 16 * VEC;  // rows per wave
  constexpr int NCOL = 16 * NB;
  constexpr int CT_LD = 17;        // one 16-column slab of the product per pass
  constexpr int RS_BYTES = kKC * NCOL * sizeof(C);
  constexpr int CT_BYTES = 4 * WROWS * CT_LD * sizeof(C);
  constexpr int U_BYTES = RS_BYTES > CT_BYTES ? RS_BYTES : CT_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char ubuf_raw[U_BYTES];  // R chunk, then product slab
  __shared__ double Rd[NCOL * NCOL];                                          // R_(i,i)
  C* ubuf = reinterpret_cast<C*>(ubuf_raw);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wrow0 = ((int64_t)blockIdx.x * 4 + wave) * WROWS;
  const int kk = lane >> 4, li = lane & 15;
  const int64_t arow = wrow0 + (int64_t)VEC * li;   // first row of this lane's A vector
  const bool afull = vec_ok && (arow + VEC <= n);

  if (Rii != nullptr) {
    for (int e = threadIdx.x; e < NCOL * NCOL; e += kUpThreads) {
      const int r = e % NCOL, c = e / NCOL;
      Rd[e] = (r < bw && c < bw) ? Rii[r + (int64_t)c * ldr] : (r == c ? 1.0 : 0.0);
    }
  }

  typename M::acc_t acc[VEC][NB];
#pragma unroll
  for (int v = 0; v < VEC; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[v][nb] = (typename M::acc_t){0, 0, 0, 0};

  // A operand group: kUnroll K-steps of 4 columns, one 16-byte load per step.
  auto load_group = [&](T (&a)[kUnroll][VEC], int kc0, int kc, int ks0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int col = kc0 + ks0 + 4 * u + kk;
      const bool colok = (ks0 + 4 * u + kk) < kc;
      const T* src = Q + arow + (int64_t)col * ldq;
      if (colok && afull) {
        typename Vec16<T>::t vv = *reinterpret_cast<const typename Vec16<T>::t*>(src);
#pragma unroll
        for (int v = 0; v < VEC; ++v) a[u][v] = vv[v];
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) a[u][v] = (colok && arow + v < n) ? src[v] : (T)0;
      }
    }
  };
  auto mma_group = [&](const T (&a)[kUnroll][VEC], int kc, int ks0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (ks0 + 4 * u < kc) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const C b = ubuf[(ks0 + 4 * u + kk) * NCOL + nb * 16 + li];
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v][nb] = M::mma((C)a[u][v], b, acc[v][nb]);
        }
      }
    }
  };

  for (int kc0 = 0; kc0 < K; kc0 += kKC) {
    const int kc = min(kKC, K - kc0);
    __syncthreads();
    for (int e = threadIdx.x; e < kKC * NCOL; e += kUpThreads) {
      const int r = e / NCOL, c = e % NCOL;
      ubuf[e] = (r < kc && c < bw) ? (C)Rk[(kc0 + r) + (int64_t)c * ldr] : (C)0;
    }
    __syncthreads();
    // ping-pong: the loads of group g+1 are in flight during the products of group g
    constexpr int GS = 4 * kUnroll;
    T a0[kUnroll][VEC], a1[kUnroll][VEC];
    load_group(a0, kc0, kc, 0);
    for (int ks0 = 0; ks0 < kc; ks0 += 2 * GS) {
      if (ks0 + GS < kc) load_group(a1, kc0, kc, ks0 + GS);
      mma_group(a0, kc, ks0);
      if (ks0 + GS < kc) {
        if (ks0 + 2 * GS < kc) load_group(a0, kc0, kc, ks0 + 2 * GS);
        mma_group(a1, kc, ks0 + GS);
      }
    }
  }
  // Epilogue: lane owns row wrow0 + lane (lanes >= WROWS idle); the product is
  // moved through LDS one 16-column slab at a time.
  C* ct = ubuf + wave * WROWS * CT_LD;
  const int64_t row = wrow0 + lane;
  const bool own = lane < WROWS && row < n;
  double x[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) x[c] = 0.0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) ct[(VEC * M::row(kk, e) + v) * CT_LD + li] = acc[v][nb][e];
    __syncthreads();
    if (own) {
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int cc = nb * 16 + c;
        if (cc < bw) {
          // step 3: Q' = W - Q R in the arithmetic C, from storage T
          const C qp = (C)W[row + (int64_t)cc * ldw] - ct[lane * CT_LD + c];
          x[cc] = (double)qp;
        }
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
  for (int c = 0; c < kMaxB; ++c) x[c] = c < bw ? (double)Qb[row + (int64_t)c * ldq] : 0.0;
  row_substitute<kMaxB>(x, Rd, bw);
#pragma unroll
  for (int c = 0; c < kMaxB; ++c)
    if (c < bw) Qb[row + (int64_t)c * ldq] = (T)x[c];
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T, typename C>
static hipError_t launch_update_t(const void* W, int64_t ldw, const void* Q, int64_t ldq,
                                  void* Qout, int64_t ldqo, const double* Rk, const double* Rii,
                                  int64_t ldr, int64_t n, int64_t K, int bw, hipStream_t st) {
  constexpr int VEC = Vec16<T>::N;
  constexpr int WROWS = 16 * VEC;
  const int vec_ok = ((ldq % VEC) == 0) && ((reinterpret_cast<uintptr_t>(Q) % 16) == 0);
  dim3 grid((unsigned)ceil_div(n, 4 * WROWS));
  if (bw <= 16)
    hipLaunchKernelGGL((update_kernel<T, C, 1>), grid, dim3(kUpThreads), 0, st, (const T*)W, ldw,
                       (const T*)Q, ldq, (T*)Qout, ldqo, Rk, Rii, ldr, n, (int)K, bw, vec_ok);
  else
    hipLaunchKernelGGL((update_kernel<T, C, 2>), grid, dim3(kUpThreads), 0, st, (const T*)W, ldw,
                       (const T*)Q, ldq, (T*)Qout, ldqo, Rk, Rii, ldr, n, (int)K, bw, vec_ok);
  return hipGetLastError();
}

hipError_t launch_update(bool f32, bool f32_math, const void* W, int64_t ldw, const void* Q,
                         int64_t ldq, void* Qout, int64_t ldqo, const double* Rk,
                         const double* Rii, int64_t ldr, int64_t n, int64_t K, int bw,
                         hipStream_t st) {
  if (f32 && f32_math)
    return launch_update_t<float, float>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  if (f32)
    return launch_update_t<float, double>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
  return launch_update_t<double, double>(W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, n, K, bw, st);
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
