// Cholesky-QR post-processing of an RBGS factorization (the remark on
// post-processing in Section 2.2): with R' the Cholesky factor of Q^T Q
// (R'^T R' = Q^T Q, upper triangular), Q <- Q R'^{-1} is orthonormal in the
// l2 sense to the accuracy of Cholesky QR on a well-conditioned Q, and
// R <- R' R keeps W = Q R.
//
// Kernels here: the Gram matrix on FP64 matrix cores (partial sums over row
// splits, reduced in a fixed order), a one-workgroup Cholesky factorization,
// and the triangular product R' R.  The substitution Q R'^{-1} reuses the
// update kernel block column by block column.
#include <algorithm>

#include "rbgs_internal.h"

namespace rbgs {

namespace {

constexpr int kGmT = 64;          // output tile (rows and columns of Q^T Q)
constexpr int kGmK = 64;          // rows of Q per LDS step
constexpr int kGmLd = kGmT + 2;   // LDS row stride (doubles)
constexpr int kGmThreads = 256;

typedef double double4_t __attribute__((ext_vector_type(4)));

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile t of the upper triangle of nt x nt tiles, row by row: (ti, tj), ti <= tj.
__device__ inline void tile_of(int t, int nt, int& ti, int& tj) {
  ti = 0;
  int row_len = nt;
  while (t >= row_len) {
    t -= row_len;
    ++ti;
    --row_len;
  }
  tj = ti + t;
}

// partial[s][i + m j] = sum over rows of split s of Q[r][i] Q[r][j] for the
// tile (blockIdx.x) of the upper triangle; wave w computes rows 16 w .. of the
// tile against all its 64 columns (four 16 x 16 accumulators).
template <typename T>
__global__ __launch_bounds__(kGmThreads) void gram_kernel(const T* __restrict__ Q, int64_t ldq,
                                                          int64_t n, int m, int64_t rows_per_split,
                                                          double* __restrict__ partial) {
  __shared__ double As[kGmK * kGmLd];
  __shared__ double Bs[kGmK * kGmLd];
  const int nt = (int)cdiv(m, kGmT);
  int ti, tj;
  tile_of(blockIdx.x, nt, ti, tj);
  const int s = blockIdx.y;
  const int64_t r_beg = (int64_t)s * rows_per_split;
  const int64_t r_end = std::min<int64_t>(n, r_beg + rows_per_split);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kk = lane >> 4, li = lane & 15;
  double4_t acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = (double4_t){0, 0, 0, 0};
  // loader: thread t covers row t % 64 of columns t / 64 + 4 q (q < 16)
  const int lr = tid & 63, lc0 = tid >> 6;
  for (int64_t r0 = r_beg; r0 < r_end; r0 += kGmK) {
    const int64_t r = r0 + lr;
    const bool rok = r < r_end;
    const int64_t rc = rok ? r : r_end - 1;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = lc0 + 4 * q;
      const int ca = ti * kGmT + c, cb = tj * kGmT + c;
      const T va = Q[rc + (int64_t)(ca < m ? ca : m - 1) * ldq];
      const T vb = Q[rc + (int64_t)(cb < m ? cb : m - 1) * ldq];
      As[lr * kGmLd + c] = (rok && ca < m) ? (double)va : 0.0;
      Bs[lr * kGmLd + c] = (rok && cb < m) ? (double)vb : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kb = 0; kb < kGmK; kb += 4) {
      const double a = As[(kb + kk) * kGmLd + 16 * w + li];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double b = Bs[(kb + kk) * kGmLd + 16 * q + li];
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
      }
    }
  }
  // accumulator q, register e: row 16 w + kk + 4 e, column 16 q + li of the tile
  double* out = partial + (int64_t)s * m * m;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = ti * kGmT + 16 * w + kk + 4 * e, j = tj * kGmT + 16 * q + li;
      if (i < m && j < m) out[i + (int64_t)m * j] = acc[q][e];
    }
}

// G[i][j] = G[j][i] = sum_s partial[s][i + m j] (s in order) for i <= j.
__global__ void gram_reduce_kernel(const double* __restrict__ partial, int S, int m,
                                   double* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  if (i > j) return;
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += partial[(int64_t)s * m * m + idx];
  G[i + (int64_t)m * j] = v;
  G[j + (int64_t)m * i] = v;
}

// Upper Cholesky factor of the m x m SPD matrix A (ld m, overwritten):
// right-looking, one pivot per step; the strict lower part is zeroed.  A
// non-positive or non-finite pivot sets *flag = j (first one) and the
// factorization continues with pivot 1 so that every step stays finite.
__global__ __launch_bounds__(1024) void cholesky_kernel(double* __restrict__ A, int m,
                                                        int64_t* flag) {
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      const double d = A[j + (int64_t)m * j];
      double r = sqrt(d);
      if (!(d > 0.0) || !isfinite(r)) {
        if (*flag < 0) *flag = j;
        r = 1.0;
      }
      A[j + (int64_t)m * j] = r;
      piv = r;
    }
    __syncthreads();
    const double r = piv;
    for (int c = j + 1 + tid; c < m; c += 1024) A[j + (int64_t)m * c] /= r;
    __syncthreads();
    const int t = m - j - 1;
    for (int64_t e = tid; e < (int64_t)t * t; e += 1024) {
      const int a = j + 1 + (int)(e % t), c = j + 1 + (int)(e / t);
      if (a <= c) A[a + (int64_t)m * c] -= A[j + (int64_t)m * a] * A[j + (int64_t)m * c];
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < (int64_t)m * m; e += 1024) {
    const int a = (int)(e % m), c = (int)(e / m);
    if (a > c) A[e] = 0.0;
  }
}

// T[i][j] = sum_{l=i..j} A[i][l] B[l][j] (i <= j, in increasing l), 0 below.
__global__ void trmm_full_kernel(const double* __restrict__ A, int64_t lda,
                                 const double* __restrict__ B, int64_t ldb, int m,
                                 double* __restrict__ T) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  double v = 0.0;
  if (i <= j)
    for (int l = i; l <= j; ++l) v = fma(A[i + lda * l], B[l + ldb * j], v);
  T[idx] = v;
}

__global__ void copy_square_kernel(const double* __restrict__ T, int m, double* __restrict__ R,
                                   int64_t ldr) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  R[(idx % m) + ldr * (idx / m)] = T[idx];
}

}  // namespace

int gram_splits(int64_t n, int64_t m) {
  const int64_t nt = cdiv(m, kGmT);
  const int64_t tiles = nt * (nt + 1) / 2;
  const int64_t S = std::min<int64_t>(cdiv(512, tiles), cdiv(n, 4 * kGmK));
  return (int)std::max<int64_t>(1, S);
}

hipError_t launch_gram(bool f32, const void* Q, int64_t ldq, int64_t n, int64_t m, double* partial,
                       double* G, hipStream_t st) {
  const int64_t nt = cdiv(m, kGmT);
  const int64_t tiles = nt * (nt + 1) / 2;
  const int S = gram_splits(n, m);
  const int64_t rps = cdiv(cdiv(n, S), kGmK) * kGmK;
  dim3 grid((unsigned)tiles, (unsigned)S);
  if (f32)
    hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(kGmThreads), 0, st, (const float*)Q, ldq, n,
                       (int)m, rps, partial);
  else
    hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(kGmThreads), 0, st, (const double*)Q, ldq,
                       n, (int)m, rps, partial);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)cdiv(m * m, 256)), dim3(256), 0, st, partial,
                     S, (int)m, G);
  return hipGetLastError();
}

hipError_t launch_cholesky(double* A, int64_t m, int64_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(1024), 0, st, A, (int)m, flag);
  return hipGetLastError();
}

hipError_t launch_trmm_full(const double* A, int64_t lda, double* R, int64_t ldr, int64_t m,
                            double* T, hipStream_t st) {
  const unsigned blocks = (unsigned)cdiv(m * m, 256);
  hipLaunchKernelGGL(trmm_full_kernel, dim3(blocks), dim3(256), 0, st, A, lda, R, ldr, (int)m, T);
  hipLaunchKernelGGL(copy_square_kernel, dim3(blocks), dim3(256), 0, st, T, (int)m, R, ldr);
  return hipGetLastError();
}

}  // namespace rbgs
