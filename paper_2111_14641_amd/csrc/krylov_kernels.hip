// Kernels of the block Krylov solvers built on RBGS (Section 4 of the paper):
//  * CSR sparse matrix times a block of vectors, Y = alpha A X + beta Y0
//    (step 2 of Algorithm RBGS-Arnoldi, W_(i) = A Q_(i-1); and the residual
//    B - A X of randomized block GMRES), FP64 arithmetic for any storage;
//  * the least-squares problem of GMRES, min_Z ||H Z - R_(1:p,1)||_F with the
//    block upper Hessenberg H = R_(1:p,2:p) (Section 4.2), by Householder
//    reflections that exploit the band (each reflector spans bs + 1 rows) and
//    back substitution, in FP64 in one workgroup;
//  * X <- X + Q Z (the GMRES correction) and sum-of-squares reductions.
// Reductions run in a fixed order.
#include "rbgs_internal.h"

namespace rbgs {

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename TX, typename TY, int MB>
__global__ __launch_bounds__(256) void spmm_csr_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ av,
                                                       const TX* __restrict__ X, int64_t ldx,
                                                       int bs, double alpha, double beta,
                                                       const double* __restrict__ Y0, int64_t ldy0,
                                                       TY* __restrict__ Y, int64_t ldy) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double acc[MB];
#pragma unroll
  for (int j = 0; j < MB; ++j) acc[j] = 0.0;
  const int64_t e0 = rp[row], e1 = rp[row + 1];
  // entries in chunks of 8: all loads of a chunk are issued before the first
  // is used (indices clamped into the row, values of padding entries zero)
  constexpr int EC = 8;
  for (int64_t eb = e0; eb < e1; eb += EC) {
    int64_t c[EC];
    double a[EC];
#pragma unroll
    for (int q = 0; q < EC; ++q) {
      const bool in = eb + q < e1;
      const int64_t e = in ? eb + q : e1 - 1;
      c[q] = ci[e];
      const double v = av[e];
      a[q] = in ? v : 0.0;
    }
#pragma unroll
    for (int q = 0; q < EC; ++q) {
      // every column slot is accumulated (slots j >= bs read column 0 and are
      // never stored), so no load sits under a branch
#pragma unroll
      for (int j = 0; j < MB; ++j)
        acc[j] = fma(a[q], (double)X[c[q] + (int64_t)(j < bs ? j : 0) * ldx], acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    if (j < bs) {
      double y = alpha * acc[j];
      if (Y0) y = fma(beta, Y0[row + j * ldy0], y);
      Y[row + j * ldy] = (TY)y;
    }
  }
}

template <typename TX, typename TY>
static void spmm_dispatch(int64_t n, const int64_t* rp, const int32_t* ci, const double* av,
                          const TX* X, int64_t ldx, int bs, double alpha, double beta,
                          const double* Y0, int64_t ldy0, TY* Y, int64_t ldy, hipStream_t st) {
  dim3 grid((unsigned)ceil_div(n, 256));
  if (bs <= 8)
    hipLaunchKernelGGL((spmm_csr_kernel<TX, TY, 8>), grid, dim3(256), 0, st, n, rp, ci, av, X, ldx,
                       bs, alpha, beta, Y0, ldy0, Y, ldy);
  else if (bs <= 16)
    hipLaunchKernelGGL((spmm_csr_kernel<TX, TY, 16>), grid, dim3(256), 0, st, n, rp, ci, av, X, ldx,
                       bs, alpha, beta, Y0, ldy0, Y, ldy);
  else
    hipLaunchKernelGGL((spmm_csr_kernel<TX, TY, 32>), grid, dim3(256), 0, st, n, rp, ci, av, X, ldx,
                       bs, alpha, beta, Y0, ldy0, Y, ldy);
}

hipError_t launch_spmm(int64_t n, const int64_t* rp, const int32_t* ci, const double* av, int tx,
                       const void* X, int64_t ldx, int bs, double alpha, double beta,
                       const double* Y0, int64_t ldy0, int ty, void* Y, int64_t ldy,
                       hipStream_t st) {
  if (bs < 1 || bs > 32) return hipErrorInvalidValue;
  // tx, ty: 4 = FP32, 8 = FP64
  if (tx == 4 && ty == 4)
    spmm_dispatch(n, rp, ci, av, (const float*)X, ldx, bs, alpha, beta, Y0, ldy0, (float*)Y, ldy, st);
  else if (tx == 4 && ty == 8)
    spmm_dispatch(n, rp, ci, av, (const float*)X, ldx, bs, alpha, beta, Y0, ldy0, (double*)Y, ldy, st);
  else if (tx == 8 && ty == 4)
    spmm_dispatch(n, rp, ci, av, (const double*)X, ldx, bs, alpha, beta, Y0, ldy0, (float*)Y, ldy, st);
  else
    spmm_dispatch(n, rp, ci, av, (const double*)X, ldx, bs, alpha, beta, Y0, ldy0, (double*)Y, ldy, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// min_Z || H Z - T ||_F for H = A[:, 0:nc] (nr x nc, zero below the band:
// A[r][c] = 0 for r > c + band) and T = A[:, nc:nc+nr_rhs], both held in the
// nr x (nc + nrhs) column-major FP64 matrix A (ld lda, overwritten).  One
// workgroup.  Step j: reflector of rows j .. min(j + band, nr - 1) of column
// j (alpha = -sign(x_0) ||x||, v = x - alpha e_1, beta = 1 / (||x|| (||x|| +
// |x_0|))), applied to every later column by one thread per column.  Then
// back substitution with the nc x nc upper triangle.  Z: nc x nrhs (ld ldz).
// resid[c] = squared norm of rows nc .. nr-1 of the transformed column c of T
// (the least-squares residual).
// ---------------------------------------------------------------------------
constexpr int kLsThreads = 1024;

__global__ __launch_bounds__(kLsThreads) void hess_ls_kernel(double* __restrict__ A, int64_t lda,
                                                             int nr, int nc, int nrhs, int band,
                                                             double* __restrict__ Z, int64_t ldz,
                                                             double* __restrict__ resid) {
  __shared__ double sc[3];  // beta, v0, alpha
  const int tid = threadIdx.x;
  const int ncols = nc + nrhs;
  for (int j = 0; j < nc; ++j) {
    const int r1 = min(nr - 1, j + band);
    double* aj = A + (int64_t)j * lda;
    if (tid == 0) {
      double s = 0.0;
      for (int r = j; r <= r1; ++r) s = fma(aj[r], aj[r], s);
      const double x0 = aj[j];
      double beta = 0.0, v0 = x0, alpha = x0;
      if (s != 0.0) {
        const double nrm = sqrt(s);
        alpha = x0 >= 0.0 ? -nrm : nrm;
        beta = 1.0 / (nrm * (nrm + fabs(x0)));
        v0 = x0 - alpha;
      }
      sc[0] = beta;
      sc[1] = v0;
      sc[2] = alpha;
    }
    __syncthreads();
    const double beta = sc[0], v0 = sc[1];
    if (beta != 0.0) {
      for (int c = j + 1 + tid; c < ncols; c += kLsThreads) {
        double* ac = A + (int64_t)c * lda;
        double d = v0 * ac[j];
        for (int r = j + 1; r <= r1; ++r) d = fma(aj[r], ac[r], d);
        const double w = beta * d;
        ac[j] = fma(-w, v0, ac[j]);
        for (int r = j + 1; r <= r1; ++r) ac[r] = fma(-w, aj[r], ac[r]);
      }
    }
    __syncthreads();
    if (tid == 0) aj[j] = sc[2];
    __syncthreads();
  }
  // residual norms of the right-hand sides
  for (int c = tid; c < nrhs; c += kLsThreads) {
    const double* t = A + (int64_t)(nc + c) * lda;
    double s = 0.0;
    for (int r = nc; r < nr; ++r) s = fma(t[r], t[r], s);
    resid[c] = s;
  }
  // back substitution, column oriented: Z_i = t_i / U_ii, then t_r -= U_ri Z_i
  for (int i = nc - 1; i >= 0; --i) {
    const double uii = A[i + (int64_t)i * lda];
    for (int c = tid; c < nrhs; c += kLsThreads) {
      double* t = A + (int64_t)(nc + c) * lda;
      const double z = t[i] / uii;
      t[i] = z;
      Z[i + (int64_t)c * ldz] = z;
    }
    __syncthreads();
    for (int e = tid; e < i * nrhs; e += kLsThreads) {
      const int r = e % i, c = e / i;
      double* t = A + (int64_t)(nc + c) * lda;
      t[r] = fma(-A[r + (int64_t)i * lda], t[i], t[r]);
    }
    __syncthreads();
  }
}

hipError_t launch_hess_ls(double* A, int64_t lda, int nr, int nc, int nrhs, int band, double* Z,
                          int64_t ldz, double* resid, hipStream_t st) {
  hipLaunchKernelGGL(hess_ls_kernel, dim3(1), dim3(kLsThreads), 0, st, A, lda, nr, nc, nrhs, band,
                     Z, ldz, resid);
  return hipGetLastError();
}

// X (n x bs, FP64) += Q (n x N, storage T) Z (N x bs, FP64); one row per thread,
// Z staged in LDS in chunks.
template <typename T>
__global__ __launch_bounds__(256) void gemm_update_kernel(int64_t n, int N, int bs,
                                                          const T* __restrict__ Q, int64_t ldq,
                                                          const double* __restrict__ Z,
                                                          int64_t ldz, double* __restrict__ X,
                                                          int64_t ldx) {
  constexpr int CH = 64;
  __shared__ double zs[CH * 32];
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = row < n;
  const int64_t rr = ok ? row : n - 1;
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int j0 = 0; j0 < N; j0 += CH) {
    const int jc = min(CH, N - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < CH * 32; e += blockDim.x) {
      const int j = e % CH, c = e / CH;
      const bool in = j < jc && c < bs;
      const double z = Z[in ? (j0 + j) + (int64_t)c * ldz : 0];
      zs[e] = in ? z : 0.0;
    }
    __syncthreads();
    // eight columns of Q per pass, loads issued together (rows of zs past jc
    // are zero, so the clamped extra loads add nothing)
    for (int j = 0; j < jc; j += 8) {
      double q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = (double)Q[rr + (int64_t)(j0 + min(j + u, jc - 1)) * ldq];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int jj = min(j + u, CH - 1);
        const double qu = j + u < jc ? q[u] : 0.0;
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] = fma(qu, zs[jj + c * CH], acc[c]);
      }
    }
  }
  double x[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) x[c] = X[rr + (int64_t)(c < bs ? c : 0) * ldx];
  if (ok) {
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c < bs) X[row + (int64_t)c * ldx] = x[c] + acc[c];
  }
}

hipError_t launch_gemm_update(bool f32, int64_t n, int N, int bs, const void* Q, int64_t ldq,
                              const double* Z, int64_t ldz, double* X, int64_t ldx,
                              hipStream_t st) {
  if (bs < 1 || bs > 32) return hipErrorInvalidValue;
  dim3 grid((unsigned)ceil_div(n, 256));
  if (f32)
    hipLaunchKernelGGL(gemm_update_kernel<float>, grid, dim3(256), 0, st, n, N, bs,
                       (const float*)Q, ldq, Z, ldz, X, ldx);
  else
    hipLaunchKernelGGL(gemm_update_kernel<double>, grid, dim3(256), 0, st, n, N, bs,
                       (const double*)Q, ldq, Z, ldz, X, ldx);
  return hipGetLastError();
}

// partial[g] = sum of x^2 over a fixed grid-stride set of entries of the
// n x bs column-major FP64 X (ld ldx); then out = sum_g partial[g] in order.
constexpr int kSsGroups = 512;

__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ X, int64_t ldx,
                                                    int64_t n, int bs, double* __restrict__ part) {
  __shared__ double w[4];
  double acc = 0.0;
  const int64_t total = n * bs;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const double v = X[(idx % n) + (idx / n) * ldx];
    acc = fma(v, v, acc);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((w[0] + w[1]) + w[2]) + w[3];
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int G, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += part[g];
    *out = s;
  }
}

size_t sumsq_scratch() { return kSsGroups; }

hipError_t launch_sumsq(const double* X, int64_t ldx, int64_t n, int bs, double* scratch,
                        double* out, hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(kSsGroups), dim3(256), 0, st, X, ldx, n, bs, scratch);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, st, scratch, kSsGroups, out);
  return hipGetLastError();
}

// Y (store) = X (FP64), n x bs
template <typename T>
__global__ void convert_kernel(const double* __restrict__ X, int64_t ldx, int64_t n, int bs,
                               T* __restrict__ Y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * bs) return;
  const int64_t r = idx % n, c = idx / n;
  Y[r + c * ldy] = (T)X[r + c * ldx];
}

hipError_t launch_convert(const double* X, int64_t ldx, int64_t n, int bs, bool f32, void* Y,
                          int64_t ldy, hipStream_t st) {
  dim3 grid((unsigned)ceil_div(n * bs, 256));
  if (f32)
    hipLaunchKernelGGL(convert_kernel<float>, grid, dim3(256), 0, st, X, ldx, n, bs, (float*)Y, ldy);
  else
    hipLaunchKernelGGL(convert_kernel<double>, grid, dim3(256), 0, st, X, ldx, n, bs, (double*)Y,
                       ldy);
  return hipGetLastError();
}

}  // namespace rbgs
