// Small FP64 factors of Algorithm RBGS (k-dimensional work):
//  * Richardson sweeps for the sketched least-squares problem of step 2
//    (supplement SM.1): Y <- Y + S^T (P - S Y), built from two kernels,
//    Y (+)= S^T E and E = P - S Y;
//  * the residual sketch S'_(i) = P_(i) - S_(1:i-1) R_(1:i-1,i) of RCholeskyQR
//    with postponed sketching (Section 2.2.3) -- the same E = P - S Y kernel;
//  * R_(i,i) = R factor of the l2 (Householder) QR of S'_(i) with positive
//    diagonal (Sections 2.2.2 and 2.2.3), as a tree of Householder QRs of row
//    chunks held in LDS (the R factor of a stack of R factors is the R factor
//    of the whole matrix, up to row signs);
//  * the certificates of step 6, Delta = ||I - S^T S||_F and
//    Delta~ = ||P - S R||_F / ||P||_F.
// Every reduction runs in a fixed order.
#include "rbgs_internal.h"

namespace rbgs {

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Householder QR of a chunk held in LDS.
// ---------------------------------------------------------------------------
constexpr int kQrThreads = 256;
constexpr int kQrLds = 4096;  // doubles of LDS for the chunk (32 KB)
constexpr int kQrMaxB = 32;

__device__ __forceinline__ int qr_chunk_rows(int bw) {
  // rows per chunk: as many as fit in LDS, at least 2*bw so the tree shrinks
  return kQrLds / bw;
}

// In-place Householder triangularization of A (rows x bw, column-major, ld
// rows) in LDS.  For column j: x = A[j:, j], alpha = -sign(x_0) ||x||,
// v = x - alpha e_1, and every later column is updated as
// a_c -= beta (v^T a_c) v with beta = 2 / (v^T v) = 1 / (||x|| (||x|| + |x_0|)).
// All dots d_c = x^T a_c (c >= j; d_j = ||x||^2) come from one reduction pass:
// thread (c, g) sums rows g, g + NG, g + 2 NG, ... of column c and the NG
// threads of a column reduce by shuffles; then v^T a_c = d_c + (v_0 - x_0) a_jc.
// On return the upper triangle holds R (a zero column gives R_jj = 0 and no
// reflection).
template <int BWP>
__device__ void householder_lds(double* A, int rows, int bw, double* red /* [kQrMaxB+1] */) {
  constexpr int NG = (kQrThreads / BWP) < 64 ? (kQrThreads / BWP) : 64;  // threads per column
  const int tid = threadIdx.x;
  const int c = tid / NG, g = tid % NG;
  const bool active = tid < BWP * NG;
  __shared__ double sc[4];  // alpha, beta, v0 - x0, flag
  for (int j = 0; j < bw && j < rows; ++j) {
    double d = 0.0;
    if (active && c >= j && c < bw) {
      const double* aj = A + j * rows;
      const double* ac = A + c * rows;
      for (int r = j + g; r < rows; r += NG) d = fma(aj[r], ac[r], d);
    }
#pragma unroll
    for (int o = 1; o < NG; o <<= 1) d += __shfl_xor(d, o, 64);
    if (active && g == 0 && c < bw) red[c] = d;
    // a_jc for this thread's column, read before any thread updates column c
    const double ajc = (active && c > j && c < bw) ? A[j + c * rows] : 0.0;
    __syncthreads();
    if (tid == 0) {
      const double sigma = red[j];
      const double x0 = A[j + j * rows];
      if (sigma == 0.0) {
        sc[0] = 0.0;
        sc[1] = 0.0;
        sc[2] = 0.0;
      } else {
        const double nrm = sqrt(sigma);
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        sc[0] = alpha;
        sc[1] = 1.0 / (nrm * (nrm + fabs(x0)));
        sc[2] = -alpha;  // v0 - x0
        A[j + j * rows] = x0 - alpha;  // v_0
      }
    }
    __syncthreads();
    const double beta = sc[1];
    if (beta != 0.0 && active && c > j && c < bw) {
      // w_c = v^T a_c = d_c + (v0 - x0) a_jc
      double* ac = A + c * rows;
      const double* v = A + j * rows;
      const double w = beta * (red[c] + sc[2] * ajc);
      for (int r = j + g; r < rows; r += NG) ac[r] = fma(-w, v[r], ac[r]);
    }
    __syncthreads();
    if (tid == 0) A[j + j * rows] = sc[0];
    // (the next iteration's reads of column j+1 start after the barrier above;
    //  A[j][j] is not read again in this factorization)
  }
  __syncthreads();
}

// One chunk of one level of the tree: chunk b of `src` (rows_in x bw, ld ld_in)
// -> its R factor (bw x bw) at rows [b*bw, b*bw+bw) of `dst` (ld ld_out).  With
// final != 0 there is one chunk and R goes to the output with a positive
// diagonal, zeros below it, and a breakdown check.  A: kQrLds doubles of LDS.
__device__ void qr_chunk(const double* __restrict__ src, int64_t ld_in, int64_t rows_in, int bw,
                         double* __restrict__ dst, int64_t ld_out, int final, int64_t* flag,
                         int64_t col0, int64_t b, double* A, double* red) {
  const int CH = qr_chunk_rows(bw);
  const int64_t r0 = b * CH;
  const int rows = (int)min((int64_t)CH, rows_in - r0);
  const int rows_p = max(rows, bw);  // pad short chunks with zero rows
  // element e = r + c rows_p of the padded chunk; every load is issued before
  // the first is used (clamped index, then select)
  constexpr int PER = kQrLds / kQrThreads;
  const int tot = rows_p * bw;
  double v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * kQrThreads;
    const int r = e % rows_p, c = e / rows_p;
    const bool ok = e < tot && r < rows;
    const double x = src[ok ? (r0 + r) + c * ld_in : 0];
    v[i] = ok ? x : 0.0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * kQrThreads;
    if (e < tot) A[e] = v[i];
  }
  __syncthreads();
  if (bw <= 4) householder_lds<4>(A, rows_p, bw, red);
  else if (bw <= 8) householder_lds<8>(A, rows_p, bw, red);
  else if (bw <= 16) householder_lds<16>(A, rows_p, bw, red);
  else householder_lds<32>(A, rows_p, bw, red);
  if (!final) {
    for (int e = threadIdx.x; e < bw * bw; e += kQrThreads) {
      const int r = e % bw, c = e / bw;
      dst[(b * bw + r) + c * ld_out] = r <= c ? A[r + c * rows_p] : 0.0;
    }
  } else {
    for (int e = threadIdx.x; e < bw * bw; e += kQrThreads) {
      const int r = e % bw, c = e / bw;
      const double d = A[r + r * rows_p];
      const double sgn = d < 0.0 ? -1.0 : 1.0;
      dst[r + c * ld_out] = r <= c ? sgn * A[r + c * rows_p] : 0.0;
    }
    if (threadIdx.x == 0 && flag != nullptr) {
      for (int j = 0; j < bw; ++j) {
        const double d = A[j + j * rows_p];
        if (!(d != 0.0) || !isfinite(d)) {
          atomicCAS((unsigned long long*)flag, (unsigned long long)(-1LL),
                    (unsigned long long)(col0 + j));
          break;
        }
      }
    }
  }
  __syncthreads();
}

size_t qr_stack_size(int64_t k, int bw) {
  const int64_t CH = kQrLds / bw;
  int64_t rows = k, total = 0;
  while (rows > CH) {
    const int64_t nch = ceil_div(rows, CH);
    total += nch * bw;
    rows = nch * bw;
  }
  return (size_t)total * bw + 1;
}

// ---------------------------------------------------------------------------
__global__ void zero_kernel(double* A, int64_t ld, int64_t rows, int64_t cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  A[(idx % rows) + (idx / rows) * ld] = 0.0;
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_zero(double* A, int64_t ld, int64_t rows, int64_t cols, hipStream_t st) {
  const int64_t total = rows * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, A, ld,
                     rows, cols);
  return hipGetLastError();
}

__global__ void set_u32_kernel(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_set_u32(unsigned* p, int n, unsigned v, hipStream_t st) {
  hipLaunchKernelGGL(set_u32_kernel, dim3((unsigned)ceil_div(n, 64)), dim3(64), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Least squares of step 2 by Richardson sweeps (supplement SM.1),
//   Y_1 = S^T P,   Y_{s+1} = Y_s + S^T (P - S Y_s) = Y_s + c - G Y_s,
// with c = S^T P and the Gram matrix G = S^T S of the sketch.  G is kept up to
// date block by block, so one pass over the k x K sketch per block gives both c
// and the new block column of G, and every further sweep only touches the
// K x K Gram matrix.  (Same iterates as the residual form in exact arithmetic;
// the limiting accuracy, u cond(S)^2, equals u up to the small factor
// (1 + Delta)^2 because S is nearly orthonormal.)
// ---------------------------------------------------------------------------

// out0[j][c] = sum_t S[t][j] X0[t][c] (c < n0), out1[j][c] = sum_t S[t][j] X1[t][c]
// (c < n1), j < K.  16 lanes per output (t strided by 16), shuffle reduction.
__global__ __launch_bounds__(256) void gram_sty_kernel(const double* __restrict__ S, int64_t k,
                                                       int64_t K, const double* __restrict__ X0,
                                                       int n0, const double* __restrict__ X1,
                                                       int n1, double* __restrict__ out0,
                                                       int64_t ldo0, double* __restrict__ out1,
                                                       int64_t ldo1, double* __restrict__ out1t,
                                                       int64_t ldo1t) {
  const int q = threadIdx.x & 15;
  const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;  // output index
  const int ncol = n0 + n1;
  const bool ok = o < K * ncol;
  const int64_t j = ok ? o % K : 0;
  const int col = ok ? (int)(o / K) : 0;
  const double* x = col < n0 ? X0 + (int64_t)col * k : X1 + (int64_t)(col - n0) * k;
  const double* sj = S + j * k;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t t = q;
  for (; t + 48 < k; t += 64) {
    a0 = fma(sj[t], x[t], a0);
    a1 = fma(sj[t + 16], x[t + 16], a1);
    a2 = fma(sj[t + 32], x[t + 32], a2);
    a3 = fma(sj[t + 48], x[t + 48], a3);
  }
  for (; t < k; t += 16) a0 = fma(sj[t], x[t], a0);
  double v = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) v += __shfl_xor(v, d, 64);
  if (ok && q == 0) {
    if (col < n0) {
      out0[j + (int64_t)col * ldo0] = v;
    } else {
      const int c = col - n0;
      out1[j + (int64_t)c * ldo1] = v;
      if (out1t) out1t[c + j * ldo1t] = v;  // symmetric half of the Gram matrix
    }
  }
}

// Ynew[j][c] = Y[j][c] + C[j][c] - sum_l G[j][l] Y[l][c].  4 lanes per output
// split l in quarters; lanes (jl, q) = (lane % 16, lane / 16) in each wave.
__global__ __launch_bounds__(256) void gram_sweep_kernel(const double* __restrict__ G, int64_t ldg,
                                                         int64_t K, const double* __restrict__ C,
                                                         const double* __restrict__ Y,
                                                         int64_t ldy, double* __restrict__ Ynew,
                                                         int64_t ldyn, int bw) {
  const int lane = threadIdx.x & 63;
  const int jl = lane & 15, q = lane >> 4;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;  // wave index
  const int64_t jblocks = (K + 15) / 16;
  const bool okw = w < jblocks * bw;
  const int64_t jb = okw ? w % jblocks : 0;
  const int c = okw ? (int)(w / jblocks) : 0;
  const int64_t j = jb * 16 + jl;
  const bool ok = okw && j < K;
  const int64_t jc = ok ? j : 0;
  const int64_t l0 = (K * q) / 4, l1 = (K * (q + 1)) / 4;
  const double* yc = Y + (int64_t)c * ldy;
  double a0 = 0.0, a1 = 0.0;
  int64_t l = l0;
  for (; l + 1 < l1; l += 2) {
    a0 = fma(G[jc + l * ldg], yc[l], a0);
    a1 = fma(G[jc + (l + 1) * ldg], yc[l + 1], a1);
  }
  if (l < l1) a0 = fma(G[jc + l * ldg], yc[l], a0);
  double v = a0 + a1;
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  if (ok && q == 0) Ynew[j + (int64_t)c * ldyn] = yc[j] + (C[j + (int64_t)c * K] - v);
}

// E[t][c] = P[t][c] - sum_j S[t][j] Y[j][c].  4 lanes per output split j in
// quarters; lanes (tl, q) = (lane % 16, lane / 16).
__global__ __launch_bounds__(256) void resid_kernel(const double* __restrict__ P,
                                                    const double* __restrict__ S, int64_t k,
                                                    int64_t K, const double* __restrict__ Y,
                                                    int64_t ldy, double* __restrict__ E, int bw) {
  const int lane = threadIdx.x & 63;
  const int tl = lane & 15, q = lane >> 4;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t tblocks = (k + 15) / 16;
  const bool okw = w < tblocks * bw;
  const int64_t tb = okw ? w % tblocks : 0;
  const int c = okw ? (int)(w / tblocks) : 0;
  const int64_t t = tb * 16 + tl;
  const bool ok = okw && t < k;
  const int64_t tc = ok ? t : 0;
  const int64_t j0 = (K * q) / 4, j1 = (K * (q + 1)) / 4;
  const double* yc = Y + (int64_t)c * ldy;
  double a0 = 0.0, a1 = 0.0;
  int64_t j = j0;
  for (; j + 1 < j1; j += 2) {
    a0 = fma(S[tc + j * k], yc[j], a0);
    a1 = fma(S[tc + (j + 1) * k], yc[j + 1], a1);
  }
  if (j < j1) a0 = fma(S[tc + j * k], yc[j], a0);
  double v = a0 + a1;
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  if (ok && q == 0) E[t + (int64_t)c * k] = P[t + (int64_t)c * k] - v;
}

__device__ __forceinline__ bool last_block_arrives(unsigned* counter, unsigned total) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == total - 1;
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// R_(i,i) (positive diagonal) of the k x bw matrix src (ld k): workgroup g
// factors chunk g in LDS; the last workgroup factors the stack of chunk R
// factors (all remaining levels of the tree) and writes R_(i,i).
__global__ __launch_bounds__(kQrThreads) void qr_fused_kernel(
    const double* __restrict__ src, int64_t k, int bw, double* __restrict__ stack,
    unsigned* counter, double* __restrict__ Rii, int64_t ldr, int64_t* flag, int64_t col0) {
  __shared__ double A[kQrLds];
  __shared__ double red[kQrMaxB + 1];
  const int CH = qr_chunk_rows(bw);
  const int64_t nch = (k + CH - 1) / CH;
  if (nch == 1) {
    qr_chunk(src, k, k, bw, Rii, ldr, 1, flag, col0, 0, A, red);
    return;
  }
  const int64_t ld1 = nch * bw;
  qr_chunk(src, k, k, bw, stack, ld1, 0, nullptr, 0, blockIdx.x, A, red);
  if (!last_block_arrives(counter, (unsigned)nch)) return;
  // remaining levels in this workgroup
  const double* lsrc = stack;
  int64_t ld_in = ld1, lrows = ld1;
  double* buf = stack + ld1 * bw;
  while (lrows > CH) {
    const int64_t n2 = (lrows + CH - 1) / CH;
    const int64_t out_rows = n2 * bw;
    for (int64_t b2 = 0; b2 < n2; ++b2)
      qr_chunk(lsrc, ld_in, lrows, bw, buf, out_rows, 0, nullptr, 0, b2, A, red);
    lsrc = buf;
    ld_in = out_rows;
    lrows = out_rows;
    buf += out_rows * bw;
  }
  qr_chunk(lsrc, ld_in, lrows, bw, Rii, ldr, 1, flag, col0, 0, A, red);
  if (threadIdx.x == 0) *counter = 0u;
}

hipError_t launch_gram_sty(const double* S, int64_t k, int64_t K, const double* X0, int n0,
                           const double* X1, int n1, double* out0, int64_t ldo0, double* out1,
                           int64_t ldo1, double* out1t, int64_t ldo1t, hipStream_t st) {
  const int64_t threads = K * (n0 + n1) * 16;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(gram_sty_kernel, dim3((unsigned)ceil_div(threads, 256)), dim3(256), 0, st, S,
                     k, K, X0, n0, X1, n1, out0, ldo0, out1, ldo1, out1t, ldo1t);
  return hipGetLastError();
}

hipError_t launch_gram_sweep(const double* G, int64_t ldg, int64_t K, const double* C,
                             const double* Y, int64_t ldy, double* Ynew, int64_t ldyn, int bw,
                             hipStream_t st) {
  const int64_t waves = ceil_div(K, 16) * bw;
  hipLaunchKernelGGL(gram_sweep_kernel, dim3((unsigned)ceil_div(waves * 64, 256)), dim3(256), 0, st,
                     G, ldg, K, C, Y, ldy, Ynew, ldyn, bw);
  return hipGetLastError();
}

hipError_t launch_resid(const double* P, const double* S, int64_t k, int64_t K, const double* Y,
                        int64_t ldy, double* E, int bw, hipStream_t st) {
  const int64_t waves = ceil_div(k, 16) * bw;
  hipLaunchKernelGGL(resid_kernel, dim3((unsigned)ceil_div(waves * 64, 256)), dim3(256), 0, st, P,
                     S, k, K, Y, ldy, E, bw);
  return hipGetLastError();
}

hipError_t launch_qr_fused(const double* src, int64_t k, int bw, double* stack, unsigned* counter,
                           double* Rii, int64_t ldr, int64_t* flag, int64_t col0, hipStream_t st) {
  if (bw > kQrMaxB) return hipErrorInvalidValue;
  const int64_t CH = kQrLds / bw;
  hipLaunchKernelGGL(qr_fused_kernel, dim3((unsigned)ceil_div(k, CH)), dim3(kQrThreads), 0, st, src,
                     k, bw, stack, counter, Rii, ldr, flag, col0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Certificates.
// ---------------------------------------------------------------------------
// scratch[a + m b] = (delta_ab - S_a . S_b)^2 ; one wave per (a, b)
__global__ __launch_bounds__(256) void gram_defect_kernel(const double* __restrict__ S, int64_t k,
                                                          int64_t m, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= m * m) return;
  const int64_t a = w % m, b = w / m;
  double acc = 0.0;
  for (int64_t t = lane; t < k; t += 64) acc = fma(S[t + a * k], S[t + b * k], acc);
  acc = wave_sum(acc);
  if (lane == 0) {
    const double d = (a == b ? 1.0 : 0.0) - acc;
    out[w] = d * d;
  }
}

// out[t + k c] = (P - S R)[t, c]^2 ; out2[t + k c] = P[t, c]^2
__global__ __launch_bounds__(256) void sketch_resid_kernel(const double* __restrict__ S,
                                                           const double* __restrict__ P,
                                                           const double* __restrict__ R,
                                                           int64_t ldr, int64_t k, int64_t m,
                                                           double* __restrict__ out,
                                                           double* __restrict__ out2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (t >= k) return;
  double acc = 0.0;
  for (int64_t j = 0; j <= c; ++j) acc = fma(S[t + j * k], R[j + c * ldr], acc);
  const double p = P[t + c * k];
  const double e = p - acc;
  out[t + c * k] = e * e;
  out2[t + c * k] = p * p;
}

__global__ __launch_bounds__(256) void finite_kernel(const double* __restrict__ S,
                                                     const double* __restrict__ R, int64_t ldr,
                                                     int64_t k, int64_t m,
                                                     double* __restrict__ out) {
  // out[idx] = 1 if the idx-th entry of S (k*m) or R (m*m) is not finite
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < k * m) {
    out[idx] = isfinite(S[idx]) ? 0.0 : 1.0;
  } else if (idx < k * m + m * m) {
    const int64_t e = idx - k * m;
    out[idx] = isfinite(R[(e % m) + (e / m) * ldr]) ? 0.0 : 1.0;
  }
}

// single workgroup, fixed order: out = sum of v[0..len)
__global__ __launch_bounds__(256) void sum_kernel(const double* __restrict__ v, int64_t len,
                                                  double* __restrict__ out) {
  __shared__ double part[4];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 256) acc += v[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((part[0] + part[1]) + part[2]) + part[3];
}

size_t cert_scratch_size(int64_t k, int64_t m) { return (size_t)(m * m + 2 * k * m + m * m); }

hipError_t launch_certificates(const double* S, const double* P, const double* R, int64_t ldr,
                               int64_t k, int64_t m, double* scratch, double* out,
                               hipStream_t st) {
  double* g = scratch;
  double* e = g + m * m;
  double* p2 = e + k * m;
  hipLaunchKernelGGL(gram_defect_kernel, dim3((unsigned)ceil_div(m * m, 4)), dim3(256), 0, st, S,
                     k, m, g);
  hipLaunchKernelGGL(sketch_resid_kernel, dim3((unsigned)ceil_div(k, 256), (unsigned)m), dim3(256),
                     0, st, S, P, R, ldr, k, m, e, p2);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, g, m * m, out + 0);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, e, k * m, out + 1);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, p2, k * m, out + 2);
  // non-finite entries: reuse the Gram area (already summed in stream order)
  double* fin = e;  // k*m + m*m entries fit in e .. p2 + k*m
  hipLaunchKernelGGL(finite_kernel, dim3((unsigned)ceil_div(k * m + m * m, 256)), dim3(256), 0, st,
                     S, R, ldr, k, m, fin);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, fin, k * m + m * m, out + 3);
  return hipGetLastError();
}

}  // namespace rbgs
