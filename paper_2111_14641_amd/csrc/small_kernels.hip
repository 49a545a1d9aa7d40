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
#include "small_device.h"

namespace rbgs {

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// R factor of chunk b of src (rows_in x bw, ld ld_in): rows [b CH, b CH + CH).
// Thread (c, g) = (tid / NG, tid % NG) keeps rows g + NG i (i < RPT) of column
// c in registers.  Householder step j: x = rows j.. of column j,
// alpha = -sign(x_0) ||x||, v = x - alpha e_j, beta = 1 / (||x|| (||x|| + |x_0|)),
// and every later column becomes a_c - beta (v^T a_c) v.  Column j and its
// squared norm are handed to all threads through LDS (double-buffered by the
// parity of j); the group owning column j + 1 publishes it right after its own
// update, so each step needs one barrier.  A zero column gives R_jj = 0 and no
// reflection.
//   final == 0: the bw x bw R goes to rows [b bw, b bw + bw) of dst (ld ld_out).
//   final != 0: R with a positive diagonal goes to dst; flag[0] gets the first
//               column col0 + j with a zero or non-finite R_jj.
template <typename T, int BWP, int RPT>
__device__ void qr_chunk_reg(const T* __restrict__ src, int64_t ld_in, int64_t rows_in,
                             int bw, double* __restrict__ dst, int64_t ld_out, int final,
                             int64_t* flag, int64_t col0, int64_t b, double* xb /* [2][NG*RPT] */,
                             double* sg /* [2 + kQrMaxB] */) {
  constexpr int NG = kQrThreads / BWP;
  constexpr int CH = NG * RPT;
  // rows g + NG i with i >= IM are >= NG IM >= bw > j: they never need a mask
  constexpr int IM0 = (BWP * BWP + kQrThreads - 1) / kQrThreads;
  constexpr int IM = IM0 < RPT ? IM0 : RPT;
  const int tid = threadIdx.x, c = tid / NG, g = tid % NG;
  const int64_t r0 = b * (int64_t)qr_chunk_rows(bw);
  const int rows = (int)min((int64_t)CH, rows_in - r0);
  const bool col_ok = c < bw;
  double a[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = g + NG * i;
    const bool ok = col_ok && r < rows;
    const double v = (double)src[ok ? (r0 + r) + (int64_t)c * ld_in : 0];
    a[i] = ok ? v : 0.0;
  }
  // publish column 0 and its squared norm
  if (c == 0) {
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      xb[g + NG * i] = a[i];
      s2 = fma(a[i], a[i], s2);
    }
    s2 = group_sum<NG>(s2);
    if (g == 0) sg[0] = s2;
  }
  __syncthreads();
  for (int j = 0; j < bw; ++j) {
    const double* xj = xb + (j & 1) * CH;
    const double sigma = sg[j & 1];
    const double x0 = xj[j];
    double alpha = 0.0, beta = 0.0, v0 = x0;
    if (sigma != 0.0) {
      const double nrm = sqrt(sigma);
      alpha = x0 >= 0.0 ? -nrm : nrm;
      beta = 1.0 / (nrm * (nrm + fabs(x0)));
      v0 = x0 - alpha;
    }
    if (c > j && col_ok && beta != 0.0) {
      double v[RPT];
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = g + NG * i;
        const double x = xj[r];
        v[i] = i >= IM ? x : (r < j ? 0.0 : (r == j ? v0 : x));
        if (i & 1) d1 = fma(v[i], a[i], d1);
        else d0 = fma(v[i], a[i], d0);
      }
      const double w = beta * group_sum<NG>(d0 + d1);
#pragma unroll
      for (int i = 0; i < RPT; ++i) a[i] = fma(-w, v[i], a[i]);
    }
    if (c == j) {
#pragma unroll
      for (int i = 0; i < IM; ++i)
        if (g + NG * i == j) a[i] = sigma != 0.0 ? alpha : 0.0;
    }
    if (c == j + 1 && col_ok) {
      // publish the next column (rows below j + 1 are masked by the reader)
      double* xn = xb + ((j + 1) & 1) * CH;
      double s2 = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = g + NG * i;
        xn[r] = a[i];
        if (i >= IM || r > j) s2 = fma(a[i], a[i], s2);
      }
      s2 = group_sum<NG>(s2);
      if (g == 0) sg[(j + 1) & 1] = s2;
    }
    __syncthreads();
  }
  // R: rows r < bw, held by g = r % NG, i = r / NG
  double* diag = sg + 2;
  if (final) {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (col_ok && g + NG * i == c) diag[c] = a[i];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = g + NG * i;
    if (col_ok && r < bw) {
      if (!final) {
        dst[(b * bw + r) + (int64_t)c * ld_out] = r <= c ? a[i] : 0.0;
      } else {
        const double sgn = diag[r] < 0.0 ? -1.0 : 1.0;
        dst[r + (int64_t)c * ld_out] = r <= c ? sgn * a[i] : 0.0;
      }
    }
  }
  if (final && threadIdx.x == 0 && flag != nullptr) {
    for (int j = 0; j < bw; ++j) {
      const double d = diag[j];
      if (!(d != 0.0) || !isfinite(d)) {
        atomicCAS((unsigned long long*)flag, (unsigned long long)(-1LL),
                  (unsigned long long)(col0 + j));
        break;
      }
    }
  }
  __syncthreads();
}

// Dispatch on the padded width; the final level of a tree uses fewer rows per
// thread when its input is short.
template <typename T>
__device__ void qr_chunk(const T* __restrict__ src, int64_t ld_in, int64_t rows_in, int bw,
                         double* __restrict__ dst, int64_t ld_out, int final, int64_t* flag,
                         int64_t col0, int64_t b, double* xb, double* sg) {
  const int bwp = qr_bwp(bw);
  const int ng = kQrThreads / bwp;
  const int64_t rows = rows_in - b * (int64_t)qr_chunk_rows(bw);
  const bool short4 = rows <= 4 * ng;
#define RBGS_QRC(BWP)                                                                            \
  if (short4)                                                                                    \
    qr_chunk_reg<T, BWP, 4>(src, ld_in, rows_in, bw, dst, ld_out, final, flag, col0, b, xb, sg); \
  else                                                                                           \
    qr_chunk_reg<T, BWP, kQrRpt>(src, ld_in, rows_in, bw, dst, ld_out, final, flag, col0, b, xb, sg);
  if (bwp == 4) { RBGS_QRC(4) }
  else if (bwp == 8) { RBGS_QRC(8) }
  else if (bwp == 16) { RBGS_QRC(16) }
  else { RBGS_QRC(32) }
#undef RBGS_QRC
}

// Stack of the tree levels: the larger of the one-group form (levels of
// re-chunked stacked rows) and the grouped form (level l holds n_l R factors,
// n_0 = chunks, n_(l+1) = ceil(n_l / FAN)).
size_t qr_stack_size(int64_t k, int bw) {
  const int64_t CH = qr_chunk_rows(bw);
  int64_t rows = k, total = 0;
  while (rows > CH) {
    const int64_t nch = ceil_div(rows, CH);
    total += nch * bw;
    rows = nch * bw;
  }
  int64_t tree = 0;
  const int64_t fan = CH / bw;
  for (int64_t n = ceil_div(k, CH); n > 1; n = ceil_div(n, fan)) tree += n * bw;
  return (size_t)std::max(total, tree) * bw + 1;
}

// ---------------------------------------------------------------------------
// Start of a factorization in one launch: R = 0 (m x m, ld ldr), the
// breakdown flag = -1 and ncnt arrival counters = 0.
__global__ void qr_init_kernel(double* R, int64_t ldr, int64_t m, int64_t* flag,
                               unsigned* counters, int ncnt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < m * m) R[(idx % m) + (idx / m) * ldr] = 0.0;
  if (idx == 0) *flag = -1;
  if (idx < ncnt) counters[idx] = 0u;
}
__global__ void set_i64_kernel(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_qr_init(double* R, int64_t ldr, int64_t m, int64_t* flag, unsigned* counters,
                          int ncnt, hipStream_t st) {
  const int64_t total = std::max<int64_t>(m * m, ncnt);
  hipLaunchKernelGGL(qr_init_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, R, ldr,
                     m, flag, counters, ncnt);
  return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void gram_sty_kernel(const double* __restrict__ S, int64_t k,
                                                       int64_t K, const double* __restrict__ X0,
                                                       int n0, const double* __restrict__ X1,
                                                       int n1, double* __restrict__ out0,
                                                       int64_t ldo0, double* __restrict__ out1,
                                                       int64_t ldo1, double* __restrict__ out1t,
                                                       int64_t ldo1t) {
  gram_sty_body(S, k, K, X0, n0, X1, n1, out0, ldo0, out1, ldo1, out1t, ldo1t, blockIdx.x);
}

// Lock-step batch (blockIdx.y = problem): c = S^T P_(i) into Cb (ld K) or
// R_(1:i-1,i), and the new Gram block from S_(i-1) (columns K - bprev ..).
__global__ __launch_bounds__(256) void gram_sty_batched_kernel(const BatchItem* items, int64_t k,
                                                               int64_t K, int bw, int bprev,
                                                               int64_t m, int to_cb) {
  const BatchItem& it = items[blockIdx.y];
  double* out0 = to_cb ? it.Cb : it.R + K * it.ldr;
  const int64_t ldo0 = to_cb ? K : it.ldr;
  gram_sty_body(it.S, k, K, it.P + K * k, bw, it.S + (K - bprev) * k, bprev, out0, ldo0,
                it.G + (K - bprev) * m, m, it.G + (K - bprev), m, blockIdx.x);
}

__global__ __launch_bounds__(256) void gram_sweep_kernel(const double* __restrict__ G, int64_t ldg,
                                                         int64_t K, const double* __restrict__ C,
                                                         const double* __restrict__ Y,
                                                         int64_t ldy, double* __restrict__ Ynew,
                                                         int64_t ldyn, int bw) {
  gram_sweep_body(G, ldg, K, C, Y, ldy, Ynew, ldyn, bw, blockIdx.x);
}

// Lock-step batch: buffers by role, 0 = Cb (ld K), 1 = Yb (ld K), 2 = R_(1:i-1,i).
__global__ __launch_bounds__(256) void gram_sweep_batched_kernel(const BatchItem* items, int64_t m,
                                                                 int64_t K, int bw, int src,
                                                                 int dst) {
  const BatchItem& it = items[blockIdx.y];
  const double* Y = src == 0 ? it.Cb : (src == 1 ? it.Yb : it.R + K * it.ldr);
  const int64_t ldy = src == 2 ? it.ldr : K;
  double* Yn = dst == 0 ? it.Cb : (dst == 1 ? it.Yb : it.R + K * it.ldr);
  const int64_t ldyn = dst == 2 ? it.ldr : K;
  gram_sweep_body(it.G, m, K, it.Cb, Y, ldy, Yn, ldyn, bw, blockIdx.x);
}

// NC columns per 16 lanes: 4 measured best for 16-column blocks (small
// factors 0.454 / 0.445 / 0.47 ms per QR at NC = 2 / 4 / 8, 0.477 with one
// column per 16 lanes; 16 leaves too few workgroups).
constexpr int kResidCols = 4;
template <int NC>
__global__ __launch_bounds__(256) void resid_cols_kernel(const double* __restrict__ P,
                                                         const double* __restrict__ S, int64_t k,
                                                         int64_t K, const double* __restrict__ Y,
                                                         int64_t ldy, double* __restrict__ E,
                                                         int bw) {
  resid_cols_body<NC>(P, S, k, K, Y, ldy, E, bw, blockIdx.x);
}

__global__ __launch_bounds__(256) void resid_batched_kernel(const BatchItem* items, int64_t k,
                                                            int64_t K, int bw) {
  const BatchItem& it = items[blockIdx.y];
  resid_body(it.P + K * k, it.S, k, K, it.R + K * it.ldr, it.ldr, it.E, bw, blockIdx.x);
}

// Arrival of a workgroup at a counter shared with total workgroups; true in
// the last one to arrive, which then sees every other workgroup's global
// writes.  Every wave first waits until its own stores have reached the L2;
// one thread then makes them visible device-wide (release: L2 write-back) and
// counts, and the last workgroup's waves acquire (L2 invalidate).  A
// device-scope fence in every wave would write back the L2 once per wave.
__device__ __forceinline__ bool last_block_arrives(unsigned* counter, unsigned total) {
  __shared__ bool last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    last = atomicAdd(counter, 1u) == total - 1;
  }
  __syncthreads();
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// Arrival counters the grouped tree needs for a k x bw sketch (0: one chunk),
// and the number of R factors one chunk of a tree level takes (FAN).
__host__ __device__ __forceinline__ int64_t qr_tree_fan(int bw) { return qr_chunk_rows(bw) / bw; }
__host__ __device__ __forceinline__ int64_t qr_tree_counters(int64_t k, int bw) {
  const int64_t fan = qr_tree_fan(bw);
  int64_t need = 0;
  for (int64_t n = (k + qr_chunk_rows(bw) - 1) / qr_chunk_rows(bw); n > 1; n = (n + fan - 1) / fan)
    need += (n + fan - 1) / fan;
  return need;
}

// R_(i,i) (positive diagonal) of the k x bw matrix src (ld k) by a Householder
// TSQR tree in one launch: workgroup g factors chunk g (level 0) and writes
// its R factor to the level-1 stack.  The R factors of a level are taken in
// groups of FAN (as many as one chunk holds); the last workgroup of a group
// to arrive (an arrival counter per group, reset to zero by that workgroup)
// factors the group's stacked R factors into one R of the next level, so the
// groups of a level proceed in parallel and the last arrival of the single
// group of the top level writes R_(i,i).  The critical path is one chunk
// factorization per level.  counters: ncnt zeroed counters; if the tree needs
// more, the last of all level-0 workgroups factors every further level
// itself (counters[0]).
__device__ __forceinline__ void qr_fused_body(const double* __restrict__ src, int64_t k, int bw,
                                              double* __restrict__ stack, unsigned* counters,
                                              int ncnt, double* __restrict__ Rii, int64_t ldr,
                                              int64_t* flag, int64_t col0, int64_t chunk) {
  __shared__ double xb[2 * (kQrThreads / 4) * kQrRpt];
  __shared__ double sg[2 + kQrMaxB];
  const int CH = qr_chunk_rows(bw);
  const int64_t nch = (k + CH - 1) / CH;
  if (nch == 1) {
    qr_chunk(src, k, k, bw, Rii, ldr, 1, flag, col0, 0, xb, sg);
    return;
  }
  const int64_t ld1 = nch * bw;
  qr_chunk(src, k, k, bw, stack, ld1, 0, nullptr, 0, chunk, xb, sg);
  if (qr_tree_counters(k, bw) <= ncnt) {
    const int64_t fan = qr_tree_fan(bw);
    const double* buf = stack;
    double* next = stack + ld1 * bw;
    int64_t ld = ld1, n = nch, pos = chunk;
    unsigned* cnt = counters;
    for (;;) {
      const int64_t ng = (n + fan - 1) / fan;  // groups (R factors of the next level)
      const int64_t g = pos / fan;
      const int64_t gs = min(fan, n - g * fan);
      if (!last_block_arrives(cnt + g, (unsigned)gs)) return;
      if (threadIdx.x == 0) cnt[g] = 0u;     // every other arrival has happened
      const double* gsrc = buf + g * fan * bw;
      if (ng == 1) {
        qr_chunk(gsrc, ld, gs * bw, bw, Rii, ldr, 1, flag, col0, 0, xb, sg);
        return;
      }
      const int64_t ld2 = ng * bw;
      qr_chunk(gsrc, ld, gs * bw, bw, next + g * bw, ld2, 0, nullptr, 0, 0, xb, sg);
      cnt += ng;
      buf = next;
      next += ld2 * bw;
      ld = ld2;
      n = ng;
      pos = g;
    }
  }
  if (!last_block_arrives(counters, (unsigned)nch)) return;
  // remaining levels in this workgroup
  const double* lsrc = stack;
  int64_t ld_in = ld1, lrows = ld1;
  double* buf = stack + ld1 * bw;
  while (lrows > CH) {
    const int64_t n2 = (lrows + CH - 1) / CH;
    const int64_t out_rows = n2 * bw;
    for (int64_t b2 = 0; b2 < n2; ++b2)
      qr_chunk(lsrc, ld_in, lrows, bw, buf, out_rows, 0, nullptr, 0, b2, xb, sg);
    lsrc = buf;
    ld_in = out_rows;
    lrows = out_rows;
    buf += out_rows * bw;
  }
  qr_chunk(lsrc, ld_in, lrows, bw, Rii, ldr, 1, flag, col0, 0, xb, sg);
  if (threadIdx.x == 0) *counters = 0u;
}

__global__ __launch_bounds__(kQrThreads) void qr_fused_kernel(
    const double* __restrict__ src, int64_t k, int bw, double* __restrict__ stack,
    unsigned* counters, int ncnt, double* __restrict__ Rii, int64_t ldr, int64_t* flag,
    int64_t col0) {
  qr_fused_body(src, k, bw, stack, counters, ncnt, Rii, ldr, flag, col0, blockIdx.x);
}

// Lock-step batch (blockIdx.y = problem): the Householder tree of S'_(i).
__global__ __launch_bounds__(kQrThreads) void qr_fused_batched_kernel(const BatchItem* items,
                                                                      int64_t k, int bw,
                                                                      int64_t c0) {
  const BatchItem& it = items[blockIdx.y];
  qr_fused_body(c0 == 0 ? it.P : it.E, k, bw, it.stack, it.counter, kQrTreeCounters,
                it.R + c0 + c0 * it.ldr, it.ldr, it.flag, c0, blockIdx.x);
}

// One level of a Householder TSQR tree over a tall rows_in x bw matrix:
// workgroup b factors chunk b.  Non-final levels stack the chunk R factors
// (rows [b bw, b bw + bw) of dst, ld ld_out); the final level (one chunk)
// writes R with a positive diagonal and raises the breakdown flag.
template <typename T>
__global__ __launch_bounds__(kQrThreads) void qr_level_kernel(
    const T* __restrict__ src, int64_t ld_in, int64_t rows_in, int bw, double* __restrict__ dst,
    int64_t ld_out, int final, int64_t* flag, int64_t col0) {
  __shared__ double xb[2 * (kQrThreads / 4) * kQrRpt];
  __shared__ double sg[2 + kQrMaxB];
  qr_chunk<T>(src, ld_in, rows_in, bw, dst, ld_out, final, flag, col0, blockIdx.x, xb, sg);
}

// R <- A R for upper triangular bw x bw A (ld lda) and R (ld ldr); only the
// upper triangles are read and written.  Entry (i, j) sums A_il R_lj for
// l = i..j in increasing l.
__global__ __launch_bounds__(1024) void trmm_upper_kernel(const double* __restrict__ A, int64_t lda,
                                                          double* __restrict__ R, int64_t ldr,
                                                          int bw) {
  const int i = threadIdx.x % kQrMaxB, j = threadIdx.x / kQrMaxB;
  const bool on = i < bw && j < bw && i <= j;
  double v = 0.0;
  if (on)
    for (int l = i; l <= j; ++l) v = fma(A[i + l * lda], R[l + j * ldr], v);
  __syncthreads();
  if (on) R[i + j * ldr] = v;
}

template <int RPT>
__global__ __launch_bounds__(kQwThreads) void qr_wave_kernel(const double* __restrict__ src,
                                                             int64_t k, int bw,
                                                             double* __restrict__ Rii, int64_t ldr,
                                                             int64_t* flag, int64_t col0) {
  __shared__ QwLds<RPT> lds;
  qr_wave_body<RPT>(src, k, bw, Rii, ldr, flag, col0, lds);
}

// Lock-step batch (blockIdx.x = problem): R_(i,i) of S'_(i) (E, or P_(1) for
// the first block).
template <int RPT>
__global__ __launch_bounds__(kQwThreads) void qr_wave_batched_kernel(const BatchItem* items,
                                                                     int64_t k, int bw,
                                                                     int64_t c0) {
  const BatchItem& it = items[blockIdx.x];
  __shared__ QwLds<RPT> lds;
  qr_wave_body<RPT>(c0 == 0 ? it.P : it.E, k, bw, it.R + c0 + c0 * it.ldr, it.ldr, it.flag, c0,
                    lds);
}

// Lock-step batch initialisation: R = 0 (m x m) and the breakdown flag.
__global__ void init_batched_kernel(const BatchItem* items, int64_t m) {
  const BatchItem& it = items[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < m * m) it.R[(idx % m) + it.ldr * (idx / m)] = 0.0;
  if (idx == 0) *it.flag = -1;
  if (idx < kQrTreeCounters) it.counter[idx] = 0u;
}

// ---------------------------------------------------------------------------
// Direct least squares of step 2 (Section 2.1): Householder QR of the sketch
// S_(1:i-1), kept up to date block by block in the form of LAPACK's geqrf (R
// on and above the diagonal of HS, the reflectors' vectors below it with a
// unit leading entry, their scalars in tau), so R_(1:i-1,i) = R_S^{-1}
// (H_(K-1) .. H_0 P_(i))[0:K].  FP64; one workgroup of 16 waves, each holding
// one or two columns of k <= 64 RPT rows in registers (lane l: rows l + 64 i).
// ---------------------------------------------------------------------------
constexpr int kHhMaxK = 1024;  // rows of the sketch and columns of S_(1:i-1)

// x <- H_j x for the column held in a[] (rows j.. of reflector j; v_j[j] = 1).
// The vector is read twice (for the dot product, then for the update; the
// second read hits the cache) rather than held, to keep the registers for the
// columns.
template <int RPT>
__device__ __forceinline__ void hh_reflect(double (&a)[RPT], const double* __restrict__ v,
                                           double t, int j, int k, int lane) {
  auto vi = [&](int i) {
    const int row = lane + 64 * i;
    const bool below = row > j && row < k;
    const double x = v[below ? row : j];
    return below ? x : (row == j ? 1.0 : 0.0);
  };
  double d0 = 0.0, d1 = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    if (i & 1) d1 = fma(vi(i), a[i], d1);
    else d0 = fma(vi(i), a[i], d0);
  }
  const double w = t * wave_total(d0 + d1);
#pragma unroll
  for (int i = 0; i < RPT; ++i) a[i] = fma(-w, vi(i), a[i]);
}

// New columns c0 .. c0 + bw - 1 of the sketch (Snew, k x bw, ld k) into the
// factorization: the reflectors 0 .. c0 - 1 applied to them, then their own
// Householder QR on rows c0 .. k - 1 (LAPACK's sign convention: beta =
// -sign(alpha) ||x||, tau = (beta - alpha) / beta, tau = 0 for a zero tail).
// Wave w holds columns w + 16 q, q < CPW (bw <= 16 CPW).
template <int RPT, int CPW>
__global__ __launch_bounds__(kQwThreads) void hh_absorb_kernel(const double* __restrict__ Snew,
                                                               int k, int c0, int bw,
                                                               double* HS, double* tau) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a[CPW][RPT];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 16 * q;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = lane + 64 * i;
      const bool ok = c < bw && row < k;
      const double x = Snew[ok ? row + (int64_t)c * k : 0];
      a[q][i] = ok ? x : 0.0;
    }
  }
  for (int j = 0; j < c0; ++j) {
    const double t = tau[j];
    if (t == 0.0) continue;
#pragma unroll
    for (int q = 0; q < CPW; ++q)
      if (w + 16 * q < bw) hh_reflect<RPT>(a[q], HS + (int64_t)j * k, t, j, k, lane);
  }
  for (int jj = 0; jj < bw; ++jj) {
    const int j = c0 + jj;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      if (w + 16 * q != jj) continue;  // the pivot column's wave
      double xs = 0.0, s2 = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int row = lane + 64 * i;
        if (row == j) xs = a[q][i];
        if (row > j && row < k) s2 = fma(a[q][i], a[q][i], s2);
      }
      const double alpha = wave_total(xs);   // one nonzero term: exact
      const double sigma = wave_total(s2);
      double beta = alpha, t = 0.0, scale = 0.0;
      if (sigma != 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, sigma));
        beta = alpha >= 0.0 ? -nrm : nrm;
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      double* col = HS + (int64_t)j * k;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int row = lane + 64 * i;
        if (row < k) col[row] = row < j ? a[q][i] : (row == j ? beta : a[q][i] * scale);
      }
      if (lane == 0) tau[j] = t;
    }
    __syncthreads();
    const double t = tau[j];
    if (t != 0.0) {
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        const int c = w + 16 * q;
        if (c < bw && c > jj) hh_reflect<RPT>(a[q], HS + (int64_t)j * k, t, j, k, lane);
      }
    }
  }
}

// Y (K x bw, ld ldy) = R_S^{-1} (H_(K-1) .. H_0 P)[0:K] for P (k x bw, ld k):
// wave w takes columns w, w + 16; the back substitution runs on the wave's
// column in LDS (y_r = c_r / R_rr, then c_l -= y_r R_lr for l < r).
template <int RPT>
__global__ __launch_bounds__(kQwThreads) void hh_solve_kernel(const double* __restrict__ HS,
                                                              const double* __restrict__ tau,
                                                              const double* __restrict__ P, int k,
                                                              int K, int bw, double* Y,
                                                              int64_t ldy) {
  __shared__ double cs[16][kHhMaxK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = w; c - w < bw; c += 16) {
    if (c >= bw) continue;  // wave-uniform
    double a[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = lane + 64 * i;
      const double x = P[(row < k ? row : 0) + (int64_t)c * k];
      a[i] = row < k ? x : 0.0;
    }
    for (int j = 0; j < K; ++j) {
      const double t = tau[j];
      if (t != 0.0) hh_reflect<RPT>(a, HS + (int64_t)j * k, t, j, k, lane);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = lane + 64 * i;
      if (row < K) cs[w][row] = a[i];
    }
    for (int r = K - 1; r >= 0; --r) {
      const double y = cs[w][r] / HS[r + (int64_t)r * k];
      const double* Rr = HS + (int64_t)r * k;
      for (int l = lane; l < r; l += 64) cs[w][l] = fma(-y, Rr[l], cs[w][l]);
      if (lane == 0) cs[w][r] = y;
    }
    for (int l = lane; l < K; l += 64) Y[l + (int64_t)c * ldy] = cs[w][l];
  }
}

bool hh_supported(int64_t k, int64_t K, int bw) {
  return k <= kHhMaxK && K <= kHhMaxK && K >= 0 && bw >= 1 && bw <= (k <= 512 ? 32 : 16);
}

hipError_t launch_hh_absorb(const double* Snew, int64_t k, int64_t c0, int bw, double* HS,
                            double* tau, hipStream_t st) {
  if (!hh_supported(k, c0, bw)) return hipErrorInvalidValue;
#define RBGS_HHA(R, C)                                                                           \
  hipLaunchKernelGGL((hh_absorb_kernel<R, C>), dim3(1), dim3(kQwThreads), 0, st, Snew, (int)k,   \
                     (int)c0, bw, HS, tau)
  if (k <= 256) RBGS_HHA(4, 2);
  else if (k <= 512) RBGS_HHA(8, 2);
  else RBGS_HHA(16, 1);
#undef RBGS_HHA
  return hipGetLastError();
}

hipError_t launch_hh_solve(const double* HS, const double* tau, const double* P, int64_t k,
                           int64_t K, int bw, double* Y, int64_t ldy, hipStream_t st) {
  if (!hh_supported(k, K, bw) || K < 1) return hipErrorInvalidValue;
#define RBGS_HHS(R)                                                                              \
  hipLaunchKernelGGL(hh_solve_kernel<R>, dim3(1), dim3(kQwThreads), 0, st, HS, tau, P, (int)k,    \
                     (int)K, bw, Y, ldy)
  if (k <= 256) RBGS_HHS(4);
  else if (k <= 512) RBGS_HHS(8);
  else RBGS_HHS(16);
#undef RBGS_HHS
  return hipGetLastError();
}

// Deterministic test matrix for the autotuner: x[r][c] = a hash of (r, c)
// mapped to [-1, 1) (full rank with overwhelming probability).
__global__ void fill_test_kernel(void* X, int f32, int64_t n, int64_t m, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t r = idx % n, c = idx / n;
  uint32_t h = (uint32_t)r * 0x9E3779B1u ^ ((uint32_t)c * 0x85EBCA77u + 0x165667B1u);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  const double v = (double)(h >> 8) * (1.0 / 8388608.0) - 1.0;
  if (f32) ((float*)X)[r + c * ld] = (float)v;
  else ((double*)X)[r + c * ld] = v;
}

hipError_t launch_fill_test(void* X, bool f32, int64_t n, int64_t m, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(fill_test_kernel, dim3((unsigned)ceil_div(n * m, 256)), dim3(256), 0, st, X,
                     f32 ? 1 : 0, n, m, ld);
  return hipGetLastError();
}

hipError_t launch_gram_sty(const double* S, int64_t k, int64_t K, const double* X0, int n0,
                           const double* X1, int n1, double* out0, int64_t ldo0, double* out1,
                           int64_t ldo1, double* out1t, int64_t ldo1t, hipStream_t st) {
  const int64_t threads = K * (n0 + n1) * 64;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(gram_sty_kernel, dim3((unsigned)ceil_div(threads, 256)), dim3(256), 0, st, S,
                     k, K, X0, n0, X1, n1, out0, ldo0, out1, ldo1, out1t, ldo1t);
  return hipGetLastError();
}

hipError_t launch_gram_sweep(const double* G, int64_t ldg, int64_t K, const double* C,
                             const double* Y, int64_t ldy, double* Ynew, int64_t ldyn, int bw,
                             hipStream_t st) {
  const int64_t threads = K * bw * 16;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(gram_sweep_kernel, dim3((unsigned)ceil_div(threads, 256)), dim3(256), 0, st,
                     G, ldg, K, C, Y, ldy, Ynew, ldyn, bw);
  return hipGetLastError();
}

hipError_t launch_resid(const double* P, const double* S, int64_t k, int64_t K, const double* Y,
                        int64_t ldy, double* E, int bw, hipStream_t st) {
  if (bw < 1 || K < 1) return hipErrorInvalidValue;
  const int64_t threads = k * ((bw + kResidCols - 1) / kResidCols) * 16;
  hipLaunchKernelGGL(resid_cols_kernel<kResidCols>, dim3((unsigned)ceil_div(threads, 256)),
                     dim3(256), 0, st, P, S, k, K, Y, ldy, E, bw);
  return hipGetLastError();
}

hipError_t launch_gram_sty_batched(const BatchItem* items, int nprob, int64_t k, int64_t K, int bw,
                                   int bprev, int64_t m, bool to_cb, hipStream_t st) {
  const int64_t threads = K * (bw + bprev) * 64;
  hipLaunchKernelGGL(gram_sty_batched_kernel, dim3((unsigned)ceil_div(threads, 256), (unsigned)nprob),
                     dim3(256), 0, st, items, k, K, bw, bprev, m, to_cb ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_sweep_batched(const BatchItem* items, int nprob, int64_t m, int64_t K, int bw,
                                int src, int dst, hipStream_t st) {
  const int64_t threads = K * bw * 16;
  hipLaunchKernelGGL(gram_sweep_batched_kernel, dim3((unsigned)ceil_div(threads, 256), (unsigned)nprob),
                     dim3(256), 0, st, items, m, K, bw, src, dst);
  return hipGetLastError();
}

hipError_t launch_resid_batched(const BatchItem* items, int nprob, int64_t k, int64_t K, int bw,
                                hipStream_t st) {
  const int64_t threads = k * bw * 16;
  hipLaunchKernelGGL(resid_batched_kernel, dim3((unsigned)ceil_div(threads, 256), (unsigned)nprob),
                     dim3(256), 0, st, items, k, K, bw);
  return hipGetLastError();
}

hipError_t launch_qr_batched(const BatchItem* items, int nprob, int64_t k, int bw, int64_t c0,
                             hipStream_t st) {
  if (bw > kQrMaxB) return hipErrorInvalidValue;
  if (bw > 16 || k > 1024) {
    const int64_t CH = qr_chunk_rows(bw);
    hipLaunchKernelGGL(qr_fused_batched_kernel, dim3((unsigned)ceil_div(k, CH), (unsigned)nprob),
                       dim3(kQrThreads), 0, st, items, k, bw, c0);
    return hipGetLastError();
  }
#define RBGS_QWB(R)                                                                            \
  hipLaunchKernelGGL(qr_wave_batched_kernel<R>, dim3((unsigned)nprob), dim3(kQwThreads), 0, st, \
                     items, k, bw, c0)
  if (k <= 256) RBGS_QWB(4);
  else if (k <= 512) RBGS_QWB(8);
  else RBGS_QWB(16);
#undef RBGS_QWB
  return hipGetLastError();
}

hipError_t launch_init_batched(const BatchItem* items, int nprob, int64_t m, hipStream_t st) {
  hipLaunchKernelGGL(init_batched_kernel, dim3((unsigned)ceil_div(m * m, 256), (unsigned)nprob),
                     dim3(256), 0, st, items, m);
  return hipGetLastError();
}

hipError_t launch_qr_fused(const double* src, int64_t k, int bw, double* stack, unsigned* counter,
                           double* Rii, int64_t ldr, int64_t* flag, int64_t col0, hipStream_t st) {
  if (bw > kQrMaxB) return hipErrorInvalidValue;
  if (bw <= 16 && k <= 1024) {
#define RBGS_QW(R)                                                                              \
  hipLaunchKernelGGL(qr_wave_kernel<R>, dim3(1), dim3(kQwThreads), 0, st, src, k, bw, Rii, ldr, \
                     flag, col0)
    if (k <= 256) RBGS_QW(4);
    else if (k <= 512) RBGS_QW(8);
    else RBGS_QW(16);
#undef RBGS_QW
    return hipGetLastError();
  }
  const int64_t CH = qr_chunk_rows(bw);
  hipLaunchKernelGGL(qr_fused_kernel, dim3((unsigned)ceil_div(k, CH)), dim3(kQrThreads), 0, st, src,
                     k, bw, stack, counter, kQrTreeCounters, Rii, ldr, flag, col0);
  return hipGetLastError();
}

hipError_t launch_qr_tall(bool f32, const void* src, int64_t ld, int64_t rows, int bw,
                          double* stack, double* R, int64_t ldr, int64_t* flag, int64_t col0,
                          hipStream_t st) {
  if (bw > kQrMaxB || bw < 1 || rows < bw) return hipErrorInvalidValue;
  const int64_t CH = qr_chunk_rows(bw);
  const int64_t nch = ceil_div(rows, CH);
  if (nch == 1) {
    if (f32)
      hipLaunchKernelGGL(qr_level_kernel<float>, dim3(1), dim3(kQrThreads), 0, st,
                         (const float*)src, ld, rows, bw, R, ldr, 1, flag, col0);
    else
      hipLaunchKernelGGL(qr_level_kernel<double>, dim3(1), dim3(kQrThreads), 0, st,
                         (const double*)src, ld, rows, bw, R, ldr, 1, flag, col0);
    return hipGetLastError();
  }
  int64_t out_rows = nch * bw;
  if (f32)
    hipLaunchKernelGGL(qr_level_kernel<float>, dim3((unsigned)nch), dim3(kQrThreads), 0, st,
                       (const float*)src, ld, rows, bw, stack, out_rows, 0, nullptr, 0);
  else
    hipLaunchKernelGGL(qr_level_kernel<double>, dim3((unsigned)nch), dim3(kQrThreads), 0, st,
                       (const double*)src, ld, rows, bw, stack, out_rows, 0, nullptr, 0);
  // the levels occupy consecutive parts of the stack (qr_stack_size(rows, bw))
  const double* lsrc = stack;
  int64_t lrows = out_rows;
  double* buf = stack + out_rows * bw;
  while (lrows > CH) {
    const int64_t n2 = ceil_div(lrows, CH);
    out_rows = n2 * bw;
    hipLaunchKernelGGL(qr_level_kernel<double>, dim3((unsigned)n2), dim3(kQrThreads), 0, st, lsrc,
                       lrows, lrows, bw, buf, out_rows, 0, nullptr, 0);
    lsrc = buf;
    lrows = out_rows;
    buf += out_rows * bw;
  }
  hipLaunchKernelGGL(qr_level_kernel<double>, dim3(1), dim3(kQrThreads), 0, st, lsrc, lrows, lrows,
                     bw, R, ldr, 1, flag, col0);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* A, int64_t lda, double* R, int64_t ldr, int bw,
                             hipStream_t st) {
  if (bw > kQrMaxB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trmm_upper_kernel, dim3(1), dim3(1024), 0, st, A, lda, R, ldr, bw);
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
