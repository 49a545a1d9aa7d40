// Device-side bodies of the small FP64 factors (least-squares products and
// sweeps, residual sketch, QR of a sketch in one workgroup) and the lane
// reductions they use, shared by the small-factor kernels and the persistent
// batch kernel.
#ifndef RBGS_SMALL_DEVICE_H
#define RBGS_SMALL_DEVICE_H

#include "rbgs_internal.h"

namespace rbgs {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Householder QR of a row chunk held in registers.
// ---------------------------------------------------------------------------
constexpr int kQrThreads = 256;
constexpr int kQrMaxB = 32;
#ifndef RBGS_QR_RPT
#define RBGS_QR_RPT 16
#endif
constexpr int kQrRpt = RBGS_QR_RPT;  // rows per thread in a chunk

// Columns padded to a power of two (>= 4); NG = 256 / BWP threads per column.
__host__ __device__ __forceinline__ int qr_bwp(int bw) {
  return bw <= 4 ? 4 : (bw <= 8 ? 8 : (bw <= 16 ? 16 : 32));
}
// Rows per chunk, NG * kQrRpt; always >= 4 bw, so every level of the tree
// shrinks the row count at least fourfold.
__host__ __device__ __forceinline__ int qr_chunk_rows(int bw) {
  return (kQrThreads / qr_bwp(bw)) * kQrRpt;
}

// Lane exchange within rows of 16 lanes by DPP (no LDS round trip), on the two
// halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16

// Sum over the NG consecutive lanes of a column group (NG a power of two, 8 <=
// NG <= 64).  Every lane ends with the same bits: each step adds a partner's
// partial sum of the same shape, and addition is commutative.
template <int NG>
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_double<kDppXor1>(v);
  v += dpp_double<kDppXor2>(v);
  v += dpp_double<kDppHalfMirror>(v);
  if (NG >= 16) v += dpp_double<kDppMirror>(v);
  if (NG >= 32) v += __shfl_xor(v, 16, 64);
  if (NG >= 64) v += __shfl_xor(v, 32, 64);
  return v;
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
// (c < n1), j < K.  One wave per output (t strided by 64), fixed reduction tree.
__device__ __forceinline__ void gram_sty_body(const double* __restrict__ S, int64_t k, int64_t K,
                                              const double* __restrict__ X0, int n0,
                                              const double* __restrict__ X1, int n1,
                                              double* __restrict__ out0, int64_t ldo0,
                                              double* __restrict__ out1, int64_t ldo1,
                                              double* __restrict__ out1t, int64_t ldo1t,
                                              int64_t bx) {
  const int lane = threadIdx.x & 63;
  const int64_t o = (bx * blockDim.x + threadIdx.x) >> 6;  // output index
  const int ncol = n0 + n1;
  const bool ok = o < K * ncol;
  const int64_t j = ok ? o % K : 0;
  const int col = ok ? (int)(o / K) : 0;
  const double* x = col < n0 ? X0 + (int64_t)col * k : X1 + (int64_t)(col - n0) * k;
  const double* sj = S + j * k;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t t = lane;
  for (; t + 192 < k; t += 256) {
    a0 = fma(sj[t], x[t], a0);
    a1 = fma(sj[t + 64], x[t + 64], a1);
    a2 = fma(sj[t + 128], x[t + 128], a2);
    a3 = fma(sj[t + 192], x[t + 192], a3);
  }
  for (; t < k; t += 64) a0 = fma(sj[t], x[t], a0);
  const double v = group_sum<64>((a0 + a1) + (a2 + a3));
  if (ok && lane == 0) {
    if (col < n0) {
      out0[j + (int64_t)col * ldo0] = v;
    } else {
      const int c = col - n0;
      out1[j + (int64_t)c * ldo1] = v;
      if (out1t) out1t[c + j * ldo1t] = v;  // symmetric half of the Gram matrix
    }
  }
}

// Ynew[j][c] = Y[j][c] + C[j][c] - sum_l G[j][l] Y[l][c], reading row j of the
// symmetric G as its column j (both halves are stored), so both operands of
// the dot are contiguous.  16 lanes per output (l strided by 16).
__device__ __forceinline__ void gram_sweep_body(const double* __restrict__ G, int64_t ldg,
                                                int64_t K, const double* __restrict__ C,
                                                const double* __restrict__ Y, int64_t ldy,
                                                double* __restrict__ Ynew, int64_t ldyn, int bw,
                                                int64_t bx) {
  const int q = threadIdx.x & 15;
  const int64_t o = (bx * blockDim.x + threadIdx.x) >> 4;
  const bool ok = o < K * bw;
  const int64_t j = ok ? o % K : 0;
  const int c = ok ? (int)(o / K) : 0;
  const double* gj = G + j * ldg;
  const double* yc = Y + (int64_t)c * ldy;
  double a0 = 0.0, a1 = 0.0;
  int64_t l = q;
  for (; l + 16 < K; l += 32) {
    a0 = fma(gj[l], yc[l], a0);
    a1 = fma(gj[l + 16], yc[l + 16], a1);
  }
  for (; l < K; l += 16) a0 = fma(gj[l], yc[l], a0);
  const double v = group_sum<16>(a0 + a1);
  if (ok && q == 0) Ynew[j + (int64_t)c * ldyn] = yc[j] + (C[j + (int64_t)c * K] - v);
}

// E[t][c] = P[t][c] - sum_j S[t][j] Y[j][c].  16 lanes per output split j
// (strided by 16); lane = q + 16 tl covers rows t = 4 tb + tl.
__device__ __forceinline__ void resid_body(const double* __restrict__ P,
                                           const double* __restrict__ S, int64_t k, int64_t K,
                                           const double* __restrict__ Y, int64_t ldy,
                                           double* __restrict__ E, int bw, int64_t bx) {
  const int q = threadIdx.x & 15;
  const int64_t o = (bx * blockDim.x + threadIdx.x) >> 4;  // output index
  const bool ok = o < k * bw;
  const int64_t t = ok ? o % k : 0;
  const int c = ok ? (int)(o / k) : 0;
  const double* yc = Y + (int64_t)c * ldy;
  double a0 = 0.0, a1 = 0.0;
  int64_t j = q;
  for (; j + 16 < K; j += 32) {
    a0 = fma(S[t + j * k], yc[j], a0);
    a1 = fma(S[t + (j + 16) * k], yc[j + 16], a1);
  }
  for (; j < K; j += 16) a0 = fma(S[t + j * k], yc[j], a0);
  const double v = group_sum<16>(a0 + a1);
  if (ok && q == 0) E[t + (int64_t)c * k] = P[t + (int64_t)c * k] - v;
}

// The same E, NC columns per group of 16 lanes (columns NC cc .. NC cc + NC - 1
// of row t): one read of S[t][j] serves NC outputs.  Every output sees the
// operations of resid_body in the same order, so the results are identical.
template <int NC>
__device__ __forceinline__ void resid_cols_body(const double* __restrict__ P,
                                                const double* __restrict__ S, int64_t k,
                                                int64_t K, const double* __restrict__ Y,
                                                int64_t ldy, double* __restrict__ E, int bw,
                                                int64_t bx) {
  const int q = threadIdx.x & 15;
  const int64_t o = (bx * blockDim.x + threadIdx.x) >> 4;
  const int ncc = (bw + NC - 1) / NC;
  const bool ok = o < k * ncc;
  const int64_t t = ok ? o % k : 0;
  const int c0 = ok ? (int)(o / k) * NC : 0;
  const double* yc[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) yc[i] = Y + (int64_t)min(c0 + i, bw - 1) * ldy;  // clamped
  double a0[NC], a1[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) a0[i] = a1[i] = 0.0;
  int64_t j = q;
  for (; j + 16 < K; j += 32) {
    const double s0 = S[t + j * k], s1 = S[t + (j + 16) * k];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      a0[i] = fma(s0, yc[i][j], a0[i]);
      a1[i] = fma(s1, yc[i][j + 16], a1[i]);
    }
  }
  for (; j < K; j += 16) {
    const double s0 = S[t + j * k];
#pragma unroll
    for (int i = 0; i < NC; ++i) a0[i] = fma(s0, yc[i][j], a0[i]);
  }
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    const double v = group_sum<16>(a0[i] + a1[i]);
    const int c = c0 + i;
    if (ok && q == 0 && c < bw) E[t + (int64_t)c * k] = P[t + (int64_t)c * k] - v;
  }
}

// ---------------------------------------------------------------------------
// R_(i,i) of a k x bw sketch with k <= 1024 and bw <= 16 CPW in one workgroup
// of 16 waves: wave w keeps columns w + 16 q (q < CPW) in registers (lane l
// holds rows l + 64 i), so every reduction is within one wave (DPP inside rows
// of 16 lanes, then the four row sums read as scalars and added in a fixed
// order: every lane gets the same bits).  Householder steps as in
// qr_chunk_reg: column j and its squared norm are published through LDS
// (double-buffered), one barrier per column.
// ---------------------------------------------------------------------------
constexpr int kQwThreads = 1024;

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_total(double v) {
  v = group_sum<16>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

template <int RPT, int CPW = 1>
struct QwLds {
  double xb[2 * 64 * RPT];
  double sg[2];
  double diag[16 * CPW];
};

template <int RPT, int CPW = 1>
__device__ __forceinline__ void qr_wave_body(const double* __restrict__ src, int64_t k, int bw,
                                             double* __restrict__ Rii, int64_t ldr, int64_t* flag,
                                             int64_t col0, QwLds<RPT, CPW>& L) {
  constexpr int CH = 64 * RPT;
  double* xb = L.xb;
  double* sg = L.sg;
  double* diag = L.diag;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a[CPW][RPT];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 16 * q;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t r = lane + 64 * i;
      const bool ok = c < bw && r < k;
      const double v = src[ok ? r + (int64_t)c * k : 0];
      a[q][i] = ok ? v : 0.0;
    }
  }
  if (w == 0) {
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      xb[lane + 64 * i] = a[0][i];
      s2 = fma(a[0][i], a[0][i], s2);
    }
    s2 = wave_total(s2);
    if (lane == 0) sg[0] = s2;
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
    // the wave's columns right of j (wave-uniform): the reflector is read once
    // for all of them
    bool right = false;
#pragma unroll
    for (int q = 0; q < CPW; ++q) right |= w + 16 * q > j && w + 16 * q < bw;
    if (right && beta != 0.0) {
      // rows lane + 64 i with i >= 1 are >= 64 > j: only i = 0 needs the mask
      auto vi = [&](int i) {
        const double x = xj[lane + 64 * i];
        return i > 0 ? x : (lane < j ? 0.0 : (lane == j ? v0 : x));
      };
      // one column per wave: the reflector is held in registers; with more,
      // it is read from LDS again for each use (register budget)
      double v[CPW == 1 ? RPT : 1];
      if constexpr (CPW == 1) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) v[i] = vi(i);
      }
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        const int c = w + 16 * q;
        if (c > j && c < bw) {
          double d0 = 0.0, d1 = 0.0;
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const double vv = CPW == 1 ? v[CPW == 1 ? i : 0] : vi(i);
            if (i & 1) d1 = fma(vv, a[q][i], d1);
            else d0 = fma(vv, a[q][i], d0);
          }
          const double wt = beta * wave_total(d0 + d1);
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const double vv = CPW == 1 ? v[CPW == 1 ? i : 0] : vi(i);
            a[q][i] = fma(-wt, vv, a[q][i]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = w + 16 * q;
      if (c == j && lane == j) a[q][0] = sigma != 0.0 ? alpha : 0.0;
      if (c == j + 1 && c < bw) {
        double* xn = xb + ((j + 1) & 1) * CH;
        double s2 = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          xn[lane + 64 * i] = a[q][i];
          if (i > 0 || lane > j) s2 = fma(a[q][i], a[q][i], s2);
        }
        s2 = wave_total(s2);
        if (lane == 0) sg[(j + 1) & 1] = s2;
      }
    }
    __syncthreads();
  }
  // R_(r,c), r <= c < bw, sits in lane r of the wave holding column c (i = 0)
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 16 * q;
    if (c < bw && lane == c) diag[c] = a[q][0];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 16 * q;
    if (c < bw && lane < bw) {
      const double sgn = diag[lane] < 0.0 ? -1.0 : 1.0;
      Rii[lane + (int64_t)c * ldr] = lane <= c ? sgn * a[q][0] : 0.0;
    }
  }
  if (threadIdx.x == 0 && flag != nullptr) {
    for (int j = 0; j < bw; ++j) {
      const double d = diag[j];
      if (!(d != 0.0) || !isfinite(d)) {
        atomicCAS((unsigned long long*)flag, (unsigned long long)(-1LL),
                  (unsigned long long)(col0 + j));
        break;
      }
    }
  }
}

// The same factorization (bw <= 16, k <= 64 RPT) by the NW waves of one
// workgroup (NW = 4 or 8; the update launch's first workgroup computes R_(i,i)
// this way while the others start their products): wave w keeps columns
// w + NW q (q < 16 / NW) and, in each step, the reflector in registers.  Every
// column sees the same operations in the same order as in qr_wave_body (dot
// product split by row parity, one wave_total, one fma per entry).
template <int RPT>
struct QwNLds {
  double xb[2 * 64 * RPT];
  double sg[2];
  double diag[16];
};

template <int RPT, int NW>
__device__ __forceinline__ void qr_waven_body(const double* __restrict__ src, int64_t k, int bw,
                                              double* __restrict__ Rii, int64_t ldr, int64_t* flag,
                                              int64_t col0, QwNLds<RPT>& L) {
  constexpr int CH = 64 * RPT;
  constexpr int CPW = 16 / NW;
  static_assert(NW * CPW == 16, "16 columns over the waves");
  double* xb = L.xb;
  double* sg = L.sg;
  double* diag = L.diag;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a[CPW][RPT];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + NW * q;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t r = lane + 64 * i;
      const bool ok = c < bw && r < k;
      const double v = src[ok ? r + (int64_t)c * k : 0];
      a[q][i] = ok ? v : 0.0;
    }
  }
  if (w == 0) {
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      xb[lane + 64 * i] = a[0][i];
      s2 = fma(a[0][i], a[0][i], s2);
    }
    s2 = wave_total(s2);
    if (lane == 0) sg[0] = s2;
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
    bool right = false;
#pragma unroll
    for (int q = 0; q < CPW; ++q) right |= w + NW * q > j && w + NW * q < bw;
    if (right && beta != 0.0) {
      double v[RPT];
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const double x = xj[lane + 64 * i];
        v[i] = i > 0 ? x : (lane < j ? 0.0 : (lane == j ? v0 : x));
      }
      double d[CPW];
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          if (i & 1) d1 = fma(v[i], a[q][i], d1);
          else d0 = fma(v[i], a[q][i], d0);
        }
        d[q] = d0 + d1;
      }
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        const int c = w + NW * q;
        if (c > j && c < bw) {
          const double wt = beta * wave_total(d[q]);
#pragma unroll
          for (int i = 0; i < RPT; ++i) a[q][i] = fma(-wt, v[i], a[q][i]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = w + NW * q;
      if (c == j && lane == j) a[q][0] = sigma != 0.0 ? alpha : 0.0;
      if (c == j + 1 && c < bw) {
        double* xn = xb + ((j + 1) & 1) * CH;
        double s2 = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          xn[lane + 64 * i] = a[q][i];
          if (i > 0 || lane > j) s2 = fma(a[q][i], a[q][i], s2);
        }
        s2 = wave_total(s2);
        if (lane == 0) sg[(j + 1) & 1] = s2;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + NW * q;
    if (c < bw && lane == c) diag[c] = a[q][0];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + NW * q;
    if (c < bw && lane < bw) {
      const double sgn = diag[lane] < 0.0 ? -1.0 : 1.0;
      Rii[lane + (int64_t)c * ldr] = lane <= c ? sgn * a[q][0] : 0.0;
    }
  }
  if (threadIdx.x == 0 && flag != nullptr) {
    for (int j = 0; j < bw; ++j) {
      const double d = diag[j];
      if (!(d != 0.0) || !isfinite(d)) {
        atomicCAS((unsigned long long*)flag, (unsigned long long)(-1LL),
                  (unsigned long long)(col0 + j));
        break;
      }
    }
  }
}

}  // namespace rbgs

#endif  // RBGS_SMALL_DEVICE_H
