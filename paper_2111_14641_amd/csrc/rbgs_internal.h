// Internal declarations of the gfx950 RBGS library: device-side definition of
// the sketching operators and the host launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace rbgs {

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// words 0 and 2 by the two Philox multipliers, swaps the high halves across,
// and mixes in the key; the key advances by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ c in one gfx950 three-input bit operation (truth table 0x96: the
// parity of the three input bits, the same for every operand order)
__device__ __forceinline__ uint32_t xor3_u32(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3_u32((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = xor3_u32((uint32_t)(p0 >> 32), c3, k1);
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

constexpr uint32_t kTagGauss = 0x47415553u;
constexpr uint32_t kTagSparse = 0x53504152u;
constexpr uint32_t kTagRademacher = 0x52414445u;
constexpr uint32_t kTagSrht = 0x53524854u;

// fp32 constants by bit pattern (correctly rounded values of the named reals).
__device__ __forceinline__ float f32c(uint32_t b) { return __uint_as_float(b); }

// n / d correctly rounded, for the operands of gauss_ln_u24 only (d = f + 1 in
// [1.7, 2.5], n = f - 1: normal, far from overflow and underflow).  The steps
// of the IEEE single-precision division: reciprocal estimate, one Newton step,
// quotient, two residual corrections by fused multiply-add (Markstein).  The
// general division adds operand scaling and special-case fix-ups, which leave
// every value in this range unchanged; so the result is the IEEE quotient.
__device__ __forceinline__ float div_rn_gauss(float n, float d) {
  float r = __builtin_amdgcn_rcpf(d);
  r = fmaf(fmaf(-d, r, 1.0f), r, r);
  float q = n * r;
  q = fmaf(fmaf(-d, q, n), r, q);
  return fmaf(fmaf(-d, q, n), r, q);
}

// sqrt(x) correctly rounded for the radius argument x = -2 ln u of gauss_pair
// (u in [2^-24, 1 - 2^-24], so x in [1.1e-7, 33.3]: normal and positive).
// Hardware estimate, then the neighbour chosen by the sign of the residual
// x - s s' (Tuckerman's rounding test).  The general square root adds scaling
// of inputs below 2^-96 and special cases for 0, inf and NaN, none of which
// occur here; so the result is the IEEE square root.
__device__ __forceinline__ float sqrt_rn_gauss(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sm = __uint_as_float(__float_as_uint(s) - 1u);
  const float sp = __uint_as_float(__float_as_uint(s) + 1u);
  const float r = fmaf(-sm, s, x) <= 0.0f ? sm : s;
  return fmaf(-sp, s, x) > 0.0f ? sp : r;
}

// Natural logarithm of u = (2*(w >> 9) + 1) * 2^-24 in single precision:
// write N = 2*(w>>9)+1 = f * 2^e with f in [sqrt(2)/2, sqrt(2)], then
// ln u = (e - 24) ln 2 + 2 atanh(s), s = (f-1)/(f+1), using the odd series of
// atanh to s^9.  Each operation is one correctly rounded IEEE fp32 operation
// (no contraction), so the result is reproducible bit for bit.
__device__ __forceinline__ float gauss_ln_u24(uint32_t w) {
#pragma clang fp contract(off)
  const uint32_t N = ((w >> 9) << 1) | 1u;
  const uint32_t bits = __float_as_uint((float)N);
  int e = (int)((bits >> 23) & 0xFFu) - 127;
  float f = __uint_as_float((bits & 0x007FFFFFu) | 0x3F800000u);
  if (f > f32c(0x3FB504F3u)) {  // sqrt(2)
    f = f * 0.5f;
    e += 1;
  }
  const float s = div_rn_gauss(f - 1.0f, f + 1.0f);
  const float s2 = s * s;
  float p = f32c(0x3E124925u) + s2 * f32c(0x3DE38E39u);  // 1/7 + s2/9
  p = f32c(0x3E4CCCCDu) + s2 * p;                         // 1/5
  p = f32c(0x3EAAAAABu) + s2 * p;                         // 1/3
  const float t = 2.0f * s;
  const float lnf = t + t * (s2 * p);
  return (float)(e - 24) * f32c(0x3F317218u) + lnf;      // ln 2
}

// cos and sin of phi = (pi/2) (q + t), q = w >> 30, t = (2*((w>>7) & 0x7FFFFF)+1) 2^-24:
// Taylor polynomials of sin a (to a^13) and cos a (to a^14) at a = t * pi/2,
// Horner form, then q quarter turns.  Single-precision, no contraction.
__device__ __forceinline__ void gauss_sincos(uint32_t w, float& c, float& s) {
#pragma clang fp contract(off)
  const uint32_t q = w >> 30;
  const uint32_t v = (w >> 7) & 0x7FFFFFu;
  const float t = (float)(2u * v + 1u) * 5.9604644775390625e-08f;  // 2^-24
  const float a = t * f32c(0x3FC90FDBu);                             // pi/2
  const float a2 = a * a;
  float ps = f32c(0xB2D7322Bu) + a2 * f32c(0x2F309231u);  // -1/11! + a2/13!
  ps = f32c(0x3638EF1Du) + a2 * ps;                         //  1/9!
  ps = f32c(0xB9500D01u) + a2 * ps;                         // -1/7!
  ps = f32c(0x3C088889u) + a2 * ps;                         //  1/5!
  ps = f32c(0xBE2AAAABu) + a2 * ps;                         // -1/3!
  const float sa = a + (a * a2) * ps;
  float pc = f32c(0x310F76C7u) + a2 * f32c(0xAD49CBA5u);   //  1/12! - a2/14!
  pc = f32c(0xB493F27Eu) + a2 * pc;                         // -1/10!
  pc = f32c(0x37D00D01u) + a2 * pc;                         //  1/8!
  pc = f32c(0xBAB60B61u) + a2 * pc;                         // -1/6!
  pc = f32c(0x3D2AAAABu) + a2 * pc;                         //  1/4!
  pc = f32c(0xBF000000u) + a2 * pc;                         // -1/2
  const float ca = 1.0f + a2 * pc;
  // q quarter turns: (cos, sin) = (ca, sa), (-sa, ca), (-ca, -sa), (sa, -ca) for q = 0..3,
  // by selects and sign-bit flips (exact negation; a 4-way switch would run every path)
  const bool sw = (q & 1u) != 0u;
  const uint32_t cneg = ((q ^ (q >> 1)) & 1u) << 31;  // q = 1, 2
  const uint32_t sneg = (q >> 1) << 31;               // q = 2, 3
  c = __uint_as_float(__float_as_uint(sw ? sa : ca) ^ cneg);
  s = __uint_as_float(__float_as_uint(sw ? ca : sa) ^ sneg);
}

// Box-Muller: radius word wr, angle word wa -> (rho cos phi, rho sin phi).
__device__ __forceinline__ void gauss_pair(uint32_t wr, uint32_t wa, float& z0, float& z1) {
#pragma clang fp contract(off)
  const float rho = sqrt_rn_gauss(-2.0f * gauss_ln_u24(wr));
  float c, s;
  gauss_sincos(wa, c, s);
  z0 = rho * c;
  z1 = rho * s;
}

// Unscaled Gaussian entries Z[4j .. 4j+3][r].
__device__ __forceinline__ void gauss4(uint64_t r, uint32_t j, uint32_t k0, uint32_t k1, float z[4]) {
  const u32x4 x = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), j, kTagGauss, k0, k1);
  gauss_pair(x.x, x.y, z[0], z[1]);
  gauss_pair(x.z, x.w, z[2], z[3]);
}

// Unscaled Rademacher entries B[4j .. 4j+3][r] = +-1: target t takes bit
// t % 32 of word (t % 128) / 32 of the Philox call (r, t / 128); bit 1 = -1.
__device__ __forceinline__ void rademacher4(uint64_t r, uint32_t j, uint32_t k0, uint32_t k1,
                                            float z[4]) {
  const u32x4 x = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), j >> 5, kTagRademacher, k0, k1);
  const uint32_t q = (j >> 3) & 3u;
  const uint32_t w = q == 0 ? x.x : (q == 1 ? x.y : (q == 2 ? x.z : x.w));
  const uint32_t bits = w >> (4u * (j & 7u));
#pragma unroll
  for (int i = 0; i < 4; ++i) z[i] = ((bits >> i) & 1u) ? -1.0f : 1.0f;
}

// SRHT random sign of global row r: bit r % 128 of the output of the Philox
// call (r / 128, 0, 0x53524854); a set bit means -1.
__device__ __forceinline__ double srht_sign(uint64_t r, uint32_t k0, uint32_t k1) {
  const uint64_t q = r >> 7;
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), 0u, kTagSrht, k0, k1);
  const uint32_t wsel = (uint32_t)(r >> 5) & 3u;
  const uint32_t w = wsel == 0 ? x.x : (wsel == 1 ? x.y : (wsel == 2 ? x.z : x.w));
  return ((w >> (r & 31u)) & 1u) ? -1.0 : 1.0;
}
// SRHT sampled row s_j of the 2^logn-point transform: the top logn bits of
// word j % 4 of the Philox call (j / 4, 0, 1, 0x53524854) (0 if logn == 0).
__device__ __forceinline__ uint64_t srht_sample(uint32_t j, int logn, uint32_t k0, uint32_t k1) {
  const u32x4 x = philox4x32_10(j >> 2, 0u, 1u, kTagSrht, k0, k1);
  const uint32_t q = j & 3u;
  const uint32_t w = q == 0 ? x.x : (q == 1 ? x.y : (q == 2 ? x.z : x.w));
  return logn == 0 ? 0ull : (uint64_t)(w >> (32 - logn));
}

// Row (target) of the nonzero of segment s of the sparse-sign column r:
// s*L + (((w_s >> 1) * L) >> 31), sign bit = w_s & 1 (1 = negative).
__device__ __forceinline__ uint32_t sparse_target(uint32_t w, uint32_t s, uint32_t L) {
  return s * L + (uint32_t)((((uint64_t)(w >> 1)) * (uint64_t)L) >> 31);
}

// The eight words of column r of the sparse sign (two Philox calls).
__device__ __forceinline__ void sparse_words(uint64_t r, uint32_t k0, uint32_t k1, uint32_t w[8]) {
  const u32x4 a = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), 0u, kTagSparse, k0, k1);
  const u32x4 b = philox4x32_10((uint32_t)r, (uint32_t)(r >> 32), 1u, kTagSparse, k0, k1);
  w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
  w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}

// ---------------------------------------------------------------------------
// Host launchers (all enqueue on `st`, return hipError_t of the launch).
// ---------------------------------------------------------------------------
enum SketchKind { kGaussian = 0, kSparse = 1, kIdentity = 2, kRademacher = 3, kSrht = 4 };

struct SketchDesc {
  int kind;
  int zeta;   // sparse sign: nonzeros per column; SRHT: log2 of the transform size
  int64_t k;
  uint32_t key0, key1;
};

// One problem of a lock-step batch (device copy; see launch_*_batched).  The
// problems of a batch share m, p, k, the sketch kind and the options; they
// differ in n, the leading dimensions, the pointers and the seed.
struct BatchItem {
  const void* W;
  void* Q;
  double *R, *S, *P, *E, *G, *Cb, *Yb, *part, *stack;
  unsigned* counter;
  const uint16_t* plan_off;
  const uint16_t* plan_ent;
  uint16_t* plan_off_w;     // the same plan, writable, for the plan kernel
  uint16_t* plan_ent_w;
  int64_t* flag;
  int64_t n, ldw, ldq, ldr;
  uint32_t key0, key1;
  int64_t plan_tile0;       // first flattened plan tile (prefix over problems)
  int64_t up_tile0;         // first flattened update tile
  int64_t up_nfull;         // update tiles on the unguarded vector path
  int64_t sk_wg0;           // first flattened sketch workgroup
  int64_t sk_tpw;           // sketch tiles per workgroup
  int32_t sk_G;             // sketch row groups (partial sums) of this problem
  int32_t pad;
};

// Workgroup -> problem for flattened grids: the last problem whose prefix
// `first(p)` is <= bx (prefixes nondecreasing, first(0) = 0).
template <typename F>
__device__ __forceinline__ int batch_find(int nprob, int64_t bx, F first) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(mid) <= bx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Lock-step batch launchers (all problems of `items`, nprob of them, device array).
hipError_t launch_plan_batched(const BatchItem* items, int nprob, int64_t total_tiles, int k,
                               int zeta, hipStream_t st);
// which = 0: all m columns of W into P; which = 1: Q_(i) (columns c0 .. c0 + ncols) into S.
hipError_t launch_sketch_batched(bool f32, const BatchItem* items, int nprob, int64_t total_wgs,
                                 int which, int64_t c0, int64_t ncols, int k, int zeta,
                                 double scale, hipStream_t st);
hipError_t launch_gram_sty_batched(const BatchItem* items, int nprob, int64_t k, int64_t K, int bw,
                                   int bprev, int64_t m, bool to_cb, hipStream_t st);
// src/dst: 0 = Cb (ld K), 1 = Yb (ld K), 2 = R_(1:i-1,i) (ld ldr)
hipError_t launch_sweep_batched(const BatchItem* items, int nprob, int64_t m, int64_t K, int bw,
                                int src, int dst, hipStream_t st);
hipError_t launch_resid_batched(const BatchItem* items, int nprob, int64_t k, int64_t K, int bw,
                                hipStream_t st);
hipError_t launch_qr_batched(const BatchItem* items, int nprob, int64_t k, int bw, int64_t c0,
                             hipStream_t st);
hipError_t launch_update_batched(bool f32, int math, const BatchItem* items, int nprob,
                                 int64_t total_tiles, int64_t K, int bw, hipStream_t st);
hipError_t launch_init_batched(const BatchItem* items, int nprob, int64_t m, hipStream_t st);
// ---------------------------------------------------------------------------
// Persistent batch: one launch runs a device queue of stages (plan, sketch of
// W, its reduction, and per block the small factors, the update, the sketch
// of Q_(i) and its reduction) for every problem of a batch; FP32 storage,
// FP64 arithmetic, low-synchronization form, sparse sign.
// ---------------------------------------------------------------------------
constexpr int kPbThreads = 1024;            // threads per workgroup (one per CU)
constexpr int kPbMaxK = 1024;               // sketch rows
constexpr int kPbMaxP = 32;                 // block width
constexpr int kPbLdsBytes = 144 * 1024;     // LDS pool shared by the stages
constexpr int kPbTileRows = 1024;           // rows per update tile for p <= 16 (half for p > 16)
constexpr int kPbSkG = 16;                  // row groups of a sketch, at most
constexpr int kPbSkMinTiles = 4;            // tiles per row group, at least (but one group)

// Stage kinds, in the order they follow one another for one problem.
enum PbKind : int32_t { kPbPlan = 0, kPbWsk, kPbRedw, kPbSmall, kPbUpd, kPbQsk, kPbReds };

struct PbProb {
  const float* W;
  float* Q;
  double *R, *S, *P, *E, *G, *Cb, *Yb, *part;
  int64_t* flag;
  uint16_t* plan_off;
  uint16_t* plan_ent;
  int64_t n, ldw, ldq, ldr;
  uint32_t key0, key1;
  int32_t m, p, k, nb;        // nb = ceil(m / p) blocks
  int32_t plan_tiles;         // tiles of kSpTile rows
  int32_t sk_G, sk_tpw;       // sketch row groups and tiles per group
  int32_t up_tiles, up_nfull; // update tiles (kPbTileRows rows, half for p > 16)
                              // and those on the vector path
};
struct PbStage {
  int32_t prob, kind, block, nitems;
};
// The queue has kPbLevels priority levels, each a FIFO over its own range of
// slots [base, end); a stage's level grows with the blocks its problem has
// left (pb_level), and workgroups take from the highest level with work.
constexpr int kPbLevels = 4;
struct PbCtl {
  unsigned head[kPbLevels], tail[kPbLevels], base[kPbLevels], end[kPbLevels];
  unsigned error, done, pad[2];  // done: problems whose last stage has finished
};
// Stages of one problem with m columns and block width p.
inline int64_t pb_stage_count(int64_t m, int64_t p) { return 4 * ((m + p - 1) / p) + 1; }
// Priority level of a stage of a problem of nb blocks: blocks left (the
// stages before the first block count as all nb) 1-2 -> 0, 3-4 -> 1, 5-6 -> 2,
// 7 or more -> 3.
__host__ __device__ inline int pb_level(int nb, int kind, int block) {
  const int rem = kind <= kPbRedw ? nb : nb - block;
  const int l = (rem - 1) / 2;
  return l < kPbLevels - 1 ? l : kPbLevels - 1;
}
// Rows of R_(1:i-1,i) staged by the persistent update form for 16 nb columns:
// K rounded up to whole pairs of the K loop's load groups (the loop has no
// partial pair; rows >= K are zero).
__host__ __device__ constexpr int up_p_kalign(int nb) { return nb == 1 ? 16 : 32; }
__host__ __device__ inline int up_p_rows(int K, int nb) {
  return (K + up_p_kalign(nb) - 1) / up_p_kalign(nb) * up_p_kalign(nb);
}
// LDS bytes the update of a block of width bw after K columns needs.
inline int64_t pb_update_lds(int64_t K, int64_t bw) {
  const int nb = bw <= 16 ? 1 : 2;
  const int64_t ncol = 16 * nb, Kp = up_p_rows((int)K, nb);
  return (Kp * ncol + ncol * ncol + ncol) * 8;
}
// Initializes the queue from the host's template (stages0 / valid0: the first
// stage of every problem in its level's range, item counts filled in on the
// device; ctl0: heads, tails, ranges)
// and, per problem, R = 0 and the breakdown flag; then runs the queue.  Both
// on st; no host synchronization.  `limit` bounds every wait of a workgroup,
// in ticks of the device's constant-rate clock (on expiry ctl->error = 1 and
// the workgroups leave).
hipError_t launch_persistent_batch(const PbProb* probs, int nprob, int64_t max_mm,
                                   const PbStage* stages0, const unsigned* valid0,
                                   const PbCtl* ctl0, PbStage* stages, unsigned* claimed,
                                   unsigned* finished, unsigned* valid, PbCtl* ctl,
                                   unsigned total, int zeta, int ls_iters, uint64_t limit,
                                   int grid, hipStream_t st);

// rows per update tile (for the flattened prefix) and the unguarded tile count
int64_t update_tile_rows(bool f32);
bool update_vec_ok(bool f32, const void* Q, int64_t ldq);
int64_t sparse_plan_tiles(int64_t n);
int64_t plan_offsets_len(const SketchDesc& sk, int64_t n);

// Number of partial blocks (row ranges) the sketch kernels use for n rows;
// max_groups > 0 caps it (a sketch that runs beside other work occupies fewer
// compute units for longer).
int sketch_num_partials(const SketchDesc& sk, int64_t n, int64_t ncols, int max_groups = 0);
// Columns handled per partial block pass.
constexpr int kSketchCols = 16;

// Sparse sign: bucket Theta's nonzeros by target once per factorization (the
// "plan"; sparse_plan_bytes of workspace), for rows [row0, row0 + n).
size_t sparse_plan_bytes(const SketchDesc& sk, int64_t n);
hipError_t launch_sparse_plan(const SketchDesc& sk, int64_t n, int64_t row0, uint16_t* plan,
                              hipStream_t st);
// partial[g][c][t] (g < G, c < ncols, t < k),
// G = sketch_num_partials(sk, n, ncols, max_groups).
// `plan` (sparse sign only) must have been built for the same rows.
hipError_t launch_sketch_partials(const SketchDesc& sk, bool f32, const void* X, int64_t ldx,
                                  int64_t n, int64_t ncols, int64_t row0, double* partial,
                                  const uint16_t* plan, hipStream_t st, int max_groups = 0);
// out[t + c*ldo] = scale * sum_g partial[g][c][t] for c < ncols; the partial
// sums hold part_cols columns per row group (0: ncols).
hipError_t launch_sketch_reduce(const double* partial, int G, int64_t k, int64_t ncols,
                                double scale, double* out, int64_t ldo, hipStream_t st,
                                int64_t part_cols = 0);
// Dense (Gaussian, Rademacher) sketch of two column blocks in one pass that
// shares every generated entry: X0 (n0 columns) into slots [0, S0), X1 (n1
// columns) into slots [S0, S0 + n1), S0 = n0 rounded up to 16;
// dense_pair_slots(n0, n1) = S0 + n1 slots of partial sums per row group
// (sketch_num_partials(sk, n, slots) row groups).
int64_t dense_pair_slots(int64_t n0, int64_t n1);
hipError_t launch_sketch_dense_pair(const SketchDesc& sk, bool f32, const void* X0, int64_t ldx0,
                                    int64_t n0, const void* X1, int64_t ldx1, int64_t n1,
                                    int64_t n, int64_t row0, double* partial, hipStream_t st);
// Identity sketch: out = X (converted to FP64).
hipError_t launch_sketch_identity(bool f32, const void* X, int64_t ldx, int64_t n, int64_t ncols,
                                  double* out, int64_t ldo, hipStream_t st);
hipError_t launch_theta_dense(const SketchDesc& sk, int64_t n, int64_t row0, float* out,
                              hipStream_t st);

// Q'_(i) = W_(i) - Q_(1:i-1) R_(1:i-1,i)  [then Q_(i) = Q'_(i) R_(i,i)^{-1} if Rii != nullptr]
//   Rk: R_(1:i-1,i) in the R array (column-major, ld ldr), K rows, bw columns.
//   Rii: R_(i,i) in the R array (ld ldr), bw x bw, or nullptr.
//   f32: storage of W/Q is FP32 (else FP64); math: kMathF64 (FP64 matrix-core
//   arithmetic), kMathF32 (FP32 matrix cores) or kMathBf16x3 (split BF16x3
//   products on the bf16 matrix cores); the last two with FP32 storage only.
constexpr int kMathF64 = 0, kMathF32 = 1, kMathBf16x3 = 2;
hipError_t launch_update(bool f32, int math, const void* W, int64_t ldw, const void* Q,
                         int64_t ldq, void* Qout, int64_t ldqo, const double* Rk,
                         const double* Rii, int64_t ldr, int64_t n, int64_t K, int bw,
                         hipStream_t st);
// The low-sync update with R_(i,i) computed in the same launch: its first
// workgroup factors the k x bw residual sketch E (ld k) into Rii (positive
// diagonal, breakdown column into flag as the QR of a sketch does) and then
// releases *ready = col0 + 1; the other workgroups run the update and wait for
// that value before their first substitution (bounded by limit ticks of the
// device's wall clock, limit > 0, after which col0 is put into flag and the
// launch completes).  *ready must start below col0 + 1.  Only where
// update_fused_ok holds: FP64 arithmetic, bw = 16, 48 <= K <= 512, k <= 1024.
bool update_fused_ok(int math, int64_t K, int bw, int64_t k);
hipError_t launch_update_fused(bool f32, const void* W, int64_t ldw, const void* Q, int64_t ldq,
                               void* Qout, int64_t ldqo, const double* Rk, double* Rii,
                               int64_t ldr, int64_t n, int64_t K, int bw, const double* E,
                               int64_t k, int64_t* flag, int64_t col0, unsigned* ready,
                               uint64_t limit, hipStream_t st);
// In place Q_(i) = Q'_(i) R_(i,i)^{-1} (forward substitution per row).
hipError_t launch_trsm(bool f32, void* Q, int64_t ldq, const double* Rii, int64_t ldr, int64_t n,
                       int bw, hipStream_t st);

// Small FP64 factors (Sections 2.1 and 2.2).  Workspace for the QR tree of a k x bw matrix.
size_t qr_stack_size(int64_t k, int bw);
// ---- block Krylov solvers --------------------------------------------------
// Y (n x bs, ld ldy, element size ty: 4 or 8) = alpha A X + beta Y0, A in CSR
// (row pointers rp[n+1] int64, column indices ci int32, values av FP64), X of
// element size tx, Y0 FP64 or NULL.  FP64 arithmetic.  bs <= 32.
hipError_t launch_spmm(int64_t n, const int64_t* rp, const int32_t* ci, const double* av, int tx,
                       const void* X, int64_t ldx, int bs, double alpha, double beta,
                       const double* Y0, int64_t ldy0, int ty, void* Y, int64_t ldy,
                       hipStream_t st);
// min_Z ||A[:, :nc] Z - A[:, nc:nc+nrhs]||_F for a matrix zero below `band`
// subdiagonals (A overwritten); Z nc x nrhs; resid[c] = squared residual norm.
hipError_t launch_hess_ls(double* A, int64_t lda, int nr, int nc, int nrhs, int band, double* Z,
                          int64_t ldz, double* resid, hipStream_t st);
// X (n x bs FP64) += Q (n x N, FP32 or FP64) Z (N x bs FP64).
hipError_t launch_gemm_update(bool f32, int64_t n, int N, int bs, const void* Q, int64_t ldq,
                              const double* Z, int64_t ldz, double* X, int64_t ldx,
                              hipStream_t st);
// out = ||X||_F^2 (n x bs FP64), scratch of sumsq_scratch() doubles; fixed order.
size_t sumsq_scratch();
hipError_t launch_sumsq(const double* X, int64_t ldx, int64_t n, int bs, double* scratch,
                        double* out, hipStream_t st);
// Y (FP32 or FP64) = X (FP64), n x bs.
hipError_t launch_convert(const double* X, int64_t ldx, int64_t n, int bs, bool f32, void* Y,
                          int64_t ldy, hipStream_t st);

// Synthetic full-rank test matrix (n x m, ld >= n) for the autotuner.
hipError_t launch_fill_test(void* X, bool f32, int64_t n, int64_t m, int64_t ld, hipStream_t st);
// out0 (K x n0, ld ldo0) = S^T X0, out1 (K x n1, ld ldo1) = S^T X1 and, if
// out1t is not null, out1t (n1 x K, ld ldo1t) = (S^T X1)^T.  S: k x K (ld k);
// X0, X1: k x n0, k x n1 (ld k).
hipError_t launch_gram_sty(const double* S, int64_t k, int64_t K, const double* X0, int n0,
                           const double* X1, int n1, double* out0, int64_t ldo0, double* out1,
                           int64_t ldo1, double* out1t, int64_t ldo1t, hipStream_t st);
// One Richardson sweep in Gram form: Ynew = Y + C - G Y (G: K x K, ld ldg;
// C: K x bw, ld K).  Ynew must not alias Y.
hipError_t launch_gram_sweep(const double* G, int64_t ldg, int64_t K, const double* C,
                             const double* Y, int64_t ldy, double* Ynew, int64_t ldyn, int bw,
                             hipStream_t st);
// E = P - S Y (k x bw, ld k; S: k x K, ld k; Y: K x bw, ld ldy; K >= 1).
hipError_t launch_resid(const double* P, const double* S, int64_t k, int64_t K, const double* Y,
                        int64_t ldy, double* E, int bw, hipStream_t st);
// R_(i,i) (positive diagonal) of src (k x bw, ld k) in one launch (tree of
// Householder QRs; counter[0 .. kQrTreeCounters) must be 0 and are left at 0;
// stack: qr_stack_size(k, bw) doubles; flag[0] is set to the first column
// col0 + j whose diagonal entry is zero or not finite, if it is still -1).
constexpr int kQrTreeCounters = 62;
hipError_t launch_qr_fused(const double* src, int64_t k, int bw, double* stack, unsigned* counter,
                           double* Rii, int64_t ldr, int64_t* flag, int64_t col0, hipStream_t st);
// R factor (positive diagonal) of the l2 QR of a tall rows x bw matrix (FP32 or
// FP64, ld ld) by a Householder TSQR tree, one launch per level; stack:
// qr_stack_size(rows, bw) doubles; flag as for launch_qr_fused.
hipError_t launch_qr_tall(bool f32, const void* src, int64_t ld, int64_t rows, int bw,
                          double* stack, double* R, int64_t ldr, int64_t* flag, int64_t col0,
                          hipStream_t st);
// R <- A R for upper triangular bw x bw A and R (upper triangles only).
hipError_t launch_trmm_upper(const double* A, int64_t lda, double* R, int64_t ldr, int bw,
                             hipStream_t st);
// Cholesky-QR post-processing pieces.
// Row splits of the Gram kernel (partial buffer: gram_splits(n, m) * m * m doubles).
int gram_splits(int64_t n, int64_t m);
// G = Q^T Q (m x m FP64, ld m, symmetric) of the n x m matrix Q (FP32 or FP64).
hipError_t launch_gram(bool f32, const void* Q, int64_t ldq, int64_t n, int64_t m, double* partial,
                       double* G, hipStream_t st);
// In place: A (m x m, ld m, SPD) <- its upper Cholesky factor; flag as above.
hipError_t launch_cholesky(double* A, int64_t m, int64_t* flag, hipStream_t st);
// R <- A R for upper triangular m x m A and R; T: m x m scratch.
hipError_t launch_trmm_full(const double* A, int64_t lda, double* R, int64_t ldr, int64_t m,
                            double* T, hipStream_t st);
// Fill an m x m column-major matrix (ld) with zeros.
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st);
// Householder least squares of step 2 (one workgroup; hh_supported: k <= 1024,
// K <= 1024, bw <= 32 for k <= 512 and bw <= 16 above):
// absorb: columns c0 .. c0 + bw - 1 of the sketch (Snew, k x bw, ld k) into
// the factorization HS (k x m, ld k: R_S on and above the diagonal, reflector
// vectors below) and tau (m); solve: Y (K x bw, ld ldy) = the least-squares
// solution of S_(1:K) Y = P (k x bw, ld k), K <= 1024.
bool hh_supported(int64_t k, int64_t K, int bw);
hipError_t launch_hh_absorb(const double* Snew, int64_t k, int64_t c0, int bw, double* HS,
                            double* tau, hipStream_t st);
hipError_t launch_hh_solve(const double* HS, const double* tau, const double* P, int64_t k,
                           int64_t K, int bw, double* Y, int64_t ldy, hipStream_t st);
// R = 0 (m x m), *flag = -1, counters[0 .. ncnt) = 0, in one launch.
hipError_t launch_qr_init(double* R, int64_t ldr, int64_t m, int64_t* flag, unsigned* counters,
                          int ncnt, hipStream_t st);
// Certificates: out[0] = ||I - S^T S||_F^2, out[1] = ||P - S R||_F^2, out[2] = ||P||_F^2,
// out[3] = 1 if any entry of R or S is not finite.  `scratch` >= cert_scratch_size(k, m).
size_t cert_scratch_size(int64_t k, int64_t m);
hipError_t launch_certificates(const double* S, const double* P, const double* R, int64_t ldr,
                               int64_t k, int64_t m, double* scratch, double* out, hipStream_t st);

}  // namespace rbgs
