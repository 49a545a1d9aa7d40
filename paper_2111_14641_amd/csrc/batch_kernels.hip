// Persistent batch of RBGS factorizations (Algorithm RBGS of Section 2, the
// low-synchronization form with the sparse-sign sketch): one launch of one
// workgroup per compute unit works through a device queue of stages until
// every problem of the batch is factored.
//
// The work of one problem is a chain of stages, each a set of independent
// items:
//   plan of Theta (per 8 tiles of 1024 rows) -> partial sums of Theta W
//   (row group x 16-column slice) -> their reduction into P = Theta W ->
//   for each block i: small factors (step 2 by Richardson sweeps in Gram
//   form on the FP64 matrix cores, Theta-QR of the sketched residual; one
//   item) -> update and substitution of steps 3-5 (16 tiles of 1024 rows,
//   512 for p > 16, per item) -> partial sums of
//   Theta Q_(i) -> their reduction into S_(i) (the last two not for the last
//   block).
// Stage s + 1 of a problem reads what every item of stage s wrote, so a stage
// enters the queue when the last item of its predecessor finishes; the first
// stage of every problem is queued at the start, largest problem first.
// Workgroups take items from the first queued stage that still has items (a
// counter of claimed items per stage), walking forward from the head, which
// moves on past stages whose items are all taken.  Different problems, and different stages of them, are in flight
// at once, so one problem's small factors (one workgroup, no HBM traffic)
// overlap the others' HBM-bound updates and sketches.
//
// Progress: an item never waits, and a workgroup waits only while the queue
// is empty, which ends when a running item finishes; a workgroup holds no item
// while it waits.  Every wait is bounded by the device's constant-rate clock
// (on expiry an error word is set and the workgroups leave).
//
// Ordering: every wave of a workgroup waits for its own memory operations and
// the workgroup meets at a barrier before one thread makes the item's writes
// visible device-wide (release) and counts the item; the last item of a
// stage acquires, writes the successor stage and publishes it with a release;
// a workgroup that takes an item acquires after it sees the stage published.
#include <algorithm>

#include "rbgs_internal.h"
#include "sketch_device.h"
#include "small_device.h"
#include "update_device.h"

namespace rbgs {

namespace {

#ifndef RBGS_PB_RED
#define RBGS_PB_RED 4          // sketch outputs per thread of a reduction item
#endif
// Measured on 512 problems (n 16k..262k, m 32..256, p = 32, k = 4m): update
// items of 4, 8, 16 and 32 tiles gave 87.4, 83.4, 82.0 and 81.4 ms (plan items
// of half as many tiles); 16 keeps more items per stage for small problems.
#ifndef RBGS_PB_PLAN_TILES
#define RBGS_PB_PLAN_TILES 8   // plan tiles per item
#endif
#ifndef RBGS_PB_UPD_TILES
#define RBGS_PB_UPD_TILES 16   // update tiles per item
#endif
constexpr int kPbRedOut = RBGS_PB_RED * kPbThreads;
constexpr int kPbPlanTiles = RBGS_PB_PLAN_TILES;
constexpr int kPbUpdTiles = RBGS_PB_UPD_TILES;

static_assert(UpPShape<float, 1, kPbThreads / 64, 4>::TILE == kPbTileRows, "update tile");
static_assert(UpPShape<float, 2, kPbThreads / 64, 2>::TILE == kPbTileRows / 2, "update tile");
static_assert(sizeof(PlanLds) <= kPbLdsBytes, "plan LDS");
static_assert(sizeof(SpqLds<float, 16, 1>) <= kPbLdsBytes, "sketch LDS");
static_assert(sizeof(QwLds<16, 2>) <= kPbLdsBytes, "QR LDS");
static_assert(kPbThreads == kSpThreads && kPbThreads == kQwThreads, "one thread count");

__device__ __forceinline__ int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
__device__ __forceinline__ int pb_bw(const PbProb& P, int block) {
  return min(P.p, P.m - block * P.p);
}
// columns per sketch item of a block of width bw
__device__ __forceinline__ int pb_qnc(int bw) { return bw > 8 ? 16 : 8; }

__device__ int pb_items(const PbProb& P, int kind, int block) {
  switch (kind) {
    case kPbPlan:
      return cdiv(P.plan_tiles, kPbPlanTiles);
    case kPbWsk:
      return P.sk_G * cdiv(P.m, 16);
    case kPbRedw:
      return cdiv((int64_t)P.k * P.m, kPbRedOut);
    case kPbSmall:
      return 1;
    case kPbUpd:
      return cdiv(P.up_tiles, kPbUpdTiles);
    case kPbQsk: {
      const int bw = pb_bw(P, block);
      return P.sk_G * cdiv(bw, pb_qnc(bw));
    }
    default:
      return cdiv((int64_t)P.k * pb_bw(P, block), kPbRedOut);
  }
}

// The stage after (kind, block) of problem P; false after the last update.
__device__ bool pb_next(const PbProb& P, int kind, int block, int& nk, int& nblk) {
  nblk = block;
  switch (kind) {
    case kPbPlan:
      nk = kPbWsk;
      return true;
    case kPbWsk:
      nk = kPbRedw;
      return true;
    case kPbRedw:
      nk = kPbSmall;
      nblk = 0;
      return true;
    case kPbSmall:
      nk = kPbUpd;
      return true;
    case kPbUpd:
      nk = kPbQsk;
      return block + 1 < P.nb;
    case kPbQsk:
      nk = kPbReds;
      return true;
    default:
      nk = kPbSmall;
      nblk = block + 1;
      return true;
  }
}

__device__ __forceinline__ unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The first wave: the next item (in lane 0's `item` and `out`), or -1 when
// every level is drained, after an error, or when a wait for a stage exceeds
// `limit` ticks (then the error word is set).  Each group of 16 lanes looks at
// 16 slots from the head of one level (the first group at the highest level)
// at once: queued?, every item taken?  The first stage with an item left, in
// that order, is tried with one atomic add, and the winner acquires.  In each
// level every stage before the first one not known to be exhausted has all its
// items taken (claim counts only grow), so that level's head moves there
// (atomic max); it never passes a stage that is not queued yet.
__device__ int pb_claim(const PbStage* stages, unsigned* claimed, const unsigned* valid,
                        PbCtl* ctl, uint64_t limit, int& item, PbStage& out) {
  const int lane = threadIdx.x & 63, grp = lane >> 4, i = lane & 15;
  const int lev = kPbLevels - 1 - grp;
  const unsigned end = ld_agent(&ctl->end[lev]);
  uint64_t t0 = wall_clock64();
  for (;;) {
    const unsigned hl = ld_agent(&ctl->head[lev]);  // the same in the 16 lanes of a group
    const unsigned slot = hl + i;
    const bool in = slot < end;
    const bool queued = in && ld_agent(&valid[in ? slot : 0]) != 0u;
    unsigned n = 0;
    bool left = false;
    if (queued) {
      n = (unsigned)ld_agent(&stages[slot].nitems);
      left = ld_agent(&claimed[slot]) < n;
    }
    const uint64_t m_left = __ballot(left);
    const uint64_t m_done = __ballot(queued && !left);  // queued, every item taken
    if (__ballot(hl < end) == 0) return -1;             // every level drained
    // this group's exhausted prefix: slots hl .. hl + g - 1
    const unsigned gd = (unsigned)(m_done >> (16 * grp)) & 0xFFFFu;
    const unsigned g = gd == 0xFFFFu ? 16u : (unsigned)__builtin_ctz(~gd);
    if (m_left == 0) {
      if (i == 0 && g > 0) atomicMax(&ctl->head[lev], hl + g);
      // a group whose 16 slots were all exhausted looks again at once
      if (__ballot(i == 0 && g == 16u) != 0) continue;
      if (__builtin_amdgcn_readfirstlane((int)ld_agent(&ctl->error)) != 0) return -1;
      if (wall_clock64() - t0 > limit) {
        if (lane == 0) atomicCAS(&ctl->error, 0u, 1u);
        return -1;
      }
      __builtin_amdgcn_s_sleep(4);
      continue;
    }
    const int f = __builtin_ctzll(m_left);
    const unsigned hs = (unsigned)__shfl((int)slot, f, 64);
    const unsigned nf = (unsigned)__shfl((int)n, f, 64);
    const unsigned gf = (unsigned)__shfl((int)g, f, 64);
    const unsigned hf = (unsigned)__shfl((int)hl, f, 64);
    const int lf = kPbLevels - 1 - (f >> 4);
    unsigned c = 0;
    if (lane == 0) c = atomicAdd(&claimed[hs], 1u);
    c = (unsigned)__shfl((int)c, 0, 64);
    if (c >= nf) continue;  // taken meanwhile
    t0 = wall_clock64();
    if (lane == 0) {
      // past the stage taken only when it ends the exhausted prefix of its
      // level and its last item was taken here
      const unsigned next = (unsigned)(f & 15) == gf && c + 1 == nf ? hs + 1 : hf + gf;
      if (next > hf) atomicMax(&ctl->head[lf], next);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      out.prob = ld_agent(&stages[hs].prob);
      out.kind = ld_agent(&stages[hs].kind);
      out.block = ld_agent(&stages[hs].block);
      out.nitems = (int)nf;
      item = (int)c;
    }
    return (int)hs;
  }
}

// One thread, after the workgroup's writes of the item are complete: count
// the item; the last one of its stage queues the successor in its level.
__device__ void pb_finish(const PbProb* probs, const PbStage& st, int slot, PbStage* stages,
                          unsigned* finished, unsigned* valid, PbCtl* ctl) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  const unsigned f = atomicAdd(&finished[slot], 1u);
  if (f + 1 != (unsigned)st.nitems) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const PbProb& P = probs[st.prob];
  int nk, nblk;
  if (!pb_next(P, st.kind, st.block, nk, nblk)) {
    atomicAdd(&ctl->done, 1u);
    return;
  }
  const int lev = pb_level(P.nb, nk, nblk);
  const unsigned t = atomicAdd(&ctl->tail[lev], 1u);
  if (t >= ld_agent(&ctl->end[lev])) {  // more stages than counted on the host: cannot happen
    atomicCAS(&ctl->error, 0u, 2u);
    return;
  }
  st_agent(&stages[t].prob, st.prob);
  st_agent(&stages[t].kind, nk);
  st_agent(&stages[t].block, nblk);
  st_agent(&stages[t].nitems, pb_items(P, nk, nblk));
  __hip_atomic_store(&valid[t], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Values read back from LDS are the same in every lane; saying so keeps them
// in scalar registers and the branches on them uniform.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// LDS shared by the stages (one stage at a time per workgroup).
__shared__ __attribute__((aligned(32))) char pb_pool[kPbLdsBytes];


// ---- the stages ------------------------------------------------------------

__device__ __forceinline__ void pb_plan(const PbProb& P, int item, int zeta) {
  PlanLds& L = *reinterpret_cast<PlanLds*>(pb_pool);
  const int t1 = min(P.plan_tiles, (item + 1) * kPbPlanTiles);
  for (int t = item * kPbPlanTiles; t < t1; ++t) {
    sparse_plan_tile(P.n, 0, P.k, zeta, P.key0, P.key1, P.plan_off, P.plan_ent, t, L);
    __syncthreads();
  }
}

// Partial sums of Theta X (ncols columns) for row group item / S, column
// slice item % S, into P.part ([sk_G][ncols][k]).
template <int NC>
__device__ __forceinline__ void pb_sketch(const float* X, int64_t ldx, const PbProb& P, int ncols, int item,
                          int zeta) {
  const int S = cdiv(ncols, NC);
  SpqLds<float, NC, 1>& L = *reinterpret_cast<SpqLds<float, NC, 1>*>(pb_pool);
  sketch_sparse_q_body<float, 1, kPbThreads, NC, 1>(X, ldx, P.n, ncols, P.k, zeta, P.plan_off,
                                                    P.plan_ent, P.sk_tpw, P.part, item / S,
                                                    item % S, L);
}

// out[idx] = scale * sum_g part[g][idx] (g in order) for kPbRedOut consecutive
// idx = column * k + row of a k x ncols sketch.
__device__ __forceinline__ void pb_reduce(const double* __restrict__ part, int G, int64_t k, int ncols,
                          double scale, double* __restrict__ out, int item) {
  const int64_t total = k * ncols;
#pragma unroll
  for (int r = 0; r < kPbRedOut / kPbThreads; ++r) {
    const int64_t idx = (int64_t)item * kPbRedOut + r * kPbThreads + threadIdx.x;
    if (idx < total) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += part[(int64_t)g * total + idx];
      out[idx] = scale * s;
    }
  }
}

// out[i, j] = add1[i, j] + (add2[i, j] + sgn sum_d op(A)[i, d] B[d, j]) for
// i < M, j < N (the addends when given), and outT[j, i] the same value when
// outT is given; op(A)[i, d] = A[d + i lda] (TA, A^T) or A[i + d lda].  One
// workgroup: each wave takes 16 x 16 output tiles in turn and accumulates them
// on the FP64 matrix cores over d in steps of 4 (lane (kk, li) supplies
// op(A)[i0 + li, d + kk] and B[d + kk, j0 + li] and ends with rows
// i0 + kk + 4 e, column j0 + li).  Loads past M, N or D are clamped and their
// values replaced by zero.  Columns of A and B are read in 32-byte runs per
// lane group, so one pass over a 128-byte line serves four steps.
template <bool TA>
__device__ __forceinline__ void pb_gemm(int M, int N, int D, const double* __restrict__ A,
                                        int64_t lda, const double* __restrict__ B, int64_t ldb,
                                        double sgn, const double* add1, int64_t ld1,
                                        const double* add2, int64_t ld2, double* out,
                                        int64_t ldo, double* outT, int64_t ldt) {
  typedef Mfma<double> Mm;
  constexpr int U = 4;  // steps of 4 whose operands are loaded together
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kk = lane >> 4, li = lane & 15;
  const int tm = (M + 15) / 16, tn = (N + 15) / 16;
  for (int tile = w; tile < tm * tn; tile += kPbThreads / 64) {
    const int i0 = (tile % tm) * 16, j0 = (tile / tm) * 16;
    const bool oka = i0 + li < M, okb = j0 + li < N;
    const int64_t ia = oka ? i0 + li : M - 1, jb = okb ? j0 + li : N - 1;
    Mm::acc_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int d0 = 0; d0 < D; d0 += 4 * U) {
      double a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int d = d0 + 4 * u + kk;
        const bool okd = d < D;
        const int64_t dc = okd ? d : D - 1;
        const double av = TA ? A[dc + ia * lda] : A[ia + dc * lda];
        const double bv = B[dc + jb * ldb];
        a[u] = oka && okd ? av : 0.0;
        b[u] = okb && okd ? bv : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc = Mm::mma(a[u], b[u], acc);
    }
    const int64_t j = j0 + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + Mm::row(kk, e);
      if (i < M && j < N) {
        double v = sgn * acc[e];
        if (add2) v = add2[i + j * ld2] + v;
        if (add1) v = add1[i + j * ld1] + v;
        out[i + j * ldo] = v;
        if (outT) outT[j + i * ldt] = v;
      }
    }
  }
}

// Steps 2 and the Theta-QR of block i (one item), in one workgroup: the least
// squares of step 2 in Gram form as the lock-step batch (c = S^T P_(i) and the
// new block column of G = S^T S, sweeps Y <- Y + c - G Y, S' = P_(i) - S Y),
// its products on the matrix cores, then the QR of S'.
__device__ __forceinline__ void pb_small(const PbProb& P, int block, int ls) {
  const int64_t k = P.k, m = P.m, ldr = P.ldr;
  const int64_t c0 = (int64_t)block * P.p, K = c0;
  const int bw = pb_bw(P, block);
  if (K > 0) {
    const int bprev = P.p;  // only the last block can be narrower
    double* const RK = P.R + K * ldr;
    double* out0 = ls > 1 ? P.Cb : RK;
    const int64_t ldo0 = ls > 1 ? K : ldr;
    pb_gemm<true>((int)K, bw, (int)k, P.S, k, P.P + K * k, k, 1.0, nullptr, 0, nullptr, 0, out0,
                  ldo0, nullptr, 0);
    pb_gemm<true>((int)K, bprev, (int)k, P.S, k, P.S + (K - bprev) * k, k, 1.0, nullptr, 0,
                  nullptr, 0, P.G + (K - bprev) * m, m, P.G + (K - bprev), m);
    __syncthreads();
    int cur = 0;  // iterate in Cb (0), Yb (1) or R_(1:i-1,i) (2); the last one in R
    for (int it = 1; it < ls; ++it) {
      const int dst = ((ls - 1 - it) & 1) == 0 ? 2 : 1;
      const double* Y = cur == 0 ? P.Cb : (cur == 1 ? P.Yb : RK);
      const int64_t ldy = cur == 2 ? ldr : K;
      double* Yn = dst == 1 ? P.Yb : RK;
      const int64_t ldyn = dst == 2 ? ldr : K;
      pb_gemm<false>((int)K, bw, (int)K, P.G, m, Y, ldy, -1.0, Y, ldy, P.Cb, K, Yn, ldyn,
                     nullptr, 0);
      __syncthreads();
      cur = dst;
    }
    pb_gemm<false>((int)k, bw, (int)K, P.S, k, RK, ldr, -1.0, P.P + K * k, k, nullptr, 0, P.E, k,
                   nullptr, 0);
    __syncthreads();
  }
  const double* src = K == 0 ? P.P : P.E;
  double* Rii = P.R + c0 + c0 * ldr;
  if (k <= 256)
    qr_wave_body<4, 2>(src, k, bw, Rii, ldr, P.flag, c0, *reinterpret_cast<QwLds<4, 2>*>(pb_pool));
  else if (k <= 512)
    qr_wave_body<8, 2>(src, k, bw, Rii, ldr, P.flag, c0, *reinterpret_cast<QwLds<8, 2>*>(pb_pool));
  else
    qr_wave_body<16, 2>(src, k, bw, Rii, ldr, P.flag, c0, *reinterpret_cast<QwLds<16, 2>*>(pb_pool));
}

// Steps 3-5 of block i for update tiles item, item + nitems, ...  NB = 2
// (block width p > 16) reads two rows per lane instead of four (512-row
// tiles), which keeps it within the register budget of 16 waves per CU.
template <int NB, int FORM>
__device__ __forceinline__ void pb_update(const PbProb& P, int block, int item, int nitems) {
  constexpr int WV = kPbThreads / 64;
  constexpr int VE = NB == 1 ? 4 : 2;
  constexpr int NCOL = 16 * NB;
  constexpr int TROWS = UpPShape<float, NB, WV, VE>::TILE;
  const int64_t c0 = (int64_t)block * P.p;
  const int K = (int)c0, Kp = up_p_rows(K, NB);
  const int bw = pb_bw(P, block);
  double* Rs = reinterpret_cast<double*>(pb_pool);
  double* Ru = Rs + (int64_t)Kp * NCOL;
  double* Rinv = Ru + NCOL * NCOL;
  update_p_stage<NCOL, kPbThreads>(P.R + c0 * P.ldr, P.R + c0 + c0 * P.ldr, P.ldr, K, Kp, bw, Rs,
                                   Ru, Rinv);
  __syncthreads();
  const float* Wi = P.W + c0 * P.ldw;
  float* Qi = P.Q + c0 * P.ldq;
  update_p_full_tiles<float, NB, FORM, false, false, WV, VE>(Wi, P.ldw, P.Q, P.ldq, Qi, P.ldq, Rs, Ru,
                                                      Rinv, true, item, nitems, P.up_nfull, K, bw);
  for (int64_t tile = item; tile < P.up_tiles; tile += nitems)
    if (tile >= P.up_nfull)
      update_p_guarded_tile<float, NB, WV, VE>(Wi, P.ldw, P.Q, P.ldq, Qi, P.ldq, Rs, Ru, Rinv,
                                               true, tile * TROWS, P.n, K, bw);
}

// One function per stage body, not inlined into the kernel: each is given the
// full register budget of the workgroup on its own (inlined together, the
// bodies' live ranges and constant-bus copies overlapped and spilled).  The
// arguments arrive in vector registers; they are the same in every lane and
// are moved to scalar registers first.
__device__ __noinline__ void pb_run_plan(const PbProb* P, int item, int zeta) {
  pb_plan(*uni(P), uni(item), uni(zeta));
}
__device__ __noinline__ void pb_run_sketch_w(const PbProb* Pp, int item, int zeta) {
  const PbProb& P = *uni(Pp);
  pb_sketch<16>(P.W, P.ldw, P, P.m, uni(item), uni(zeta));
}
template <int NC>
__device__ __noinline__ void pb_run_sketch_q(const PbProb* Pp, int block, int item, int zeta) {
  const PbProb& P = *uni(Pp);
  block = uni(block);
  pb_sketch<NC>(P.Q + (int64_t)block * P.p * P.ldq, P.ldq, P, pb_bw(P, block), uni(item),
                uni(zeta));
}
// block < 0: the sketch of W into P; else that of Q_(block) into S.
__device__ __noinline__ void pb_run_reduce(const PbProb* Pp, int block, int item, int zeta) {
  const PbProb& P = *uni(Pp);
  block = uni(block);
  const double scale = 1.0 / sqrt((double)uni(zeta));
  if (block < 0)
    pb_reduce(P.part, P.sk_G, P.k, P.m, scale, P.P, uni(item));
  else
    pb_reduce(P.part, P.sk_G, P.k, pb_bw(P, block), scale, P.S + (int64_t)block * P.p * P.k,
              uni(item));
}
__device__ __noinline__ void pb_run_small(const PbProb* P, int block, int ls) {
  pb_small(*uni(P), uni(block), uni(ls));
}
template <int NB, int FORM>
__device__ __noinline__ void pb_run_update(const PbProb* P, int block, int item, int nitems) {
  pb_update<NB, FORM>(*uni(P), uni(block), uni(item), uni(nitems));
}
// the update in the form its block needs (up_p_form), each a function of its own
template <int NB>
__device__ __forceinline__ void pb_run_update_form(const PbProb* P, int block, int item,
                                                   int nitems) {
  switch (up_p_form(block * P->p, pb_bw(*P, block), NB)) {
    case 0: pb_run_update<NB, 0>(P, block, item, nitems); break;
    case 1: pb_run_update<NB, 1>(P, block, item, nitems); break;
    case 2: pb_run_update<NB, 2>(P, block, item, nitems); break;
    default: pb_run_update<NB, 3>(P, block, item, nitems); break;
  }
}

}  // namespace

// The queue's arguments are copied to LDS at the start and read back after
// every item (a barrier orders the reads), so that none of them holds a
// register through the items.
__global__ __launch_bounds__(kPbThreads, 1) void persistent_batch_kernel(
    const PbProb* probs, PbStage* stages, unsigned* claimed, unsigned* finished, unsigned* valid,
    PbCtl* ctl, unsigned total, int zeta, int ls, uint64_t limit) {
  struct Args {
    const PbProb* probs;
    PbStage* stages;
    unsigned *claimed, *finished, *valid;
    PbCtl* ctl;
    unsigned total;
    int zeta, ls;
    uint64_t limit;
  };
  __shared__ Args a;
  __shared__ int s_slot, s_item;
  __shared__ PbStage s_st;
  if (threadIdx.x == 0) {
    a.probs = probs;
    a.stages = stages;
    a.claimed = claimed;
    a.finished = finished;
    a.valid = valid;
    a.ctl = ctl;
    a.total = total;
    a.zeta = zeta;
    a.ls = ls;
    a.limit = limit;
  }
  for (;;) {
    __syncthreads();
    if (threadIdx.x < 64) {
      int item = 0;
      PbStage e;
      const int slot = pb_claim(a.stages, a.claimed, a.valid, a.ctl, a.limit, item, e);
      if (threadIdx.x == 0) {
        s_slot = slot;
        s_item = item;
        s_st = e;
      }
    }
    __syncthreads();
    const int slot = uni(s_slot);
    if (slot < 0) break;
    const int kind = uni(s_st.kind), block = uni(s_st.block), item = uni(s_item);
    const PbProb* P = uni(a.probs) + uni(s_st.prob);
    switch (kind) {
      case kPbPlan:
        pb_run_plan(P, item, a.zeta);
        break;
      case kPbWsk:
        pb_run_sketch_w(P, item, a.zeta);
        break;
      case kPbRedw:
        pb_run_reduce(P, -1, item, a.zeta);
        break;
      case kPbSmall:
        pb_run_small(P, block, a.ls);
        break;
      case kPbUpd:
        if (P->p <= 16) pb_run_update_form<1>(P, block, item, uni(s_st.nitems));
        else pb_run_update_form<2>(P, block, item, uni(s_st.nitems));
        break;
      case kPbQsk:
        if (pb_bw(*P, block) > 8) pb_run_sketch_q<16>(P, block, item, a.zeta);
        else pb_run_sketch_q<8>(P, block, item, a.zeta);
        break;
      default:
        pb_run_reduce(P, block, item, a.zeta);
        break;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
      pb_finish(a.probs, s_st, s_slot, a.stages, a.finished, a.valid, a.ctl);
  }
}

// y < nprob: R = 0 and the breakdown flag of problem y; y = nprob: the queue,
// from the host's template.
__global__ __launch_bounds__(256) void persistent_init_kernel(
    const PbProb* __restrict__ probs, int nprob, const PbStage* __restrict__ stages0,
    const unsigned* __restrict__ valid0, const PbCtl* __restrict__ ctl0, PbStage* stages,
    unsigned* claimed, unsigned* finished, unsigned* valid, PbCtl* ctl, unsigned total) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((int)blockIdx.y < nprob) {
    const PbProb& P = probs[blockIdx.y];
    if (idx < (int64_t)P.m * P.m) P.R[(idx % P.m) + P.ldr * (idx / P.m)] = 0.0;
    if (idx == 0) *P.flag = -1;
    return;
  }
  if (idx < total) {
    claimed[idx] = 0u;
    finished[idx] = 0u;
    PbStage e = stages0[idx];
    if (valid0[idx] != 0u) e.nitems = pb_items(probs[e.prob], e.kind, e.block);
    stages[idx] = e;
    valid[idx] = valid0[idx];
  }
  if (idx == 0) *ctl = *ctl0;
}

static int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_persistent_batch(const PbProb* probs, int nprob, int64_t max_mm,
                                   const PbStage* stages0, const unsigned* valid0,
                                   const PbCtl* ctl0, PbStage* stages, unsigned* claimed,
                                   unsigned* finished, unsigned* valid, PbCtl* ctl,
                                   unsigned total, int zeta, int ls_iters, uint64_t limit,
                                   int grid, hipStream_t st) {
  if (nprob < 1 || nprob >= 65535 || grid < 1 || zeta < 1 || zeta > kSpMaxZeta)
    return hipErrorInvalidValue;
  const int64_t gx = std::max(ceil_div64(max_mm, 256), ceil_div64(total, 256));
  hipLaunchKernelGGL(persistent_init_kernel, dim3((unsigned)gx, (unsigned)nprob + 1), dim3(256), 0,
                     st, probs, nprob, stages0, valid0, ctl0, stages, claimed, finished, valid,
                     ctl, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(persistent_batch_kernel, dim3((unsigned)grid), dim3(kPbThreads), 0, st, probs,
                     stages, claimed, finished, valid, ctl, total, zeta, ls_iters, limit);
  return hipGetLastError();
}

}  // namespace rbgs
