// C ABI of the RBGS library: argument validation, workspace, and the block
// loop of Algorithm RBGS (Section 2) for both inter-block variants of
// Section 2.2.  Every step is enqueued on the caller's stream; nothing waits
// on the host unless a certificate is requested.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rbgs.h"
#include "rbgs_internal.h"

using namespace rbgs;

namespace {

constexpr int kProfClasses = 5;
enum ProfClass { kProfUpdate = 0, kProfSketch = 1, kProfReduce = 2, kProfSmall = 3, kProfTrsm = 4 };

struct ProfRec {
  int which;
  hipEvent_t a, b;
  double bytes;
};

}  // namespace

struct rbgs_handle_s {
  int device = 0;
  std::string last_error;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t prof_mask = 0;  // bit c: record launches of kernel class c
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[kProfClasses] = {0};
  int64_t prof_cnt[kProfClasses] = {0};
  double prof_bytes[kProfClasses] = {0};
  double* host_cert = nullptr;  // pinned, 4 doubles + flag
  hipStream_t side = nullptr;   // sketches of later blocks of W run here (default priority)
  std::vector<hipEvent_t> sync_ev;  // ordering between the caller's stream and `side`
  bool no_overlap = false;      // set on the lanes of a batch: everything on one stream
  // batched calls: lanes (child handles with their own stream and workspace)
  std::vector<rbgs_handle> lanes;
  std::vector<hipStream_t> lane_streams;
  std::vector<hipEvent_t> lane_ev;
  // graph of the last batch enqueued with graph capture, and its key
  std::vector<int64_t> graph_key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // autotuner: (m, ceil log2 n, store, math, kind, variant) -> (p, k)
  std::vector<std::pair<std::vector<int64_t>, std::pair<int64_t, int64_t>>> tuned;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

rbgs_status fail(rbgs_handle h, rbgs_status s, const std::string& msg) {
  if (h) h->last_error = msg;
  return s;
}

rbgs_status hip_fail(rbgs_handle h, hipError_t e, const char* where) {
  std::string msg = std::string(where) + ": " + hipGetErrorString(e);
  return fail(h, RBGS_EDEVICE, msg);
}

#define HIP_TRY(h, expr, where)                        \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return hip_fail(h, _e, where); \
  } while (0)

hipEvent_t take_event(rbgs_handle h) {
  hipEvent_t e;
  if (!h->pool.empty()) {
    e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Wraps one kernel launch (or launch sequence) with profiling events.
struct ProfScope {
  rbgs_handle h;
  int which;
  double bytes;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(rbgs_handle h_, int which_, double bytes_, hipStream_t st_)
      : h(h_), which(which_), bytes(bytes_), st(st_) {
    if ((h->prof_mask >> which) & 1u) {
      a = take_event(h);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = take_event(h);
      if (b) {
        (void)hipEventRecord(b, st);
        h->recs.push_back({which, a, b, bytes});
      } else {
        h->pool.push_back(a);
      }
    }
  }
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

#ifndef RBGS_SIDE_GROUPS
#define RBGS_SIDE_GROUPS 128
#endif
constexpr int kSideGroups = RBGS_SIDE_GROUPS;  // partial groups of a side-stream sketch

// The side stream (created once, default priority, not blocking on the null
// stream) and at least `nev` ordering events.
rbgs_status ensure_side(rbgs_handle h, size_t nev) {
  if (!h->side && hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    h->side = nullptr;
    return fail(h, RBGS_EDEVICE, "side stream creation failed");
  }
  while (h->sync_ev.size() < nev) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, RBGS_EDEVICE, "event creation failed");
    }
    h->sync_ev.push_back(e);
  }
  return RBGS_OK;
}

rbgs_status ensure_ws(rbgs_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return RBGS_OK;
  if (h->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)1 << 20);
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, RBGS_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  h->ws_bytes = want;
  return RBGS_OK;
}

bool valid_sketch(const rbgs_sketch* sk, int64_t n, std::string& why) {
  if (!sk) { why = "sketch descriptor is NULL"; return false; }
  if (sk->k < 1) { why = "sketch dimension k must be >= 1"; return false; }
  switch (sk->kind) {
    case RBGS_SKETCH_GAUSSIAN:
      if (sk->k % 4) { why = "Gaussian sketch needs k % 4 == 0"; return false; }
      if (sk->k > (int64_t)1 << 20) { why = "k too large"; return false; }
      return true;
    case RBGS_SKETCH_SPARSE_SIGN:
      if (sk->zeta < 1 || sk->zeta > 8) { why = "sparse sign needs 1 <= zeta <= 8"; return false; }
      if (sk->k % sk->zeta) { why = "sparse sign needs k % zeta == 0"; return false; }
      if (sk->k > 2048) { why = "sparse sign supports k <= 2048"; return false; }
      return true;
    case RBGS_SKETCH_IDENTITY:
      if (sk->k != n) { why = "identity sketch needs k == n"; return false; }
      return true;
    default:
      why = "unknown sketch kind";
      return false;
  }
}

SketchDesc make_desc(const rbgs_sketch* sk) {
  SketchDesc d;
  d.kind = sk->kind;
  d.zeta = sk->zeta;
  d.k = sk->k;
  d.key0 = (uint32_t)(sk->seed & 0xFFFFFFFFull);
  d.key1 = (uint32_t)(sk->seed >> 32);
  return d;
}

double sketch_scale(const SketchDesc& d) {
  if (d.kind == kGaussian) return 1.0 / sqrt((double)d.k);
  if (d.kind == kSparse) return 1.0 / sqrt((double)d.zeta);
  return 1.0;
}

size_t sketch_partial_doubles(const SketchDesc& d, int64_t n, int64_t ncols, int max_groups = 0) {
  if (d.kind == kIdentity) return 0;
  return (size_t)sketch_num_partials(d, n, ncols, max_groups) * (size_t)ncols * (size_t)d.k;
}

// out = Theta X (k x ncols, ld ldo)
rbgs_status do_sketch(rbgs_handle h, const SketchDesc& d, bool f32, const void* X, int64_t ldx,
                      int64_t n, int64_t ncols, int64_t row0, double* out, int64_t ldo,
                      double* partial, const uint16_t* plan, hipStream_t st, int max_groups = 0) {
  const double s = f32 ? 4.0 : 8.0;
  if (d.kind == kIdentity) {
    ProfScope ps(h, kProfSketch, s * n * ncols + 8.0 * n * ncols, st);
    HIP_TRY(h, launch_sketch_identity(f32, X, ldx, n, ncols, out, ldo, st), "sketch_identity");
    return RBGS_OK;
  }
  const int G = sketch_num_partials(d, n, ncols, max_groups);
  {
    ProfScope ps(h, kProfSketch, s * n * ncols, st);
    HIP_TRY(h, launch_sketch_partials(d, f32, X, ldx, n, ncols, row0, partial, plan, st, max_groups),
            "sketch");
  }
  {
    ProfScope ps(h, kProfReduce, 8.0 * d.k * ncols, st);
    HIP_TRY(h, launch_sketch_reduce(partial, G, d.k, ncols, sketch_scale(d), out, ldo, st),
            "sketch_reduce");
  }
  return RBGS_OK;
}

}  // namespace

static rbgs_status validate_qr(rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m,
                               int64_t p, const rbgs_sketch* sk, const rbgs_opts* opts, void* Q,
                               int64_t ldq, double* R, int64_t ldr) {
  // ---- host-side validation (nothing is enqueued on failure) -------------
  if (!W || !Q || !R) return fail(h, RBGS_EINVAL, "W, Q and R must be non-NULL");
  if (!opts) return fail(h, RBGS_EINVAL, "options are NULL");
  if (n < 1 || m < 1) return fail(h, RBGS_EINVAL, "n and m must be >= 1");
  if (m > n) return fail(h, RBGS_EINVAL, "m must not exceed n");
  if (p < 1) return fail(h, RBGS_EINVAL, "block width p must be >= 1");
  if (ldw < n || ldq < n) return fail(h, RBGS_EINVAL, "leading dimensions of W and Q must be >= n");
  if (ldr < m) return fail(h, RBGS_EINVAL, "leading dimension of R must be >= m");
  std::string why;
  if (!valid_sketch(sk, n, why)) return fail(h, RBGS_EINVAL, why);
  if (sk->k < m) return fail(h, RBGS_EINVAL, "sketch dimension k must be >= m");
  if (sk->k > n) return fail(h, RBGS_EINVAL, "sketch dimension k must be <= n");
  if (opts->store != RBGS_STORE_F64 && opts->store != RBGS_STORE_F32)
    return fail(h, RBGS_EINVAL, "unknown storage type");
  if (opts->math != RBGS_MATH_F64 && opts->math != RBGS_MATH_F32)
    return fail(h, RBGS_EINVAL, "unknown arithmetic");
  if (opts->store == RBGS_STORE_F64 && opts->math != RBGS_MATH_F64)
    return fail(h, RBGS_EINVAL, "FP64 storage needs FP64 arithmetic");
  if (opts->variant != RBGS_VARIANT_PLAIN && opts->variant != RBGS_VARIANT_LOWSYNC)
    return fail(h, RBGS_EINVAL, "unknown variant");
  if (opts->ls_iters < 1 || opts->ls_iters > 16)
    return fail(h, RBGS_EINVAL, "ls_iters must be in [1, 16]");
  if (p > 32) return fail(h, RBGS_EUNSUPPORTED, "block width p > 32 is not implemented");
  const size_t es = opts->store == RBGS_STORE_F32 ? 4 : 8;
  {
    // Q == W (same ld) is the in-place factorization; any other overlap is invalid.
    const char* w0 = (const char*)W;
    const char* w1 = w0 + es * (size_t)(ldw * (m - 1) + n);
    const char* q0 = (const char*)Q;
    const char* q1 = q0 + es * (size_t)(ldq * (m - 1) + n);
    const bool same = (w0 == q0) && (ldw == ldq);
    if (!same && q0 < w1 && w0 < q1) return fail(h, RBGS_EINVAL, "Q overlaps W (only Q == W is allowed)");
    const char* r0 = (const char*)R;
    const char* r1 = r0 + 8 * (size_t)(ldr * (m - 1) + m);
    if ((r0 < w1 && w0 < r1) || (r0 < q1 && q0 < r1)) return fail(h, RBGS_EINVAL, "R overlaps W or Q");
  }

  return RBGS_OK;
}

extern "C" {

rbgs_status rbgs_create(rbgs_handle* h, int device) {
  if (!h || device < 0) return RBGS_EINVAL;
  rbgs_handle p = new (std::nothrow) rbgs_handle_s();
  if (!p) return RBGS_ENOMEM;
  p->device = device;
  *h = p;
  return RBGS_OK;
}

rbgs_status rbgs_destroy(rbgs_handle h) {
  if (!h) return RBGS_OK;
  for (auto c : h->lanes) rbgs_destroy(c);
  if (h->ws || !h->recs.empty() || !h->pool.empty() || h->host_cert || h->side ||
      !h->lane_streams.empty() || h->graph) {
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    for (auto& r : h->recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    for (auto e : h->sync_ev) (void)hipEventDestroy(e);
    if (h->side) (void)hipStreamDestroy(h->side);
    for (auto e : h->lane_ev) (void)hipEventDestroy(e);
    for (auto q : h->lane_streams) (void)hipStreamDestroy(q);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->ws) (void)hipFree(h->ws);
    if (h->host_cert) (void)hipHostFree(h->host_cert);
  }
  delete h;
  return RBGS_OK;
}

const char* rbgs_status_string(rbgs_status s) {
  switch (s) {
    case RBGS_OK: return "success";
    case RBGS_EINVAL: return "invalid argument";
    case RBGS_ENOMEM: return "out of device memory";
    case RBGS_EDEVICE: return "HIP runtime error";
    case RBGS_EBREAKDOWN: return "breakdown: zero or non-finite diagonal entry of R";
    case RBGS_ENOTCONV: return "not converged";
    case RBGS_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* rbgs_last_error(rbgs_handle h) { return h ? h->last_error.c_str() : ""; }

rbgs_status rbgs_qr(rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m, int64_t p,
                    const rbgs_sketch* sk, const rbgs_opts* opts, void* Q, int64_t ldq,
                    double* R, int64_t ldr, double* S_out, rbgs_cert* cert) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  {
    const rbgs_status vs = validate_qr(h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr);
    if (vs != RBGS_OK) return vs;
  }
  const bool f32 = opts->store == RBGS_STORE_F32;
  const bool f32_math = opts->math == RBGS_MATH_F32;
  const size_t es = f32 ? 4 : 8;

  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)opts->stream;
  const SketchDesc d = make_desc(sk);
  const int64_t k = d.k;
  const int b = (int)p;

  // ---- workspace ---------------------------------------------------------
  size_t off = 0;
  auto carve = [&](size_t doubles) {
    size_t o = off;
    off += ((doubles * 8 + 255) / 256) * 256;
    return o;
  };
  const size_t o_S = S_out ? 0 : carve((size_t)k * m);
  const size_t o_P = carve((size_t)k * m);
  const size_t o_E = carve((size_t)k * b);
  // partial sums for every sketch width used: all of W, a full block, the last block
  size_t part_need = std::max(sketch_partial_doubles(d, n, m), sketch_partial_doubles(d, n, std::min<int64_t>(b, m)));
  if (m % b) part_need = std::max(part_need, sketch_partial_doubles(d, n, m % b));
  const size_t o_part = carve(part_need);
  // The sketches of blocks 1.. of W run on a side stream while the main
  // stream works through earlier blocks (they only read W and the plan); the
  // small factors of a block use few compute units, so these sketches mostly
  // fill idle ones.  Block i waits for its sketch before its least squares.
  const int64_t nblk = (m + b - 1) / b;
  const bool overlap = !h->no_overlap && d.kind != kIdentity && nblk > 1;
  size_t part2_need = 0;
  if (overlap) {
    part2_need = sketch_partial_doubles(d, n, std::min<int64_t>(b, m), kSideGroups);
    if (m % b) part2_need = std::max(part2_need, sketch_partial_doubles(d, n, m % b, kSideGroups));
  }
  const size_t o_part2 = carve(part2_need);
  const size_t o_stack = carve(qr_stack_size(k, b));
  const size_t o_plan = d.kind == kSparse ? carve((sparse_plan_bytes(d, n) + 7) / 8) : 0;
  const size_t o_flag = carve(1);
  const size_t o_cnt = carve(1);
  const size_t o_G = carve((size_t)m * m);   // Gram matrix S^T S of the blocks done
  const size_t o_C = carve((size_t)m * b);   // c = S^T P_(i)
  const size_t o_Y = carve((size_t)m * b);   // Richardson iterate
  const size_t o_cs = carve(cert_scratch_size(k, m));
  const size_t o_cout = carve(4);
  rbgs_status rs = ensure_ws(h, off);
  if (rs != RBGS_OK) return rs;
  char* base = (char*)h->ws;
  double* S = S_out ? S_out : (double*)(base + o_S);
  double* P = (double*)(base + o_P);
  double* E = (double*)(base + o_E);
  double* part = (double*)(base + o_part);
  double* part2 = (double*)(base + o_part2);
  double* stack = (double*)(base + o_stack);
  uint16_t* plan = d.kind == kSparse ? (uint16_t*)(base + o_plan) : nullptr;
  int64_t* flag = (int64_t*)(base + o_flag);
  unsigned* counters = (unsigned*)(base + o_cnt);  // [1]: QR tree arrivals
  double* G = (double*)(base + o_G);
  double* Cb = (double*)(base + o_C);
  double* Yb = (double*)(base + o_Y);
  double* cscratch = (double*)(base + o_cs);
  double* cout = (double*)(base + o_cout);

  HIP_TRY(h, launch_zero(R, ldr, m, m, st), "zero R");
  HIP_TRY(h, launch_set_i64(flag, -1, st), "flag");
  HIP_TRY(h, launch_set_u32(counters, 2, 0u, st), "counters");
  if (plan) {
    ProfScope ps(h, kProfSketch, 0.0, st);
    HIP_TRY(h, launch_sparse_plan(d, n, 0, plan, st), "sketch plan");
  }

  // ---- step 1 ahead of the loop: P = Theta W (W_(i) is not modified before
  // block i, so sketching it early gives the same P_(i)) --------------------
  if (!overlap) {
    rs = do_sketch(h, d, f32, W, ldw, n, m, 0, P, k, part, plan, st);
    if (rs != RBGS_OK) return rs;
  } else {
    rs = ensure_side(h, (size_t)nblk + 1);
    if (rs != RBGS_OK) return rs;
    hipEvent_t ev_start = h->sync_ev[nblk];
    HIP_TRY(h, hipEventRecord(ev_start, st), "event record");
    HIP_TRY(h, hipStreamWaitEvent(h->side, ev_start, 0), "stream wait");
    rs = do_sketch(h, d, f32, W, ldw, n, std::min<int64_t>(b, m), 0, P, k, part, plan, st);
    if (rs != RBGS_OK) return rs;
    for (int64_t blk = 1; blk < nblk; ++blk) {
      const int64_t c0 = blk * b;
      const int64_t bwb = std::min<int64_t>(b, m - c0);
      rs = do_sketch(h, d, f32, (const char*)W + es * (size_t)(c0 * ldw), ldw, n, bwb, 0,
                     P + c0 * k, k, part2, plan, h->side, kSideGroups);
      if (rs != RBGS_OK) return rs;
      HIP_TRY(h, hipEventRecord(h->sync_ev[blk], h->side), "event record");
    }
  }

  const char* Wb = (const char*)W;
  char* Qb = (char*)Q;
  const int l = opts->ls_iters;
  for (int64_t c0 = 0; c0 < m; c0 += b) {
    const int bw = (int)std::min<int64_t>(b, m - c0);
    const int64_t K = c0;
    const double* Pi = P + c0 * k;
    double* Rk = R + c0 * ldr;            // R_(1:i-1,i): rows [0, K), columns [c0, c0+bw)
    double* Rii = R + c0 + c0 * ldr;      // R_(i,i)
    const void* Wi = Wb + es * (size_t)(c0 * ldw);
    void* Qi = Qb + es * (size_t)(c0 * ldq);

    if (overlap && K > 0) HIP_TRY(h, hipStreamWaitEvent(st, h->sync_ev[c0 / b], 0), "stream wait");
    // ---- step 2: sketched least squares by l Richardson sweeps ----------
    // One pass over S gives c = S^T P_(i) (sweep 1: R_(1:i-1,i) = c) and the
    // Gram block S^T S_(i-1); sweeps 2..l use the Gram matrix.
    if (K > 0) {
      ProfScope ps(h, kProfSmall, 0.0, st);
      const int bprev = b;  // width of block i-1 (only the last block can be narrower)
      const double* Sprev = S + (K - bprev) * k;
      double* Ccol = (l > 1) ? Cb : Rk;
      const int64_t ldc = (l > 1) ? K : ldr;
      HIP_TRY(h, launch_gram_sty(S, k, K, Pi, bw, Sprev, bprev, Ccol, ldc, G + (K - bprev) * m, m,
                                 G + (K - bprev), m, st),
              "least squares: sketch products");
      // sweeps: Y_1 = c, Y_{s+1} = Y_s + c - G Y_s.  Targets alternate between
      // R_(1:i-1,i) and Yb so that the last sweep lands in R and no sweep
      // writes its own input.
      const double* Ycur = Cb;
      int64_t ldycur = K;
      for (int it = 1; it < l; ++it) {
        const bool toR = ((l - 1 - it) & 1) == 0;
        double* Ynext = toR ? Rk : Yb;
        const int64_t ldn = toR ? ldr : K;
        HIP_TRY(h, launch_gram_sweep(G, m, K, Cb, Ycur, ldycur, Ynext, ldn, bw, st),
                "least squares: sweep");
        Ycur = Ynext;
        ldycur = ldn;
      }
    }
    const double ub = (double)es * (double)n * (double)(K + 2 * bw);
    if (opts->variant == RBGS_VARIANT_LOWSYNC) {
      // ---- steps 4-5 with postponed sketching: S'_(i) = P_(i) - S R_(1:i-1,i)
      {
        ProfScope ps(h, kProfSmall, 0.0, st);
        const double* Sp = Pi;
        if (K > 0) {
          HIP_TRY(h, launch_resid(Pi, S, k, K, Rk, ldr, E, bw, st), "S'");
          Sp = E;
        }
        HIP_TRY(h, launch_qr_fused(Sp, k, bw, stack, counters + 1, Rii, ldr, flag, c0, st),
                "qr of sketch");
      }
      // ---- step 3 + substitution in one pass --------------------------
      {
        ProfScope ps(h, kProfUpdate, ub, st);
        HIP_TRY(h, launch_update(f32, f32_math, Wi, ldw, Q, ldq, Qi, ldq, Rk, Rii, ldr, n, K, bw, st),
                "update");
      }
    } else {
      // ---- step 3: Q'_(i), stored in Q_(i) ------------------------------
      {
        ProfScope ps(h, kProfUpdate, ub, st);
        HIP_TRY(h, launch_update(f32, f32_math, Wi, ldw, Q, ldq, Qi, ldq, Rk, nullptr, ldr, n, K, bw, st),
                "update");
      }
      // ---- step 4: S'_(i) = Theta Q'_(i), R_(i,i), substitution -----------
      rs = do_sketch(h, d, f32, Qi, ldq, n, bw, 0, E, k, part, plan, st);
      if (rs != RBGS_OK) return rs;
      {
        ProfScope ps(h, kProfSmall, 0.0, st);
        HIP_TRY(h, launch_qr_fused(E, k, bw, stack, counters + 1, Rii, ldr, flag, c0, st),
                "qr of sketch");
      }
      {
        ProfScope ps(h, kProfTrsm, 2.0 * es * n * bw, st);
        HIP_TRY(h, launch_trsm(f32, Qi, ldq, Rii, ldr, n, bw, st), "substitution");
      }
    }
    // ---- step 5: S_(i) = Theta Q_(i) ----------------------------------------
    rs = do_sketch(h, d, f32, Qi, ldq, n, bw, 0, S + c0 * k, k, part, plan, st);
    if (rs != RBGS_OK) return rs;
  }

  if (!cert) return RBGS_OK;
  // ---- step 6: certificates (host waits) ---------------------------------
  HIP_TRY(h, launch_certificates(S, P, R, ldr, k, m, cscratch, cout, st), "certificates");
  if (!h->host_cert) HIP_TRY(h, hipHostMalloc((void**)&h->host_cert, 8 * sizeof(double)), "hipHostMalloc");
  HIP_TRY(h, hipMemcpyAsync(h->host_cert, cout, 4 * sizeof(double), hipMemcpyDeviceToHost, st),
          "copy certificate");
  HIP_TRY(h, hipMemcpyAsync(h->host_cert + 4, flag, sizeof(int64_t), hipMemcpyDeviceToHost, st),
          "copy flag");
  HIP_TRY(h, hipStreamSynchronize(st), "stream synchronize");
  const double* hc = h->host_cert;
  int64_t bcol;
  memcpy(&bcol, hc + 4, sizeof(int64_t));
  const double pn2 = hc[2];
  cert->delta = sqrt(hc[0]);
  cert->delta_tilde = pn2 > 0 ? sqrt(hc[1] / pn2) : 0.0;
  cert->breakdown_col = bcol;
  cert->nonfinite = hc[3] != 0.0 ? 1 : 0;
  cert->reserved = 0;
  if (bcol >= 0) {
    char buf[128];
    snprintf(buf, sizeof buf, "R(%lld,%lld) is zero or not finite", (long long)bcol, (long long)bcol);
    return fail(h, RBGS_EBREAKDOWN, buf);
  }
  return RBGS_OK;
}

// ---------------------------------------------------------------------------
// Batched factorizations and the autotuner.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr int kBatchLanes = 4;  // internal streams of a batch

rbgs_status ensure_lanes(rbgs_handle h, int L) {
  while ((int)h->lanes.size() < L) {
    rbgs_handle c = nullptr;
    if (rbgs_create(&c, h->device) != RBGS_OK) return fail(h, RBGS_ENOMEM, "lane handle");
    c->no_overlap = true;
    h->lanes.push_back(c);
  }
  while ((int)h->lane_streams.size() < L) {
    hipStream_t q;
    HIP_TRY(h, hipStreamCreateWithFlags(&q, hipStreamNonBlocking), "lane stream");
    h->lane_streams.push_back(q);
  }
  while ((int)h->lane_ev.size() < L + 1) {
    hipEvent_t e;
    HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "lane event");
    h->lane_ev.push_back(e);
  }
  return RBGS_OK;
}

int64_t ceil_log2(int64_t n) {
  int64_t b = 0;
  while (((int64_t)1 << b) < n) ++b;
  return b;
}

double batch_bytes(const rbgs_problem& pr, size_t es) {
  double tot = 0.0;
  for (int64_t c0 = 0; c0 < pr.m; c0 += pr.p) {
    const int64_t bw = std::min<int64_t>(pr.p, pr.m - c0);
    tot += (double)(c0 + 2 * bw) * (double)pr.n * (double)es;
  }
  return tot;
}

// Enqueue every problem on its lane; lanes fork from and join back to st.
rbgs_status enqueue_batch(rbgs_handle h, int64_t count, rbgs_problem* probs,
                          const rbgs_sketch* sk, const rbgs_opts* opts,
                          const std::vector<std::vector<int64_t>>& lane_items) {
  hipStream_t st = (hipStream_t)opts->stream;
  const int L = (int)lane_items.size();
  HIP_TRY(h, hipEventRecord(h->lane_ev[L], st), "event record");
  for (int l = 0; l < L; ++l)
    HIP_TRY(h, hipStreamWaitEvent(h->lane_streams[l], h->lane_ev[L], 0), "stream wait");
  for (int l = 0; l < L; ++l) {
    for (int64_t i : lane_items[l]) {
      rbgs_problem& pr = probs[i];
      rbgs_sketch ski = *sk;
      ski.k = pr.k;
      ski.seed = sk->seed + (uint64_t)i;
      rbgs_opts oi = *opts;
      oi.stream = h->lane_streams[l];
      pr.status = rbgs_qr(h->lanes[l], pr.W, pr.ldw, pr.n, pr.m, pr.p, &ski, &oi, pr.Q, pr.ldq,
                          pr.R, pr.ldr, nullptr, nullptr);
      if (pr.status != RBGS_OK)
        return fail(h, (rbgs_status)pr.status,
                    "problem " + std::to_string(i) + ": " + h->lanes[l]->last_error);
    }
  }
  for (int l = 0; l < L; ++l) {
    HIP_TRY(h, hipEventRecord(h->lane_ev[l], h->lane_streams[l]), "event record");
    HIP_TRY(h, hipStreamWaitEvent(st, h->lane_ev[l], 0), "stream wait");
  }
  return RBGS_OK;
}

}  // namespace

extern "C" {

rbgs_status rbgs_autotune(rbgs_handle h, int64_t n, int64_t m, const rbgs_sketch* sk,
                          const rbgs_opts* opts, int64_t* p_out, int64_t* k_out) {
  if (!h) return RBGS_EINVAL;
  if (!sk || !opts || !p_out || !k_out) return fail(h, RBGS_EINVAL, "NULL argument");
  if (n < 1 || m < 1 || m > n) return fail(h, RBGS_EINVAL, "need 1 <= m <= n");
  const std::vector<int64_t> key = {m, ceil_log2(n), opts->store, opts->math, sk->kind, sk->zeta,
                                    opts->variant};
  for (auto& e : h->tuned)
    if (e.first == key) {
      *p_out = e.second.first;
      *k_out = e.second.second;
      return RBGS_OK;
    }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  rbgs_status rs = ensure_lanes(h, 1);
  if (rs != RBGS_OK) return rs;
  rbgs_handle lane = h->lanes[0];
  const bool f32 = opts->store == RBGS_STORE_F32;
  const size_t es = f32 ? 4 : 8;
  const int64_t step = sk->kind == RBGS_SKETCH_SPARSE_SIGN ? std::max<int64_t>(4, sk->zeta) * 4 : 4;
  std::vector<int64_t> ps, ks;
  for (int64_t pc : {16, 32}) {
    const int64_t pp = std::min<int64_t>(pc, m);
    if (std::find(ps.begin(), ps.end(), pp) == ps.end()) ps.push_back(pp);
  }
  for (int64_t mult : {2, 3, 4}) {
    int64_t kc = ((mult * m + step - 1) / step) * step;
    if (sk->kind == RBGS_SKETCH_SPARSE_SIGN) kc = ((kc + sk->zeta - 1) / sk->zeta) * sk->zeta;
    kc = std::min<int64_t>(kc, n);
    if (kc >= m && std::find(ks.begin(), ks.end(), kc) == ks.end()) ks.push_back(kc);
  }
  if (ks.empty()) return fail(h, RBGS_EINVAL, "no admissible sketch size for this n, m");
  void* W = nullptr;
  void* Q = nullptr;
  double* R = nullptr;
  auto cleanup = [&]() {
    (void)hipDeviceSynchronize();
    if (W) (void)hipFree(W);
    if (Q) (void)hipFree(Q);
    if (R) (void)hipFree(R);
  };
  if (hipMalloc(&W, es * (size_t)(n * m)) != hipSuccess || hipMalloc(&Q, es * (size_t)(n * m)) != hipSuccess ||
      hipMalloc((void**)&R, 8 * (size_t)(m * m)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(h, RBGS_ENOMEM, "autotuner buffers");
  }
  hipStream_t st = h->lane_streams[0];
  hipEvent_t e0 = h->lane_ev[0], e1 = h->lane_ev[1];
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    cleanup();
    return fail(h, RBGS_EDEVICE, "event creation failed");
  }
  (void)e0;
  (void)e1;
  double best = 1e300;
  int64_t bp = ps[0], bk = ks[0];
  rbgs_status out = RBGS_OK;
  if (launch_fill_test(W, f32, n, m, n, st) != hipSuccess) out = fail(h, RBGS_EDEVICE, "fill");
  for (int64_t pp : ps) {
    for (int64_t kc : ks) {
      if (out != RBGS_OK) break;
      rbgs_sketch ski = *sk;
      ski.k = kc;
      rbgs_opts oi = *opts;
      oi.stream = st;
      float ms = 0.f;
      for (int rep = 0; rep < 3 && out == RBGS_OK; ++rep) {
        if (rep == 1) (void)hipEventRecord(t0, st);
        out = rbgs_qr(lane, W, n, n, m, pp, &ski, &oi, Q, n, R, m, nullptr, nullptr);
        if (out != RBGS_OK) h->last_error = lane->last_error;
      }
      if (out != RBGS_OK) break;
      (void)hipEventRecord(t1, st);
      if (hipEventSynchronize(t1) != hipSuccess || hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
        out = fail(h, RBGS_EDEVICE, "autotuner timing");
        break;
      }
      if (ms < best) {
        best = ms;
        bp = pp;
        bk = kc;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  cleanup();
  if (out != RBGS_OK) return out;
  h->tuned.push_back({key, {bp, bk}});
  *p_out = bp;
  *k_out = bk;
  return RBGS_OK;
}

rbgs_status rbgs_qr_batched(rbgs_handle h, int64_t count, rbgs_problem* probs,
                            const rbgs_sketch* sk, const rbgs_opts* opts, int32_t graph) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  if (count < 1 || !probs || !sk || !opts) return fail(h, RBGS_EINVAL, "empty batch or NULL argument");
  if (graph != 0 && graph != 1) return fail(h, RBGS_EINVAL, "graph must be 0 or 1");
  // tune the problems that ask for it, then validate every problem
  for (int64_t i = 0; i < count; ++i) {
    rbgs_problem& pr = probs[i];
    if (pr.p < 0 || pr.k < 0) {
      pr.status = RBGS_EINVAL;
      return fail(h, RBGS_EINVAL, "problem " + std::to_string(i) + ": negative p or k");
    }
    if (pr.p == 0 || pr.k == 0) {
      if (pr.n < 1 || pr.m < 1 || pr.m > pr.n) {
        pr.status = RBGS_EINVAL;
        return fail(h, RBGS_EINVAL, "problem " + std::to_string(i) + ": need 1 <= m <= n");
      }
      int64_t tp = 0, tk = 0;
      const rbgs_status ts = rbgs_autotune(h, pr.n, pr.m, sk, opts, &tp, &tk);
      if (ts != RBGS_OK) {
        pr.status = ts;
        return ts;
      }
      if (pr.p == 0) pr.p = tp;
      if (pr.k == 0) pr.k = tk;
    }
  }
  for (int64_t i = 0; i < count; ++i) {
    rbgs_problem& pr = probs[i];
    rbgs_sketch ski = *sk;
    ski.k = pr.k;
    ski.seed = sk->seed + (uint64_t)i;
    pr.status = validate_qr(h, pr.W, pr.ldw, pr.n, pr.m, pr.p, &ski, opts, pr.Q, pr.ldq, pr.R, pr.ldr);
    if (pr.status != RBGS_OK) {
      h->last_error = "problem " + std::to_string(i) + ": " + h->last_error;
      return (rbgs_status)pr.status;
    }
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)opts->stream;
  const bool use_graph = graph == 1 && st != nullptr;
  std::vector<int64_t> key = {count, opts->store, opts->math, opts->variant, opts->ls_iters,
                              (int64_t)(intptr_t)st, sk->kind, sk->zeta, (int64_t)sk->seed};
  for (int64_t i = 0; i < count; ++i) {
    const rbgs_problem& pr = probs[i];
    for (int64_t v : {(int64_t)(intptr_t)pr.W, pr.ldw, pr.n, pr.m, (int64_t)(intptr_t)pr.Q, pr.ldq,
                      (int64_t)(intptr_t)pr.R, pr.ldr, pr.p, pr.k})
      key.push_back(v);
  }
  if (use_graph && h->graph_exec && key == h->graph_key) {
    HIP_TRY(h, hipGraphLaunch(h->graph_exec, st), "hipGraphLaunch");
    for (int64_t i = 0; i < count; ++i) probs[i].status = RBGS_OK;
    return RBGS_OK;
  }
  // largest problem first, each to the least loaded lane
  const int L = (int)std::min<int64_t>(kBatchLanes, count);
  rbgs_status rs = ensure_lanes(h, L);
  if (rs != RBGS_OK) return rs;
  const size_t es = opts->store == RBGS_STORE_F32 ? 4 : 8;
  std::vector<int64_t> order(count);
  for (int64_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return batch_bytes(probs[a], es) > batch_bytes(probs[b], es);
  });
  std::vector<std::vector<int64_t>> lane_items(L);
  std::vector<double> load(L, 0.0);
  for (int64_t i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lane_items[l].push_back(i);
    load[l] += batch_bytes(probs[i], es);
  }
  rs = enqueue_batch(h, count, probs, sk, opts, lane_items);
  if (rs != RBGS_OK || !use_graph) return rs;
  // record the same enqueue sequence as a graph for later identical calls
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  h->graph_key.clear();
  HIP_TRY(h, hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  rs = enqueue_batch(h, count, probs, sk, opts, lane_items);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(st, &g);
  if (rs != RBGS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rs;
  }
  if (ce != hipSuccess) return hip_fail(h, ce, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(h, ie, "hipGraphInstantiate");
  }
  h->graph = g;
  h->graph_exec = ex;
  h->graph_key = key;
  return RBGS_OK;
}

rbgs_status rbgs_sketch_apply(rbgs_handle h, const rbgs_sketch* sk, int32_t store, const void* X,
                              int64_t ldx, int64_t n, int64_t c, int64_t row0, double* out,
                              int64_t ldo, void* stream) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  if (!X || !out) return fail(h, RBGS_EINVAL, "X and out must be non-NULL");
  if (n < 1 || c < 1 || ldx < n || row0 < 0) return fail(h, RBGS_EINVAL, "bad sizes");
  if (store != RBGS_STORE_F64 && store != RBGS_STORE_F32) return fail(h, RBGS_EINVAL, "unknown storage type");
  std::string why;
  if (sk && sk->kind == RBGS_SKETCH_IDENTITY) {
    if (sk->k != n || row0 != 0) return fail(h, RBGS_EINVAL, "identity sketch needs k == n and row0 == 0");
  } else if (!valid_sketch(sk, n, why)) {
    return fail(h, RBGS_EINVAL, why);
  }
  if (ldo < sk->k) return fail(h, RBGS_EINVAL, "ldo must be >= k");
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  const SketchDesc d = make_desc(sk);
  const size_t part_bytes = ((sketch_partial_doubles(d, n, c) * 8 + 255) / 256) * 256;
  const size_t plan_bytes = d.kind == kSparse ? sparse_plan_bytes(d, n) : 0;
  rbgs_status rs = ensure_ws(h, part_bytes + plan_bytes + 256);
  if (rs != RBGS_OK) return rs;
  hipStream_t st = (hipStream_t)stream;
  uint16_t* plan = d.kind == kSparse ? (uint16_t*)((char*)h->ws + part_bytes) : nullptr;
  if (plan) HIP_TRY(h, launch_sparse_plan(d, n, row0, plan, st), "sketch plan");
  return do_sketch(h, d, store == RBGS_STORE_F32, X, ldx, n, c, row0, out, ldo, (double*)h->ws,
                   plan, st);
}

rbgs_status rbgs_theta_dense(rbgs_handle h, const rbgs_sketch* sk, int64_t n, int64_t row0,
                             float* out, void* stream) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  if (!out || n < 1 || row0 < 0) return fail(h, RBGS_EINVAL, "bad arguments");
  std::string why;
  if (!sk) return fail(h, RBGS_EINVAL, "sketch descriptor is NULL");
  if (sk->kind != RBGS_SKETCH_IDENTITY && !valid_sketch(sk, n, why)) return fail(h, RBGS_EINVAL, why);
  if (sk->kind == RBGS_SKETCH_IDENTITY && sk->k < 1) return fail(h, RBGS_EINVAL, "k must be >= 1");
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  HIP_TRY(h, launch_theta_dense(make_desc(sk), n, row0, out, (hipStream_t)stream), "theta_dense");
  return RBGS_OK;
}

rbgs_status rbgs_profile_enable(rbgs_handle h, int32_t enable) {
  if (!h) return RBGS_EINVAL;
  h->prof_mask = (uint32_t)enable & ((1u << kProfClasses) - 1u);
  for (int i = 0; i < kProfClasses; ++i) {
    h->prof_ms[i] = 0;
    h->prof_cnt[i] = 0;
    h->prof_bytes[i] = 0;
  }
  return RBGS_OK;
}

rbgs_status rbgs_profile_get(rbgs_handle h, int32_t which, double* ms, int64_t* launches,
                             double* bytes) {
  if (!h || which < 0 || which >= kProfClasses) return RBGS_EINVAL;
  if (!h->recs.empty()) {
    DeviceGuard guard(h->device);
    for (auto& r : h->recs) {
      HIP_TRY(h, hipEventSynchronize(r.b), "hipEventSynchronize");
      float t = 0.f;
      HIP_TRY(h, hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
      h->prof_ms[r.which] += t;
      h->prof_cnt[r.which] += 1;
      h->prof_bytes[r.which] += r.bytes;
      h->pool.push_back(r.a);
      h->pool.push_back(r.b);
    }
    h->recs.clear();
  }
  if (ms) *ms = h->prof_ms[which];
  if (launches) *launches = h->prof_cnt[which];
  if (bytes) *bytes = h->prof_bytes[which];
  return RBGS_OK;
}

}  // extern "C"
