// C ABI of the RBGS library: argument validation, workspace, and the block
// loop of Algorithm RBGS (Section 2) for the inter-block variants of
// Section 2.2.  Every step is enqueued on the caller's stream; nothing waits
// on the host unless a certificate is requested.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
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

constexpr int kHostWords = 16;  // pinned host words of a handle
static_assert(sizeof(rbgs::PbCtl) <= kHostWords * sizeof(double), "queue state");

struct rbgs_handle_s {
  int device = 0;
  int clock_khz = 0;  // rate of the device's wall clock (bounded waits); 0 if unknown
  std::string last_error;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t prof_mask = 0;  // bit c: record launches of kernel class c
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[kProfClasses] = {0};
  int64_t prof_cnt[kProfClasses] = {0};
  double prof_bytes[kProfClasses] = {0};
  double* host_cert = nullptr;  // pinned, kHostWords doubles (certificates, queue state)
  // batched calls: lanes (child handles with their own stream and workspace)
  std::vector<rbgs_handle> lanes;
  std::vector<hipStream_t> lane_streams;
  std::vector<hipEvent_t> lane_ev;
  // graph of the last batch enqueued with graph capture, and its key
  std::vector<int64_t> graph_key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // block GMRES: basis, R, residual and least-squares buffers (grown on demand)
  void* kry = nullptr;
  size_t kry_bytes = 0;
  // autotuner: (m, ceil log2 n, store, math, kind, variant) -> (p, k)
  std::vector<std::pair<std::vector<int64_t>, std::pair<int64_t, int64_t>>> tuned;
  // lock-step and persistent batches: workspace of every problem and the
  // device descriptors
  void* bws = nullptr;
  size_t bws_bytes = 0;
  PbCtl* pb_ctl = nullptr;  // control words of the last persistent batch (in bws)
  unsigned pb_nprob = 0;  // its problems
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

// Workspace of the no-allocation entry point: one copy of this array per
// device, kept until the process ends.  Host code never uses the array's name
// as an address: the device address of each device's copy is looked up once
// with hipGetSymbolAddress (with that device current) and kept in
// g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static_assert(kScratchBytes == (size_t)RBGS_NOALLOC_SCRATCH_BYTES, "scratch size");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of this device's scratch array; the device must be
// current.
rbgs_status scratch_for_device(rbgs_handle h, void** out) {
  if (h->device >= kMaxScratchDevices) return fail(h, RBGS_EUNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[h->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(h, RBGS_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[h->device] = p;
  }
  *out = g_scratch_ptr[h->device];
  return RBGS_OK;
}

bool valid_sketch(const rbgs_sketch* sk, int64_t n, std::string& why) {
  if (!sk) { why = "sketch descriptor is NULL"; return false; }
  if (sk->k < 1) { why = "sketch dimension k must be >= 1"; return false; }
  switch (sk->kind) {
    case RBGS_SKETCH_GAUSSIAN:
    case RBGS_SKETCH_RADEMACHER:
      if (sk->k % 4) { why = "dense sketches need k % 4 == 0"; return false; }
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
    case RBGS_SKETCH_SRHT:
      if (sk->k > 2048) { why = "SRHT supports k <= 2048"; return false; }
      if (sk->zeta < 0 || sk->zeta > 32) { why = "SRHT needs 0 <= log2 of the transform size <= 32"; return false; }
      if (sk->zeta > 0 && n > ((int64_t)1 << sk->zeta)) {
        why = "SRHT transform size 2^zeta is smaller than the number of rows";
        return false;
      }
      if (sk->zeta == 0 && n > ((int64_t)1 << 32)) { why = "SRHT supports at most 2^32 rows"; return false; }
      return true;
    default:
      why = "unknown sketch kind";
      return false;
  }
}

// rows_total: the global row count the sketch must cover (the SRHT transform
// size defaults to the smallest power of two >= rows_total).
SketchDesc make_desc(const rbgs_sketch* sk, int64_t rows_total) {
  SketchDesc d;
  d.kind = sk->kind;
  d.zeta = sk->zeta;
  if (sk->kind == RBGS_SKETCH_SRHT && sk->zeta == 0) {
    int l = 0;
    while (((int64_t)1 << l) < rows_total) ++l;
    d.zeta = l;
  }
  d.k = sk->k;
  d.key0 = (uint32_t)(sk->seed & 0xFFFFFFFFull);
  d.key1 = (uint32_t)(sk->seed >> 32);
  return d;
}

double sketch_scale(const SketchDesc& d) {
  if (d.kind == kGaussian || d.kind == kRademacher || d.kind == kSrht) return 1.0 / sqrt((double)d.k);
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
  if (opts->math != RBGS_MATH_F64 && opts->math != RBGS_MATH_F32 && opts->math != RBGS_MATH_BF16X3)
    return fail(h, RBGS_EINVAL, "unknown arithmetic");
  if (opts->store == RBGS_STORE_F64 && opts->math != RBGS_MATH_F64)
    return fail(h, RBGS_EINVAL, "FP64 storage needs FP64 arithmetic");
  if (opts->variant < RBGS_VARIANT_PLAIN || opts->variant > RBGS_VARIANT_L2QR)
    return fail(h, RBGS_EINVAL, "unknown variant");
  if (opts->ls_iters < 0 || opts->ls_iters > 16)
    return fail(h, RBGS_EINVAL, "ls_iters must be in [0, 16]");
  if (opts->ls_iters == 0 && p <= 32 &&
      !hh_supported(sk->k, ((m - 1) / p) * p, (int)std::min<int64_t>(p, m)))
    return fail(h, RBGS_EUNSUPPORTED,
                "ls_iters = 0 (Householder least squares) needs k <= 1024, at most 1024 columns "
                "before the last block, and p <= 16 when k > 512");
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
  // queried once here, outside any stream capture; a device that cannot say
  // leaves 0 (the bounded waits then assume 100 MHz) and no error behind
  if (hipDeviceGetAttribute(&p->clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess) {
    p->clock_khz = 0;
    (void)hipGetLastError();
  }
  *h = p;
  return RBGS_OK;
}

rbgs_status rbgs_destroy(rbgs_handle h) {
  if (!h) return RBGS_OK;
  for (auto c : h->lanes) rbgs_destroy(c);
  if (h->ws || !h->recs.empty() || !h->pool.empty() || h->host_cert ||
      !h->lane_streams.empty() || h->graph || h->kry || h->bws) {
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    for (auto& r : h->recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    for (auto e : h->lane_ev) (void)hipEventDestroy(e);
    for (auto q : h->lane_streams) (void)hipStreamDestroy(q);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->kry) (void)hipFree(h->kry);
    if (h->bws) (void)hipFree(h->bws);
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

}  // extern "C"

namespace {

// State of one RBGS factorization in progress: the blocks are processed one
// at a time, so a caller can form W_(i) from Q_(i-1) between blocks (block
// Arnoldi) or hand all of W at once (rbgs_qr).
struct QrRun {
  rbgs_handle h;
  SketchDesc d;
  bool f32;
  int math;  // kMathF64 / kMathF32 / kMathBf16x3
  size_t es;
  hipStream_t st;
  int64_t n, m, k;
  int b, l, variant;
  const char* Wb;
  int64_t ldw;
  char* Qb;
  void* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
  double *S, *P, *E, *part, *stack, *G, *Cb, *Yb, *cscratch, *cout, *Rt, *tall;
  double *HS, *tau;  // Householder factorization of S_(1:i-1) (ls_iters = 0)
  uint16_t* plan;
  int64_t* flag;
  unsigned* counters;
  bool pair;     // dense sketches: W_(i+1) sketched together with Q_(i) (rbgs_qr only)
  bool last_s = true;  // take S_(i) = Theta Q_(i) of the last block (for S_out or certificates)
};

// Workspace, zeroed R, breakdown flag, sketch plan.  `hoist` says whether all
// of W is available now (its sketch may be taken ahead of the loop).
rbgs_status qr_begin(QrRun& r, rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m,
                     int64_t p, const rbgs_sketch* sk, const rbgs_opts* opts, void* Q, int64_t ldq,
                     double* R, int64_t ldr, double* S_out, bool hoist, void* ext_ws = nullptr,
                     size_t ext_bytes = 0) {
  r.h = h;
  r.d = make_desc(sk, n);
  r.f32 = opts->store == RBGS_STORE_F32;
  r.math = opts->math;
  r.es = r.f32 ? 4 : 8;
  r.st = (hipStream_t)opts->stream;
  r.n = n;
  r.m = m;
  r.k = r.d.k;
  r.b = (int)p;
  r.l = opts->ls_iters;
  r.variant = opts->variant;
  r.Wb = (const char*)W;
  r.ldw = ldw;
  r.Qb = (char*)Q;
  r.Q = Q;
  r.ldq = ldq;
  r.R = R;
  r.ldr = ldr;
  const SketchDesc& d = r.d;
  const int64_t k = r.k;
  const int b = r.b;
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
  const bool dense = d.kind == kGaussian || d.kind == kRademacher;
  r.pair = hoist && dense && (m + b - 1) / b > 1;
  size_t part_need = std::max(hoist && !r.pair ? sketch_partial_doubles(d, n, m) : 0,
                              sketch_partial_doubles(d, n, std::min<int64_t>(b, m)));
  if (m % b) part_need = std::max(part_need, sketch_partial_doubles(d, n, m % b));
  if (r.pair) {
    for (int64_t bw1 : {(int64_t)b, m % b}) {
      if (bw1 == 0) continue;
      const int64_t slots = dense_pair_slots(b, bw1);
      part_need = std::max(part_need, (size_t)sketch_num_partials(d, n, slots, 0) * slots * k);
    }
  }
  const size_t o_part = carve(part_need);
  const size_t o_stack = carve(qr_stack_size(k, b));
  const size_t o_plan = d.kind == kSparse ? carve((sparse_plan_bytes(d, n) + 7) / 8) : 0;
  const size_t o_flag = carve(1);
  const size_t o_cnt = carve((size_t)(2 + kQrTreeCounters) / 2);  // [0] R_(i,i) ready, [1 ..] QR tree
  const size_t o_G = carve((size_t)m * m);   // Gram matrix S^T S of the blocks done
  const size_t o_C = carve((size_t)m * b);   // c = S^T P_(i)
  const size_t o_Y = carve((size_t)m * b);   // Richardson iterate
  const size_t o_cs = carve(cert_scratch_size(k, m));
  const size_t o_cout = carve(4);
  const bool twice = r.variant == RBGS_VARIANT_TWICE || r.variant == RBGS_VARIANT_L2QR;
  const size_t o_Rt = twice ? carve((size_t)b * b) : 0;   // second R factor of a block
  size_t tall_need = 0;                                   // TSQR tree of Q'_(i)
  if (r.variant == RBGS_VARIANT_L2QR) {
    tall_need = qr_stack_size(n, (int)std::min<int64_t>(b, m));
    if (m % b) tall_need = std::max(tall_need, qr_stack_size(n, (int)(m % b)));
  }
  const size_t o_tall = tall_need ? carve(tall_need) : 0;
  const bool hh = r.l == 0;
  const size_t o_HS = hh ? carve((size_t)k * m) : 0;
  const size_t o_tau = hh ? carve((size_t)m) : 0;
  char* base;
  if (ext_ws) {
    if (off > ext_bytes)
      return fail(h, RBGS_ENOMEM, "this factorization needs " + std::to_string(off) +
                                      " bytes of workspace; the no-allocation entry point has " +
                                      std::to_string(ext_bytes));
    base = (char*)ext_ws;
  } else {
    rbgs_status rs = ensure_ws(h, off);
    if (rs != RBGS_OK) return rs;
    base = (char*)h->ws;
  }
  r.S = S_out ? S_out : (double*)(base + o_S);
  r.P = (double*)(base + o_P);
  r.E = (double*)(base + o_E);
  r.part = (double*)(base + o_part);
  r.stack = (double*)(base + o_stack);
  r.plan = d.kind == kSparse ? (uint16_t*)(base + o_plan) : nullptr;
  r.flag = (int64_t*)(base + o_flag);
  r.counters = (unsigned*)(base + o_cnt);  // [0]: R_(i,i) ready (fused update), [1 ..]: QR tree
  r.G = (double*)(base + o_G);
  r.Cb = (double*)(base + o_C);
  r.Yb = (double*)(base + o_Y);
  r.cscratch = (double*)(base + o_cs);
  r.cout = (double*)(base + o_cout);
  r.Rt = twice ? (double*)(base + o_Rt) : nullptr;
  r.tall = tall_need ? (double*)(base + o_tall) : nullptr;
  r.HS = hh ? (double*)(base + o_HS) : nullptr;
  r.tau = hh ? (double*)(base + o_tau) : nullptr;
  hipStream_t st = r.st;
  HIP_TRY(h, launch_qr_init(R, ldr, m, r.flag, r.counters, 1 + kQrTreeCounters, st), "init");
  if (r.plan) {
    ProfScope ps(h, kProfSketch, 0.0, st);
    HIP_TRY(h, launch_sparse_plan(d, n, 0, r.plan, st), "sketch plan");
  }
  if (!hoist) return RBGS_OK;
  // ---- step 1 ahead of the loop: P = Theta W (W_(i) is not modified before
  // block i, so sketching it early gives the same P_(i)) --------------------
  // Dense sketches: P_(1) here, P_(i+1) with S_(i) at the end of block i.
  if (r.pair) return do_sketch(h, d, r.f32, W, ldw, n, std::min<int64_t>(b, m), 0, r.P, k, r.part,
                               r.plan, st);
  return do_sketch(h, d, r.f32, W, ldw, n, m, 0, r.P, k, r.part, r.plan, st);
}

// Steps 1 (unless hoisted) to 5 of block i = c0 / b, reading W_(i) at Wi (ld
// ldwi) and writing Q_(i); the column block of R is filled.
rbgs_status qr_block(QrRun& r, int64_t c0, const void* Wi, int64_t ldwi, bool sketch_w) {
  rbgs_handle h = r.h;
  const SketchDesc& d = r.d;
  hipStream_t st = r.st;
  const int64_t k = r.k, n = r.n, m = r.m;
  const int b = r.b, l = r.l;
  const int bw = (int)std::min<int64_t>(b, m - c0);
  const int64_t K = c0;
  double* Pi = r.P + c0 * k;
  double* Rk = r.R + c0 * r.ldr;          // R_(1:i-1,i): rows [0, K), columns [c0, c0+bw)
  double* Rii = r.R + c0 + c0 * r.ldr;    // R_(i,i)
  const int64_t ldr = r.ldr;
  void* Qi = r.Qb + r.es * (size_t)(c0 * r.ldq);
  // the update's wait for R_(i,i) gives up after 4 s (the QR takes microseconds)
  const uint64_t wait_limit = (uint64_t)(h->clock_khz > 0 ? h->clock_khz : 100000) * 4000ull;
  rbgs_status rs;
  if (sketch_w) {
    rs = do_sketch(h, d, r.f32, Wi, ldwi, n, bw, 0, Pi, k, r.part, r.plan, st);
    if (rs != RBGS_OK) return rs;
  }
  // ---- step 2: sketched least squares ----------------------------------
  // l = 0: Householder (the factorization of S_(1:i-1) is kept up to date).
  if (K > 0 && l == 0) {
    ProfScope ps(h, kProfSmall, 0.0, st);
    HIP_TRY(h, launch_hh_solve(r.HS, r.tau, Pi, k, K, bw, Rk, ldr, st),
            "least squares: Householder");
  }
  // l >= 1 Richardson sweeps: one pass over S gives c = S^T P_(i) (sweep 1:
  // R_(1:i-1,i) = c) and the Gram block S^T S_(i-1); sweeps 2..l use the Gram
  // matrix.
  if (K > 0 && l > 0) {
    ProfScope ps(h, kProfSmall, 0.0, st);
    const int bprev = b;  // width of block i-1 (only the last block can be narrower)
    const double* Sprev = r.S + (K - bprev) * k;
    double* Ccol = (l > 1) ? r.Cb : Rk;
    const int64_t ldc = (l > 1) ? K : ldr;
    HIP_TRY(h, launch_gram_sty(r.S, k, K, Pi, bw, Sprev, bprev, Ccol, ldc, r.G + (K - bprev) * m,
                               m, r.G + (K - bprev), m, st),
            "least squares: sketch products");
    // sweeps: Y_1 = c, Y_{s+1} = Y_s + c - G Y_s.  Targets alternate between
    // R_(1:i-1,i) and Yb so that the last sweep lands in R and no sweep
    // writes its own input.
    const double* Ycur = r.Cb;
    int64_t ldycur = K;
    for (int it = 1; it < l; ++it) {
      const bool toR = ((l - 1 - it) & 1) == 0;
      double* Ynext = toR ? Rk : r.Yb;
      const int64_t ldn = toR ? ldr : K;
      HIP_TRY(h, launch_gram_sweep(r.G, m, K, r.Cb, Ycur, ldycur, Ynext, ldn, bw, st),
              "least squares: sweep");
      Ycur = Ynext;
      ldycur = ldn;
    }
  }
  const double ub = (double)r.es * (double)n * (double)(K + 2 * bw);
  if (r.variant == RBGS_VARIANT_LOWSYNC && update_fused_ok(r.math, K, bw, k)) {
    // ---- steps 4-5 with postponed sketching; the QR of S'_(i) runs inside
    // the update launch (its first workgroup), overlapping the products
    {
      ProfScope ps(h, kProfSmall, 0.0, st);
      HIP_TRY(h, launch_resid(Pi, r.S, k, K, Rk, ldr, r.E, bw, st), "S'");
    }
    {
      ProfScope ps(h, kProfUpdate, ub, st);
      HIP_TRY(h, launch_update_fused(r.f32, Wi, ldwi, r.Q, r.ldq, Qi, r.ldq, Rk, Rii, ldr, n, K,
                                     bw, r.E, k, r.flag, c0, r.counters, wait_limit, st),
              "update with the QR of the sketch");
    }
  } else if (r.variant == RBGS_VARIANT_LOWSYNC) {
    // ---- steps 4-5 with postponed sketching: S'_(i) = P_(i) - S R_(1:i-1,i)
    {
      ProfScope ps(h, kProfSmall, 0.0, st);
      const double* Sp = Pi;
      if (K > 0) {
        HIP_TRY(h, launch_resid(Pi, r.S, k, K, Rk, ldr, r.E, bw, st), "S'");
        Sp = r.E;
      }
      HIP_TRY(h, launch_qr_fused(Sp, k, bw, r.stack, r.counters + 1, Rii, ldr, r.flag, c0, st),
              "qr of sketch");
    }
    // ---- step 3 + substitution in one pass --------------------------
    {
      ProfScope ps(h, kProfUpdate, ub, st);
      HIP_TRY(h, launch_update(r.f32, r.math, Wi, ldwi, r.Q, r.ldq, Qi, r.ldq, Rk, Rii, ldr, n,
                               K, bw, st),
              "update");
    }
  } else {
    // ---- step 3: Q'_(i), stored in Q_(i) ------------------------------
    {
      ProfScope ps(h, kProfUpdate, ub, st);
      HIP_TRY(h, launch_update(r.f32, r.math, Wi, ldwi, r.Q, r.ldq, Qi, r.ldq, Rk, nullptr, ldr,
                               n, K, bw, st),
              "update");
    }
    if (r.variant == RBGS_VARIANT_L2QR) {
      // ---- step 4, l2 part: Q'_(i) = Q* R' (R' by TSQR), Q* = Q'_(i) R'^-1
      {
        ProfScope ps(h, kProfTrsm, r.es * n * bw, st);
        HIP_TRY(h, launch_qr_tall(r.f32, Qi, r.ldq, n, bw, r.tall, Rii, ldr, r.flag, c0, st),
                "l2 qr of the block");
      }
      {
        ProfScope ps(h, kProfTrsm, 2.0 * r.es * n * bw, st);
        HIP_TRY(h, launch_trsm(r.f32, Qi, r.ldq, Rii, ldr, n, bw, st), "substitution");
      }
    } else {
      // ---- step 4: S'_(i) = Theta Q'_(i), R_(i,i), substitution ---------
      rs = do_sketch(h, d, r.f32, Qi, r.ldq, n, bw, 0, r.E, k, r.part, r.plan, st);
      if (rs != RBGS_OK) return rs;
      {
        ProfScope ps(h, kProfSmall, 0.0, st);
        HIP_TRY(h, launch_qr_fused(r.E, k, bw, r.stack, r.counters + 1, Rii, ldr, r.flag, c0, st),
                "qr of sketch");
      }
      {
        ProfScope ps(h, kProfTrsm, 2.0 * r.es * n * bw, st);
        HIP_TRY(h, launch_trsm(r.f32, Qi, r.ldq, Rii, ldr, n, bw, st), "substitution");
      }
    }
    if (r.Rt) {
      // ---- RCholeskyQR of the current Q_(i) = Q_(i) R2; R_(i,i) <- R2 R_(i,i)
      rs = do_sketch(h, d, r.f32, Qi, r.ldq, n, bw, 0, r.E, k, r.part, r.plan, st);
      if (rs != RBGS_OK) return rs;
      {
        ProfScope ps(h, kProfSmall, 0.0, st);
        HIP_TRY(h, launch_qr_fused(r.E, k, bw, r.stack, r.counters + 1, r.Rt, b, r.flag, c0, st),
                "qr of sketch");
      }
      {
        ProfScope ps(h, kProfTrsm, 2.0 * r.es * n * bw, st);
        HIP_TRY(h, launch_trsm(r.f32, Qi, r.ldq, r.Rt, b, n, bw, st), "substitution");
      }
      {
        ProfScope ps(h, kProfSmall, 0.0, st);
        HIP_TRY(h, launch_trmm_upper(r.Rt, b, Rii, ldr, bw, st), "R2 R1");
      }
    }
  }
  // ---- step 5: S_(i) = Theta Q_(i) ----------------------------------------
  if (r.pair && c0 + b < m) {
    // ... together with step 1 of block i+1, P_(i+1) = Theta W_(i+1): one pass
    // over Theta, one reduction per block (the low-synchronization form)
    const int64_t bw1 = std::min<int64_t>(b, m - c0 - b);
    const void* W1 = r.Wb + r.es * (size_t)((c0 + b) * r.ldw);
    const int64_t slots = dense_pair_slots(bw, bw1);
    const int G = sketch_num_partials(d, n, slots, 0);
    const double sc = sketch_scale(d);
    {
      ProfScope ps(h, kProfSketch, r.es * (double)n * (bw + bw1), st);
      HIP_TRY(h, launch_sketch_dense_pair(d, r.f32, Qi, r.ldq, bw, W1, r.ldw, bw1, n, 0, r.part, st),
              "sketch of Q_(i) and W_(i+1)");
    }
    ProfScope ps(h, kProfReduce, 8.0 * k * (bw + bw1), st);
    HIP_TRY(h, launch_sketch_reduce(r.part, G, k, bw, sc, r.S + c0 * k, k, st, slots),
            "sketch reduction");
    HIP_TRY(h, launch_sketch_reduce(r.part + (slots - bw1) * k, G, k, bw1, sc, r.P + (c0 + b) * k, k,
                                    st, slots),
            "sketch reduction");
  } else {
    // the sketch of the last block is used only by S_out and the certificates
    if (!r.last_s && c0 + bw >= m) return RBGS_OK;
    rs = do_sketch(h, d, r.f32, Qi, r.ldq, n, bw, 0, r.S + c0 * k, k, r.part, r.plan, st);
    if (rs != RBGS_OK) return rs;
  }
  if (l == 0 && c0 + bw < m) {
    ProfScope ps(h, kProfSmall, 0.0, st);
    HIP_TRY(h, launch_hh_absorb(r.S + c0 * k, k, c0, bw, r.HS, r.tau, st),
            "least squares: Householder update");
  }
  return RBGS_OK;
}

// Step 6: certificates; the host waits for the stream.
rbgs_status qr_certify(QrRun& r, rbgs_cert* cert) {
  rbgs_handle h = r.h;
  hipStream_t st = r.st;
  HIP_TRY(h, launch_certificates(r.S, r.P, r.R, r.ldr, r.k, r.m, r.cscratch, r.cout, st),
          "certificates");
  if (!h->host_cert) HIP_TRY(h, hipHostMalloc((void**)&h->host_cert, kHostWords * sizeof(double)), "hipHostMalloc");
  HIP_TRY(h, hipMemcpyAsync(h->host_cert, r.cout, 4 * sizeof(double), hipMemcpyDeviceToHost, st),
          "copy certificate");
  HIP_TRY(h, hipMemcpyAsync(h->host_cert + 4, r.flag, sizeof(int64_t), hipMemcpyDeviceToHost, st),
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

}  // namespace

extern "C" {

rbgs_status rbgs_qr(rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m, int64_t p,
                    const rbgs_sketch* sk, const rbgs_opts* opts, void* Q, int64_t ldq,
                    double* R, int64_t ldr, double* S_out, rbgs_cert* cert) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  {
    const rbgs_status vs = validate_qr(h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr);
    if (vs != RBGS_OK) return vs;
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  QrRun r;
  rbgs_status rs = qr_begin(r, h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr, S_out, true);
  if (rs != RBGS_OK) return rs;
  r.last_s = S_out != nullptr || cert != nullptr;
  for (int64_t c0 = 0; c0 < m; c0 += p) {
    rs = qr_block(r, c0, r.Wb + r.es * (size_t)(c0 * ldw), ldw, false);
    if (rs != RBGS_OK) return rs;
  }
  if (!cert) return RBGS_OK;
  return qr_certify(r, cert);
}

rbgs_status rbgs_qr_noalloc(rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m,
                            int64_t p, const rbgs_sketch* sk, const rbgs_opts* opts, void* Q,
                            int64_t ldq, double* R, int64_t ldr, double* S_out) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  {
    const rbgs_status vs = validate_qr(h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr);
    if (vs != RBGS_OK) return vs;
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  void* ws = nullptr;
  rbgs_status rs = scratch_for_device(h, &ws);
  if (rs != RBGS_OK) return rs;
  // profiling events are created on demand, so the call records none
  const uint32_t mask = h->prof_mask;
  h->prof_mask = 0;
  QrRun r;
  rs = qr_begin(r, h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr, S_out, true, ws, kScratchBytes);
  r.last_s = S_out != nullptr;
  for (int64_t c0 = 0; rs == RBGS_OK && c0 < m; c0 += p)
    rs = qr_block(r, c0, r.Wb + r.es * (size_t)(c0 * ldw), ldw, false);
  h->prof_mask = mask;
  return rs;
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

// Grows the batch arena to `bytes` (waiting for the device and dropping the
// old contents when it must move).
rbgs_status arena_reserve(rbgs_handle h, size_t bytes) {
  if (bytes <= h->bws_bytes) return RBGS_OK;
  if (h->bws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->bws);
    h->bws = nullptr;
    h->bws_bytes = 0;
    h->pb_ctl = nullptr;
  }
  if (hipMalloc(&h->bws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    h->bws = nullptr;
    return fail(h, RBGS_ENOMEM, "batch workspace of " + std::to_string(bytes) + " bytes");
  }
  h->bws_bytes = bytes;
  return RBGS_OK;
}

// Enqueue every problem on its lane; lanes fork from and join back to st.
// ---------------------------------------------------------------------------
// Lock-step groups: problems with the same m, p and k (low-sync form, sparse
// sign, p <= 32, k <= 2048) advance block by block together, each kernel of
// a block step launched once for the whole group over a device array of
// per-problem descriptors (pointers, n, seed, prefix sums of the flattened
// grids).  The descriptors and every problem's workspace live in the
// handle's batch arena, laid out and uploaded before anything is enqueued.
// ---------------------------------------------------------------------------
struct LockGroup {
  std::vector<int64_t> idx;   // problem indices
  int64_t m = 0, p = 0, k = 0;
  BatchItem* items = nullptr; // device array in the arena
  int64_t plan_tiles = 0, up_tiles = 0, sk_wgs = 0;
};

bool lockstep_ok(const rbgs_problem& pr, const rbgs_sketch* sk, const rbgs_opts* opts) {
  return opts->variant == RBGS_VARIANT_LOWSYNC && sk->kind == RBGS_SKETCH_SPARSE_SIGN &&
         opts->ls_iters >= 1 && pr.p <= 32 && pr.k <= 2048;
}

// Groups, arena layout and descriptor upload (waits for the copy).
rbgs_status lockstep_setup(rbgs_handle h, int64_t count, const rbgs_problem* probs,
                           const rbgs_sketch* sk, const rbgs_opts* opts,
                           std::vector<LockGroup>& groups, std::vector<int64_t>& rest) {
  groups.clear();
  rest.clear();
  for (int64_t i = 0; i < count; ++i) {
    const rbgs_problem& pr = probs[i];
    if (!lockstep_ok(pr, sk, opts)) {
      rest.push_back(i);
      continue;
    }
    LockGroup* g = nullptr;
    for (auto& gg : groups)
      if (gg.m == pr.m && gg.p == pr.p && gg.k == pr.k) g = &gg;
    if (!g) {
      groups.emplace_back();
      g = &groups.back();
      g->m = pr.m;
      g->p = pr.p;
      g->k = pr.k;
    }
    g->idx.push_back(i);
  }
  // groups of one problem gain nothing: run them on the lanes
  for (size_t gi = 0; gi < groups.size();) {
    if (groups[gi].idx.size() < 2) {
      rest.push_back(groups[gi].idx[0]);
      groups.erase(groups.begin() + gi);
    } else {
      ++gi;
    }
  }
  if (groups.empty()) return RBGS_OK;
  // an earlier batch may still run out of the arena: wait before it is rewritten
  if (h->bws) HIP_TRY(h, hipDeviceSynchronize(), "synchronize before batch setup");
  const bool f32 = opts->store == RBGS_STORE_F32;
  const int64_t tile_rows = update_tile_rows(f32);
  auto r256 = [](size_t bytes) { return ((bytes + 255) / 256) * 256; };
  size_t off = 0;
  std::vector<std::vector<BatchItem>> host(groups.size());
  std::vector<size_t> items_off(groups.size());
  std::vector<std::vector<size_t>> offs(groups.size());  // per problem: 12 buffer offsets
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    LockGroup& g = groups[gi];
    const int64_t np = (int64_t)g.idx.size();
    items_off[gi] = off;
    off += r256(sizeof(BatchItem) * (size_t)np);
    host[gi].resize(np);
    const int64_t target_g = std::max<int64_t>(4, (1024 + np - 1) / np);
    for (int64_t q = 0; q < np; ++q) {
      const int64_t i = g.idx[q];
      const rbgs_problem& pr = probs[i];
      BatchItem& it = host[gi][q];
      memset(&it, 0, sizeof it);
      rbgs_sketch ski = *sk;
      ski.k = pr.k;
      ski.seed = sk->seed + (uint64_t)i;
      const SketchDesc d = make_desc(&ski, pr.n);
      const int64_t tiles = sparse_plan_tiles(pr.n);
      const int64_t G = std::min<int64_t>(tiles, target_g);
      const int64_t tpw = (tiles + G - 1) / G;
      it.W = pr.W;
      it.Q = pr.Q;
      it.n = pr.n;
      it.ldw = pr.ldw;
      it.ldq = pr.ldq;
      it.ldr = pr.ldr;
      it.R = pr.R;
      it.key0 = d.key0;
      it.key1 = d.key1;
      it.plan_tile0 = g.plan_tiles;
      g.plan_tiles += tiles;
      it.up_tile0 = g.up_tiles;
      const int64_t ut = (pr.n + tile_rows - 1) / tile_rows;
      it.up_nfull = update_vec_ok(f32, pr.Q, pr.ldq) ? pr.n / tile_rows : 0;
      g.up_tiles += ut;
      it.sk_wg0 = g.sk_wgs;
      it.sk_G = (int32_t)G;
      it.sk_tpw = tpw;
      g.sk_wgs += G;
      const int64_t m = g.m, k = g.k, b = g.p;
      std::vector<size_t> o;
      for (size_t doubles : {(size_t)(k * m), (size_t)(k * m), (size_t)(k * b), (size_t)(m * m),
                             (size_t)(m * b), (size_t)(m * b), (size_t)(G * k * m), (size_t)1,
                             qr_stack_size(k, (int)b), (size_t)(kQrTreeCounters + 1) / 2}) {
        o.push_back(off);
        off += r256(doubles * 8);
      }
      o.push_back(off);  // plan
      off += r256(sparse_plan_bytes(d, pr.n));
      o.push_back((size_t)plan_offsets_len(d, pr.n));  // entry offset (elements)
      offs[gi].insert(offs[gi].end(), o.begin(), o.end());
    }
  }
  h->pb_ctl = nullptr;
  const rbgs_status rs = arena_reserve(h, off);
  if (rs != RBGS_OK) return rs;
  char* base = (char*)h->bws;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    LockGroup& g = groups[gi];
    const size_t np = g.idx.size();
    for (size_t q = 0; q < np; ++q) {
      BatchItem& it = host[gi][q];
      const size_t* o = &offs[gi][q * 12];
      it.S = (double*)(base + o[0]);
      it.P = (double*)(base + o[1]);
      it.E = (double*)(base + o[2]);
      it.G = (double*)(base + o[3]);
      it.Cb = (double*)(base + o[4]);
      it.Yb = (double*)(base + o[5]);
      it.part = (double*)(base + o[6]);
      it.flag = (int64_t*)(base + o[7]);
      it.stack = (double*)(base + o[8]);
      it.counter = (unsigned*)(base + o[9]);
      uint16_t* plan = (uint16_t*)(base + o[10]);
      it.plan_off_w = plan;
      it.plan_ent_w = plan + o[11];
      it.plan_off = plan;
      it.plan_ent = plan + o[11];
    }
    g.items = (BatchItem*)(base + items_off[gi]);
    HIP_TRY(h, hipMemcpy(g.items, host[gi].data(), sizeof(BatchItem) * np, hipMemcpyHostToDevice),
            "upload batch descriptors");
  }
  return RBGS_OK;
}

// ---------------------------------------------------------------------------
// Persistent batch: every problem it can take (FP32 storage, FP64
// arithmetic, low-sync form, sparse sign, p <= 32, k <= 1024, the factors of
// the last block within the kernel's LDS) runs in one launch that works
// through a device queue of stages (batch_kernels.hip).  The descriptors, the
// queue and every problem's workspace live in the batch arena.
// ---------------------------------------------------------------------------
struct PersistBatch {
  std::vector<int64_t> idx;  // problem indices
  PbProb* probs = nullptr;   // device arrays in the arena
  PbStage* stages0 = nullptr;  // the queue at the start (template)
  unsigned* valid0 = nullptr;
  PbCtl* ctl0 = nullptr;
  PbStage* stages = nullptr;
  unsigned *claimed = nullptr, *finished = nullptr, *valid = nullptr;
  PbCtl* ctl = nullptr;
  unsigned total = 0;
  int64_t max_mm = 0;
};

bool persist_ok(const rbgs_problem& pr, const rbgs_sketch* sk, const rbgs_opts* opts) {
  if (opts->variant != RBGS_VARIANT_LOWSYNC || sk->kind != RBGS_SKETCH_SPARSE_SIGN ||
      opts->store != RBGS_STORE_F32 || opts->math != RBGS_MATH_F64 || sk->zeta > 8 ||
      opts->ls_iters < 1)
    return false;
  if (pr.p > kPbMaxP || pr.k > kPbMaxK) return false;
  const int64_t last_c0 = ((pr.m - 1) / pr.p) * pr.p;  // columns before the last block
  return pb_update_lds(last_c0, pr.p) <= kPbLdsBytes;
}

bool aligned16(const void* ptr, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(ptr) % 16) == 0 && ld % 4 == 0;
}

// Arena layout and descriptor upload (waits for the copy).
rbgs_status persist_setup(rbgs_handle h, int64_t count, const rbgs_problem* probs,
                          const rbgs_sketch* sk, const rbgs_opts* opts, PersistBatch& pb,
                          std::vector<int64_t>& rest) {
  pb = PersistBatch();
  rest.clear();
  h->pb_ctl = nullptr;
  for (int64_t i = 0; i < count; ++i)
    (persist_ok(probs[i], sk, opts) ? pb.idx : rest).push_back(i);
  if (pb.idx.empty()) return RBGS_OK;
  if ((int64_t)pb.idx.size() >= 65535)
    return fail(h, RBGS_EUNSUPPORTED, "persistent batch of more than 65534 problems");
  if (h->bws) HIP_TRY(h, hipDeviceSynchronize(), "synchronize before batch setup");
  const int64_t np = (int64_t)pb.idx.size();
  auto r256 = [](size_t bytes) { return ((bytes + 255) / 256) * 256; };
  std::vector<PbProb> host(np);
  std::vector<size_t> offs;  // per problem: S, P, E, G, Cb, Yb, part, flag, plan
  size_t off = 0;
  const size_t o_probs = off;
  off += r256(sizeof(PbProb) * np);
  // stages per priority level: the kinds of a problem's chain in order
  auto chain = [](int nb, auto&& visit) {
    visit(kPbPlan, 0);
    visit(kPbWsk, 0);
    visit(kPbRedw, 0);
    for (int b = 0; b < nb; ++b) {
      visit(kPbSmall, b);
      visit(kPbUpd, b);
      if (b + 1 < nb) {
        visit(kPbQsk, b);
        visit(kPbReds, b);
      }
    }
  };
  int64_t per_level[kPbLevels] = {0};
  for (int64_t q = 0; q < np; ++q) {
    const rbgs_problem& pr = probs[pb.idx[q]];
    const int nb = (int)((pr.m + pr.p - 1) / pr.p);
    chain(nb, [&](int kind, int b) { ++per_level[pb_level(nb, kind, b)]; });
  }
  int64_t total = 0;
  for (int l = 0; l < kPbLevels; ++l) total += per_level[l];
  if (total >= (int64_t)1 << 31) return fail(h, RBGS_EUNSUPPORTED, "persistent batch too large");
  const size_t o_stages0 = off;
  off += r256(sizeof(PbStage) * total);
  const size_t o_valid0 = off;
  off += r256(sizeof(unsigned) * total);
  const size_t o_ctl0 = off;
  off += r256(sizeof(PbCtl));
  const size_t o_stages = off;
  off += r256(sizeof(PbStage) * total);
  const size_t o_claimed = off;
  off += r256(sizeof(unsigned) * total);
  const size_t o_finished = off;
  off += r256(sizeof(unsigned) * total);
  const size_t o_valid = off;
  off += r256(sizeof(unsigned) * total);
  const size_t o_ctl = off;
  off += r256(sizeof(PbCtl));
  std::vector<double> work(np);
  for (int64_t q = 0; q < np; ++q) {
    const int64_t i = pb.idx[q];
    const rbgs_problem& pr = probs[i];
    rbgs_sketch ski = *sk;
    ski.k = pr.k;
    ski.seed = sk->seed + (uint64_t)i;
    const SketchDesc d = make_desc(&ski, pr.n);
    PbProb& P = host[q];
    memset(&P, 0, sizeof P);
    P.W = (const float*)pr.W;
    P.Q = (float*)pr.Q;
    P.R = pr.R;
    P.n = pr.n;
    P.ldw = pr.ldw;
    P.ldq = pr.ldq;
    P.ldr = pr.ldr;
    P.key0 = d.key0;
    P.key1 = d.key1;
    P.m = (int32_t)pr.m;
    P.p = (int32_t)pr.p;
    P.k = (int32_t)pr.k;
    P.nb = (int32_t)((pr.m + pr.p - 1) / pr.p);
    const int64_t tiles = sparse_plan_tiles(pr.n);
    P.plan_tiles = (int32_t)tiles;
    const int64_t tpw = std::min(tiles, std::max<int64_t>((tiles + kPbSkG - 1) / kPbSkG,
                                                          kPbSkMinTiles));
    P.sk_tpw = (int32_t)tpw;
    P.sk_G = (int32_t)((tiles + tpw - 1) / tpw);
    const int64_t rows = pr.p <= 16 ? kPbTileRows : kPbTileRows / 2;
    P.up_tiles = (int32_t)((pr.n + rows - 1) / rows);
    P.up_nfull = aligned16(pr.W, pr.ldw) && aligned16(pr.Q, pr.ldq) ? (int32_t)(pr.n / rows) : 0;
    pb.max_mm = std::max<int64_t>(pb.max_mm, pr.m * pr.m);
    work[q] = batch_bytes(pr, 4);
    const int64_t m = pr.m, k = pr.k, b = pr.p;
    for (size_t doubles : {(size_t)(k * m), (size_t)(k * m), (size_t)(k * b), (size_t)(m * m),
                           (size_t)(m * b), (size_t)(m * b), (size_t)(P.sk_G * k * m), (size_t)1}) {
      offs.push_back(off);
      off += r256(doubles * 8);
    }
    offs.push_back(off);
    off += r256(sparse_plan_bytes(d, pr.n));
    offs.push_back((size_t)plan_offsets_len(d, pr.n));  // entry offset (elements)
  }
  rbgs_status rs = arena_reserve(h, off);
  if (rs != RBGS_OK) return rs;
  char* base = (char*)h->bws;
  for (int64_t q = 0; q < np; ++q) {
    PbProb& P = host[q];
    const size_t* o = &offs[q * 10];
    P.S = (double*)(base + o[0]);
    P.P = (double*)(base + o[1]);
    P.E = (double*)(base + o[2]);
    P.G = (double*)(base + o[3]);
    P.Cb = (double*)(base + o[4]);
    P.Yb = (double*)(base + o[5]);
    P.part = (double*)(base + o[6]);
    P.flag = (int64_t*)(base + o[7]);
    P.plan_off = (uint16_t*)(base + o[8]);
    P.plan_ent = P.plan_off + o[9];
  }
  // the queue at the start: the first stage of every problem in its level,
  // the largest problem of a level first
  std::vector<int32_t> order(np);
  for (int64_t q = 0; q < np; ++q) order[q] = (int32_t)q;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
  PbCtl c0;
  memset(&c0, 0, sizeof c0);
  for (int l = 0, b = 0; l < kPbLevels; b += (int)per_level[l], ++l) {
    c0.base[l] = c0.head[l] = c0.tail[l] = (unsigned)b;
    c0.end[l] = (unsigned)(b + per_level[l]);
  }
  std::vector<PbStage> stages0((size_t)total);
  std::vector<unsigned> valid0((size_t)total, 0u);
  for (auto& e : stages0) e = PbStage{-1, -1, -1, 0};
  for (int32_t q : order) {
    const int l = pb_level(host[q].nb, kPbPlan, 0);
    const unsigned t = c0.tail[l]++;
    stages0[t] = PbStage{q, kPbPlan, 0, 0};  // items: filled in on the device
    valid0[t] = 1u;
  }
  pb.probs = (PbProb*)(base + o_probs);
  pb.stages0 = (PbStage*)(base + o_stages0);
  pb.valid0 = (unsigned*)(base + o_valid0);
  pb.ctl0 = (PbCtl*)(base + o_ctl0);
  pb.stages = (PbStage*)(base + o_stages);
  pb.claimed = (unsigned*)(base + o_claimed);
  pb.finished = (unsigned*)(base + o_finished);
  pb.valid = (unsigned*)(base + o_valid);
  pb.ctl = (PbCtl*)(base + o_ctl);
  pb.total = (unsigned)total;
  HIP_TRY(h, hipMemcpy(pb.probs, host.data(), sizeof(PbProb) * np, hipMemcpyHostToDevice),
          "upload batch descriptors");
  HIP_TRY(h, hipMemcpy(pb.stages0, stages0.data(), sizeof(PbStage) * total, hipMemcpyHostToDevice),
          "upload queue");
  HIP_TRY(h, hipMemcpy(pb.valid0, valid0.data(), sizeof(unsigned) * total, hipMemcpyHostToDevice),
          "upload queue");
  HIP_TRY(h, hipMemcpy(pb.ctl0, &c0, sizeof c0, hipMemcpyHostToDevice), "upload queue");
  h->pb_ctl = pb.ctl;
  h->pb_nprob = (unsigned)np;
  return RBGS_OK;
}

rbgs_status enqueue_persistent(rbgs_handle h, const PersistBatch& pb, const rbgs_sketch* sk,
                               const rbgs_opts* opts, hipStream_t st) {
  int cus = 0, rate_khz = 0;
  HIP_TRY(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device),
          "compute unit count");
  HIP_TRY(h, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, h->device),
          "wall clock rate");
  // every wait of a workgroup: at most 4 s (a stage takes milliseconds)
  const uint64_t limit = (uint64_t)std::max(rate_khz, 1) * 4000ull;
  HIP_TRY(h, launch_persistent_batch(pb.probs, (int)pb.idx.size(), pb.max_mm, pb.stages0, pb.valid0,
                                     pb.ctl0, pb.stages, pb.claimed, pb.finished, pb.valid, pb.ctl,
                                     pb.total, (int)sk->zeta, (int)opts->ls_iters, limit, cus, st),
          "persistent batch");
  return RBGS_OK;
}

// Waits for st and reads the persistent queue's control word.
rbgs_status persist_check(rbgs_handle h, hipStream_t st) {
  if (!h->pb_ctl) return RBGS_OK;
  if (!h->host_cert) HIP_TRY(h, hipHostMalloc((void**)&h->host_cert, kHostWords * sizeof(double)), "hipHostMalloc");
  HIP_TRY(h, hipMemcpyAsync(h->host_cert, h->pb_ctl, sizeof(PbCtl), hipMemcpyDeviceToHost, st),
          "copy queue state");
  HIP_TRY(h, hipStreamSynchronize(st), "persistent batch");
  PbCtl c;
  memcpy(&c, h->host_cert, sizeof c);
  if (c.error == 1u)
    return fail(h, RBGS_EDEVICE, "persistent batch: a workgroup waited too long for a stage");
  if (c.error != 0u) return fail(h, RBGS_EDEVICE, "persistent batch: queue overflow");
  bool full = true;
  for (int l = 0; l < kPbLevels; ++l) full = full && c.tail[l] == c.end[l] && c.head[l] == c.end[l];
  if (!full || c.done != h->pb_nprob)
    return fail(h, RBGS_EDEVICE, "persistent batch: " + std::to_string(h->pb_nprob - c.done) +
                                     " problems not finished");
  return RBGS_OK;
}

// Enqueue one lock-step group on st.
rbgs_status enqueue_group(rbgs_handle h, const LockGroup& g, const rbgs_sketch* sk,
                          const rbgs_opts* opts, hipStream_t st) {
  const bool f32 = opts->store == RBGS_STORE_F32;
  const int math = opts->math;
  const int np = (int)g.idx.size();
  const int64_t m = g.m, p = g.p, k = g.k;
  const int l = opts->ls_iters;
  const int zeta = sk->zeta;
  const double scale = 1.0 / sqrt((double)zeta);
  HIP_TRY(h, launch_init_batched(g.items, np, m, st), "batch init");
  HIP_TRY(h, launch_plan_batched(g.items, np, g.plan_tiles, (int)k, zeta, st), "batch plan");
  HIP_TRY(h, launch_sketch_batched(f32, g.items, np, g.sk_wgs, 0, 0, m, (int)k, zeta, scale, st),
          "batch sketch of W");
  for (int64_t c0 = 0; c0 < m; c0 += p) {
    const int bw = (int)std::min<int64_t>(p, m - c0);
    const int64_t K = c0;
    if (K > 0) {
      HIP_TRY(h, launch_gram_sty_batched(g.items, np, k, K, bw, (int)p, m, l > 1, st),
              "batch least squares: sketch products");
      int cur = 0;
      for (int it = 1; it < l; ++it) {
        const int dst = ((l - 1 - it) & 1) == 0 ? 2 : 1;
        HIP_TRY(h, launch_sweep_batched(g.items, np, m, K, bw, cur, dst, st), "batch sweep");
        cur = dst;
      }
      HIP_TRY(h, launch_resid_batched(g.items, np, k, K, bw, st), "batch S'");
    }
    HIP_TRY(h, launch_qr_batched(g.items, np, k, bw, c0, st), "batch qr of sketch");
    HIP_TRY(h, launch_update_batched(f32, math, g.items, np, g.up_tiles, K, bw, st),
            "batch update");
    HIP_TRY(h, launch_sketch_batched(f32, g.items, np, g.sk_wgs, 1, c0, bw, (int)k, zeta, scale, st),
            "batch sketch of Q");
  }
  return RBGS_OK;
}

rbgs_status enqueue_batch(rbgs_handle h, int64_t count, rbgs_problem* probs,
                          const rbgs_sketch* sk, const rbgs_opts* opts,
                          const std::vector<std::vector<int64_t>>& lane_items,
                          const std::vector<LockGroup>& groups, const PersistBatch& pb) {
  hipStream_t st = (hipStream_t)opts->stream;
  const int L = (int)lane_items.size();
  if (L > 0) HIP_TRY(h, hipEventRecord(h->lane_ev[L], st), "event record");
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
  for (const LockGroup& g : groups) {
    const rbgs_status rs = enqueue_group(h, g, sk, opts, st);
    if (rs != RBGS_OK) return rs;
    for (int64_t i : g.idx) probs[i].status = RBGS_OK;
  }
  if (!pb.idx.empty()) {
    const rbgs_status rs = enqueue_persistent(h, pb, sk, opts, st);
    if (rs != RBGS_OK) return rs;
    for (int64_t i : pb.idx) probs[i].status = RBGS_OK;
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
  if (graph < 0 || graph > 3) return fail(h, RBGS_EINVAL, "graph must be 0, 1, 2 or 3");
  const bool persistent = (graph & 2) != 0;
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
  const bool use_graph = (graph & 1) != 0 && st != nullptr;
  std::vector<int64_t> key = {count, opts->store, opts->math, opts->variant, opts->ls_iters,
                              (int64_t)(intptr_t)st, sk->kind, sk->zeta, (int64_t)sk->seed, graph};
  for (int64_t i = 0; i < count; ++i) {
    const rbgs_problem& pr = probs[i];
    for (int64_t v : {(int64_t)(intptr_t)pr.W, pr.ldw, pr.n, pr.m, (int64_t)(intptr_t)pr.Q, pr.ldq,
                      (int64_t)(intptr_t)pr.R, pr.ldr, pr.p, pr.k})
      key.push_back(v);
  }
  if (use_graph && h->graph_exec && key == h->graph_key) {
    HIP_TRY(h, hipGraphLaunch(h->graph_exec, st), "hipGraphLaunch");
    for (int64_t i = 0; i < count; ++i) probs[i].status = RBGS_OK;
    return persistent ? persist_check(h, st) : RBGS_OK;
  }
  // a recorded graph refers to the batch arena, which the setup below lays out anew
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  h->graph_key.clear();
  // lock-step groups on the caller's stream; the other problems on the lanes
  std::vector<LockGroup> groups;
  std::vector<int64_t> rest;
  PersistBatch pb;
  rbgs_status rs = persistent ? persist_setup(h, count, probs, sk, opts, pb, rest)
                              : lockstep_setup(h, count, probs, sk, opts, groups, rest);
  if (rs != RBGS_OK) return rs;
  // largest problem first, each to the least loaded lane
  const int L = (int)std::min<int64_t>(kBatchLanes, (int64_t)rest.size());
  rs = ensure_lanes(h, std::max(L, 1));
  if (rs != RBGS_OK) return rs;
  const size_t es = opts->store == RBGS_STORE_F32 ? 4 : 8;
  std::vector<int64_t> order = rest;
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
  rs = enqueue_batch(h, count, probs, sk, opts, lane_items, groups, pb);
  if (rs == RBGS_OK && !pb.idx.empty()) rs = persist_check(h, st);
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
  rs = enqueue_batch(h, count, probs, sk, opts, lane_items, groups, pb);
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

// ---------------------------------------------------------------------------
// Block Krylov solvers (Section 4).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

rbgs_status validate_csr(rbgs_handle h, const rbgs_csr* A) {
  if (!A) return fail(h, RBGS_EINVAL, "A is NULL");
  if (A->n < 1 || A->nnz < 0) return fail(h, RBGS_EINVAL, "A needs n >= 1 and nnz >= 0");
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(h, RBGS_EINVAL, "A has NULL arrays");
  if (A->n > INT32_MAX) return fail(h, RBGS_EUNSUPPORTED, "n above 2^31 - 1");
  return RBGS_OK;
}

int store_bytes(int32_t store) { return store == RBGS_STORE_F32 ? 4 : 8; }

rbgs_status ensure_kry(rbgs_handle h, size_t bytes) {
  if (bytes <= h->kry_bytes) return RBGS_OK;
  if (h->kry) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->kry);
    h->kry = nullptr;
    h->kry_bytes = 0;
  }
  if (hipMalloc(&h->kry, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, RBGS_ENOMEM, "Krylov buffers of " + std::to_string(bytes) + " bytes");
  }
  h->kry_bytes = bytes;
  return RBGS_OK;
}

// RBGS-Arnoldi on a caller-validated configuration: W_(1) at B (ld ldb),
// W_(i) = A Q_(i-1) formed in place in Q.
rbgs_status arnoldi_run(rbgs_handle h, const rbgs_csr* A, const void* B, int64_t ldb, int64_t bs,
                        int64_t nblocks, const rbgs_sketch* sk, const rbgs_opts* opts, void* Q,
                        int64_t ldq, double* R, int64_t ldr, rbgs_cert* cert) {
  const int64_t n = A->n, m = nblocks * bs;
  const int es = store_bytes(opts->store);
  QrRun r;
  rbgs_status rs = qr_begin(r, h, Q, ldq, n, m, bs, sk, opts, Q, ldq, R, ldr, nullptr, false);
  if (rs != RBGS_OK) return rs;
  rs = qr_block(r, 0, B, ldb, true);
  if (rs != RBGS_OK) return rs;
  char* Qb = (char*)Q;
  for (int64_t i = 1; i < nblocks; ++i) {
    void* Qi = Qb + (size_t)es * (size_t)(i * bs * ldq);
    const void* Qp = Qb + (size_t)es * (size_t)((i - 1) * bs * ldq);
    HIP_TRY(h, launch_spmm(n, A->row_ptr, A->col_idx, A->val, es, Qp, ldq, (int)bs, 1.0, 0.0,
                           nullptr, 0, es, Qi, ldq, r.st),
            "A Q_(i-1)");
    rs = qr_block(r, i * bs, Qi, ldq, true);
    if (rs != RBGS_OK) return rs;
  }
  return cert ? qr_certify(r, cert) : RBGS_OK;
}

}  // namespace

extern "C" {

rbgs_status rbgs_spmm(rbgs_handle h, const rbgs_csr* A, int32_t xstore, const void* X, int64_t ldx,
                      int64_t bs, double alpha, double beta, const double* Y0, int64_t ldy0,
                      int32_t ystore, void* Y, int64_t ldy, void* stream) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  rbgs_status vs = validate_csr(h, A);
  if (vs != RBGS_OK) return vs;
  if (!X || !Y) return fail(h, RBGS_EINVAL, "X and Y must be non-NULL");
  if (bs < 1 || bs > 32) return fail(h, bs < 1 ? RBGS_EINVAL : RBGS_EUNSUPPORTED, "need 1 <= bs <= 32");
  if ((xstore != RBGS_STORE_F32 && xstore != RBGS_STORE_F64) ||
      (ystore != RBGS_STORE_F32 && ystore != RBGS_STORE_F64))
    return fail(h, RBGS_EINVAL, "unknown storage type");
  const int64_t n = A->n;
  if (ldx < n || ldy < n || (Y0 && ldy0 < n)) return fail(h, RBGS_EINVAL, "leading dimensions must be >= n");
  {
    const char* x0 = (const char*)X;
    const char* x1 = x0 + (size_t)store_bytes(xstore) * (size_t)(ldx * (bs - 1) + n);
    const char* y0 = (const char*)Y;
    const char* y1 = y0 + (size_t)store_bytes(ystore) * (size_t)(ldy * (bs - 1) + n);
    if (y0 < x1 && x0 < y1) return fail(h, RBGS_EINVAL, "Y overlaps X");
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  HIP_TRY(h, launch_spmm(n, A->row_ptr, A->col_idx, A->val, store_bytes(xstore), X, ldx, (int)bs,
                         alpha, beta, Y0, ldy0, store_bytes(ystore), Y, ldy, (hipStream_t)stream),
          "spmm");
  return RBGS_OK;
}

rbgs_status rbgs_block_arnoldi(rbgs_handle h, const rbgs_csr* A, const void* B, int64_t ldb,
                               int64_t bs, int64_t nblocks, const rbgs_sketch* sk,
                               const rbgs_opts* opts, void* Q, int64_t ldq, double* R, int64_t ldr,
                               rbgs_cert* cert) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  rbgs_status vs = validate_csr(h, A);
  if (vs != RBGS_OK) return vs;
  if (!B) return fail(h, RBGS_EINVAL, "B is NULL");
  if (bs < 1 || nblocks < 1) return fail(h, RBGS_EINVAL, "need bs >= 1 and nblocks >= 1");
  const int64_t n = A->n, m = nblocks * bs;
  if (ldb < n) return fail(h, RBGS_EINVAL, "ldb must be >= n");
  // Q plays W (formed block by block in place): the checks of rbgs_qr apply
  vs = validate_qr(h, Q, ldq, n, m, bs, sk, opts, Q, ldq, R, ldr);
  if (vs != RBGS_OK) return vs;
  {
    const size_t es = (size_t)store_bytes(opts->store);
    const char* b0 = (const char*)B;
    const char* b1 = b0 + es * (size_t)(ldb * (bs - 1) + n);
    const char* q0 = (const char*)Q;
    const char* q1 = q0 + es * (size_t)(ldq * (m - 1) + n);
    if (b0 < q1 && q0 < b1) return fail(h, RBGS_EINVAL, "B overlaps Q");
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  return arnoldi_run(h, A, B, ldb, bs, nblocks, sk, opts, Q, ldq, R, ldr, cert);
}

rbgs_status rbgs_block_gmres(rbgs_handle h, const rbgs_csr* A, const double* B, double* X,
                             int64_t bs, int64_t blocks_per_cycle, int64_t max_cycles, double tol,
                             const rbgs_sketch* sk, const rbgs_opts* opts, int64_t* iters,
                             double* relres, double* history) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  rbgs_status vs = validate_csr(h, A);
  if (vs != RBGS_OK) return vs;
  if (!B || !X || !iters || !relres) return fail(h, RBGS_EINVAL, "NULL argument");
  if (bs < 1 || bs > 32) return fail(h, bs < 1 ? RBGS_EINVAL : RBGS_EUNSUPPORTED, "need 1 <= bs <= 32");
  if (blocks_per_cycle < 1 || max_cycles < 1 || !(tol >= 0.0))
    return fail(h, RBGS_EINVAL, "need blocks_per_cycle >= 1, max_cycles >= 1, tol >= 0");
  const int64_t n = A->n, nb = blocks_per_cycle + 1, m = nb * bs;
  if (m > n) return fail(h, RBGS_EINVAL, "(blocks_per_cycle + 1) bs must not exceed n");
  if ((const void*)B == (const void*)X) return fail(h, RBGS_EINVAL, "B and X must differ");
  const size_t es = (size_t)store_bytes(opts ? opts->store : RBGS_STORE_F64);
  // buffers: basis | R | T (residual) | LS matrix | Z | resid | sumsq scratch | norms
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    size_t o = off;
    off += ((bytes + 255) / 256) * 256;
    return o;
  };
  const size_t o_Q = carve(es * (size_t)(n * m));
  const size_t o_R = carve(8 * (size_t)(m * m));
  const size_t o_T = carve(8 * (size_t)(n * bs));
  const size_t o_A = carve(8 * (size_t)(m * m));
  const size_t o_Z = carve(8 * (size_t)(m * bs));
  const size_t o_res = carve(8 * (size_t)bs);
  const size_t o_ss = carve(8 * sumsq_scratch());
  const size_t o_nrm = carve(8 * 2);
  // validate the Arnoldi configuration with the basis location as a stand-in
  // (device pointers are not dereferenced by validation)
  {
    const char* fake = (const char*)(uintptr_t)0x1000;
    vs = validate_qr(h, fake, n, n, m, bs, sk, opts, (void*)fake, n, (double*)(fake + es * (size_t)(n * m) + 4096), m);
    if (vs != RBGS_OK) return vs;
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  rbgs_status rs = ensure_kry(h, off);
  if (rs != RBGS_OK) return rs;
  if (!h->host_cert) HIP_TRY(h, hipHostMalloc((void**)&h->host_cert, kHostWords * sizeof(double)), "hipHostMalloc");
  char* base = (char*)h->kry;
  void* Qb = base + o_Q;
  double* Rm = (double*)(base + o_R);
  double* T = (double*)(base + o_T);
  double* Als = (double*)(base + o_A);
  double* Z = (double*)(base + o_Z);
  double* res = (double*)(base + o_res);
  double* ss = (double*)(base + o_ss);
  double* nrm = (double*)(base + o_nrm);
  hipStream_t st = (hipStream_t)opts->stream;
  const bool f32 = opts->store == RBGS_STORE_F32;
  auto norm2_to_host = [&](const double* Y, double* out) -> rbgs_status {
    HIP_TRY(h, launch_sumsq(Y, n, n, (int)bs, ss, nrm, st), "norm");
    HIP_TRY(h, hipMemcpyAsync(h->host_cert, nrm, sizeof(double), hipMemcpyDeviceToHost, st), "copy norm");
    HIP_TRY(h, hipStreamSynchronize(st), "stream synchronize");
    *out = h->host_cert[0];
    return RBGS_OK;
  };
  auto residual = [&](double* out_rel) -> rbgs_status {
    HIP_TRY(h, launch_spmm(n, A->row_ptr, A->col_idx, A->val, 8, X, n, (int)bs, -1.0, 1.0, B, n, 8,
                           T, n, st),
            "residual");
    double rr = 0.0;
    rbgs_status r2 = norm2_to_host(T, &rr);
    if (r2 != RBGS_OK) return r2;
    *out_rel = rr;
    return RBGS_OK;
  };
  double bb = 0.0;
  rs = norm2_to_host(B, &bb);
  if (rs != RBGS_OK) return rs;
  if (history)
    for (int64_t c = 0; c <= max_cycles; ++c) history[c] = -1.0;
  const double bnorm = sqrt(bb);
  int64_t done = 0;
  double rel = 0.0;
  bool converged = false;
  int64_t c = 0;
  for (; c < max_cycles; ++c) {
    double rr = 0.0;
    rs = residual(&rr);
    if (rs != RBGS_OK) return rs;
    rel = bnorm > 0 ? sqrt(rr) / bnorm : sqrt(rr);
    if (history) history[c] = rel;
    if (rel <= tol) {
      converged = true;
      break;
    }
    // W_(1) = R0 in the basis precision, then RBGS-Arnoldi in place
    HIP_TRY(h, launch_convert(T, n, n, (int)bs, f32, Qb, n, st), "residual to basis");
    rs = arnoldi_run(h, A, Qb, n, bs, nb, sk, opts, Qb, n, Rm, m, nullptr);
    if (rs != RBGS_OK) return rs;
    // min_Z ||H Z - R_(1:p,1)||, H = R[:, bs:m] (block upper Hessenberg)
    const int64_t nc = m - bs;
    HIP_TRY(h, hipMemcpyAsync(Als, Rm + bs * m, 8 * (size_t)(m * nc), hipMemcpyDeviceToDevice, st),
            "copy H");
    HIP_TRY(h, hipMemcpyAsync(Als + nc * m, Rm, 8 * (size_t)(m * bs), hipMemcpyDeviceToDevice, st),
            "copy R_(1:p,1)");
    HIP_TRY(h, launch_hess_ls(Als, m, (int)m, (int)nc, (int)bs, (int)bs, Z, nc, res, st),
            "Hessenberg least squares");
    HIP_TRY(h, launch_gemm_update(f32, n, (int)nc, (int)bs, Qb, n, Z, nc, X, n, st), "X += Q Z");
    done += blocks_per_cycle;
  }
  if (!converged) {
    double rr = 0.0;
    rs = residual(&rr);
    if (rs != RBGS_OK) return rs;
    rel = bnorm > 0 ? sqrt(rr) / bnorm : sqrt(rr);
    if (history) history[c] = rel;
    converged = rel <= tol;
  }
  *iters = done;
  *relres = rel;
  if (!converged) return fail(h, RBGS_ENOTCONV, "relative residual " + std::to_string(rel) + " above tol");
  return RBGS_OK;
}

rbgs_status rbgs_cholqr_post(rbgs_handle h, int32_t store, void* Q, int64_t ldq, int64_t n,
                             int64_t m, double* R, int64_t ldr, int64_t* breakdown_col,
                             void* stream) {
  if (!h) return RBGS_EINVAL;
  h->last_error.clear();
  if (!Q || !R) return fail(h, RBGS_EINVAL, "Q and R must be non-NULL");
  if (n < 1 || m < 1 || m > n) return fail(h, RBGS_EINVAL, "need 1 <= m <= n");
  if (m > 8192) return fail(h, RBGS_EUNSUPPORTED, "m > 8192 is not implemented");
  if (ldq < n || ldr < m) return fail(h, RBGS_EINVAL, "bad leading dimension");
  if (store != RBGS_STORE_F64 && store != RBGS_STORE_F32) return fail(h, RBGS_EINVAL, "unknown storage type");
  const bool f32 = store == RBGS_STORE_F32;
  const size_t es = f32 ? 4 : 8;
  {
    const char* q0 = (const char*)Q;
    const char* q1 = q0 + es * (size_t)(ldq * (m - 1) + n);
    const char* r0 = (const char*)R;
    const char* r1 = r0 + 8 * (size_t)(ldr * (m - 1) + m);
    if (r0 < q1 && q0 < r1) return fail(h, RBGS_EINVAL, "R overlaps Q");
  }
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  const size_t mm = (size_t)m * m;
  const size_t part = (size_t)gram_splits(n, m) * mm;
  auto r256 = [](size_t doubles) { return ((doubles * 8 + 255) / 256) * 256; };
  rbgs_status rs = ensure_ws(h, r256(part) + 2 * r256(mm) + 256);
  if (rs != RBGS_OK) return rs;
  char* base = (char*)h->ws;
  double* partial = (double*)base;
  double* G = (double*)(base + r256(part));
  double* T = (double*)(base + r256(part) + r256(mm));
  int64_t* flag = (int64_t*)(base + r256(part) + 2 * r256(mm));
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(h, launch_set_i64(flag, -1, st), "flag");
  HIP_TRY(h, launch_gram(f32, Q, ldq, n, m, partial, G, st), "gram");
  HIP_TRY(h, launch_cholesky(G, m, flag, st), "cholesky");
  // Q <- Q R'^{-1} block column by block column: X_b = (Q_b - X_(1:b-1) R'_(1:b-1,b)) R'_bb^{-1}
  for (int64_t b0 = 0; b0 < m; b0 += 16) {
    const int bw = (int)std::min<int64_t>(16, m - b0);
    char* Qb = (char*)Q + es * (size_t)(b0 * ldq);
    HIP_TRY(h, launch_update(f32, kMathF64, Qb, ldq, Q, ldq, Qb, ldq, G + b0 * m, G + b0 + b0 * m, m, n,
                             b0, bw, st),
            "substitution");
  }
  HIP_TRY(h, launch_trmm_full(G, m, R, ldr, m, T, st), "R' R");
  if (!breakdown_col) return RBGS_OK;
  if (!h->host_cert) HIP_TRY(h, hipHostMalloc((void**)&h->host_cert, kHostWords * sizeof(double)), "hipHostMalloc");
  HIP_TRY(h, hipMemcpyAsync(h->host_cert + 4, flag, sizeof(int64_t), hipMemcpyDeviceToHost, st),
          "copy flag");
  HIP_TRY(h, hipStreamSynchronize(st), "stream synchronize");
  memcpy(breakdown_col, h->host_cert + 4, sizeof(int64_t));
  if (*breakdown_col >= 0) return fail(h, RBGS_EBREAKDOWN, "Q^T Q is not positive definite in FP64");
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
  if (sk->kind == RBGS_SKETCH_SRHT && sk->zeta > 0 && row0 + n > ((int64_t)1 << sk->zeta))
    return fail(h, RBGS_EINVAL, "rows beyond the SRHT transform size 2^zeta");
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  const SketchDesc d = make_desc(sk, row0 + n);
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
  if (sk->kind == RBGS_SKETCH_SRHT && sk->zeta > 0 && row0 + n > ((int64_t)1 << sk->zeta))
    return fail(h, RBGS_EINVAL, "rows beyond the SRHT transform size 2^zeta");
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, RBGS_EDEVICE, "hipSetDevice failed");
  HIP_TRY(h, launch_theta_dense(make_desc(sk, row0 + n), n, row0, out, (hipStream_t)stream),
          "theta_dense");
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
