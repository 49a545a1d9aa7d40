// Drives the library's host code against the recording HIP stand-in
// (mock_hip.cpp): one rbgs_qr call per invocation, with the caller's W, Q, R
// and S allocated through the stand-in, so that every address a kernel is given
// can be matched to an allocation (test infrastructure).
//   driver n m p k kind store math variant ls_iters want_S want_cert [noalloc]
// noalloc = 1: rbgs_qr_noalloc (the library's scratch array; want_cert ignored),
// called twice, the second time on the first half of the rows.
// kind: 0 Gaussian, 1 sparse sign, 3 Rademacher, 4 SRHT; store/math/variant as
// in include/rbgs.h.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "rbgs.h"

// driver batch count p kmult ragged_ld: rbgs_qr_batched with the persistent
// queue (graph = 2) over `count` FP32 problems of mixed shapes (n from 1000 to
// 262144, m from 32 to 256), block width p, k = min(kmult m, 1024); ragged_ld
// = 1 gives every odd problem a leading dimension one larger than n.
// driver batchs "n,m,p,k,ld;...": the same with the problems listed (ld 0: n).
static int batch_main(int argc, char** argv) {
  if (argc < 3) return 2;
  struct Spec {
    int64_t n, m, p, k, ld;
  };
  std::vector<Spec> specs;
  if (argv[1][5] == 's') {
    const char* c = argv[2];
    while (*c) {
      Spec sp;
      if (sscanf(c, "%lld,%lld,%lld,%lld,%lld", (long long*)&sp.n, (long long*)&sp.m,
                 (long long*)&sp.p, (long long*)&sp.k, (long long*)&sp.ld) != 5)
        return 2;
      if (sp.ld == 0) sp.ld = sp.n;
      specs.push_back(sp);
      while (*c && *c != ';') ++c;
      if (*c == ';') ++c;
    }
  } else {
    if (argc < 6) return 2;
    const int count = atoi(argv[2]);
    const int64_t p = atoll(argv[3]), kmult = atoll(argv[4]);
    const int ragged = atoi(argv[5]);
    static const int64_t ns[] = {16384, 20001, 65573, 262144, 4097, 1000, 131072, 8191};
    static const int64_t ms[] = {32, 64, 128, 256, 40, 200, 100, 72};
    for (int i = 0; i < count; ++i) {
      Spec sp;
      sp.n = ns[i % 8];
      sp.m = ms[(i / 2) % 8];
      if (sp.m > sp.n) sp.m = 32;
      sp.ld = sp.n + ((ragged && (i & 1)) ? 1 : 0);
      sp.p = p < sp.m ? p : sp.m;
      int64_t k = kmult * sp.m;
      k = k < 1024 ? k : 1024;
      k = (k + 7) / 8 * 8;
      sp.k = k < sp.n ? k : sp.n / 8 * 8;
      specs.push_back(sp);
    }
  }
  const int count = (int)specs.size();
  rbgs_problem* probs = new rbgs_problem[count];
  for (int i = 0; i < count; ++i) {
    rbgs_problem& pr = probs[i];
    pr.n = specs[i].n;
    pr.m = specs[i].m;
    pr.ldw = pr.ldq = specs[i].ld;
    pr.ldr = pr.m;
    void *W, *Q, *R;
    (void)hipMalloc(&W, 4 * (size_t)pr.ldw * (size_t)pr.m);
    (void)hipMalloc(&Q, 4 * (size_t)pr.ldq * (size_t)pr.m);
    (void)hipMalloc(&R, 8 * (size_t)pr.m * (size_t)pr.m);
    pr.W = W;
    pr.Q = Q;
    pr.R = (double*)R;
    pr.p = specs[i].p;
    pr.k = specs[i].k;
    pr.status = 0;
    pr.reserved = 0;
  }
  rbgs_handle h;
  rbgs_create(&h, 0);
  rbgs_sketch sk;
  sk.kind = RBGS_SKETCH_SPARSE_SIGN;
  sk.zeta = 8;
  sk.k = 0;
  sk.seed = 0x2111146414ull;
  rbgs_opts o;
  o.store = RBGS_STORE_F32;
  o.math = RBGS_MATH_F64;
  o.variant = RBGS_VARIANT_LOWSYNC;
  o.ls_iters = 4;
  o.stream = nullptr;
  const rbgs_status st = rbgs_qr_batched(h, count, probs, &sk, &o, 2);
  printf("status %d %s\n", (int)st, rbgs_last_error(h));
  rbgs_destroy(h);
  delete[] probs;
  return st == RBGS_OK ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc > 1 && argv[1][0] == 'b') return batch_main(argc, argv);
  if (argc < 12) {
    fprintf(stderr, "usage: driver n m p k kind store math variant ls_iters want_S want_cert\n");
    return 2;
  }
  const int64_t n = atoll(argv[1]), m = atoll(argv[2]), p = atoll(argv[3]), k = atoll(argv[4]);
  const int kind = atoi(argv[5]), store = atoi(argv[6]), math = atoi(argv[7]);
  const int variant = atoi(argv[8]), ls = atoi(argv[9]), want_S = atoi(argv[10]);
  const int want_cert = atoi(argv[11]);
  const size_t es = store == RBGS_STORE_F32 ? 4 : 8;
  void *W, *Q, *R, *S = nullptr;
  (void)hipMalloc(&W, es * (size_t)n * (size_t)m);
  (void)hipMalloc(&Q, es * (size_t)n * (size_t)m);
  (void)hipMalloc(&R, 8 * (size_t)m * (size_t)m);
  if (want_S) (void)hipMalloc(&S, 8 * (size_t)k * (size_t)m);
  rbgs_handle h;
  rbgs_create(&h, 0);
  rbgs_sketch sk;
  sk.kind = kind;
  sk.zeta = kind == RBGS_SKETCH_SPARSE_SIGN ? 8 : 0;
  sk.k = k;
  sk.seed = 0x2111146412ull;
  rbgs_opts o;
  o.store = store;
  o.math = math;
  o.variant = variant;
  o.ls_iters = ls;
  o.stream = nullptr;
  rbgs_cert cert;
  const int noalloc = argc > 12 ? atoi(argv[12]) : 0;
  rbgs_status st;
  if (noalloc) {
    st = rbgs_qr_noalloc(h, W, n, n, m, p, &sk, &o, Q, n, (double*)R, m, (double*)S);
    if (st == RBGS_OK)
      st = rbgs_qr_noalloc(h, W, n, n / 2, m, p, &sk, &o, Q, n, (double*)R, m, (double*)S);
  } else {
    st = rbgs_qr(h, W, n, n, m, p, &sk, &o, Q, n, (double*)R, m, (double*)S,
                 want_cert ? &cert : nullptr);
  }
  printf("status %d %s\n", (int)st, rbgs_last_error(h));
  rbgs_destroy(h);
  return st == RBGS_OK ? 0 : 1;
}
