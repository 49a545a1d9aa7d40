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

#include "rbgs.h"

int main(int argc, char** argv) {
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
