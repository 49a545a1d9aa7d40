"""RBGS QR on the GPU (through the C ABI) against the FP64 oracle.

Every comparison of Q, R and S is made entry by entry against a per-entry
scale derived from a perturbation bound (tests/parity_checks.py), and the
certificates Delta, Delta~ are compared with the oracle's certificate routine
evaluated on the GPU's own S and R.  The relative Frobenius checks stay beside
them.  Tolerances (u = 2^-53, u32 = 2^-24):
* FP64 storage, same Theta bits on both sides, so the two computations differ
  only in summation order (and the GPU's multiplication by 1/R_cc in the
  substitution).  Entry-wise: |x - x_or| <= TOL64 * scale with TOL64 = 4096 u
  (a reordering of the oracle's own sums gives at most about 30 u on these
  scales).  Norm-wise: R <= 1e-12, Q <= 1e-12 for cond(W) = 1e2 and <= 1e-6
  for cond(W) = 1e8.
* FP32 storage with FP64 arithmetic (only Q'_(i) is rounded to FP32) is
  compared with the oracle run on the same fp32-rounded input: the rounding of
  each stored Q_(i) (u32 |Q_(i)|) propagates through R^{-1}, so entry-wise
  |x - x_or| <= 64 u32 cond(W) * scale, and the benchmark spec's metrics
  ||W - QR||_F/||W||_F <= 1e-6 and cond2(Q) <= 10.
"""
import sys

import numpy as np
import pytest

import oracle.rbgs as orb
import parity_checks as pc
from oracle.metrics import cond2, factorization_error
from oracle.theta import Sketch
from paper_2111_14641_amd.workloads import svd_matrix, small_single_qr, THETA_SEED_SMALL

pytestmark = pytest.mark.gpu

U64 = 2.0**-53
U32 = 2.0**-24
TOL64 = 4096 * U64


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_qr(W, b, kind, k, seed, variant, store="f64", ls_iters=2, zeta=None, inplace=False, math="f64"):
    import torch
    from paper_2111_14641_amd import binding as B
    n, m = W.shape
    dt = torch.float64 if store == "f64" else torch.float32
    Wt = B.colmajor(n, m, dt)
    Wt.copy_(torch.from_numpy(np.asarray(W, dtype=np.float64)))
    Q, R, S, cert = B.rbgs_qr(Wt, b, kind, k, seed, zeta, variant, ls_iters,
                              Q=Wt if inplace else None, want_S=True, want_cert=True, math=math)
    torch.cuda.synchronize()
    to = lambda t: np.ascontiguousarray(t.cpu().numpy()).astype(np.float64)
    return to(Q), to(R), to(S), cert


def oracle_qr(W, b, kind, k, seed, variant, ls_iters=2, zeta=None):
    th = Sketch(kind, k, seed=seed, zeta=zeta).materialize(W.shape[0])
    o = orb.rbgs(W, b, th, variant, "richardson", ls_iters)
    o["absT"] = pc.abs_theta(th, W.shape[0])
    return o


def check_entrywise(W, Q, R, S, cert, o, tol_r, tol_q=None, tol_s=None, certs=True):
    """Entry-wise Q, R, S against the oracle and the certificates against the
    oracle's routine on the GPU's S and R."""
    pc.assert_qrs_entrywise(Q, R, S, o, o["absT"], tol_r, tol_q if tol_q is not None else tol_r,
                            tol_s)
    if certs and cert is not None and S is not None:
        pc.check_certificates(cert, S, R, o["P"], pc.abs_theta_w_fro(o["absT"], W), W.shape[0])


@pytest.fixture(scope="module")
def small():
    return small_single_qr()


@pytest.mark.parametrize("variant", ["plain", "lowsync"])
def test_small_workload_fp64_matches_oracle(gpu_lib, small, variant):
    """n = 10 000, m = 64, p = 8, Gaussian k = 256, cond(W) = 1e8."""
    W = small
    say("small fp64", variant)
    Q, R, S, cert = gpu_qr(W, 8, "gaussian", 256, THETA_SEED_SMALL, variant)
    o = oracle_qr(W, 8, "gaussian", 256, THETA_SEED_SMALL, variant)
    assert rel(R, o["R"]) < 1e-12
    assert rel(Q, o["Q"]) < 1e-6
    assert rel(S, o["S"]) < 1e-6
    check_entrywise(W, Q, R, S, cert, o, TOL64)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert factorization_error(W, Q, R) < 1e-14
    assert abs(cond2(Q) - cond2(o["Q"])) < 1e-6
    assert cert["breakdown_col"] == -1 and cert["nonfinite"] == 0
    assert cert["delta"] == pytest.approx(o["delta"], rel=0.5, abs=1e-12)
    assert cert["delta_tilde"] < 1e-14


@pytest.mark.parametrize("variant", ["plain", "lowsync"])
@pytest.mark.parametrize("kind,k", [("gaussian", 256), ("sparse", 256), ("rademacher", 256),
                                    ("srht", 256)])
def test_well_conditioned_fp64_elementwise(gpu_lib, variant, kind, k):
    W = svd_matrix(10_000, 64, np.logspace(0, -2, 64), seed=5)
    say("well-conditioned", variant, kind)
    Q, R, S, cert = gpu_qr(W, 8, kind, k, 17, variant)
    o = oracle_qr(W, 8, kind, k, 17, variant)
    assert rel(R, o["R"]) < 1e-12
    assert rel(Q, o["Q"]) < 1e-12
    assert rel(S, o["S"]) < 1e-12
    check_entrywise(W, Q, R, S, cert, o, TOL64)
    assert cert["delta"] < 1e-12


@pytest.mark.parametrize("n,m,b,k,kind,variant", [
    (4097, 30, 8, 128, "sparse", "lowsync"),       # ragged rows and last block
    (4097, 30, 8, 128, "gaussian", "plain"),
    (5000, 17, 1, 64, "sparse", "plain"),           # single-column blocks
    (3000, 24, 24, 96, "gaussian", "lowsync"),      # one block
    (2000, 1, 4, 8, "sparse", "lowsync"),           # m = 1
    (1000, 32, 32, 32, "gaussian", "lowsync"),      # k = m, widest block
    (64, 16, 4, 64, "identity", "plain"),           # Theta = I
    (300, 20, 6, 300, "identity", "lowsync"),
    (9000, 40, 16, 2048, "sparse", "lowsync"),      # largest sparse k
    (5000, 96, 32, 256, "gaussian", "lowsync"),     # widest blocks after the first (2 x 16 columns)
    (5000, 96, 32, 256, "sparse", "plain"),
    (3000, 70, 32, 512, "sparse", "lowsync"),       # 32-wide tree over 4 chunks, ragged last block
    (4000, 72, 24, 256, "gaussian", "plain"),       # width 24 padded to 32 in the tree
    (4097, 30, 8, 132, "rademacher", "lowsync"),    # Rademacher, partial last Philox call
    (3000, 40, 16, 256, "rademacher", "plain"),
    (4097, 30, 8, 128, "sparse", "twice"),          # two-pass forms: ragged rows and last block
    (5000, 17, 1, 64, "gaussian", "l2qr"),          # TSQR of single columns
    (3000, 70, 32, 512, "sparse", "l2qr"),          # 32-wide TSQR over four tree levels
    (4000, 72, 24, 256, "rademacher", "twice"),
    (4097, 75, 24, 256, "sparse", "lowsync"),       # 24-wide blocks: the 32-column update form
    (6000, 64, 32, 2048, "sparse", "lowsync"),      # QR tree of the sketch: 16 chunks, 4 groups, 2 levels
    (5000, 72, 24, 1536, "gaussian", "lowsync"),    # ragged groups (5 R factors of 24 rows per chunk)
    (8192, 40, 32, 8192, "identity", "plain"),      # 64 chunks, three levels of groups
    (9000, 96, 32, 512, "gaussian", "plain"),
    (64, 16, 4, 64, "identity", "l2qr"),
    (300, 20, 6, 300, "identity", "twice"),
    (4097, 30, 8, 128, "srht", "lowsync"),          # SRHT: ragged chunk, transform of 2^13
    (3000, 40, 16, 2048, "srht", "plain"),          # SRHT with two outputs per thread
])
def test_shapes_fp64(gpu_lib, n, m, b, k, kind, variant):
    W = svd_matrix(n, m, np.logspace(0, -2, m), seed=n + m + b)
    say("shape", n, m, b, k, kind, variant)
    Q, R, S, cert = gpu_qr(W, b, kind, k, 23, variant)
    o = oracle_qr(W, b, kind, k, 23, variant)
    assert rel(R, o["R"]) < 1e-12
    assert rel(Q, o["Q"]) < 1e-11
    check_entrywise(W, Q, R, S, cert, o, TOL64)
    assert factorization_error(W, Q, R) < 1e-14
    if kind == "identity":
        Qh, Rh = np.linalg.qr(W)
        d = np.sign(np.diag(Rh))
        assert rel(R, d[:, None] * Rh) < 1e-13


@pytest.mark.parametrize("variant", ["plain", "lowsync", "twice", "l2qr"])
@pytest.mark.parametrize("decades", [2, 8])
def test_fp32_storage_fp64_arithmetic(gpu_lib, variant, decades):
    """FP32 storage, FP64 products: Q'_(i) is accurate to u32 relative to itself,
    so the result matches the oracle on the same fp32 input to O(u32 cond) and
    stays well conditioned even when W is numerically rank deficient in FP32."""
    W = svd_matrix(10_000, 64, np.logspace(0, -decades, 64), seed=31).astype(np.float32).astype(np.float64)
    say("fp32 storage fp64 math", variant, decades)
    Q, R, S, cert = gpu_qr(W, 8, "gaussian", 256, THETA_SEED_SMALL, variant, store="f32")
    o = oracle_qr(W, 8, "gaussian", 256, THETA_SEED_SMALL, variant)
    assert factorization_error(W, Q, R) <= 1e-6
    assert cond2(Q) <= 10
    assert np.all(np.diag(R) > 0)
    assert cert["delta"] < 1e-4
    assert rel(R, o["R"]) <= 64 * 2.0**-24 * 10**decades
    if decades == 2:
        assert rel(Q, o["Q"]) <= 64 * 2.0**-24 * 1e2
    # entry-wise against the oracle on the same fp32 input; Q and S (whose
    # columns inherit the FP32 rounding of the stored blocks) where W is
    # numerically full rank in FP32
    tol = 64 * U32 * 10**decades
    check_entrywise(W, Q, R, S if decades == 2 else None, cert, o, tol,
                    tol_q=tol if decades == 2 else np.inf)
    pc.check_certificates(cert, S, R, o["P"], pc.abs_theta_w_fro(o["absT"], W), W.shape[0])


@pytest.mark.parametrize("variant", ["plain", "lowsync"])
@pytest.mark.parametrize("n,m,b", [
    (7777, 40, 5),      # K = 5, 10, ..: steps past K - K % 4 read a clamped column
    (7777, 42, 6),      # K % 4 = 2, ragged last block of 2 columns
    (5000, 70, 10),     # partial 16-column group in every block
    (9000, 100, 16),    # full 16-column blocks (row-layout epilogue) and a last block of 4
    (300, 48, 16),      # one full tile and a ragged one: a workgroup's first tile is its last
])
def test_fp32_storage_update_block_widths(gpu_lib, variant, n, m, b):
    """FP32 storage with FP64 arithmetic on the persistent update's forms:
    block widths below 16 (partial column groups), K not a multiple of 4,
    full 16-column blocks, ragged tiles; entry-wise against the oracle on the
    same FP32 input."""
    decades = 2
    W = svd_matrix(n, m, np.logspace(0, -decades, m), seed=n + m + b).astype(np.float32)
    W = W.astype(np.float64)
    say("fp32 storage update widths", variant, n, m, b)
    Q, R, S, cert = gpu_qr(W, b, "sparse", 256, THETA_SEED_SMALL, variant, store="f32", ls_iters=4)
    o = oracle_qr(W, b, "sparse", 256, THETA_SEED_SMALL, variant, ls_iters=4)
    assert factorization_error(W, Q, R) <= 1e-6
    assert np.all(np.diag(R) > 0)
    tol = 64 * U32 * 10**decades
    check_entrywise(W, Q, R, S, cert, o, tol)


@pytest.mark.parametrize("variant", ["plain", "lowsync"])
def test_fp32_arithmetic(gpu_lib, variant):
    """FP32 products with FP32 accumulation: fine on a well-conditioned W,
    while on a W that is numerically rank deficient in FP32 the factorization
    error stays at u32 but the sketched orthogonality is lost -- and the
    certificate Delta reports it."""
    W = svd_matrix(10_000, 64, np.logspace(0, -2, 64), seed=31).astype(np.float32).astype(np.float64)
    say("fp32 math", variant)
    Q, R, S, cert = gpu_qr(W, 8, "gaussian", 256, THETA_SEED_SMALL, variant, store="f32", math="f32")
    o = oracle_qr(W, 8, "gaussian", 256, THETA_SEED_SMALL, variant)
    assert rel(R, o["R"]) <= 64 * 2.0**-24 * 1e2
    check_entrywise(W, Q, R, S, cert, o, 64 * U32 * 1e2)
    assert cond2(Q) <= 10 and cert["delta"] < 1e-3
    W8 = svd_matrix(10_000, 64, np.logspace(0, -8, 64), seed=31).astype(np.float32).astype(np.float64)
    Q, R, S, cert = gpu_qr(W8, 8, "gaussian", 256, THETA_SEED_SMALL, variant, store="f32", math="f32")
    assert factorization_error(W8, Q, R) <= 1e-6
    assert cert["delta"] > 0.1                 # certificate: not stable
    assert cond2(Q) > 10
    # the certificate reports what the GPU's own S and R show
    th8 = Sketch("gaussian", 256, seed=THETA_SEED_SMALL).materialize(W8.shape[0])
    P8 = th8(W8)
    pc.check_certificates(cert, S, R, P8, pc.abs_theta_w_fro(pc.abs_theta(th8, W8.shape[0]), W8),
                          W8.shape[0])


EPS_BF3 = 3 * 2.0**-16


@pytest.mark.parametrize("variant", ["lowsync", "plain"])
@pytest.mark.parametrize("m,b,k", [(64, 8, 256), (70, 16, 256), (96, 32, 384)])
def test_bf16x3_arithmetic(gpu_lib, variant, m, b, k):
    """Split BF16x3 products with FP32 accumulation on a well-conditioned W
    (cond 1e2), against the oracle run on the same FP32-rounded input.
    Tolerances: each split product a_hi b_hi + a_hi b_lo + a_lo b_hi differs
    from a b by at most about EPS_BF3 = 3 2^-16 |a b| (the dropped a_lo b_lo and
    the parts of a and b beyond two bf16 pieces), more than the FP32
    accumulation (at most (K/32 + 3) u32) and the FP32 storage of Q (u32), so
    * ||W - QR||_F <= EPS_BF3 || |Q| |R| ||_F (the update error of every block
      is the factorization error of that block);
    * entry-wise, the update error EPS_BF3 |Q| |R| reaches Q through R^{-1} and
      later blocks through the least-squares step, so |x - x_or| <= EPS_BF3
      cond(W) scale as for FP32 storage (tests/parity_checks.py);
    * the first diagonal block involves no update: R_(1,1) to 4096 u;
    * the certificates equal the oracle's routine on the GPU's S and R.
    (A product missing one of its cross terms errs by about 2^-9 |a b| and
    breaks the first bound by a factor of 7 or more.)"""
    W = svd_matrix(10_000, m, np.logspace(0, -2, m), seed=41).astype(np.float32).astype(np.float64)
    say("bf16x3 math", variant, m, b, k)
    Q, R, S, cert = gpu_qr(W, b, "gaussian", k, THETA_SEED_SMALL, variant, store="f32", math="bf16x3")
    o = oracle_qr(W, b, "gaussian", k, THETA_SEED_SMALL, variant)
    err = factorization_error(W, Q, R)
    bound = EPS_BF3 * np.linalg.norm(np.abs(Q) @ np.abs(R)) / np.linalg.norm(W)
    say("bf16x3 factorization error", err, "bound", bound)
    assert err <= bound
    check_entrywise(W, Q, R, S, cert, o, EPS_BF3 * 1e2)
    pc.assert_entrywise(R[:b, :b], o["R"][:b, :b], pc.scale_R(o["R"][:b, :b]), TOL64, "R_(1,1)")
    assert cond2(Q) <= 10 and cert["delta"] < 1e-2


def test_bf16x3_certificate_on_rank_deficient_input(gpu_lib):
    """cond(W) = 1e8, numerically rank deficient at the precision of the split
    products: the factorization error stays at the products' level, the
    sketched orthogonality is lost, and the certificate Delta reports it (equal
    to the oracle's certificate routine on the GPU's S and R)."""
    W8 = svd_matrix(10_000, 64, np.logspace(0, -8, 64), seed=31).astype(np.float32).astype(np.float64)
    Q, R, S, cert = gpu_qr(W8, 8, "sparse", 256, THETA_SEED_SMALL, "lowsync", store="f32",
                           math="bf16x3")
    err = factorization_error(W8, Q, R)
    say("bf16x3 rank deficient", err, cert["delta"], cond2(Q))
    assert err <= EPS_BF3 * np.linalg.norm(np.abs(Q) @ np.abs(R)) / np.linalg.norm(W8)
    assert cert["delta"] > 0.1 and cond2(Q) > 10
    th8 = Sketch("sparse", 256, seed=THETA_SEED_SMALL).materialize(W8.shape[0])
    pc.check_certificates(cert, S, R, th8(W8), pc.abs_theta_w_fro(pc.abs_theta(th8, W8.shape[0]), W8),
                          W8.shape[0])


@pytest.mark.parametrize("variant", ["twice", "l2qr"])
@pytest.mark.parametrize("kind,k", [("gaussian", 256), ("sparse", 256)])
def test_two_pass_forms_fp64_elementwise(gpu_lib, variant, kind, k):
    W = svd_matrix(10_000, 64, np.logspace(0, -2, 64), seed=5)
    say("two-pass", variant, kind)
    Q, R, S, cert = gpu_qr(W, 8, kind, k, 17, variant)
    o = oracle_qr(W, 8, kind, k, 17, variant)
    assert rel(R, o["R"]) < 1e-12
    assert rel(Q, o["Q"]) < 1e-12
    assert rel(S, o["S"]) < 1e-12
    check_entrywise(W, Q, R, S, cert, o, TOL64)
    assert cert["delta"] < 1e-12


@pytest.mark.parametrize("decades", [8, 12])
def test_second_pass_restores_sketched_orthogonality(gpu_lib, decades):
    """One block with cond(W) = 10^decades: the certificate Delta of RCholeskyQR
    grows like u cond(W), that of the two-pass forms stays at a few u m
    (Section 2.2.4), on the GPU as in the oracle; R agrees with the oracle's
    to ~u cond of the block's sketch."""
    W = svd_matrix(4000, 16, np.logspace(0, -decades, 16), seed=3)
    say("second pass", decades)
    _, Rp, _, cp = gpu_qr(W, 16, "gaussian", 128, 4, "plain")
    assert cp["delta"] > 1e-3 * 2.0**-53 * 10.0**decades
    for variant in ("twice", "l2qr"):
        Q, R, S, cert = gpu_qr(W, 16, "gaussian", 128, 4, variant)
        o = oracle_qr(W, 16, "gaussian", 128, 4, variant)
        assert cert["delta"] < 100 * 2.0**-53 * 16
        assert cert["delta_tilde"] < 100 * 2.0**-53 * 16
        assert factorization_error(W, Q, R) < 100 * 2.0**-53 * 16
        assert rel(R, o["R"]) < 1e-13 * 10.0**(decades / 2)
        pc.assert_entrywise(R, o["R"], pc.scale_R(o["R"]), 1e-13 * 10.0**(decades / 2), "R")
        pc.check_certificates(cert, S, R, o["P"], pc.abs_theta_w_fro(o["absT"], W), W.shape[0])


@pytest.mark.parametrize("n,m,b,store", [(10_000, 64, 8, "f64"), (7777, 70, 16, "f64"),
                                         (10_000, 64, 8, "f32"), (3000, 200, 16, "f64")])
def test_cholqr_post_processing(gpu_lib, n, m, b, store):
    """Post-processing on the GPU against the oracle's on the same RBGS output
    (FP64: elementwise; the Gram matrix and the Cholesky factor differ only in
    summation order) and against LAPACK's QR of W."""
    import torch
    from paper_2111_14641_amd import binding as B
    W = svd_matrix(n, m, np.logspace(0, -3, m), seed=n + m)
    if store == "f32":
        W = W.astype(np.float32).astype(np.float64)
    say("cholqr post", n, m, b, store)
    dt = torch.float64 if store == "f64" else torch.float32
    Wt = B.colmajor(n, m, dt)
    Wt.copy_(torch.from_numpy(W))
    Q, R, _, _ = B.rbgs_qr(Wt, b, "sparse", 4 * m, 5, None, "lowsync", 4, want_cert=True)
    torch.cuda.synchronize()
    Q0 = np.ascontiguousarray(Q.cpu().numpy()).astype(np.float64)
    R0 = R.cpu().numpy().astype(np.float64)
    B.cholqr_post(Q, R)
    torch.cuda.synchronize()
    Qg = np.ascontiguousarray(Q.cpu().numpy()).astype(np.float64)
    Rg = R.cpu().numpy().astype(np.float64)
    Qo, Ro = orb.cholqr_post(Q0, R0)
    u = 2.0**-53 if store == "f64" else 2.0**-24
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0)
    assert np.linalg.norm(np.eye(m) - Qg.T @ Qg) < 100 * u * m
    assert factorization_error(W, Qg, Rg) < 100 * u * m
    tol = 1e-12 if store == "f64" else 64 * u
    assert rel(Rg, Ro) < tol
    assert rel(Qg, Qo) < tol
    # entry-wise: R' R by the column scale; Q R'^{-1} by the scale of Q = W R^{-1}
    etol = TOL64 if store == "f64" else 64 * u
    pc.assert_entrywise(Rg, Ro, pc.scale_R(Ro), etol, "R post")
    pc.assert_entrywise(Qg, Qo, pc.scale_Q(Qo, Ro), etol, "Q post")
    Qh, Rh = np.linalg.qr(W)
    d = np.sign(np.diag(Rh))
    assert rel(Rg, d[:, None] * Rh) < (1e-12 if store == "f64" else 1e-5)


def test_cholqr_post_breakdown(gpu_lib):
    import torch
    from paper_2111_14641_amd import binding as B
    say("cholqr post breakdown")
    Q = B.colmajor(500, 6, torch.float64)
    Q.copy_(torch.from_numpy(np.random.default_rng(0).standard_normal((500, 6))))
    Q[:, 3] = 0.0
    R = torch.eye(6, dtype=torch.float64, device="cuda").t().contiguous().t()
    with pytest.raises(RuntimeError, match="positive definite"):
        B.cholqr_post(Q, R)


def test_determinism_and_in_place(gpu_lib, small):
    say("determinism")
    a = gpu_qr(small, 8, "sparse", 256, 5, "lowsync")
    b = gpu_qr(small, 8, "sparse", 256, 5, "lowsync")
    c = gpu_qr(small, 8, "sparse", 256, 5, "lowsync", inplace=True)
    for x, y, z in zip(a[:3], b[:3], c[:3]):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_zero_column_breakdown(gpu_lib):
    W = svd_matrix(3000, 12, np.logspace(0, -1, 12), seed=3)
    W[:, 7] = 0.0
    say("breakdown")
    Q, R, S, cert = gpu_qr(W, 4, "sparse", 64, 1, "lowsync")
    assert cert["status"] == -4
    assert cert["breakdown_col"] == 7
    assert np.all(np.diag(R)[:4] > 0)       # blocks before the breakdown are valid


def test_nonfinite_input_flagged(gpu_lib):
    W = svd_matrix(2000, 8, np.logspace(0, -1, 8), seed=4)
    W[10, 2] = np.nan
    say("nan")
    Q, R, S, cert = gpu_qr(W, 4, "gaussian", 32, 1, "plain")
    assert cert["status"] == -4 and cert["breakdown_col"] >= 0
    assert cert["nonfinite"] == 1


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_rank_deficient_in_fp64(gpu_lib, store):
    """The oscillatory matrix (n = 10^5 here) is numerically rank deficient even
    in FP64 (sigma_min / sigma_max ~ 1e-15), so the least-squares step must be
    solved to backward-stable accuracy: with 4 Richardson sweeps both GPU forms
    and the oracle (Householder solver) keep cond2(Q) ~ 3."""
    from paper_2111_14641_amd.workloads import oscillatory_matrix, THETA_SEED_LARGE
    W = oscillatory_matrix(100_000, 256, 0xDA7A01)
    if store == "f32":
        W = W.astype(np.float32).astype(np.float64)
    say("rank deficient", store)
    Q, R, S, cert = gpu_qr(W, 16, "sparse", 1024, THETA_SEED_LARGE, "lowsync", store=store, ls_iters=4)
    th = Sketch("sparse", 1024, seed=THETA_SEED_LARGE).materialize(W.shape[0])
    o = orb.rbgs(W, 16, th, "lowsync", "householder")
    cq, co = cond2(Q), cond2(o["Q"])
    assert cq <= 10 and co <= 10
    assert abs(cq - co) / co < 0.05
    assert factorization_error(W, Q, R) <= (1e-13 if store == "f64" else 1e-6)
    assert cert["delta"] < 0.1 and cert["delta_tilde"] < 1e-6
    # the first block is well conditioned: its R factor is unique
    assert rel(R[:16, :16], o["R"][:16, :16]) < (1e-12 if store == "f64" else 1e-6)
    R11 = o["R"][:16, :16]
    pc.assert_entrywise(R[:16, :16], R11, pc.scale_R(R11), TOL64 if store == "f64" else 64 * U32,
                        "R_(1,1)")


@pytest.mark.parametrize("kind,store", [("sparse", "f32"), ("gaussian", "f64"), ("srht", "f32")])
def test_last_sketch_skipped_without_outputs(gpu_lib, kind, store):
    """Without S_out and a certificate the sketch of the last block (used by
    nothing else) is not taken: Q and R are bit for bit those of the call that
    returns S, which equals the oracle's sketch of the GPU's Q."""
    import torch
    from paper_2111_14641_amd import binding as B
    n, m, b, k = 6000, 40, 16, 256
    W = svd_matrix(n, m, np.logspace(0, -3, m), seed=77)
    dt = torch.float64 if store == "f64" else torch.float32
    Wt = B.colmajor(n, m, dt)
    Wt.copy_(torch.from_numpy(W))
    Q1, R1, S1, _ = B.rbgs_qr(Wt, b, kind, k, 9, None, "lowsync", 4, want_S=True)
    Q2, R2, _, _ = B.rbgs_qr(Wt, b, kind, k, 9, None, "lowsync", 4)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
    th = Sketch(kind, k, seed=9).materialize(n)
    Qh = np.asfortranarray(Q1.double().cpu().numpy())
    So = th(Qh[:, 32:])
    scale = np.abs(Qh[:, 32:]).sum(axis=0) if kind != "sparse" else np.linalg.norm(Qh[:, 32:], axis=0)
    assert np.all(np.abs(S1.cpu().numpy()[:, 32:] - So) <= 1e-12 * scale[None, :])


@pytest.mark.parametrize("b,m", [(16, 560), (32, 544)])
def test_update_falls_back_past_lds_capacity(gpu_lib, b, m):
    """Blocks whose K = c0 exceeds the rows of R the persistent update keeps in
    LDS (512 for 16-column blocks, 480 for 32-column blocks) take the general
    update kernel; both forms in one factorization agree with the oracle at the
    FP64 tolerance."""
    n, k = 3000, 576
    W = svd_matrix(n, m, np.logspace(0, -2, m), seed=91)
    say("update forms", n, m, b, k)
    Q, R, S, cert = gpu_qr(W, b, "sparse", k, 29, "lowsync")
    o = oracle_qr(W, b, "sparse", k, 29, "lowsync")
    assert rel(R, o["R"]) < 1e-12
    assert rel(Q, o["Q"]) < 1e-11
    check_entrywise(W, Q, R, S, cert, o, TOL64)
    assert factorization_error(W, Q, R) < 1e-14


@pytest.mark.parametrize("b", [16, 32])
@pytest.mark.parametrize("store", ["f64", "f32"])
@pytest.mark.parametrize("ldw_pad,ldq_pad", [(0, 0), (8, 4), (3, 5), (4, 1)])
def test_leading_dimensions_give_identical_results(gpu_lib, store, ldw_pad, ldq_pad, b):
    """W and Q inside larger column-major buffers (ld > n): 16-byte aligned
    leading dimensions keep the vector path, others take the guarded path for
    every tile.  Every element is computed by the same operations in the same
    order either way, so the results equal those with ld = n bit for bit.  With
    m = 64 and 16-column blocks the last block (K = 48) takes the update launch
    that also factors the sketch, whose workgroups then reach the wait for
    R_(i,i) from the guarded tiles."""
    import torch
    from paper_2111_14641_amd import binding as B
    n, m, k = 5000, 64, 256
    W = svd_matrix(n, m, np.logspace(0, -3, m), seed=5)
    dt = torch.float64 if store == "f64" else torch.float32
    say("leading dimensions", store, ldw_pad, ldq_pad)
    W0 = B.colmajor(n, m, dt)
    W0.copy_(torch.from_numpy(W))
    Q0, R0, _, _ = B.rbgs_qr(W0, b, "sparse", k, 3, None, "lowsync", 4)
    Wb = B.colmajor(n + ldw_pad, m, dt)
    Wb.fill_(float("nan"))          # padding rows must never be read into a result
    Wv = Wb[:n]
    Wv.copy_(W0)
    Qb = B.colmajor(n + ldq_pad, m, dt)
    Qb.fill_(7.0)
    Qv = Qb[:n]
    Q1, R1, _, _ = B.rbgs_qr(Wv, b, "sparse", k, 3, None, "lowsync", 4, Q=Qv)
    torch.cuda.synchronize()
    assert torch.equal(R1, R0)
    assert torch.equal(Q1, Q0)
    if ldq_pad:
        assert bool((Qb[n:] == 7.0).all())   # nothing written past row n


# ---------------------------------------------------------------------------
# Direct (Householder) least squares of step 2: ls_iters = 0
# ---------------------------------------------------------------------------
def oracle_qr_householder(W, b, kind, k, seed, variant, zeta=None):
    th = Sketch(kind, k, seed=seed, zeta=zeta).materialize(W.shape[0])
    o = orb.rbgs(W, b, th, variant, "householder")
    o["absT"] = pc.abs_theta(th, W.shape[0])
    return o


@pytest.mark.parametrize("n,m,b,k,kind,variant", [
    (10_000, 64, 8, 256, "gaussian", "lowsync"),
    (10_000, 64, 8, 256, "gaussian", "plain"),
    (7777, 70, 16, 1024, "sparse", "lowsync"),      # k = 1024: 16 rows per lane, ragged last block
    (5000, 96, 32, 512, "sparse", "lowsync"),       # 32-wide blocks (two columns per wave)
    (4097, 40, 32, 132, "rademacher", "plain"),     # Rademacher, k not a multiple of 64
    (4097, 30, 8, 128, "sparse", "twice"),
    (3000, 70, 16, 256, "srht", "lowsync"),
    (2000, 1, 4, 8, "sparse", "lowsync"),           # m = 1: no least squares at all
    (3000, 24, 24, 96, "gaussian", "lowsync"),      # one block
    (5000, 17, 1, 64, "sparse", "plain"),           # single-column blocks: 16 factorization updates
])
def test_householder_least_squares_fp64(gpu_lib, n, m, b, k, kind, variant):
    """The GPU's Householder least squares (QR of S_(1:i-1) extended block by
    block) against the oracle's direct solver (LAPACK QR of S_(1:i-1))."""
    W = svd_matrix(n, m, np.logspace(0, -2, m), seed=n + m + 3 * b)
    say("householder", n, m, b, k, kind, variant)
    Q, R, S, cert = gpu_qr(W, b, kind, k, 31, variant, ls_iters=0)
    o = oracle_qr_householder(W, b, kind, k, 31, variant)
    assert rel(R, o["R"]) < 1e-12
    assert rel(Q, o["Q"]) < 1e-11
    check_entrywise(W, Q, R, S, cert, o, TOL64)
    assert factorization_error(W, Q, R) < 1e-14


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_householder_matches_sweeps_on_rank_deficient_input(gpu_lib, store):
    """On a numerically rank-deficient W (cond 1e14) the direct solver and 4
    Richardson sweeps give the same factorization quality (the sweeps' error
    Delta^4 |y| is below the rounding of step 3), and the direct GPU result
    matches the oracle's direct result in the metrics."""
    n, m, b, k = 20_000, 96, 16, 512
    W = svd_matrix(n, m, np.logspace(0, -14, m), seed=77)
    if store == "f32":
        W = W.astype(np.float32).astype(np.float64)
    say("householder rank deficient", store)
    Qh, Rh, Sh, ch = gpu_qr(W, b, "sparse", k, 5, "lowsync", store=store, ls_iters=0)
    Qr, Rr, Sr, cr = gpu_qr(W, b, "sparse", k, 5, "lowsync", store=store, ls_iters=4)
    o = oracle_qr_householder(W, b, "sparse", k, 5, "lowsync")
    target = 1e-14 if store == "f64" else 1e-6
    for Q, R in ((Qh, Rh), (Qr, Rr)):
        assert factorization_error(W, Q, R) < target
        assert cond2(Q) <= 10
    assert abs(cond2(Qh) - cond2(o["Q"])) <= 0.05 * cond2(o["Q"])
    assert abs(cond2(Qh) - cond2(Qr)) <= 0.05 * cond2(Qr)


def test_householder_in_a_batch(gpu_lib):
    """Batched problems with ls_iters = 0 run one by one (the lock-step and
    persistent forms use the sweeps) and each matches the oracle."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("householder batch")
    shapes = [(3000, 32, 16, 96), (5000, 48, 8, 128), (4097, 40, 32, 160)]
    Wh, Ws = [], []
    for i, (n, m, b, k) in enumerate(shapes):
        W = svd_matrix(n, m, np.logspace(0, -2, m), seed=400 + i)
        Wt = B.colmajor(n, m, torch.float64)
        Wt.copy_(torch.from_numpy(W))
        Wh.append(W)
        Ws.append(Wt)
    for persistent in (False, True):
        Qs, Rs, _, _ = B.rbgs_qr_batched(Ws, [s[2] for s in shapes], [s[3] for s in shapes],
                                         seed=50, ls_iters=0, persistent=persistent)
        torch.cuda.synchronize()
        for i, (W, Q, R) in enumerate(zip(Wh, Qs, Rs)):
            n, m, b, k = shapes[i]
            o = oracle_qr_householder(W, b, "sparse", k, 50 + i, "lowsync")
            Rg = np.ascontiguousarray(R.cpu().numpy())
            Qg = np.ascontiguousarray(Q.cpu().numpy())
            assert rel(Rg, o["R"]) < 1e-12, (persistent, i)
            pc.assert_qrs_entrywise(Qg, Rg, None, o, None, TOL64, TOL64)
