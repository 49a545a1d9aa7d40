"""Block Krylov solvers on the GPU against the FP64 oracle: CSR SpMM,
RBGS-Arnoldi (elementwise and through the Arnoldi identity), randomized block
GMRES (exact solution when the Krylov space is everything; convergence and
solution on a larger grid), and a few cycles on the 1024 x 1024 grid."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import parity_checks as pc
from oracle import krylov
from oracle.theta import Sketch
from paper_2111_14641_amd.workloads import convection_diffusion_csr, gmres_rhs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def host_csr(N):
    indptr, indices, data = convection_diffusion_csr(N)
    return (indptr, indices, data), sp.csr_matrix((data, indices, indptr), shape=(N * N, N * N))


def dev(X, dtype):
    import torch
    from paper_2111_14641_amd import binding as B
    Xt = B.colmajor(X.shape[0], X.shape[1], dtype)
    Xt.copy_(torch.from_numpy(np.asarray(X, dtype=np.float64)))
    return Xt


def to_np(t):
    return np.ascontiguousarray(t.double().cpu().numpy())


@pytest.mark.parametrize("bs", [1, 8, 13])
@pytest.mark.parametrize("xdt,ydt", [("f64", "f64"), ("f32", "f32"), ("f64", "f32")])
def test_spmm_matches_library_product(gpu_lib, bs, xdt, ydt):
    import torch
    from paper_2111_14641_amd import binding as B
    say("spmm", bs, xdt, ydt)
    arrs, A = host_csr(37)
    n = A.shape[0]
    rng = np.random.default_rng(bs)
    X = rng.standard_normal((n, bs))
    Y0 = rng.standard_normal((n, bs))
    tx = torch.float64 if xdt == "f64" else torch.float32
    ty = torch.float64 if ydt == "f64" else torch.float32
    if xdt == "f32":
        X = X.astype(np.float32).astype(np.float64)
    Ad = B.CSR(*arrs)
    Y = to_np(B.spmm(Ad, dev(X, tx), alpha=-1.5, beta=0.5, Y0=dev(Y0, torch.float64), out_dtype=ty))
    ref = -1.5 * (A @ X) + 0.5 * Y0
    scale = 1.5 * (abs(A) @ np.abs(X)) + 0.5 * np.abs(Y0)
    tol = (4e-16 if ydt == "f64" else 2 ** -24) * 8 * scale
    assert np.all(np.abs(Y - ref) <= tol + 1e-300)


@pytest.mark.parametrize("kind", ["sparse", "gaussian"])
def test_arnoldi_matches_oracle(gpu_lib, kind):
    import torch
    from paper_2111_14641_amd import binding as B
    say("arnoldi", kind)
    N, bs, nb, k = 64, 4, 10, 160
    arrs, A = host_csr(N)
    n = N * N
    Bh = gmres_rhs(n, bs, seed=11)
    Q, R, cert = B.block_arnoldi(B.CSR(*arrs), dev(Bh, torch.float64), nb, kind, k, seed=21,
                                 ls_iters=2, want_cert=True)
    Qg, Rg = to_np(Q), to_np(R)
    th = Sketch(kind, k, seed=21).materialize(n)
    Qo, Ro, So = krylov.rbgs_arnoldi(A, Bh, nb, th, "lowsync", "richardson", 2)
    m = nb * bs
    assert np.linalg.norm(Rg - Ro) <= 1e-11 * np.linalg.norm(Ro)
    assert np.linalg.norm(Qg - Qo) <= 1e-10 * np.linalg.norm(Qo)
    # entry-wise: R by its column norms; Q by the largest entry of its column
    # (W_(i) = A Q_(i-1) depends on the basis, so Q = W R^{-1} gives no finer scale)
    pc.assert_entrywise(Rg, Ro, pc.scale_R(Ro), 1e-11, "Arnoldi R")
    pc.assert_entrywise(Qg, Qo, np.broadcast_to(np.abs(Qo).max(axis=0)[None, :], Qo.shape), 1e-10,
                        "Arnoldi Q")
    An = np.linalg.norm(A.toarray(), 2)
    assert np.linalg.norm(A @ Qg[:, :m - bs] - Qg @ Rg[:, bs:]) <= 1e-12 * An * np.linalg.norm(Qg)
    assert cert["delta"] < 1e-10 and cert["breakdown_col"] == -1


def test_gmres_exact_solution_small(gpu_lib):
    import torch
    from paper_2111_14641_amd import binding as B
    say("gmres exact")
    N, bs = 8, 2
    arrs, A = host_csr(N)
    n = N * N
    Bh = gmres_rhs(n, bs, seed=4)
    X, iters, rel, hist, ok = B.block_gmres(B.CSR(*arrs), dev(Bh, torch.float64), None,
                                           n // bs - 1, 2, 1e-10, kind="identity", k=n,
                                           store="f64", variant="plain")
    Xd = spla.spsolve(A.tocsc(), Bh)
    assert ok and rel <= 1e-10
    assert np.linalg.norm(to_np(X) - Xd) <= 1e-9 * np.linalg.norm(Xd)


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_gmres_converges_like_the_oracle(gpu_lib, store):
    import torch
    from paper_2111_14641_amd import binding as B
    say("gmres", store)
    N, bs, p, k = 32, 4, 20, 512
    arrs, A = host_csr(N)
    n = N * N
    Bh = gmres_rhs(n, bs, seed=5)
    X, iters, rel, hist, ok = B.block_gmres(B.CSR(*arrs), dev(Bh, torch.float64), None, p, 30, 1e-8,
                                           kind="sparse", k=k, seed=6, store=store)
    Xo, ho = krylov.block_gmres(A, Bh, np.zeros((n, bs)), p, 30, 1e-8,
                                Sketch("sparse", k, seed=6).materialize(n))
    assert ok and rel <= 1e-8 and ho[-1] <= 1e-8
    # same number of cycles give or take one; same solution
    assert abs(len(hist) - len(ho)) <= 1
    Xd = spla.spsolve(A.tocsc(), Bh)
    assert np.linalg.norm(to_np(X) - Xd) <= 1e-5 * np.linalg.norm(Xd)
    if store == "f64":
        np.testing.assert_allclose(hist[:3], ho[:3], rtol=1e-6)


def test_gmres_history_matches_oracle_where_it_converges(gpu_lib):
    """The workload's settings (8 right-hand sides, 40 blocks per cycle,
    k = 1280, sparse sign) on the 64 x 64 grid, where restarted GMRES converges
    without a preconditioner (the oracle reaches 1e-8 in 9 cycles): FP64 basis,
    the relative residual at the start of every cycle and at the end against the
    oracle's, entry by entry.

    Tolerance per entry: 1e-6 relative, plus n u cond2(A) absolute (n = 4096,
    u = 2^-53, cond2(A) = 408 from the singular values below, about 1.9e-10):
    the forward error of a backward-stable FP64 solve, the level at which two
    such solvers of one system can disagree once the residual approaches it.
    The two solutions differ by at most ||A^-1||_2 (||r_gpu|| + ||r_oracle||)
    (both residuals recomputed here in FP64)."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("gmres history 64^2")
    N, bs, p, k, seed = 64, 8, 40, 1280, 0x2111146413
    arrs, A = host_csr(N)
    n = N * N
    Bh = gmres_rhs(n, bs)
    X, iters, rel, hist, ok = B.block_gmres(B.CSR(*arrs), dev(Bh, torch.float64), None, p, 12, 1e-8,
                                           kind="sparse", k=k, seed=seed, store="f64")
    Xo, ho = krylov.block_gmres(A, Bh, np.zeros((n, bs)), p, 12, 1e-8,
                                Sketch("sparse", k, seed=seed).materialize(n))
    say("history gpu", hist)
    say("history oracle", ho)
    assert ok and ho[-1] <= 1e-8
    assert len(hist) == len(ho)
    sv = np.linalg.svd(A.toarray(), compute_uv=False)
    atol = n * 2.0**-53 * sv[0] / sv[-1]
    say("entry-wise history tolerance", atol)
    np.testing.assert_allclose(hist, ho, rtol=1e-6, atol=atol)
    Xg = to_np(X)
    res = np.linalg.norm(Bh - A @ Xg) + np.linalg.norm(Bh - A @ Xo)
    assert np.linalg.norm(Xg - Xo) <= 1.001 * res / sv[-1]


def test_gmres_full_grid_first_cycles(gpu_lib):
    """The 1024 x 1024 operator, 8 right-hand sides, 40 blocks per cycle,
    k = 1280, FP32 basis: three cycles reduce the residual."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("gmres 1024^2")
    N, bs = 1024, 8
    arrs, _ = host_csr(N)
    n = N * N
    Bh = gmres_rhs(n, bs)
    X, iters, rel, hist, ok = B.block_gmres(B.CSR(*arrs), dev(Bh, torch.float64), None, 40, 3, 1e-8,
                                           kind="sparse", k=1280, seed=7, store="f32")
    say("history", hist)
    assert iters == 120 and len(hist) == 4
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert np.isfinite(to_np(X)).all()
