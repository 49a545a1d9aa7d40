"""Pins of the RBGS oracle against things other than itself (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle.rbgs as orb
from oracle.metrics import cond2, factorization_error, orthogonality_loss, cond2_from_gram
from oracle.theta import Sketch
from paper_2111_14641_amd.workloads import svd_matrix, small_single_qr, THETA_SEED_SMALL

U64 = 2.0**-53


def lapack_qr_posdiag(W):
    Qh, Rh = np.linalg.qr(W)
    d = np.sign(np.diag(Rh))
    return Qh * d[None, :], d[:, None] * Rh


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small_case():
    W = small_single_qr()
    th = Sketch("gaussian", 256, seed=THETA_SEED_SMALL).materialize(W.shape[0])
    return W, th


# -- Theta = I: RBGS is block Gram-Schmidt with exact projections -------------
@pytest.mark.parametrize("variant", ["plain", "lowsync", "twice", "l2qr"])
@pytest.mark.parametrize("ls,iters", [("householder", 0), ("richardson", 2)])
@pytest.mark.parametrize("n,m,b", [(48, 12, 4), (64, 16, 5), (30, 7, 3), (20, 20, 20), (33, 9, 1)])
def test_identity_sketch_equals_householder_qr(variant, ls, iters, n, m, b):
    W = svd_matrix(n, m, np.logspace(0, -3, m), seed=n * m + b)
    out = orb.rbgs(W, b, Sketch("identity", n), variant, ls, iters)
    Qh, Rh = lapack_qr_posdiag(W)
    assert rel(out["R"], Rh) < 1e-13
    assert rel(out["Q"], Qh) < 1e-12
    assert np.allclose(out["S"], out["Q"])


# -- the exact-arithmetic closed form -----------------------------------------
@pytest.mark.parametrize("kind", ["gaussian", "sparse", "rademacher", "srht"])
def test_closed_form_well_conditioned(kind):
    W = svd_matrix(10_000, 64, np.logspace(0, -2, 64), seed=5)
    th = Sketch(kind, 256, seed=17).materialize(W.shape[0])
    Qc, Rc = orb.rbgs_closed_form(W, th)
    for variant in ("plain", "lowsync", "twice", "l2qr"):
        out = orb.rbgs(W, 8, th, variant)
        assert rel(out["R"], Rc) < 1e-12
        assert rel(out["Q"], Qc) < 1e-12


def test_closed_form_ill_conditioned(small_case):
    """cond(W) = 1e8: R is still determined to ~u, Q to ~u cond(W) poly(m)."""
    W, th = small_case
    Qc, Rc = orb.rbgs_closed_form(W, th)
    out = orb.rbgs(W, 8, th, "plain")
    assert rel(out["R"], Rc) < 1e-12
    assert rel(out["Q"], Qc) < 1e-6


# -- invariants and certificates ----------------------------------------------
@pytest.mark.parametrize("variant", ["plain", "lowsync", "twice", "l2qr"])
def test_invariants_and_certificates(small_case, variant):
    W, th = small_case
    out = orb.rbgs(W, 8, th, variant)
    R = out["R"]
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R) > 0)
    # S really is the sketch of Q and P the sketch of W
    assert rel(out["S"], th(out["Q"])) < 1e-14
    assert rel(out["P"], th(W)) < 1e-15
    assert out["delta"] == pytest.approx(orthogonality_loss(out["S"]), rel=1e-12)
    # a priori bounds of the stability theorem (Section 3.2, u_crs = u_fine = u)
    m = W.shape[1]
    assert out["delta_tilde"] <= 6 * U64 * m**1.5
    assert out["delta"] <= 20 * U64 * m**2 * 1e8
    assert factorization_error(W, out["Q"], R) < 1e-14


def _cert_case():
    """S = U diag(sqrt(1 + e_j)) with U orthonormal gives S^T S = diag(1 + e_j),
    so Delta = ||e||_2 exactly.  P = S R + F with S^T F = 0 gives P - S R = F
    and ||P||_F^2 = ||S R||_F^2 + ||F||_F^2, so Delta~ = ||F||_F /
    sqrt(||S R||_F^2 + ||F||_F^2).  ||P||_F is about 30, so dropping the
    normalization (or applying it twice, or to the squares only) changes Delta~
    by a large factor."""
    rng = np.random.default_rng(7)
    k, m = 40, 6
    Ufull, _ = np.linalg.qr(rng.standard_normal((k, k)))
    U, Uperp = Ufull[:, :m], Ufull[:, m:]
    e = np.array([0.3, -0.2, 0.1, 0.05, -0.4, 0.25])
    S = U * np.sqrt(1.0 + e)[None, :]
    R = np.triu(rng.standard_normal((m, m))) * 10.0 + np.diag(np.full(m, 5.0))
    F = Uperp @ rng.standard_normal((k - m, m)) * 0.7
    nF = np.linalg.norm(F)
    nP = np.sqrt(np.linalg.norm(S @ R) ** 2 + nF ** 2)
    return S, S @ R + F, R, float(np.linalg.norm(e)), float(nF / nP), nP


def _cert_pin_holds():
    S, P, R, delta_ref, dt_ref, _ = _cert_case()
    delta, delta_tilde = orb.certificates(S, P, R)
    return (abs(delta - delta_ref) <= 1e-13 * delta_ref
            and abs(delta_tilde - dt_ref) <= 1e-12 * dt_ref)


def test_certificates_on_known_matrices(monkeypatch):
    """Step 6 of Algorithm RBGS on matrices whose certificates are known in
    closed form (_cert_case), and planted mistakes in the certificate formulas
    that this pin must catch."""
    S, P, R, delta_ref, dt_ref, nP = _cert_case()
    assert nP > 20.0
    assert _cert_pin_holds()
    # an exact factorization has Delta~ = 0 whatever the scale of P
    assert orb.certificates(S, S @ R, R)[1] < 1e-15
    # Delta~ is invariant under a common scaling of P and R (a normalized residual)
    assert orb.certificates(S, 3.0 * P, 3.0 * R)[1] == pytest.approx(dt_ref, rel=1e-12)
    # orthonormal columns: Delta = 0
    U = S / np.linalg.norm(S, axis=0)[None, :]
    assert orb.certificates(U, P, R)[0] < 1e-14
    good = orb.certificates
    fro = lambda A: np.linalg.norm(A, "fro")
    mistakes = {
        "Delta~ not normalized": lambda S, P, R: (good(S, P, R)[0], fro(P - S @ R)),
        "Delta~ normalized twice": lambda S, P, R: (good(S, P, R)[0], fro(P - S @ R) / fro(P) ** 2),
        "Delta~ squares normalized": lambda S, P, R: (good(S, P, R)[0], fro(P - S @ R) ** 2 / fro(P) ** 2),
        "Delta~ with R transposed": lambda S, P, R: (good(S, P, R)[0], fro(P - S @ R.T) / fro(P)),
        "Delta from S S^T": lambda S, P, R: (fro(np.eye(S.shape[0]) - S @ S.T), good(S, P, R)[1]),
        "Delta squared": lambda S, P, R: (fro(np.eye(S.shape[1]) - S.T @ S) ** 2, good(S, P, R)[1]),
    }
    for name, bad in mistakes.items():
        monkeypatch.setattr(orb, "certificates", bad)
        assert not _cert_pin_holds(), name
        monkeypatch.setattr(orb, "certificates", good)
    assert _cert_pin_holds()


def test_condition_number_equals_that_of_sketched_basis(small_case):
    """In exact arithmetic sigma(Q) = 1/sigma(Theta U) for U an orthonormal basis
    of range(W), so cond(Q) = cond(Theta U)."""
    W, th = small_case
    out = orb.rbgs(W, 8, th, "lowsync")
    U = np.linalg.svd(W, full_matrices=False)[0]
    sU = np.linalg.svd(th(U), compute_uv=False)
    cq = cond2(out["Q"])
    assert abs(cq - sU[0] / sU[-1]) / cq < 1e-6
    assert cq < 10
    assert cond2_from_gram(out["Q"].T @ out["Q"]) == pytest.approx(cq, rel=1e-6)


def test_a_posteriori_condition_bound():
    """A posteriori theorem (Section 3.2): if Theta is an eps-embedding (eps <=
    1/2) of W and Q and Delta, Delta~ <= 0.1, then
    (1+eps)^(-1/2) (1 - Delta - 0.1u) <= sigma(Q) <= (1-eps)^(-1/2) (1 + Delta + 0.1u).
    k = 32 m keeps eps below 1/2 for the Gaussian operator."""
    W = svd_matrix(8000, 16, np.logspace(0, -6, 16), seed=21)
    th = Sketch("gaussian", 512, seed=22).materialize(8000)
    out = orb.rbgs(W, 4, th, "plain")
    # eps for range([W, Q]) (= range(W) in exact arithmetic; include both)
    U = np.linalg.svd(np.hstack([W / np.linalg.norm(W), out["Q"] / np.linalg.norm(out["Q"])]),
                      full_matrices=False)[0][:, :16]
    sU = np.linalg.svd(th(U), compute_uv=False)
    eps = np.max(np.abs(sU**2 - 1))
    d = out["delta"]
    assert eps <= 0.5 and d <= 0.1 and out["delta_tilde"] <= 0.1
    sq = np.linalg.svd(out["Q"], compute_uv=False)
    lo = (1 + eps) ** -0.5 * (1 - d - 0.1 * U64)
    hi = (1 - eps) ** -0.5 * (1 + d + 0.1 * U64)
    assert lo <= sq[-1] and sq[0] <= hi


def test_a_posteriori_factorization_bound(small_case):
    W, th = small_case
    out = orb.rbgs(W, 8, th, "plain")
    m = W.shape[1]
    assert out["delta"] <= 0.1 and out["delta_tilde"] <= 0.1
    err = np.linalg.norm(W - out["Q"] @ out["R"])
    assert err <= 4 * U64 * m**1.5 * np.linalg.norm(W)
    sk = np.linalg.norm(th(W - out["Q"] @ out["R"]))
    assert sk <= 5 * U64 * m**1.5 * np.linalg.norm(W)


# -- variants and least-squares solvers ---------------------------------------
def test_plain_and_lowsync_agree(small_case):
    W, th = small_case
    a = orb.rbgs(W, 8, th, "plain")
    b = orb.rbgs(W, 8, th, "lowsync")
    assert rel(a["R"], b["R"]) < 1e-12
    assert rel(a["Q"], b["Q"]) < 1e-6


@pytest.mark.parametrize("decades", [8, 12])
def test_second_pass_restores_sketched_orthogonality(decades):
    """Section 2.2.4: running RCholeskyQR twice, or after an l2-QR, makes the
    block's sketched orthogonality independent of its conditioning.  One
    block (b = m) with cond(W) = 10^decades: RCholeskyQR leaves
    Delta ~ u cond(W), the two-pass forms Delta ~ u m; R2 of the second pass
    is I up to ~u cond(W)."""
    W = svd_matrix(4000, 16, np.logspace(0, -decades, 16), seed=3)
    th = Sketch("gaussian", 128, seed=4).materialize(4000)
    plain = orb.rbgs(W, 16, th, "plain")
    assert plain["delta"] > 1e-3 * U64 * 10.0**decades
    for variant in ("twice", "l2qr"):
        out = orb.rbgs(W, 16, th, variant)
        assert out["delta"] < 100 * U64 * 16
        assert out["delta_tilde"] < 100 * U64 * 16
        assert factorization_error(W, out["Q"], out["R"]) < 100 * U64 * 16
        assert np.all(np.diag(out["R"]) > 0) and np.all(np.tril(out["R"], -1) == 0)
    # the first pass of "twice" is the plain result: R2 = R_twice R_plain^{-1} ~ I
    tw = orb.rbgs(W, 16, th, "twice")
    R2 = sla.solve_triangular(plain["R"].T, tw["R"].T, lower=True).T
    assert np.linalg.norm(R2 - np.eye(16)) < 100 * U64 * 10.0**decades


def test_cholqr_post_processing_gives_householder_qr():
    """Post-processing (remark in Section 2.2): after RBGS, Cholesky QR of the
    well-conditioned Q gives an l2-orthonormal Q, keeps W = Q R, and -- QR
    with positive diagonal being unique -- reproduces LAPACK's Householder
    QR of W."""
    W = svd_matrix(6000, 40, np.logspace(0, -3, 40), seed=12)
    th = Sketch("gaussian", 160, seed=13).materialize(6000)
    out = orb.rbgs(W, 8, th, "lowsync")
    Qn, Rn = orb.cholqr_post(out["Q"], out["R"])
    Qh, Rh = lapack_qr_posdiag(W)
    assert np.linalg.norm(np.eye(40) - Qn.T @ Qn) < 50 * U64 * 40
    assert factorization_error(W, Qn, Rn) < 10 * U64 * 40
    assert rel(Rn, Rh) < 1e-13
    assert rel(Qn, Qh) < 1e-12
    assert np.all(np.tril(Rn, -1) == 0) and np.all(np.diag(Rn) > 0)


def test_ragged_last_block():
    W = svd_matrix(5000, 30, np.logspace(0, -3, 30), seed=9)
    th = Sketch("sparse", 128, seed=2).materialize(5000)
    Qc, Rc = orb.rbgs_closed_form(W, th)
    out = orb.rbgs(W, 8, th, "lowsync", "richardson", 2)     # blocks 8, 8, 8, 6
    assert rel(out["R"], Rc) < 1e-12 and rel(out["Q"], Qc) < 1e-11


def test_richardson_error_bound():
    """Supplement SM.1: ||x_j - y_j|| <= (Delta^(i-1))^l ||y_j|| where y is the
    exact least-squares solution (here: the Householder solution)."""
    rng = np.random.default_rng(3)
    k, mcols, c = 200, 40, 6
    # a nearly orthonormal S with a controlled Delta
    U, _ = np.linalg.qr(rng.standard_normal((k, mcols)))
    S = U @ (np.eye(mcols) + 3e-3 * rng.standard_normal((mcols, mcols)))
    P = rng.standard_normal((k, c))
    Y = orb.ls_householder(S, P)
    delta = orthogonality_loss(S)
    assert 0.01 < delta < 0.5
    for l in (1, 2, 3, 5, 8):
        X = orb.ls_richardson(S, P, l)
        for j in range(c):
            assert np.linalg.norm(X[:, j] - Y[:, j]) <= delta**l * np.linalg.norm(Y[:, j]) * (1 + 1e-8) + 1e-13
    # one sweep is the sketched block CGS projection S^T P
    assert np.allclose(orb.ls_richardson(S, P, 1), S.T @ P, rtol=0, atol=1e-14)


def test_householder_ls_solves_normal_equations():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((100, 20))
    P = rng.standard_normal((100, 3))
    Y = orb.ls_householder(S, P)
    assert np.allclose(S.T @ (S @ Y - P), 0, atol=1e-12)
    ref = np.linalg.lstsq(S, P, rcond=None)[0]
    assert np.allclose(Y, ref, atol=1e-13)


# -- planted mistakes must be caught by the pins above ------------------------
def _identity_pin_holds():
    W = svd_matrix(40, 12, np.logspace(0, -2, 12), seed=1)
    out = orb.rbgs(W, 4, Sketch("identity", 40), "plain")
    Qh, Rh = lapack_qr_posdiag(W)
    return (rel(out["R"], Rh) < 1e-13 and rel(out["Q"], Qh) < 1e-12
            and np.all(np.diag(out["R"]) > 0))


def _ls_pin_holds():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((100, 20))
    P = rng.standard_normal((100, 3))
    return np.allclose(orb.ls_householder(S, P), np.linalg.lstsq(S, P, rcond=None)[0], atol=1e-12)


def _closed_form_pin_holds():
    W = svd_matrix(600, 12, np.logspace(0, -2, 12), seed=2)
    th = Sketch("sparse", 48, seed=3).materialize(600)
    Qc, Rc = orb.rbgs_closed_form(W, th)
    out = orb.rbgs(W, 4, th, "lowsync")
    return rel(out["R"], Rc) < 1e-12 and rel(out["Q"], Qc) < 1e-12


def _pins_hold():
    return _identity_pin_holds() and _ls_pin_holds() and _closed_form_pin_holds()


def test_planted_mistakes_break_a_pin(monkeypatch):
    assert _pins_hold()
    good_ls, good_qr, good_rbgs = orb.ls_householder, orb.qr_r_posdiag, orb.rbgs

    def transposed_solve(S, P):
        if S.shape[1] == 0:
            return good_ls(S, P)
        Qs, Rs = np.linalg.qr(S)
        return sla.solve_triangular(Rs.T, Qs.T @ P, lower=True)

    ls_mistakes = {
        "dropped projection": lambda S, P: 0 * good_ls(S, P),
        "wrong sign": lambda S, P: -good_ls(S, P),
        "transposed solve": transposed_solve,
    }
    for name, bad in ls_mistakes.items():
        monkeypatch.setattr(orb, "ls_householder", bad)
        assert not _pins_hold(), name
        monkeypatch.setattr(orb, "ls_householder", good_ls)
    qr_mistakes = {
        "negative diagonal kept": lambda A: np.linalg.qr(A, mode="r"),
        "R of the Gram matrix": lambda A: good_qr(A.T @ A),
        "transposed R": lambda A: good_qr(A).T,
    }
    for name, bad in qr_mistakes.items():
        monkeypatch.setattr(orb, "qr_r_posdiag", bad)
        assert not _pins_hold(), name
        monkeypatch.setattr(orb, "qr_r_posdiag", good_qr)
    assert _pins_hold()
