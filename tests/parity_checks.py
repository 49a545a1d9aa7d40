"""Element-wise comparisons of GPU results with the oracle's.

Each comparison is |x_gpu - x_or| <= tol * scale, entry by entry, with a
per-entry scale taken from a first-order perturbation bound of the quantity
(so a single wrong column, row range or tile cannot hide inside a norm):

* R.  Entry (j, c) above the diagonal block solves the sketched least-squares
  problem of step 2 of Algorithm RBGS for column c of P = Theta W, and the
  diagonal block is the R factor of a k x b sketch whose column c has norm
  ||R_(:,c)||_2 (Theta Q is nearly orthonormal).  Rounding in either step is
  bounded by a multiple of u ||P_c||_2 = u ||R_(:,c)||_2, hence
  scale_R[j, c] = ||R_(:,c)||_2.
* Q.  For full-rank W the result is Q = W R^{-1}.  A relative perturbation
  |dR| <= e |R| changes Q by dQ = -Q dR R^{-1}, so |dQ| <= e |Q| |R| |R^{-1}|
  componentwise, hence scale_Q = |Q| (|R| |R^{-1}|).
* S = Theta Q.  |dS| <= |Theta| |dQ| plus the rounding of the sketch,
  gamma |Theta| |Q|, hence scale_S = |Theta| scale_Q.

Certificates (step 6): Delta = ||I - S^T S||_F and Delta~ = ||P - S R||_F /
||P||_F are recomputed by the oracle's certificate routine from the GPU's own
S and R (and the oracle's P).  The GPU's values may differ only by the rounding
of the Gram matrix, |dDelta| <= ||dG||_F <= gamma_k ||S||_F^2, and of the
residual, |dDelta~| <= (||P_gpu - P_or||_F + gamma_m || |S| |R| ||_F) / ||P||_F
with ||P_gpu - P_or||_F <= gamma_n || |Theta| |W| ||_F.
"""
import sys

import numpy as np
import scipy.linalg as sla

U64 = 2.0**-53


def say(*a):
    print("[parity]", *a, file=sys.stderr, flush=True)


def abs_theta(th, n):
    """A function Y -> |Theta| Y for an oracle Sketch over n rows (Y >= 0)."""
    if th.kind == "sparse":
        A = abs(th.materialize(n)._csr) * th.scale
        return lambda Y: np.asarray(A @ Y)
    if th.kind == "identity":
        return lambda Y: np.asarray(Y)
    if th.kind in ("rademacher", "srht"):
        # every entry is +-1/sqrt(k) (SRHT: P H D with H and D of +-1 entries)
        return lambda Y: np.repeat(th.scale * np.asarray(Y).sum(axis=0, keepdims=True), th.k, axis=0)
    A = np.abs(th.dense(n))
    return lambda Y: A @ Y


def scale_R(R):
    """Per-entry scale of R: the 2-norm of its column."""
    return np.broadcast_to(np.linalg.norm(R, axis=0)[None, :], R.shape)


def scale_Q(Q, R):
    """Per-entry scale of Q = W R^{-1}: |Q| (|R| |R^{-1}|)."""
    Rinv = sla.solve_triangular(R, np.eye(R.shape[0]), lower=False)
    return np.abs(Q) @ (np.abs(R) @ np.abs(Rinv))


def scale_S(absT, sQ):
    """Per-entry scale of S = Theta Q: |Theta| scale_Q."""
    return absT(sQ)


def assert_entrywise(x, ref, scale, tol, what):
    """|x - ref| <= tol * scale entry by entry; entries whose scale is zero must
    match exactly.  Returns the largest ratio |x - ref| / scale."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    d = np.abs(x - ref)
    zero = scale == 0
    assert np.all(d[zero] == 0), f"{what}: nonzero difference where the scale is zero"
    ratio = np.zeros_like(d)
    ratio[~zero] = d[~zero] / scale[~zero]
    worst = float(ratio.max()) if ratio.size else 0.0
    idx = np.unravel_index(int(np.argmax(ratio)), ratio.shape) if ratio.size else ()
    say(f"{what}: max |x - x_or| / scale = {worst:.3e} at {tuple(int(i) for i in idx)} (tol {tol:.1e})")
    assert np.all(np.isfinite(x)), f"{what}: non-finite entries"
    assert worst <= tol, f"{what}: max ratio {worst:.3e} > {tol:.1e} at {idx}"
    return worst


def assert_qrs_entrywise(Q, R, S, o, absT, tol_r, tol_q, tol_s=None):
    """Q, R (and S) of the GPU against the oracle's result dict `o`."""
    assert_entrywise(R, o["R"], scale_R(o["R"]), tol_r, "R")
    sQ = scale_Q(o["Q"], o["R"])
    assert_entrywise(Q, o["Q"], sQ, tol_q, "Q")
    if S is not None:
        assert_entrywise(S, o["S"], scale_S(absT, sQ), tol_s if tol_s is not None else tol_q, "S")


def check_certificates(cert, S, R, P_or, absTW_fro, n, c=8.0, what="cert"):
    """The GPU's Delta and Delta~ against the oracle's certificate routine on
    the GPU's S and R (bounds in the module docstring)."""
    from oracle.rbgs import certificates
    d_or, dt_or = certificates(S, P_or, R)
    k, m = S.shape
    Pn = np.linalg.norm(P_or)
    tol_d = c * k * U64 * np.linalg.norm(S) ** 2
    tol_dt = c * U64 * (n * absTW_fro + m * np.linalg.norm(np.abs(S) @ np.abs(np.triu(R)))) / Pn
    say(f"{what}: Delta gpu {cert['delta']:.6e} oracle {d_or:.6e} (tol {tol_d:.1e}); "
        f"Delta~ gpu {cert['delta_tilde']:.6e} oracle {dt_or:.6e} (tol {tol_dt:.1e})")
    assert abs(cert["delta"] - d_or) <= tol_d, (cert["delta"], d_or, tol_d)
    assert abs(cert["delta_tilde"] - dt_or) <= tol_dt, (cert["delta_tilde"], dt_or, tol_dt)
    return d_or, dt_or


def abs_theta_w_fro(absT, W):
    """|| |Theta| |W| ||_F."""
    return float(np.linalg.norm(absT(np.abs(W))))
