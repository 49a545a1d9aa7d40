"""Block Krylov methods on top of RBGS, FP64 (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* `rbgs_arnoldi`: Algorithm RBGS-Arnoldi (Section 4.1).  W_(1) = B; for
  i = 2..p, W_(i) = A Q_(i-1); after each W_(i), iteration i of Algorithm RBGS
  (the same steps as `oracle.rbgs.rbgs`: sketch, sketched least squares,
  projection, sketched QR of the projection by RCholeskyQR or RCholeskyQR with
  postponed sketching, substitution, re-sketch).  The Arnoldi identity is
  A Q_(1:p-1) = Q R_(1:p,2:p).
* `block_gmres`: restarted randomized block GMRES (Section 4.2).  Each cycle:
  R0 = B - A X; RBGS-Arnoldi with blocks_per_cycle + 1 blocks from W_(1) = R0;
  Z = argmin ||H Z - R_(1:p,1)||_F with H = R_(1:p,2:p) (a library
  least-squares solve, numpy's lstsq); X <- X + Q_(1:p-1) Z.

Parity: pinned in tests/test_oracle_krylov.py -- with Theta = I the basis is
l2-orthonormal and equals, up to column signs, the orthonormal basis of the
block Krylov matrix [B, A B, ..., A^(p-1) B] obtained by a library QR; the
Arnoldi identity holds to rounding for any Theta; GMRES reaches the exact
solution (a library sparse direct solve) once the Krylov space is the whole
space, and its residual never exceeds the initial one.
"""
import numpy as np
import scipy.linalg as sla

from oracle.rbgs import block_ranges, ls_householder, ls_richardson, qr_r_posdiag


def rbgs_arnoldi(A, B, nblocks, theta, variant="lowsync", ls="richardson", ls_iters=4):
    """Q (n x nblocks bs), R (m x m) and S = Theta Q of RBGS-Arnoldi."""
    B = np.asarray(B, dtype=np.float64)
    n, bs = B.shape
    m = nblocks * bs
    Q = np.zeros((n, m))
    R = np.zeros((m, m))
    S = None
    for i, (c0, c1) in enumerate(block_ranges(m, bs)):
        Wi = B if i == 0 else A @ Q[:, c0 - bs:c0]
        Pi = theta(Wi)
        if S is None:
            S = np.zeros((Pi.shape[0], m))
        if c0 == 0:
            Rij = np.zeros((0, c1 - c0))
        elif ls == "householder":
            Rij = ls_householder(S[:, :c0], Pi)
        else:
            Rij = ls_richardson(S[:, :c0], Pi, ls_iters)
        R[:c0, c0:c1] = Rij
        Qp = Wi - Q[:, :c0] @ Rij
        Sp = theta(Qp) if variant == "plain" else Pi - S[:, :c0] @ Rij
        Rii = qr_r_posdiag(Sp)
        R[c0:c1, c0:c1] = Rii
        Qi = sla.solve_triangular(Rii.T, Qp.T, lower=True).T
        Q[:, c0:c1] = Qi
        S[:, c0:c1] = theta(Qi)
    return Q, R, S


def block_gmres(A, B, X0, blocks_per_cycle, max_cycles, tol, theta, variant="lowsync",
                ls="richardson", ls_iters=4):
    """Returns (X, history of relative residuals at each cycle start and at the end)."""
    B = np.asarray(B, dtype=np.float64)
    X = np.array(X0, dtype=np.float64, copy=True)
    bs = B.shape[1]
    nb = blocks_per_cycle + 1
    bnorm = np.linalg.norm(B)
    hist = []
    for _ in range(max_cycles):
        R0 = B - A @ X
        rel = np.linalg.norm(R0) / bnorm
        hist.append(rel)
        if rel <= tol:
            return X, hist
        Q, R, _ = rbgs_arnoldi(A, R0, nb, theta, variant, ls, ls_iters)
        H = R[:, bs:]
        Z = np.linalg.lstsq(H, R[:, :bs], rcond=None)[0]
        X = X + Q[:, :nb * bs - bs] @ Z
    hist.append(np.linalg.norm(B - A @ X) / bnorm)
    return X, hist
