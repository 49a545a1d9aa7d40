"""Randomized block Gram-Schmidt QR, FP64 (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation follows the paper: W = [W_(1) ... W_(p)] is n x m, split into blocks of
m_p columns (here the width is called `b`; the last block may be narrower);
Theta is the k x n sketching operator; P_(i) = Theta W_(i); S_(i) = Theta Q_(i);
Q'_(i) is the projection of W_(i); R is m x m upper triangular with positive
diagonal.

`rbgs` performs Algorithm "RBGS" (Section 2):
  1. P_(i) = Theta W_(i)
  2. R_(1:i-1,i) = argmin_Y || S_(1:i-1) Y - P_(i) ||_F      (Section 2.1)
  3. Q'_(i) = W_(i) - Q_(1:i-1) R_(1:i-1,i)
  4-5. sketched QR Q'_(i) = Q_(i) R_(i,i) and S_(i) = Theta Q_(i), either by
       RCholeskyQR ("plain", the algorithm of Section 2.2.2: S'_(i) = Theta Q'_(i))
       or by RCholeskyQR with postponed sketching ("lowsync", Section 2.2.3:
       S'_(i) = P_(i) - S_(1:i-1) R_(1:i-1,i)); in both, R_(i,i) is the R factor
       of the l2-QR of S'_(i) and Q_(i) = Q'_(i) R_(i,i)^{-1} by substitution.
       Two more stable forms of Section 2.2.4: "twice" runs RCholeskyQR on
       the Q-factor of the first RCholeskyQR (Q'_(i) = Q* R1, Q* = Q_(i) R2,
       R_(i,i) = R2 R1), and "l2qr" first takes the l2 (Householder) QR
       Q'_(i) = Q* R', then RCholeskyQR Q* = Q_(i) R'' and R_(i,i) = R'' R'.
  6. Delta = ||I - S^T S||_F and Delta~ = ||P - S R||_F / ||P||_F.

Least-squares solvers for step 2:
  * Householder (Section 2.1, the direct backward-stable solver): QR of
    S_(1:i-1) by LAPACK Householder, then a triangular solve.
  * Richardson with l sweeps (supplement, Section SM.1):
    X <- X + S^T (P - S X), starting from X = 0.

Parity: pinned (tests/test_oracle_rbgs.py) -- with Theta = I the result must
equal LAPACK Householder QR with a positive diagonal; for full-rank W it must
equal the closed form R = R-factor(Theta W), Q = W R^{-1} (the exact-arithmetic
result of RBGS); plain and low-sync variants must agree; R must be upper
triangular with positive diagonal; Richardson with l = 1 must equal the
sketched block CGS projection S^T P and its error must respect the bound
(Delta^(i-1))^l ||y|| of the supplement; the a-posteriori bound of the
stability theorem must hold.
"""
import numpy as np
import scipy.linalg as sla


def qr_r_posdiag(A):
    """R factor of the l2 (Householder) QR of A with a positive diagonal.

    The paper requires R with positive diagonal entries (Section 1); LAPACK's
    Householder QR may return negative diagonal entries, which are made
    positive by flipping the sign of the corresponding rows of R (and, implicitly,
    columns of the orthogonal factor)."""
    R = np.linalg.qr(A, mode="r")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return d[:, None] * R


def ls_householder(S, P):
    """argmin_Y ||S Y - P||_F via Householder QR of S (direct solver)."""
    if S.shape[1] == 0:
        return np.zeros((0, P.shape[1]))
    Qs, Rs = np.linalg.qr(S, mode="reduced")
    return sla.solve_triangular(Rs, Qs.T @ P, lower=False)


def ls_richardson(S, P, l):
    """l Richardson sweeps X <- X + S^T (P - S X) from X = 0 (supplement SM.1)."""
    X = np.zeros((S.shape[1], P.shape[1]))
    for _ in range(l):
        X = X + S.T @ (P - S @ X)
    return X


def block_ranges(m, b):
    """Column ranges [c0, c1) of the blocks W_(1), ..., W_(p); the last block is
    narrower when b does not divide m."""
    return [(c0, min(m, c0 + b)) for c0 in range(0, m, b)]


def rbgs(W, b, theta, variant="plain", ls="householder", ls_iters=2):
    """RBGS QR of W (n x m, FP64) with block width b and sketch `theta`
    (a callable X -> Theta X, e.g. oracle.theta.Sketch).

    variant: "plain" (RCholeskyQR in steps 4-5), "lowsync" (RCholeskyQR with
             postponed sketching), "twice" (RCholeskyQR twice) or "l2qr"
             (l2-QR + RCholeskyQR).
    ls:      "householder" or "richardson" (with `ls_iters` sweeps).
    Returns a dict with Q, R, S (= Theta Q), P (= Theta W), delta, delta_tilde.
    """
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    Q = np.zeros((n, m))
    R = np.zeros((m, m))
    S = None
    P = None
    for (c0, c1) in block_ranges(m, b):
        Wi = W[:, c0:c1]
        # 1. sketch of W_(i)
        Pi = theta(Wi)
        if S is None:
            k = Pi.shape[0]
            S = np.zeros((k, m))
            P = np.zeros((k, m))
        P[:, c0:c1] = Pi
        # 2. sketched least-squares problem
        if c0 == 0:
            Rij = np.zeros((0, c1 - c0))
        elif ls == "householder":
            Rij = ls_householder(S[:, :c0], Pi)
        elif ls == "richardson":
            Rij = ls_richardson(S[:, :c0], Pi, ls_iters)
        else:
            raise ValueError(ls)
        R[:c0, c0:c1] = Rij
        # 3. projection
        Qp = Wi - Q[:, :c0] @ Rij
        # 4. sketch of Q'_(i) and R_(i,i)
        if variant in ("plain", "twice"):
            Qi, Rii = rcholeskyqr(Qp, theta(Qp))
            if variant == "twice":
                Qi, R2 = rcholeskyqr(Qi, theta(Qi))
                Rii = R2 @ Rii
        elif variant == "lowsync":
            Qi, Rii = rcholeskyqr(Qp, Pi - S[:, :c0] @ Rij)
        elif variant == "l2qr":
            Qs, Rp = l2_qr_posdiag(Qp)
            Qi, R2 = rcholeskyqr(Qs, theta(Qs))
            Rii = R2 @ Rp
        else:
            raise ValueError(variant)
        R[c0:c1, c0:c1] = Rii
        Q[:, c0:c1] = Qi
        # 5. sketch of Q_(i)
        S[:, c0:c1] = theta(Qi)
    delta, delta_tilde = certificates(S, P, R)
    return dict(Q=Q, R=R, S=S, P=P, delta=delta, delta_tilde=delta_tilde)


def rcholeskyqr(Qp, Sp):
    """Steps 4-5 core of RCholeskyQR (Section 2.2.2): R = R factor of the l2-QR
    of the sketch Sp = Theta Qp (positive diagonal) and Q = Qp R^{-1} by
    substitution -- solve Q R = Qp, i.e. R^T Q^T = Qp^T (lower triangular,
    forward substitution)."""
    Rf = qr_r_posdiag(Sp)
    return sla.solve_triangular(Rf.T, Qp.T, lower=True).T, Rf


def l2_qr_posdiag(A):
    """Householder (LAPACK) QR A = Q R of a tall matrix with R's diagonal made
    positive (the columns of Q flipped with the rows of R)."""
    Qh, Rh = np.linalg.qr(A, mode="reduced")
    d = np.sign(np.diag(Rh))
    d[d == 0] = 1.0
    return Qh * d[None, :], d[:, None] * Rh


def certificates(S, P, R):
    """Step 6: Delta = ||I - S^T S||_F, Delta~ = ||P - S R||_F / ||P||_F."""
    m = S.shape[1]
    delta = np.linalg.norm(np.eye(m) - S.T @ S, "fro")
    pn = np.linalg.norm(P, "fro")
    delta_tilde = np.linalg.norm(P - S @ R, "fro") / pn if pn > 0 else 0.0
    return float(delta), float(delta_tilde)


def cholqr_post(Q, R):
    """Cholesky-QR post-processing (remark on post-processing, Section 2.2):
    R' = upper Cholesky factor of Q^T Q, Q <- Q R'^{-1} (substitution),
    R <- R' R."""
    Rp = np.linalg.cholesky(Q.T @ Q).T
    Qn = sla.solve_triangular(Rp.T, Q.T, lower=True).T
    return Qn, Rp @ R


def rbgs_closed_form(W, theta):
    """Exact-arithmetic result of RBGS for full-rank W: Theta W = (Theta Q) R with
    Theta Q orthonormal, so R is the positive-diagonal R factor of Theta W and
    Q = W R^{-1} (cf. the remark relating RBGS to RCholeskyQR, Section 2.2.3)."""
    R = qr_r_posdiag(theta(W))
    Q = sla.solve_triangular(R.T, np.asarray(W, dtype=np.float64).T, lower=True).T
    return Q, R
