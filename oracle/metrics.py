"""Result metrics (oracle side, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* factorization_error: ||W - Q R||_F / ||W||_F (the error studied in the
  paper's first numerical example, Section 5.1).
* cond2: 2-norm condition number of Q (ratio of extreme singular values).
* orthogonality_loss: Delta = ||I - S^T S||_F for a sketch S = Theta Q
  (step 6 of the RBGS algorithm).

Parity: these are plain definitions written out with LAPACK SVD / BLAS; the
tests pin them on matrices with known values (orthogonal Q -> cond 1, scaled
columns -> known cond).
"""
import numpy as np


def factorization_error(W, Q, R):
    W = np.asarray(W, dtype=np.float64)
    return float(np.linalg.norm(W - np.asarray(Q, np.float64) @ np.asarray(R, np.float64), "fro")
                 / np.linalg.norm(W, "fro"))


def cond2(Q):
    s = np.linalg.svd(np.asarray(Q, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")


def cond2_from_gram(G):
    """cond2 of Q from its Gram matrix G = Q^T Q (eigenvalues are sigma^2)."""
    ev = np.linalg.eigvalsh(np.asarray(G, dtype=np.float64))
    if ev[0] <= 0:
        return float("inf")
    return float(np.sqrt(ev[-1] / ev[0]))


def orthogonality_loss(S):
    S = np.asarray(S, dtype=np.float64)
    return float(np.linalg.norm(np.eye(S.shape[1]) - S.T @ S, "fro"))
