"""Pins of the oracle's metrics on matrices with known values (CPU only)."""
import numpy as np

from oracle.metrics import cond2, cond2_from_gram, factorization_error, orthogonality_loss


def test_cond2_known_values():
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((500, 8)))
    assert abs(cond2(U) - 1) < 1e-12
    D = U * np.array([1, 2, 3, 4, 5, 6, 7, 50.0])[None, :]
    assert abs(cond2(D) - 50) < 1e-10
    assert abs(cond2_from_gram(D.T @ D) - 50) < 1e-8


def test_orthogonality_loss_and_error_known_values():
    rng = np.random.default_rng(1)
    U, _ = np.linalg.qr(rng.standard_normal((300, 5)))
    assert orthogonality_loss(U) < 1e-14
    assert abs(orthogonality_loss(2 * U) - 3 * np.sqrt(5)) < 1e-12
    R = np.triu(rng.standard_normal((5, 5)))
    W = U @ R
    assert factorization_error(W, U, R) < 1e-15
    assert abs(factorization_error(W, U, 0.5 * R) - 0.5) < 1e-14
