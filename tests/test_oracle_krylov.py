"""Pins of the block Krylov oracle and of the convection-diffusion operator
(CPU)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import krylov
from oracle.theta import Sketch
from paper_2111_14641_amd.workloads import convection_diffusion_csr, gmres_rhs


def csr(N, beta=50.0):
    indptr, indices, data = convection_diffusion_csr(N, beta)
    return sp.csr_matrix((data, indices, indptr), shape=(N * N, N * N))


def test_operator_equals_kronecker_sum():
    """The stencil assembly equals I (x) T + T (x) I with the 1-D operator
    T = tridiag(-1 - beta h, 2 + beta h, -1) (second difference plus upwind
    first difference, scaled by h^2)."""
    N, beta = 13, 50.0
    h = 1.0 / (N + 1)
    T = sp.diags([np.full(N - 1, -1.0 - beta * h), np.full(N, 2.0 + beta * h), np.full(N - 1, -1.0)],
                 [-1, 0, 1])
    I = sp.identity(N)
    K = (sp.kron(I, T) + sp.kron(T, I)).toarray()
    A = csr(N, beta).toarray()
    assert np.allclose(A, K, rtol=0, atol=1e-14)
    indptr, indices, _ = convection_diffusion_csr(N, beta)
    assert indptr[-1] == 5 * N * N - 4 * N
    for r in range(N * N):   # sorted columns per row
        cols = indices[indptr[r]:indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


def test_arnoldi_identity_sketch_is_block_arnoldi():
    """Theta = I: the basis is l2-orthonormal, spans the block Krylov space
    (projector equal to the one of a library QR of [B, AB, A^2 B]), and the
    Arnoldi identity holds."""
    N, bs, nb = 8, 2, 3
    A = csr(N)
    n = N * N
    B = gmres_rhs(n, bs, seed=1)
    Q, R, _ = krylov.rbgs_arnoldi(A, B, nb, Sketch("identity", n), "plain", "householder")
    m = nb * bs
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) < 1e-12
    Kr = np.hstack([B, A @ B, A @ (A @ B)])
    U = np.linalg.qr(Kr)[0]
    assert np.linalg.norm(Q @ Q.T - U @ U.T) < 1e-9
    assert np.linalg.norm(A @ Q[:, :m - bs] - Q @ R[:, bs:]) < 1e-12 * np.linalg.norm(A.toarray())
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


@pytest.mark.parametrize("kind", ["sparse", "gaussian"])
def test_arnoldi_identity_with_sketch(kind):
    N, bs, nb = 16, 4, 6
    A = csr(N)
    n = N * N
    B = gmres_rhs(n, bs, seed=2)
    th = Sketch(kind, 96, seed=3).materialize(n)
    Q, R, S = krylov.rbgs_arnoldi(A, B, nb, th, "lowsync", "richardson", 4)
    m = nb * bs
    assert np.linalg.norm(S.T @ S - np.eye(m)) < 1e-10          # sketched orthonormality
    An = np.linalg.norm(A.toarray(), 2)
    assert np.linalg.norm(A @ Q[:, :m - bs] - Q @ R[:, bs:]) < 1e-12 * An * np.linalg.norm(Q)
    assert np.allclose(R[:bs, :bs], np.linalg.qr(th(B), mode="r") * np.sign(np.diag(np.linalg.qr(th(B), mode="r")))[:, None])


def test_gmres_exact_when_the_krylov_space_is_everything():
    N, bs = 8, 2
    A = csr(N)
    n = N * N
    B = gmres_rhs(n, bs, seed=4)
    X, hist = krylov.block_gmres(A, B, np.zeros((n, bs)), n // bs - 1, 2, 1e-10,
                                 Sketch("identity", n), "plain", "householder")
    Xd = spla.spsolve(A.tocsc(), B)
    assert hist[-1] < 1e-10
    assert np.linalg.norm(X - Xd) < 1e-9 * np.linalg.norm(Xd)


def test_gmres_converges_with_a_sparse_sketch():
    N, bs = 16, 4
    A = csr(N)
    n = N * N
    B = gmres_rhs(n, bs, seed=5)
    X, hist = krylov.block_gmres(A, B, np.zeros((n, bs)), 15, 20, 1e-8,
                                 Sketch("sparse", 256, seed=6).materialize(n))
    assert hist[0] == pytest.approx(1.0)
    assert hist[-1] <= 1e-8
    Xd = spla.spsolve(A.tocsc(), B)
    assert np.linalg.norm(X - Xd) < 1e-5 * np.linalg.norm(Xd)
