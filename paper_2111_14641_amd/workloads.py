"""Seeded synthetic input matrices for RBGS QR.

This module only builds inputs; it contains none of the method's arithmetic
and is shared by the tests, the benchmark and the smoke check.  All matrices are
returned in FP64, column-major (Fortran order), so that column j is contiguous.

* `svd_matrix(n, m, sigma, seed)`: W = U diag(sigma) V^T with U the
  orthonormal factor of a seeded n x m Gaussian matrix and V that of a seeded
  m x m Gaussian matrix (both sign-fixed so the factor is unique); cond(W) is
  sigma[0] / sigma[-1].  With n = 10 000, m = 64 and sigma = logspace(0, -8, 64)
  this is the small FP64 single-QR workload.
* `oscillatory_matrix(n, m, seed)`: w_ij = sin(10 (mu_j x_i + 1)) /
  (cos(100 mu_j x_i - 100 mu_j) + 1.1), x_i = i / (n - 1), mu_j ~ U[0, 1]
  drawn from a seeded generator.  A smooth parametric family, numerically
  rank-deficient, which stands in for the matrix of the paper's first numerical
  example (Section 5.1), whose exact generator differs; with n = 10^6 and
  m = 256 this is the large single-QR workload.
* `svd_matrix_gpu(n, m, sigma, seed, dtypes)`: the same construction as
  `svd_matrix` built on the GPU in row chunks, for sizes whose FP64 factors do
  not fit comfortably in host memory: G is a seeded device Gaussian generated
  chunk by chunk (chunk c from its own generator seeded with seed + c, so any
  chunk can be regenerated), U = G M1 with M1 = L1^{-T} L2^{-T} from two rounds
  of Cholesky orthonormalization whose Gram matrices are summed over the
  chunks in a fixed order, V on the host, and W = G (M1 diag(sigma) V^T)
  written chunk by chunk into one output tensor per requested dtype.  No torch
  operation touches more than one chunk (2^18 rows).  With n = 4 10^6, m = 512
  and sigma = logspace(0, -10, 512) this is the mixed-precision workload.
* `batched_problems(count, seed)`: the batched workload, `count` FP32
  matrices on the GPU with n = round(2^u), u ~ U[14, 18], m drawn from
  {32, 64, 128, 256} and W = G diag(sigma) V^T, G a seeded Gaussian n x m
  (cond(G) <= (1 + sqrt(m/n)) / (1 - sqrt(m/n)) < 1.3), sigma =
  logspace(0, -c, m), c ~ U[2, 10], V a seeded orthogonal m x m matrix: so
  cond(W) is 10^c up to that factor.
* `convection_diffusion_csr(N, beta)`: the block GMRES operator, the 2-D
  convection-diffusion operator -Laplace(u) + beta (1, 1) . grad(u) on the
  unit square with homogeneous Dirichlet conditions, discretized on the N x N
  interior grid (h = 1 / (N + 1)) by the 5-point stencil with first-order
  upwind convection and scaled by h^2: diagonal 4 + 2 beta h, west and south
  -1 - beta h, east and north -1.  Unknown (i, j) (1-based) is row
  (i - 1) + N (j - 1).  Returns CSR arrays (indptr int64, indices int32,
  data float64), columns sorted within each row.  N = 1024 gives n = 1048576
  with 5 n - 4 N nonzeros.
* `gmres_rhs(n, bs, seed)`: the block of right-hand sides, seeded standard
  Gaussian n x bs (FP64, column-major).
"""
import numpy as np


def _orthonormal(rng, n, m):
    G = rng.standard_normal((n, m))
    U, Rg = np.linalg.qr(G)
    d = np.sign(np.diag(Rg))
    d[d == 0] = 1.0
    return U * d[None, :]


def svd_matrix(n, m, sigma, seed):
    rng = np.random.default_rng(seed)
    U = _orthonormal(rng, n, m)
    V = _orthonormal(rng, m, m)
    sigma = np.asarray(sigma, dtype=np.float64)
    return np.asfortranarray((U * sigma[None, :]) @ V.T)


def small_single_qr(seed=0xDA7A00, n=10_000, m=64, decades=8.0):
    """The small FP64 single-QR workload (cond(W) = 10^decades)."""
    return svd_matrix(n, m, np.logspace(0.0, -decades, m), seed)


def oscillatory_matrix(n, m, seed, dtype=np.float64, chunk=1 << 17):
    rng = np.random.default_rng(seed)
    mu = rng.random(m)
    W = np.empty((n, m), dtype=dtype, order="F")
    denom_n = max(n - 1, 1)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        x = np.arange(r0, r1, dtype=np.float64)[:, None] / denom_n
        mx = mu[None, :] * x
        W[r0:r1, :] = np.sin(10.0 * (mx + 1.0)) / (np.cos(100.0 * mx - 100.0 * mu[None, :]) + 1.1)
    return W


def _gpu_gaussian_chunk(r0, r1, m, seed, chunk, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) + r0 // chunk) & 0x7FFFFFFFFFFFFFFF)
    return torch.randn((r1 - r0, m), generator=g, dtype=torch.float64, device=device)


def svd_matrix_gpu(n, m, sigma, seed, device="cuda", dtypes=("float64",), chunk=1 << 18):
    """W = U diag(sigma) V^T as column-major tensors on `device`, one per
    entry of `dtypes` (torch dtype names), built in row chunks."""
    import torch
    ranges = [(r0, min(n, r0 + chunk)) for r0 in range(0, n, chunk)]
    # two rounds of Cholesky orthonormalization of G; M1 = L1^{-T} L2^{-T}
    M1 = np.eye(m)
    for _ in range(2):
        Mt = torch.from_numpy(M1).to(device)
        A = np.zeros((m, m))
        for r0, r1 in ranges:
            X = _gpu_gaussian_chunk(r0, r1, m, seed, chunk, device) @ Mt
            A += (X.t() @ X).cpu().numpy()
            del X
        A = 0.5 * (A + A.T)
        L = np.linalg.cholesky(A)
        M1 = M1 @ np.linalg.inv(L).T
    V = _orthonormal(np.random.default_rng(seed), m, m)
    M = torch.from_numpy(M1 @ (np.asarray(sigma, dtype=np.float64)[:, None] * V.T)).to(device)
    outs = [torch.empty((m, n), dtype=getattr(torch, d), device=device).t() for d in dtypes]
    for r0, r1 in ranges:
        Wc = _gpu_gaussian_chunk(r0, r1, m, seed, chunk, device) @ M
        for o in outs:
            o[r0:r1].copy_(Wc)
        del Wc
    return outs[0] if len(outs) == 1 else tuple(outs)


def mixed_single_qr_gpu(seed=0xDA7A02, n=4_000_000, m=512, decades=10.0,
                        dtypes=("float64",)):
    """The mixed-precision single-QR workload (cond(W) = 10^decades), on the GPU."""
    return svd_matrix_gpu(n, m, np.logspace(0.0, -decades, m), seed, dtypes=dtypes)


def batched_problems(count=512, seed=0xDA7A04, device="cuda"):
    """List of (W (FP32, column-major, on `device`), n, m, c)."""
    import torch
    rng = np.random.default_rng(seed)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    out = []
    for _ in range(count):
        n = int(round(2.0 ** rng.uniform(14.0, 18.0)))
        m = int(rng.choice([32, 64, 128, 256]))
        c = float(rng.uniform(2.0, 10.0))
        V = _orthonormal(rng, m, m)
        M = torch.from_numpy(np.logspace(0.0, -c, m)[:, None] * V.T).to(device)
        G = torch.randn((n, m), generator=g, dtype=torch.float64, device=device)
        W = torch.empty((m, n), dtype=torch.float32, device=device).t()
        W.copy_(G @ M)
        del G
        out.append((W, n, m, c))
    return out


def convection_diffusion_csr(N, beta=50.0):
    h = 1.0 / (N + 1)
    n = N * N
    r = np.arange(n, dtype=np.int64)
    i = r % N
    j = r // N
    cols, vals, valid = [], [], []
    # neighbours in increasing column order: south, west, centre, east, north
    for dc, ok, v in ((-N, j > 0, -1.0 - beta * h), (-1, i > 0, -1.0 - beta * h),
                      (0, np.ones(n, bool), 4.0 + 2.0 * beta * h), (1, i < N - 1, -1.0),
                      (N, j < N - 1, -1.0)):
        cols.append(r + dc)
        vals.append(np.full(n, v))
        valid.append(ok)
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    M = np.stack(valid, axis=1)
    counts = M.sum(axis=1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    indices = C[M].astype(np.int32)
    data = V[M].astype(np.float64)
    return indptr, indices, data


def gmres_rhs(n, bs, seed=0xDA7A03):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, bs)))


def large_single_qr(seed=0xDA7A01, n=1_000_000, m=256, dtype=np.float64):
    """The large single-QR workload (n = 10^6, m = 256)."""
    return oscillatory_matrix(n, m, seed, dtype=dtype)


# Default seeds of the sketching operators for each workload.
THETA_SEED_SMALL = 0x2111146410
THETA_SEED_LARGE = 0x2111146411
THETA_SEED_MIXED = 0x2111146412
