"""GPU sketching operators against the oracle's definition (bit-exact Theta,
FP64-accurate sketches)."""
import sys

import numpy as np
import pytest

from oracle import theta as th

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def to_np(t):
    return np.ascontiguousarray(t.detach().cpu().numpy())


@pytest.mark.parametrize("k,n,row0,seed", [
    (256, 1000, 0, 0x2111146410),
    (64, 333, 12345, 7),
    (1024, 300, 2**32 - 100, 99),      # crosses the 32-bit boundary of the row counter
    # 2^25 Box-Muller pairs: about 98 % of the 2^23 values of each word the
    # logarithm, square root and sine/cosine read
    (1024, 65536, 5, 0x5EED),
])
def test_gaussian_theta_bit_exact(gpu_lib, k, n, row0, seed):
    from paper_2111_14641_amd import binding as B
    say("theta gaussian", k, n, row0, seed)
    Zg = to_np(B.theta_dense("gaussian", k, seed, n, row0))
    Zo = np.ascontiguousarray(th.gaussian_z(np.arange(row0, row0 + n, dtype=np.uint64), k, seed).T)
    mism = np.count_nonzero(Zg.view(np.uint32) != Zo.view(np.uint32))
    assert mism == 0, f"{mism} of {Zg.size} entries differ; max abs diff {np.max(np.abs(Zg - Zo))}"


@pytest.mark.parametrize("k,zeta,n,row0,seed", [
    (1024, 8, 2000, 0, 0x2111146411), (64, 8, 500, 777, 3), (60, 5, 100, 2**33, 5), (2048, 8, 300, 0, 1),
])
def test_sparse_theta_bit_exact(gpu_lib, k, zeta, n, row0, seed):
    from paper_2111_14641_amd import binding as B
    say("theta sparse", k, zeta, n, row0, seed)
    Bg = to_np(B.theta_dense("sparse", k, seed, n, row0, zeta=zeta))
    S = th.Sketch("sparse", k, seed=seed, zeta=zeta)
    idx, sgn = th.sparse_sign_entries(np.arange(row0, row0 + n, dtype=np.uint64), k, zeta, seed)
    Bo = np.zeros((k, n), dtype=np.float32)
    Bo[idx.ravel(), np.repeat(np.arange(n), zeta)] = sgn.ravel()
    assert np.array_equal(Bg, Bo)
    assert S.scale == 1 / np.sqrt(zeta)


@pytest.mark.parametrize("k,n,row0,seed", [
    (256, 1000, 0, 0x2111146412),
    (100, 333, 12345, 7),               # k not a multiple of 128: a partial last Philox call
    (260, 300, 2**32 - 100, 99),        # crosses the 32-bit boundary of the row counter
])
def test_rademacher_theta_bit_exact(gpu_lib, k, n, row0, seed):
    from paper_2111_14641_amd import binding as B
    say("theta rademacher", k, n, row0, seed)
    Bg = to_np(B.theta_dense("rademacher", k, seed, n, row0))
    Bo = th.rademacher_b(np.arange(row0, row0 + n, dtype=np.uint64), k, seed).T.astype(np.float32)
    assert np.array_equal(Bg, Bo)


def srht_entries(k, seed, rows, L):
    """Unscaled SRHT entries d_r (-1)^popcount(s_t & r) for the given global
    rows (the closed form of H, pinned against scipy's Hadamard matrix)."""
    s = th.srht_samples(k, L, seed)
    d = th.srht_signs(rows, seed)
    par = np.zeros((k, len(rows)), dtype=np.int64)
    x = s[:, None] & np.asarray(rows, dtype=np.uint64)[None, :]
    while np.any(x):
        par ^= (x & np.uint64(1)).astype(np.int64)
        x = x >> np.uint64(1)
    return (np.where(par == 1, -1.0, 1.0) * d[None, :]).astype(np.float32)


@pytest.mark.parametrize("k,n,row0,L,seed", [
    (256, 1000, 0, 10, 0x2111146413),
    (100, 333, 12345, 15, 7),
    (2048, 300, 2**31 + 5, 32, 99),     # widest transform, row index above 2^31
    (64, 50, 0, 6, 3),                  # transform smaller than one 1024-row chunk
])
def test_srht_theta_bit_exact(gpu_lib, k, n, row0, L, seed):
    from paper_2111_14641_amd import binding as B
    say("theta srht", k, n, row0, L, seed)
    Tg = to_np(B.theta_dense("srht", k, seed, n, row0, zeta=L))
    To = srht_entries(k, seed, np.arange(row0, row0 + n, dtype=np.uint64), L)
    assert np.array_equal(Tg, To)
    if row0 == 0:
        Td = th.Sketch("srht", k, seed=seed, zeta=L).dense(n) * np.sqrt(k)
        assert np.array_equal(To.astype(np.float64), np.round(Td))


def abs_sketch(kind, k, seed, X, row0, zeta=8):
    """|Theta| |X| (the scale of the rounding-error bound of a sketch)."""
    import scipy.sparse as sp
    n = X.shape[0]
    rows = np.arange(row0, row0 + n, dtype=np.uint64)
    if kind == "gaussian":
        out = np.zeros((k, X.shape[1]))
        for r0 in range(0, n, 8192):
            Z = th.gaussian_z(rows[r0:r0 + 8192], k, seed).astype(np.float64)
            out += np.abs(Z).T @ np.abs(X[r0:r0 + 8192])
        return out / np.sqrt(k)
    if kind in ("rademacher", "srht"):
        return np.broadcast_to(np.abs(X).sum(axis=0) / np.sqrt(k), (k, X.shape[1]))
    idx, _ = th.sparse_sign_entries(rows, k, zeta, seed)
    Bm = sp.csr_matrix((np.ones(idx.size), (idx.ravel().astype(np.int64), np.repeat(np.arange(n), zeta))),
                       shape=(k, n))
    return (Bm @ np.abs(X)) / np.sqrt(zeta)


@pytest.mark.parametrize("kind,k", [("gaussian", 256), ("gaussian", 100), ("sparse", 1024),
                                    ("sparse", 2048), ("sparse", 64), ("rademacher", 256),
                                    ("rademacher", 100), ("srht", 256), ("srht", 2048),
                                    ("srht", 30)])
@pytest.mark.parametrize("n,c,row0", [(4097, 16, 0), (1000, 5, 31), (70000, 33, 1 << 20), (3, 1, 0),
                                      (3000, 70, 5)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sketch_apply_matches_oracle(gpu_lib, kind, k, n, c, row0, dtype):
    """FP64 accumulation of exact products (fp32 entries of Z or +-1 times the
    data): GPU and oracle differ by summation order only, within
    c u sqrt(n) |Theta| |X| elementwise."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("sketch", kind, k, n, c, row0, dtype)
    rng = np.random.default_rng(n + c + k)
    X = rng.standard_normal((n, c))
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Xt = B.colmajor(n, c, tdt)
    Xt.copy_(torch.from_numpy(X))
    got = to_np(B.sketch_apply(Xt, kind, k, seed=11, row0=row0))
    ref = th.Sketch(kind, k, seed=11).apply(X, row0=row0)
    # the transform of the SRHT adds log2 N levels of pairwise sums
    depth = np.sqrt(n) if kind != "srht" else np.sqrt(n) + th.ceil_log2(row0 + n)
    tol = 1e-15 * (10 + depth) * abs_sketch(kind, k, 11, X, row0)
    assert np.all(np.abs(got - ref) <= tol)


def test_identity_sketch_copies(gpu_lib):
    import torch
    from paper_2111_14641_amd import binding as B
    say("sketch identity")
    X = np.random.default_rng(0).standard_normal((50, 3))
    Xt = B.colmajor(50, 3, torch.float64)
    Xt.copy_(torch.from_numpy(X))
    assert np.array_equal(to_np(B.sketch_apply(Xt, "identity", 50, seed=0)), X)


@pytest.mark.parametrize("kind,k", [("sparse", 1024), ("gaussian", 256), ("rademacher", 256),
                                    ("srht", 1024)])
def test_row_shards_sum_to_the_whole(gpu_lib, kind, k):
    """Theta's columns are addressed by the global row index, so sketching G row
    ranges with their row offsets and adding the parts in a fixed order gives
    the sketch of the whole matrix (up to summation order): the one exchange a
    row-sharded run needs per block."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("virtual shards", kind, k)
    n, c = 300_001, 16
    X = np.random.default_rng(5).standard_normal((n, c))
    Xt = B.colmajor(n, c, torch.float64)
    Xt.copy_(torch.from_numpy(X))
    z = th.ceil_log2(n) if kind == "srht" else None   # one SRHT size for every range
    whole = to_np(B.sketch_apply(Xt, kind, k, seed=21, zeta=z))
    bounds = [0, 70_000, 150_123, 299_999, n]
    parts = np.zeros_like(whole)
    for a, b in zip(bounds[:-1], bounds[1:]):
        parts += to_np(B.sketch_apply(Xt[a:b], kind, k, seed=21, row0=a, zeta=z))
    tol = 1e-15 * (10 + np.sqrt(n)) * abs_sketch(kind, k, 21, X, 0)
    assert np.all(np.abs(parts - whole) <= tol)
