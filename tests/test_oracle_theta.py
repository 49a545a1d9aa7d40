"""Pins of the oracle's sketching operators (CPU only)."""
import numpy as np
import pytest
import scipy.stats as st

from oracle import theta as th


def test_ln_u24_exhaustive_against_libm():
    """All 2^23 inputs of the fp32 logarithm against numpy's FP64 log."""
    v = np.arange(1 << 23, dtype=np.uint32)
    w = v << np.uint32(9)
    got = th.ln_u24(w).astype(np.float64)
    u = (v.astype(np.float64) * 2 + 1) * 2.0**-24
    ex = np.log(u)
    ulp = np.spacing(np.abs(ex).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ex) / ulp) <= 3.0


def test_sincos_against_libm():
    rng = np.random.default_rng(3)
    w = rng.integers(0, 2**32, size=1 << 22, dtype=np.uint64).astype(np.uint32)
    w[:4] = [0, 0xFFFFFFFF, 0x40000000, 0xBFFFFF80]
    c, s = th.sincos_quarter(w)
    q = (w >> np.uint32(30)).astype(np.float64)
    t = (((w >> np.uint32(7)) & np.uint32(0x7FFFFF)).astype(np.float64) * 2 + 1) * 2.0**-24
    phi = 0.5 * np.pi * (q + t)
    assert np.max(np.abs(c - np.cos(phi))) < 4e-7
    assert np.max(np.abs(s - np.sin(phi))) < 4e-7
    # unit circle to fp32 accuracy
    c64, s64 = c.astype(np.float64), s.astype(np.float64)
    assert np.max(np.abs(c64 * c64 + s64 * s64 - 1)) < 1e-6


def test_gaussian_entries_are_standard_normal():
    z = th.gaussian_z(np.arange(4096), 256, seed=0x5EED).astype(np.float64)
    x = z.ravel()
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs((x**4).mean() - 3) < 5 * np.sqrt(96 / n)
    assert st.kstest(x, "norm").pvalue > 1e-3
    # entries from the two halves of a Box-Muller pair and from neighbouring
    # targets / columns are uncorrelated
    for a, b in [(z[:, 0::4], z[:, 1::4]), (z[:, 0::4], z[:, 2::4]), (z[:-1], z[1:])]:
        r = np.corrcoef(a.ravel(), b.ravel())[0, 1]
        assert abs(r) < 5 / np.sqrt(a.size)


def test_gaussian_depends_on_seed_row_and_target():
    a = th.gaussian_z(np.arange(8), 16, seed=1)
    b = th.gaussian_z(np.arange(8), 16, seed=2)
    c = th.gaussian_z(np.arange(1, 9), 16, seed=1)
    assert not np.any(a == b)
    assert np.array_equal(a[1:], c[:-1])       # columns are addressed by global row
    assert len(np.unique(a)) == a.size
    big = th.gaussian_z(np.array([2**32 + 5, 5], dtype=np.uint64), 16, seed=1)
    assert not np.any(big[0] == big[1])        # the high word of the row index counts


def test_rademacher_bits_by_pure_python():
    """Entry t of column r is bit t % 128 of the 128-bit output of Philox call
    (r, t // 128): checked bit by bit with integer arithmetic in plain Python."""
    from oracle.philox import philox4x32_10, split_seed
    seed, k = 0x0123456789ABCDEF, 260
    rows = [0, 7, 2**32 + 3]
    B = th.rademacher_b(np.array(rows, dtype=np.uint64), k, seed)
    k0, k1 = split_seed(seed)
    for i, r in enumerate(rows):
        for q in range((k + 127) // 128):
            w = philox4x32_10(np.uint32(r & 0xFFFFFFFF), np.uint32(r >> 32), np.uint32(q),
                              np.uint32(th.TAG_RADEMACHER), k0, k1)
            big = sum(int(x) << (32 * e) for e, x in enumerate(w))
            for b in range(128):
                t = 128 * q + b
                if t < k:
                    assert B[i, t] == (-1 if (big >> b) & 1 else 1)


def test_rademacher_entries_distribution():
    """Section 1.3: i.i.d. +-1/sqrt(k), each sign with probability 1/2."""
    B = th.rademacher_b(np.arange(4096), 256, seed=0x5EED).astype(np.float64)
    assert set(np.unique(B)) == {-1.0, 1.0}
    n = B.size
    assert abs(B.mean()) < 5 / np.sqrt(n)
    # neighbouring bits, bits of different words and calls, neighbouring columns
    for a, b in [(B[:, :-1], B[:, 1:]), (B[:, :224], B[:, 32:]), (B[:, :128], B[:, 128:]),
                 (B[:-1], B[1:])]:
        assert abs(np.mean(a * b)) < 5 / np.sqrt(a.size)
    # every target row is balanced over the columns
    col = B.mean(axis=0)
    assert np.max(np.abs(col)) < 5 / np.sqrt(B.shape[0])
    a = th.rademacher_b(np.arange(8), 128, seed=1)
    b = th.rademacher_b(np.arange(8), 128, seed=2)
    c = th.rademacher_b(np.arange(1, 9), 128, seed=1)
    assert np.mean(a == b) < 0.6
    assert np.array_equal(a[1:], c[:-1])
    T = th.Sketch("rademacher", 64, seed=3).dense(100)
    assert np.allclose(np.abs(T), 1 / 8.0, rtol=0, atol=0)


@pytest.mark.parametrize("N", [1, 2, 16, 1024])
def test_fwht_equals_scipy_hadamard(N):
    """The butterfly transform against scipy's Sylvester-construction
    Hadamard matrix (an independent implementation of H)."""
    import scipy.linalg as sla
    X = np.random.default_rng(N).integers(-50, 50, size=(N, 3)).astype(np.float64)
    assert np.array_equal(th.fwht(X), sla.hadamard(N) @ X)


def test_srht_signs_and_samples_by_pure_python():
    """d_r is bit r % 128 of the call (r // 128, 0, 0) and s_j the top L bits of
    word j % 4 of the call (j // 4, 0, 1): checked with plain integer code."""
    from oracle.philox import philox4x32_10, split_seed
    seed = 0xFEEDFACE12345
    k0, k1 = split_seed(seed)
    tag = np.uint32(th.TAG_SRHT)
    rows = [0, 1, 127, 128, 5000, 2**32 + 77, 2**35 + 3]
    d = th.srht_signs(np.array(rows, dtype=np.uint64), seed)
    for r, dr in zip(rows, d):
        q = r >> 7
        w = philox4x32_10(np.uint32(q & 0xFFFFFFFF), np.uint32(q >> 32), np.uint32(0), tag, k0, k1)
        big = sum(int(x) << (32 * e) for e, x in enumerate(w))
        assert dr == (-1.0 if (big >> (r & 127)) & 1 else 1.0)
    for L in (1, 10, 20, 32):
        s = th.srht_samples(9, L, seed)
        for j in range(9):
            w = philox4x32_10(np.uint32(j >> 2), np.uint32(0), np.uint32(1), tag, k0, k1)
            assert int(s[j]) == int(w[j & 3]) >> (32 - L)


def test_srht_distribution_and_unbiasedness():
    """Signs balanced, samples uniform on [0, 2^L); E[Theta^T Theta] = I
    (Monte Carlo over seeds; exact expectation of the definition)."""
    d = th.srht_signs(np.arange(200_000), seed=3)
    assert abs(d.mean()) < 5 / np.sqrt(d.size)
    s = th.srht_samples(100_000, 6, seed=4)
    counts = np.bincount(s.astype(np.int64), minlength=64)
    chi = ((counts - counts.mean())**2 / counts.mean()).sum()
    assert st.chi2.sf(chi, 63) > 1e-4
    n, k, reps = 6, 4, 3000
    acc = np.zeros((n, n))
    for rep in range(reps):
        T = th.Sketch("srht", k, seed=1000 + rep).dense(n)
        acc += T.T @ T
    acc /= reps
    # each entry of Theta^T Theta is a mean of k products of +-1/k; its
    # standard deviation over seeds is <= 1/sqrt(k)
    assert np.max(np.abs(acc - np.eye(n))) < 5 / np.sqrt(k * reps)
    T = th.Sketch("srht", 64, seed=3).dense(100)
    assert np.allclose(np.abs(T), 1 / 8.0, rtol=0, atol=0)


def test_srht_zero_padding_and_explicit_size():
    """Zero padding: the sketch of n rows with transform size 2^L equals the
    same rows embedded in any larger power of two only if L is the same; a
    given L (zeta) fixes Theta for every row range."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((3000, 4))
    S = th.Sketch("srht", 64, seed=9, zeta=13)
    whole = S.apply(X)
    parts = S.apply(X[:1234], row0=0) + S.apply(X[1234:], row0=1234)
    assert np.allclose(parts, whole, rtol=0, atol=1e-12 * np.abs(X).sum())
    T = S.dense(3000)
    assert np.allclose(T @ X, whole, rtol=0, atol=1e-12 * np.abs(X).sum())


def test_sparse_sign_structure():
    n, k, zeta = 20000, 1024, 8
    idx, sgn = th.sparse_sign_entries(np.arange(n), k, zeta, seed=99)
    L = k // zeta
    # exactly one nonzero in each segment of L rows
    seg = idx // L
    assert np.array_equal(seg, np.broadcast_to(np.arange(zeta), seg.shape))
    assert len(np.unique(idx[0])) == zeta
    # rows within a segment are uniform (chi-square) and signs are balanced
    counts = np.bincount((idx % L).ravel(), minlength=L)
    chi = ((counts - counts.mean())**2 / counts.mean()).sum()
    assert st.chi2.sf(chi, L - 1) > 1e-4
    assert abs((sgn == 1).mean() - 0.5) < 5 * 0.5 / np.sqrt(sgn.size)
    # unit column norms of Theta (zeta entries of magnitude 1/sqrt(zeta))
    T = th.Sketch("sparse", 64, seed=3).dense(500)
    assert np.allclose((T**2).sum(axis=0), 1.0, rtol=0, atol=1e-15)
    assert np.all((T != 0).sum(axis=0) == 8)


@pytest.mark.parametrize("kind", ["gaussian", "sparse", "rademacher", "srht"])
def test_apply_matches_dense(kind):
    n, k, c = 3000, 64, 5
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, c))
    # (the SRHT transform size is fixed explicitly so row ranges share Theta)
    S = th.Sketch(kind, k, seed=11, chunk_rows=700, zeta=12 if kind == "srht" else None)
    T = S.dense(n)
    got = S.apply(X)
    assert np.allclose(got, T @ X, rtol=0, atol=1e-12 * np.abs(T) .sum(axis=1).max() * np.abs(X).max())
    # a row offset addresses the global columns of Theta
    got2 = S.apply(X[1000:2000], row0=1000)
    assert np.allclose(got2, T[:, 1000:2000] @ X[1000:2000], rtol=0, atol=1e-11)


def test_frobenius_norm_of_theta():
    """Corollary on ||Theta||_F: E||Theta||_F^2 = n for every operator (exact for
    the sparse sign, the Rademacher matrix and the SRHT)."""
    n = 4000
    Tg = th.Sketch("gaussian", 128, seed=5).dense(n)
    fro2 = (Tg**2).sum()
    assert abs(fro2 - n) < 5 * np.sqrt(2 * n)      # chi-square(kn)/k
    Ts = th.Sketch("sparse", 128, seed=5).dense(n)
    assert abs((Ts**2).sum() - n) < 1e-9
    Tr = th.Sketch("rademacher", 128, seed=5).dense(n)
    assert abs((Tr**2).sum() - n) < 1e-9
    Th = th.Sketch("srht", 128, seed=5).dense(n)
    assert abs((Th**2).sum() - n) < 1e-9


@pytest.mark.parametrize("kind", ["gaussian", "sparse", "rademacher", "srht"])
def test_subspace_embedding_distortion(kind):
    """For a fixed d-dimensional subspace and k = 8d the singular values of
    Theta U (U orthonormal) lie in a band of width about sqrt(d/k) around 1, as
    for an epsilon-embedding with epsilon ~ 2 sqrt(d/k) + d/k."""
    n, d, k = 20000, 16, 128
    rng = np.random.default_rng(6)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    s = np.linalg.svd(th.Sketch(kind, k, seed=7).apply(U), compute_uv=False)
    eps = np.max(np.abs(s**2 - 1))
    assert eps < 2.5 * np.sqrt(d / k) + d / k
