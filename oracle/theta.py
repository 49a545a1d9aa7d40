"""Sketching operators Theta (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper (Section 1.3, random sketching) requires Theta in R^{k x n} to be an
epsilon-embedding of the subspaces of interest and notes that a seeded random
number generator lets Theta be applied without being stored.  The paper itself
reports results for SRHT and Rademacher matrices; this build uses a Gaussian
operator and a sparse-sign operator whose entries are *defined* from
Philox-4x32-10 output as follows (each side -- this oracle and the GPU
library -- implements the definition independently).

Common: key = (seed mod 2^32, seed >> 32).  Column r of Theta corresponds to
row r of the sketched matrix (the global row index, 0 <= r < n).

Gaussian, Theta = c_k * Z with c_k = fl64(1 / sqrt(k)) and Z an fp32 matrix:
  for target group j (0 <= j < k/4) and column r, the counter
  (r mod 2^32, r >> 32, j, 0x47415553) gives words (x0, x1, x2, x3); the pair
  (x0, x1) gives Z[4j, r], Z[4j+1, r] and the pair (x2, x3) gives
  Z[4j+2, r], Z[4j+3, r] through the Box-Muller transform (Box & Muller 1958)
  evaluated with single-precision IEEE operations (+, -, *, /, sqrt, each
  correctly rounded, no fused multiply-add) in the exact order of
  `box_muller_f32` below.  Requires k % 4 == 0.

Sparse sign (block CountSketch), Theta = c_z * B with c_z = fl64(1/sqrt(zeta)):
  the counters (r mod 2^32, r >> 32, c, 0x53504152) for c = 0, 1 give eight
  words w_0..w_7; for segment s < zeta (zeta <= 8, k % zeta == 0, L = k/zeta)
  column r of B has the entry sign_s at row
        s*L + (((w_s >> 1) * L) >> 31),   sign_s = -1 if w_s & 1 else +1,
  so every column has exactly zeta nonzeros, one per segment of L rows.

Rademacher, Theta = c_k * B with c_k = fl64(1 / sqrt(k)) (Section 1.3: i.i.d.
  entries +-1/sqrt(k) with probability 1/2 each): the counter
  (r mod 2^32, r >> 32, q, 0x52414445) gives 128 bits x0 | x1 << 32 |
  x2 << 64 | x3 << 96; entry B[t, r] for t = 128 q + b is -1 if bit b is set,
  +1 otherwise.  Requires k % 4 == 0.

SRHT (Section 1.3: random signs, Walsh-Hadamard matrix, uniform row sampling,
  scale 1/sqrt(k), zero padding to a power of two), Theta = c_k * P H D with
  c_k = fl64(1 / sqrt(k)), for a transform size N = 2^L >= n:
    D = diag(d_r): d_r = -1 if bit (r mod 128) of the 128-bit output of the
        counter (q mod 2^32, q >> 32, 0, 0x53524854), q = r >> 7, is set
        (bits numbered as for the Rademacher operator);
    H[s, r] = (-1)^popcount(s & r) (Sylvester's construction);
    P selects rows s_0 .. s_{k-1}: s_j = word (j mod 4) of the counter
        (j >> 2, 0, 1, 0x53524854), shifted right by 32 - L (its top L bits),
        i.e. uniform on [0, N) and drawn with replacement.
  L is given (`zeta`) or, if 0, the smallest L with 2^L >= the row count.

Identity: Theta = I (requires k == n).  RBGS with Theta = I is block
Gram-Schmidt with exact least-squares projections (Section 2), which the tests
use to pin the oracle against Householder QR.

Sketches are always formed as c * (Z @ X) (or c * (B @ X)) in FP64.

Parity: pinned (tests/test_oracle_theta.py): the fp32 logarithm and sine /
cosine polynomials against numpy's FP64 functions to a few fp32 ulps, the
Gaussian samples against the normal distribution (moments, Kolmogorov-Smirnov),
the Rademacher entries against their distribution (values +-1, sign balance,
pairwise independence of targets and of columns), the sparse-sign columns
against their defining invariants (exactly zeta
distinct rows, one per segment, unit column norm, uniform row distribution),
and the blocked application against explicit dense products.
"""
import numpy as np
import scipy.sparse as sp

from .philox import philox4x32_10, split_seed

TAG_GAUSS = 0x47415553
TAG_SPARSE = 0x53504152
TAG_RADEMACHER = 0x52414445
TAG_SRHT = 0x53524854

F32 = np.float32


def _c(bits):
    """fp32 constant from its IEEE bit pattern."""
    return np.array([bits], dtype=np.uint32).view(np.float32)[0]


# fp32 constants (correctly rounded values of the named reals).
SQRT2 = _c(0x3FB504F3)      # sqrt(2)
LN2 = _c(0x3F317218)        # ln 2
HALF_PI = _c(0x3FC90FDB)    # pi / 2
INV3, INV5, INV7, INV9 = _c(0x3EAAAAAB), _c(0x3E4CCCCD), _c(0x3E124925), _c(0x3DE38E39)
# Taylor coefficients (-1)^j / (2j+1)! and (-1)^j / (2j)!
S3, S5, S7, S9, S11, S13 = (_c(0xBE2AAAAB), _c(0x3C088889), _c(0xB9500D01),
                            _c(0x3638EF1D), _c(0xB2D7322B), _c(0x2F309231))
C2, C4, C6, C8, C10, C12, C14 = (_c(0xBF000000), _c(0x3D2AAAAB), _c(0xBAB60B61),
                                 _c(0x37D00D01), _c(0xB493F27E), _c(0x310F76C7),
                                 _c(0xAD49CBA5))
TWO_M24 = F32(2.0 ** -24)


def ln_u24(word):
    """fp32 approximation of ln(u), u = (2*(word >> 9) + 1) * 2^-24 in (0, 1).

    ln(u) = (e - 24) ln 2 + ln f, where N = 2*(word>>9)+1 = f * 2^e with f in
    [sqrt2/2, sqrt2]; ln f = 2 atanh(s), s = (f-1)/(f+1), by its odd series up
    to s^9.  Every operation is a single correctly rounded fp32 operation.
    """
    N = (word.astype(np.uint32) >> np.uint32(9)) * np.uint32(2) + np.uint32(1)
    mant, ex = np.frexp(N.astype(np.float32))     # N = mant * 2^ex, mant in [0.5, 1)
    f = (mant * F32(2.0)).astype(np.float32)      # exact
    e = (ex - 1).astype(np.int32)
    big = f > SQRT2
    f = np.where(big, f * F32(0.5), f).astype(np.float32)   # exact
    e = np.where(big, e + 1, e)
    s = ((f - F32(1.0)) / (f + F32(1.0))).astype(np.float32)
    s2 = (s * s).astype(np.float32)
    p = (INV7 + s2 * INV9).astype(np.float32)
    p = (INV5 + s2 * p).astype(np.float32)
    p = (INV3 + s2 * p).astype(np.float32)
    t = (F32(2.0) * s).astype(np.float32)
    lnf = (t + t * (s2 * p)).astype(np.float32)
    return ((e - 24).astype(np.float32) * LN2 + lnf).astype(np.float32)


def sincos_quarter(word):
    """fp32 (cos(phi), sin(phi)) with phi = 2*pi*(q + t)/4 for the quadrant
    q = word >> 30 and t = (2*((word >> 7) & 0x7FFFFF) + 1) * 2^-24 in (0, 1).

    a = t * (pi/2); sin a and cos a by Taylor polynomials (to a^13 and a^14),
    Horner form; the quadrant turns (cos a, sin a) by q quarter turns.
    """
    w = word.astype(np.uint32)
    q = (w >> np.uint32(30)).astype(np.int32)
    v = (w >> np.uint32(7)) & np.uint32(0x7FFFFF)
    t = ((v * np.uint32(2) + np.uint32(1)).astype(np.float32) * TWO_M24).astype(np.float32)
    a = (t * HALF_PI).astype(np.float32)
    a2 = (a * a).astype(np.float32)
    ps = (S11 + a2 * S13).astype(np.float32)
    ps = (S9 + a2 * ps).astype(np.float32)
    ps = (S7 + a2 * ps).astype(np.float32)
    ps = (S5 + a2 * ps).astype(np.float32)
    ps = (S3 + a2 * ps).astype(np.float32)
    sin_a = (a + (a * a2) * ps).astype(np.float32)
    pc = (C12 + a2 * C14).astype(np.float32)
    pc = (C10 + a2 * pc).astype(np.float32)
    pc = (C8 + a2 * pc).astype(np.float32)
    pc = (C6 + a2 * pc).astype(np.float32)
    pc = (C4 + a2 * pc).astype(np.float32)
    pc = (C2 + a2 * pc).astype(np.float32)
    cos_a = (F32(1.0) + a2 * pc).astype(np.float32)
    c = np.select([q == 0, q == 1, q == 2], [cos_a, -sin_a, -cos_a], sin_a).astype(np.float32)
    s = np.select([q == 0, q == 1, q == 2], [sin_a, cos_a, -sin_a], -cos_a).astype(np.float32)
    return c, s


def box_muller_f32(wr, wa):
    """Two fp32 standard normals from two words: radius word wr, angle word wa.

    z0 = rho * cos(phi), z1 = rho * sin(phi), rho = sqrt(-2 ln u).
    """
    rho = np.sqrt((F32(-2.0) * ln_u24(wr)).astype(np.float32)).astype(np.float32)
    c, s = sincos_quarter(wa)
    return (rho * c).astype(np.float32), (rho * s).astype(np.float32)


def gaussian_z(rows, k, seed):
    """Unscaled Gaussian entries Z[:, rows] as an fp32 array of shape
    (len(rows), k): out[i, t] = Z[t, rows[i]]."""
    if k % 4:
        raise ValueError("Gaussian sketch needs k % 4 == 0")
    rows = np.asarray(rows, dtype=np.uint64)
    k0, k1 = split_seed(seed)
    j = np.arange(k // 4, dtype=np.uint32)
    r_lo = (rows & np.uint64(0xFFFFFFFF)).astype(np.uint32)[:, None]
    r_hi = (rows >> np.uint64(32)).astype(np.uint32)[:, None]
    x0, x1, x2, x3 = philox4x32_10(r_lo, r_hi, j[None, :], np.uint32(TAG_GAUSS), k0, k1)
    z = np.empty((rows.shape[0], k), dtype=np.float32)
    z[:, 0::4], z[:, 1::4] = box_muller_f32(x0, x1)
    z[:, 2::4], z[:, 3::4] = box_muller_f32(x2, x3)
    return z


def rademacher_b(rows, k, seed):
    """Unscaled Rademacher entries B[:, rows] as an int8 array of shape
    (len(rows), k) with values +-1: out[i, t] = B[t, rows[i]]."""
    if k % 4:
        raise ValueError("Rademacher sketch needs k % 4 == 0")
    rows = np.asarray(rows, dtype=np.uint64)
    k0, k1 = split_seed(seed)
    nq = (k + 127) // 128
    q = np.arange(nq, dtype=np.uint32)
    r_lo = (rows & np.uint64(0xFFFFFFFF)).astype(np.uint32)[:, None]
    r_hi = (rows >> np.uint64(32)).astype(np.uint32)[:, None]
    words = philox4x32_10(r_lo, r_hi, q[None, :], np.uint32(TAG_RADEMACHER), k0, k1)
    # bits[i, q, w, b] = bit b of word w of call q; target t = 128 q + 32 w + b
    W = np.stack(words, axis=2)                                       # (len, nq, 4)
    bits = (W[..., None] >> np.arange(32, dtype=np.uint32)) & np.uint32(1)
    bits = bits.reshape(rows.shape[0], nq * 128)[:, :k]
    return np.where(bits == 1, -1, 1).astype(np.int8)


def _bits128(q, tag, c2, seed):
    """Bits of the 128-bit Philox outputs for counters (q lo, q hi, c2, tag):
    array (len(q), 128) of 0/1, bit b of word w at position 32 w + b."""
    q = np.asarray(q, dtype=np.uint64)
    k0, k1 = split_seed(seed)
    words = philox4x32_10((q & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                          (q >> np.uint64(32)).astype(np.uint32),
                          np.uint32(c2), np.uint32(tag), k0, k1)
    W = np.stack(words, axis=-1)                                      # (len, 4)
    return ((W[..., None] >> np.arange(32, dtype=np.uint32)) & np.uint32(1)).reshape(q.shape[0], 128)


def srht_signs(rows, seed):
    """d_r for the global rows `rows` (+1 / -1 as float64)."""
    rows = np.asarray(rows, dtype=np.uint64)
    if rows.size == 0:
        return np.zeros(0)
    q = rows >> np.uint64(7)
    uq, inv = np.unique(q, return_inverse=True)
    bits = _bits128(uq, TAG_SRHT, 0, seed)[inv, (rows & np.uint64(127)).astype(np.int64)]
    return np.where(bits == 1, -1.0, 1.0)


def srht_samples(k, L, seed):
    """Sampled rows s_0 .. s_{k-1} of the 2^L-point transform (uint64)."""
    k0, k1 = split_seed(seed)
    j = np.arange(k, dtype=np.uint64)
    words = philox4x32_10((j >> np.uint64(2)).astype(np.uint32), np.uint32(0), np.uint32(1),
                          np.uint32(TAG_SRHT), k0, k1)
    w = np.stack(words, axis=-1)[np.arange(k), (j & np.uint64(3)).astype(np.int64)].astype(np.uint64)
    return (w >> np.uint64(32 - L)) if L > 0 else np.zeros(k, dtype=np.uint64)


def fwht(A):
    """Unnormalized Walsh-Hadamard transform H A along axis 0 (length a power
    of two), H[s, r] = (-1)^popcount(s & r): log2(N) butterfly stages, stage h
    combining rows i and i + h of every block of 2h rows into their sum and
    difference."""
    A = np.array(A, dtype=np.float64, copy=True)
    N = A.shape[0]
    if N & (N - 1):
        raise ValueError("length must be a power of two")
    h = 1
    while h < N:
        B = A.reshape(N // (2 * h), 2, h, *A.shape[1:])
        top = B[:, 0] + B[:, 1]
        bot = B[:, 0] - B[:, 1]
        B[:, 0], B[:, 1] = top, bot
        A = B.reshape(A.shape)
        h *= 2
    return A


def ceil_log2(n):
    L = 0
    while (1 << L) < n:
        L += 1
    return L


def sparse_sign_entries(rows, k, zeta, seed):
    """Row indices (uint32, shape (len(rows), zeta)) and signs (+1/-1 int8) of
    the nonzeros of the unscaled sparse-sign columns B[:, rows]."""
    if not (1 <= zeta <= 8) or k % zeta:
        raise ValueError("sparse-sign sketch needs 1 <= zeta <= 8 and k % zeta == 0")
    rows = np.asarray(rows, dtype=np.uint64)
    k0, k1 = split_seed(seed)
    r_lo = (rows & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    r_hi = (rows >> np.uint64(32)).astype(np.uint32)
    a = philox4x32_10(r_lo, r_hi, np.uint32(0), np.uint32(TAG_SPARSE), k0, k1)
    b = philox4x32_10(r_lo, r_hi, np.uint32(1), np.uint32(TAG_SPARSE), k0, k1)
    words = np.stack(list(a) + list(b), axis=1)[:, :zeta]          # (len, zeta)
    L = np.uint64(k // zeta)
    seg = np.arange(zeta, dtype=np.uint64)[None, :]
    idx = seg * L + (((words.astype(np.uint64) >> np.uint64(1)) * L) >> np.uint64(31))
    sign = np.where(words & np.uint32(1), -1, 1).astype(np.int8)
    return idx.astype(np.uint32), sign


class Sketch:
    """A sketching operator Theta in R^{k x n} defined by (kind, k, seed, zeta).

    kind: "gaussian", "sparse", "rademacher", "srht" or "identity".  For
    "srht", `zeta` is log2 of the transform size (0: the smallest power of two
    covering the rows of the call).
    """

    def __init__(self, kind, k, seed=0, zeta=None, chunk_rows=8192):
        if zeta is None:
            zeta = 0 if kind == "srht" else 8
        self.kind, self.k, self.seed, self.zeta = kind, int(k), int(seed), int(zeta)
        self.chunk_rows = chunk_rows
        if kind in ("gaussian", "rademacher", "srht"):
            self.scale = 1.0 / np.sqrt(float(self.k))
        elif kind == "sparse":
            self.scale = 1.0 / np.sqrt(float(self.zeta))
        elif kind == "identity":
            self.scale = 1.0
        else:
            raise ValueError(kind)
        self._dense = None
        self._csr = None
        self._csr_n = 0

    def srht_L(self, rows):
        return self.zeta if self.zeta > 0 else ceil_log2(rows)

    def _srht_apply(self, X, row0):
        """c_k (H D X_pad)[s, :], X_pad holding X at rows row0 .. of N = 2^L."""
        n_loc, c = X.shape
        L = self.srht_L(row0 + n_loc)
        N = 1 << L
        if row0 + n_loc > N:
            raise ValueError("rows beyond the SRHT transform size")
        Xp = np.zeros((N, c))
        Xp[row0:row0 + n_loc] = srht_signs(np.arange(row0, row0 + n_loc), self.seed)[:, None] * X
        Y = fwht(Xp)
        return self.scale * Y[srht_samples(self.k, L, self.seed).astype(np.int64)]

    def materialize(self, n):
        """Form Theta explicitly once and apply it by a product from then on:
        a dense k x n FP64 matrix, or for the sparse sign a compressed sparse
        row matrix of the unscaled +-1 entries (so large n stays cheap)."""
        if self.kind == "srht":
            return self       # applied by the fast transform every time
        if self.kind == "sparse":
            idx, sign = sparse_sign_entries(np.arange(n), self.k, self.zeta, self.seed)
            cols = np.repeat(np.arange(n), self.zeta)
            self._csr = sp.csr_matrix((sign.ravel().astype(np.float64),
                                       (idx.ravel().astype(np.int64), cols)), shape=(self.k, n))
            self._csr_n = n
        else:
            self._dense = self.dense(n)
        return self

    # -- explicit form -------------------------------------------------
    def dense(self, n):
        """Explicit Theta (k x n, FP64).  Only for small n."""
        if self.kind == "identity":
            if n != self.k:
                raise ValueError("identity sketch needs k == n")
            return np.eye(n)
        if self.kind == "gaussian":
            return self.scale * gaussian_z(np.arange(n), self.k, self.seed).T.astype(np.float64)
        if self.kind == "rademacher":
            return self.scale * rademacher_b(np.arange(n), self.k, self.seed).T.astype(np.float64)
        if self.kind == "srht":
            # columns of Theta are the transforms of the unit vectors
            L = self.srht_L(n)
            H = fwht(np.eye(1 << L)[:, :n])
            return self.scale * H[srht_samples(self.k, L, self.seed).astype(np.int64)] * \
                srht_signs(np.arange(n), self.seed)[None, :]
        idx, sign = sparse_sign_entries(np.arange(n), self.k, self.zeta, self.seed)
        T = np.zeros((self.k, n))
        cols = np.repeat(np.arange(n), self.zeta)
        T[idx.ravel(), cols] = sign.ravel()
        return self.scale * T

    def unscaled_dense(self, n):
        """Z (fp32 values) or B (+-1) or I, as FP64, k x n."""
        return self.dense(n) / self.scale

    # -- application ---------------------------------------------------
    def apply(self, X, row0=0):
        """Theta[:, row0:row0+X.shape[0]] @ X in FP64 (k x X.shape[1])."""
        X = np.asarray(X, dtype=np.float64)
        if X.ndim == 1:
            return self.apply(X[:, None], row0)[:, 0]
        n_loc, c = X.shape
        if self._dense is not None:
            return self._dense[:, row0:row0 + n_loc] @ X
        if self._csr is not None and row0 == 0 and n_loc == self._csr_n:
            return self.scale * (self._csr @ X)
        if self.kind == "identity":
            if row0 != 0 or n_loc != self.k:
                raise ValueError("identity sketch needs k == n")
            return X.copy()
        if self.kind == "srht":
            return self._srht_apply(X, row0)
        if self.kind == "sparse":
            idx, sign = sparse_sign_entries(np.arange(row0, row0 + n_loc), self.k,
                                            self.zeta, self.seed)
            cols = np.repeat(np.arange(n_loc), self.zeta)
            B = sp.csr_matrix((sign.ravel().astype(np.float64),
                               (idx.ravel().astype(np.int64), cols)), shape=(self.k, n_loc))
            return self.scale * (B @ X)
        out = np.zeros((self.k, c))
        for r0 in range(0, n_loc, self.chunk_rows):
            r1 = min(n_loc, r0 + self.chunk_rows)
            rows = np.arange(row0 + r0, row0 + r1)
            if self.kind == "rademacher":
                Z = rademacher_b(rows, self.k, self.seed)
            else:
                Z = gaussian_z(rows, self.k, self.seed)
            out += Z.T.astype(np.float64) @ X[r0:r1]
        return self.scale * out

    def __call__(self, X, row0=0):
        return self.apply(X, row0)
