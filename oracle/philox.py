"""Philox-4xW-R counter-based random number generator (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, Section 4): the state is a counter of four W-bit words
(c0, c1, c2, c3) and a key of two W-bit words (k0, k1).  One round maps

    (c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),
                         hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

where hi/lo are the upper and lower W bits of the 2W-bit product.  Between
rounds the key is bumped by the Weyl constants: k0 += W0, k1 += W1 (mod 2^W).
Philox-4xW-R applies R rounds (the first with the unbumped key).

Two instances are provided:
  * 4x32-10: the generator the sketching operators use (both the oracle and
    the GPU library implement it independently from this definition).
  * 4x64-10: the same construction with 64-bit words; it exists so the
    shared round/key-schedule structure can be pinned against NumPy's
    independent Philox implementation (numpy.random.Philox), which is
    Philox-4x64-10.

Parity: pinned (tests/test_oracle_philox.py) -- the 4x64 instance must
reproduce numpy.random.Philox bit for bit; the 4x32 instance, which differs
only in word size and constants, is checked by statistical tests (bit
balance, avalanche) since no reference output for it is available here.
"""
import numpy as np

# Multipliers and Weyl increments from the Philox paper (Section 4 / Table 2).
PHILOX4x32 = dict(bits=32, M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85)
PHILOX4x64 = dict(bits=64, M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
                  W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B)

_MASK32 = np.uint64(0xFFFFFFFF)


def _mulhilo32(a, m):
    """(hi, lo) 32-bit halves of a*m for uint32 arrays a and a constant m."""
    p = a.astype(np.uint64) * np.uint64(m)
    return (p >> np.uint64(32)).astype(np.uint32), (p & _MASK32).astype(np.uint32)


def _mulhilo64(a, m):
    """(hi, lo) 64-bit halves of a*m for uint64 arrays a and a constant m,
    computed from 32-bit partial products (numpy has no 128-bit integers)."""
    a = a.astype(np.uint64)
    s32 = np.uint64(32)
    a_lo, a_hi = a & _MASK32, a >> s32
    m_lo, m_hi = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    ll = a_lo * m_lo
    hl = a_hi * m_lo
    lh = a_lo * m_hi
    hh = a_hi * m_hi
    cross = (ll >> s32) + (hl & _MASK32) + lh          # < 2^64, no wrap
    hi = hh + (hl >> s32) + (cross >> s32)
    lo = (cross << s32) | (ll & _MASK32)
    return hi, lo


def philox(counter, key, spec=PHILOX4x32, rounds=10):
    """Apply Philox-4xW-`rounds` to a batch of counters.

    counter: sequence of four integer arrays (broadcastable) -- words c0..c3.
    key:     sequence of two integers or arrays -- words k0, k1.
    Returns a tuple of four arrays (uint32 for W=32, uint64 for W=64).
    """
    bits = spec["bits"]
    dt = np.uint32 if bits == 32 else np.uint64
    mulhilo = _mulhilo32 if bits == 32 else _mulhilo64
    c = [np.asarray(x).astype(dt) for x in counter]
    shape = np.broadcast_shapes(*[x.shape for x in c])
    c = [np.broadcast_to(x, shape).copy() for x in c]
    k0 = np.asarray(key[0]).astype(dt)
    k1 = np.asarray(key[1]).astype(dt)
    w0, w1 = dt(spec["W0"]), dt(spec["W1"])
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + w0).astype(dt)
                k1 = (k1 + w1).astype(dt)
            hi0, lo0 = mulhilo(c[0], spec["M0"])
            hi1, lo1 = mulhilo(c[2], spec["M1"])
            c = [(hi1 ^ c[1] ^ k0).astype(dt), lo1.astype(dt),
                 (hi0 ^ c[3] ^ k1).astype(dt), lo0.astype(dt)]
    return tuple(c)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox-4x32-10 on counter (c0..c3) and key (k0, k1); uint32 outputs."""
    return philox((c0, c1, c2, c3), (k0, k1), PHILOX4x32, 10)


def split_seed(seed):
    """Key words of a 64-bit seed: (low 32 bits, high 32 bits)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.uint32(seed & 0xFFFFFFFF), np.uint32(seed >> 32)
