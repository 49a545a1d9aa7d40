"""Pins of the oracle's Philox implementation (CPU only)."""
import numpy as np
import pytest

from oracle import philox as ph


def test_mulhilo32_matches_python_integers():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**32, size=5000, dtype=np.uint64).astype(np.uint32)
    for m in (ph.PHILOX4x32["M0"], ph.PHILOX4x32["M1"]):
        hi, lo = ph._mulhilo32(a, m)
        for ai, h, l in zip(a[:500], hi[:500], lo[:500]):
            p = int(ai) * m
            assert int(h) == p >> 32 and int(l) == p & 0xFFFFFFFF


def test_mulhilo64_matches_python_integers():
    rng = np.random.default_rng(2)
    a = rng.integers(0, 2**64, size=2000, dtype=np.uint64)
    a[:4] = [0, 1, 2**64 - 1, 2**63]
    for m in (ph.PHILOX4x64["M0"], ph.PHILOX4x64["M1"]):
        hi, lo = ph._mulhilo64(a, m)
        for ai, h, l in zip(a, hi, lo):
            p = int(ai) * m
            assert int(h) == p >> 64 and int(l) == p & (2**64 - 1)


@pytest.mark.parametrize("key", [(0, 0), (1, 2), (0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF)])
@pytest.mark.parametrize("ctr", [(1, 0, 0, 0), (2**64 - 1, 5, 7, 2**63), (12345, 0, 99, 1)])
def test_philox4x64_matches_numpy(key, ctr):
    """The shared round and key-schedule structure, instantiated with 64-bit
    words, must reproduce NumPy's independent Philox-4x64-10.  NumPy increments
    its counter before each block, so it is started one below `ctr`."""
    c = np.array(ctr, dtype=np.uint64)
    start = c.copy()
    # decrement with borrow
    for w in range(4):
        if start[w] > 0:
            start[w] -= np.uint64(1)
            break
        start[w] = np.uint64(2**64 - 1)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    expect = bg.random_raw(4)
    got = ph.philox(tuple(np.array([x], dtype=np.uint64) for x in ctr),
                    (np.uint64(key[0]), np.uint64(key[1])), ph.PHILOX4x64, 10)
    assert [int(g[0]) for g in got] == [int(e) for e in expect]


def test_philox4x32_bit_balance_and_avalanche():
    n = 1 << 16
    r = np.arange(n, dtype=np.uint32)
    out = np.stack(ph.philox4x32_10(r, 0, 7, 0x47415553, 0x12345678, 0x9ABCDEF0), axis=1)
    bits = np.unpackbits(out.view(np.uint8)).reshape(n, 128)
    freq = bits.mean(axis=0)
    # every output bit is 1 with probability 1/2 (5 sigma band)
    assert np.all(np.abs(freq - 0.5) < 5 * 0.5 / np.sqrt(n))
    # flipping one counter bit flips about half of the 128 output bits
    out2 = np.stack(ph.philox4x32_10(r ^ np.uint32(1 << 13), 0, 7, 0x47415553,
                                     0x12345678, 0x9ABCDEF0), axis=1)
    flips = np.unpackbits((out ^ out2).view(np.uint8)).reshape(n, 128).sum(axis=1)
    assert abs(flips.mean() - 64) < 0.2
    # different keys give unrelated streams
    out3 = np.stack(ph.philox4x32_10(r, 0, 7, 0x47415553, 0x12345679, 0x9ABCDEF0), axis=1)
    same = (out == out3).mean()
    assert same < 1e-3


def test_planted_mistake_in_round_is_caught():
    """A plausible slip in the round (swapping the two multipliers) must break
    the NumPy pin."""
    bad = dict(ph.PHILOX4x64)
    bad["M0"], bad["M1"] = bad["M1"], bad["M0"]
    bg = np.random.Philox(key=np.array([1, 2], dtype=np.uint64),
                          counter=np.zeros(4, dtype=np.uint64))
    expect = [int(x) for x in bg.random_raw(4)]
    got = ph.philox((np.array([1], np.uint64), 0, 0, 0), (np.uint64(1), np.uint64(2)), bad, 10)
    assert [int(g[0]) for g in got] != expect
