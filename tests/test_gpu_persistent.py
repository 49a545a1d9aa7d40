"""Persistent batch (rbgs_qr_batched with RBGS_BATCH_PERSISTENT): every
problem the device queue takes runs in one launch.  Each problem against the
FP64 oracle, element by element; run-to-run determinism (the queue's order
changes from run to run, the arithmetic of every stage does not); HIP-graph
record and replay; factorization in place (Q = W); problems the queue does not
take (k > 1024) running beside it on the streams."""
import sys

import numpy as np
import pytest

import oracle.rbgs as orb
import parity_checks as pc
from oracle.metrics import cond2, factorization_error
from oracle.theta import Sketch
from paper_2111_14641_amd.workloads import svd_matrix

pytestmark = pytest.mark.gpu

# n, m, p, k, leading dimension (0: n).  Ragged row counts cover partial plan
# and update tiles; ld = n + 1 sends every tile of that problem down the
# guarded (element-load) path of the update; widths 8, 16 and 32 (17..32: two
# 16-column groups, 512-row update tiles) with narrower last blocks; k from 64
# to 1024 covers the three register shapes of the sketch QR.
SHAPES = [
    (3000, 48, 16, 128, 0),
    (20001, 48, 16, 128, 0),
    (1025, 40, 32, 96, 0),
    (70000, 48, 32, 128, 0),
    (4096, 40, 8, 96, 0),
    (9999, 72, 32, 256, 10000),
    (5000, 64, 16, 520, 5001),
    (4500, 100, 32, 1024, 0),
    (2000, 20, 20, 64, 0),
    (6001, 56, 24, 384, 6003),
]
# with problems the queue does not take (k > 1024: the single-problem path)
STREAM_SHAPES = [(3000, 40, 16, 1104, 0), (4096, 40, 8, 96, 0), (2000, 32, 16, 1040, 0),
                 (8000, 48, 32, 192, 0)]
TOL32 = 64 * 2.0**-24  # entry-wise, times 10**decades, per-entry scales of parity_checks


def random_shapes(seed, count):
    """Seeded random shapes the queue takes: n from 300 (less than one tile)
    to 30000, m from 1 to 120, p from 1 to 32 (not above m), k a multiple of 8
    from m to min(4m, 1024, n), leading dimension n or n + 1..3."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.integers(300, 30001))
        m = int(rng.integers(1, 121))
        if 8 * ((m + 7) // 8) > n:
            continue
        p = int(rng.integers(1, 33))
        p = min(p, m)
        kmin = 8 * ((m + 7) // 8)
        kmax = min(4 * m, 1024, n) // 8 * 8
        k = int(rng.integers(kmin // 8, max(kmin, kmax) // 8 + 1)) * 8
        ld = n + int(rng.integers(0, 4)) * int(rng.integers(0, 2))
        out.append((n, m, p, k, ld))
    return out


RANDOM_SHAPES = random_shapes(2024, 24)


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def to_np(t):
    return np.ascontiguousarray(t.double().cpu().numpy())


def make_batch(shapes, decades, seed0):
    import torch
    from paper_2111_14641_amd import binding as B
    Wh, Ws = [], []
    for i, (n, m, p, k, ld) in enumerate(shapes):
        W = svd_matrix(n, m, np.logspace(0, -decades, m), seed=seed0 + i).astype(np.float32)
        W = W.astype(np.float64)
        Wt = B.colmajor(ld or n, m, torch.float32)[:n]
        Wt.copy_(torch.from_numpy(W))
        Wh.append(W)
        Ws.append(Wt)
    return Wh, Ws


def out_like(shapes):
    import torch
    from paper_2111_14641_amd import binding as B
    Qs = [B.colmajor(ld or n, m, torch.float32)[:n] for n, m, p, k, ld in shapes]
    Rs = [B.colmajor(m, m, torch.float64) for n, m, p, k, ld in shapes]
    return Qs, Rs


def check_oracle(Wh, Qs, Rs, shapes, seed, ls, decades):
    for i, (W, Q, R) in enumerate(zip(Wh, Qs, Rs)):
        n, m, p, k, ld = shapes[i]
        th = Sketch("sparse", k, seed=seed + i).materialize(n)
        o = orb.rbgs(W, p, th, "lowsync", "richardson", ls)
        Rg, Qg = to_np(R), to_np(Q)
        say("problem", i, (n, m, p, k, ld))
        assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0), i
        tol = TOL32 * 10**decades
        assert np.linalg.norm(Rg - o["R"]) <= tol * np.linalg.norm(o["R"]), i
        pc.assert_qrs_entrywise(Qg, Rg, None, o, None, tol, tol)
        assert factorization_error(W, Qg, Rg) <= 1e-6, i
        # cond2(Q) = cond2(Theta U) is the method's (about 6 at k = 2m, more
        # for k nearer m): the GPU's must be the oracle's
        c_or = cond2(o["Q"])
        assert abs(cond2(Qg) - c_or) <= 1e-3 * c_or, i
        if k >= 2 * m:
            assert c_or <= 10, i


@pytest.mark.parametrize("ls", [4, 1, 2])
def test_persistent_matches_oracle(gpu_lib, ls):
    from paper_2111_14641_amd import binding as B
    say("persistent batch vs oracle, ls", ls)
    decades = 2.0
    Wh, Ws = make_batch(SHAPES, decades, 900)
    Qs, Rs = out_like(SHAPES)
    ps = [s[2] for s in SHAPES]
    ks = [s[3] for s in SHAPES]
    B.rbgs_qr_batched(Ws, ps, ks, kind="sparse", seed=61, variant="lowsync", ls_iters=ls,
                      Qs=Qs, Rs=Rs, persistent=True)
    check_oracle(Wh, Qs, Rs, SHAPES, 61, ls, decades)


def test_persistent_deterministic_graph_and_in_place(gpu_lib):
    """Two eager runs and three graph replays give the same bits; a graph
    replay reads the current W; in place (Q = W) gives the same bits."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("persistent determinism, graph, in place")
    Wh, Ws = make_batch(SHAPES, 4.0, 950)
    ps = [s[2] for s in SHAPES]
    ks = [s[3] for s in SHAPES]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Qa, Ra = out_like(SHAPES)
        B.rbgs_qr_batched(Ws, ps, ks, seed=8, Qs=Qa, Rs=Ra, persistent=True)
        ref = [(to_np(Q), to_np(R)) for Q, R in zip(Qa, Ra)]
        Qb, Rb = out_like(SHAPES)
        B.rbgs_qr_batched(Ws, ps, ks, seed=8, Qs=Qb, Rs=Rb, persistent=True)
        for (Q, R), (q0, r0) in zip(zip(Qb, Rb), ref):
            assert np.array_equal(to_np(Q), q0) and np.array_equal(to_np(R), r0)
        Qg, Rg = out_like(SHAPES)
        B.rbgs_qr_batched(Ws, ps, ks, seed=8, Qs=Qg, Rs=Rg, graph=True, persistent=True)
        for rep in range(3):
            for Q, R in zip(Qg, Rg):
                Q.zero_()
                R.fill_(7.0)
            B.rbgs_qr_batched(Ws, ps, ks, seed=8, Qs=Qg, Rs=Rg, graph=True, persistent=True)
            torch.cuda.synchronize()
            for (Q, R), (q0, r0) in zip(zip(Qg, Rg), ref):
                assert np.array_equal(to_np(Q), q0) and np.array_equal(to_np(R), r0), rep
        Wc = [W.clone() for W in Ws]
        Ri = [torch.zeros_like(R) for R in Ra]
        B.rbgs_qr_batched(Wc, ps, ks, seed=8, Qs=Wc, Rs=Ri, persistent=True)
        torch.cuda.synchronize()
        for Q, R, (q0, r0) in zip(Wc, Ri, ref):
            assert np.array_equal(to_np(Q), q0) and np.array_equal(to_np(R), r0)
        # new W, same graph
        for W in Ws:
            W.mul_(2.0)
        B.rbgs_qr_batched(Ws, ps, ks, seed=8, Qs=Qg, Rs=Rg, graph=True, persistent=True)
        torch.cuda.synchronize()
    for R, (q0, r0) in zip(Rg, ref):
        assert np.allclose(to_np(R), 2.0 * r0, rtol=1e-6, atol=0)


def test_persistent_with_problems_on_the_streams(gpu_lib):
    """Problems the queue does not take (k > 1024) run on the internal
    streams in the same call; all match the oracle."""
    from paper_2111_14641_amd import binding as B
    say("persistent batch with stream problems")
    shapes = STREAM_SHAPES
    decades = 2.0
    Wh, Ws = make_batch(shapes, decades, 990)
    Qs, Rs = out_like(shapes)
    B.rbgs_qr_batched(Ws, [s[2] for s in shapes], [s[3] for s in shapes], seed=13, ls_iters=4,
                      Qs=Qs, Rs=Rs, persistent=True)
    check_oracle(Wh, Qs, Rs, shapes, 13, 4, decades)


def test_persistent_random_shapes(gpu_lib):
    """24 seeded random shapes (n below one tile, odd leading dimensions,
    widths 1..32 with ragged last blocks, k from m to 1024) in one batch."""
    from paper_2111_14641_amd import binding as B
    say("persistent batch, random shapes")
    decades = 2.0
    Wh, Ws = make_batch(RANDOM_SHAPES, decades, 1300)
    Qs, Rs = out_like(RANDOM_SHAPES)
    B.rbgs_qr_batched(Ws, [s[2] for s in RANDOM_SHAPES], [s[3] for s in RANDOM_SHAPES], seed=29,
                      ls_iters=4, Qs=Qs, Rs=Rs, persistent=True)
    check_oracle(Wh, Qs, Rs, RANDOM_SHAPES, 29, 4, decades)
