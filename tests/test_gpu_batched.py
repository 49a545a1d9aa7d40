"""Batched RBGS QR (independent problems of uneven n, m in one call) on the
GPU: each problem against the FP64 oracle, determinism, HIP-graph replay
(identical results, and replays read the current W), and the autotuner's
choices."""
import sys

import numpy as np
import pytest

import oracle.rbgs as orb
import parity_checks as pc
from oracle.metrics import cond2, factorization_error
from oracle.theta import Sketch
from paper_2111_14641_amd.workloads import svd_matrix

pytestmark = pytest.mark.gpu

TOL64 = 4096 * 2.0**-53   # entry-wise, per-entry scales of tests/parity_checks.py

SHAPES = [  # n, m, p, k
    (3000, 32, 16, 96),
    (20000, 48, 8, 128),
    (65537, 64, 32, 256),
    (5000, 20, 16, 64),
    (12000, 64, 16, 160),
    (40000, 40, 32, 120),
]


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def to_np(t):
    return np.ascontiguousarray(t.double().cpu().numpy())


def make_batch(store, decades=2.0, seed0=100):
    import torch
    from paper_2111_14641_amd import binding as B
    dt = torch.float64 if store == "f64" else torch.float32
    Wh, Ws = [], []
    for i, (n, m, p, k) in enumerate(SHAPES):
        W = svd_matrix(n, m, np.logspace(0, -decades, m), seed=seed0 + i)
        if store == "f32":
            W = W.astype(np.float32).astype(np.float64)
        Wt = B.colmajor(n, m, dt)
        Wt.copy_(torch.from_numpy(W))
        Wh.append(W)
        Ws.append(Wt)
    return Wh, Ws


@pytest.mark.parametrize("kind", ["sparse", "gaussian"])
def test_batched_matches_oracle(gpu_lib, kind):
    from paper_2111_14641_amd import binding as B
    say("batched vs oracle", kind)
    Wh, Ws = make_batch("f64")
    ps = [s[2] for s in SHAPES]
    ks = [s[3] for s in SHAPES]
    Qs, Rs, p_used, k_used = B.rbgs_qr_batched(Ws, ps, ks, kind=kind, seed=77, variant="lowsync",
                                               ls_iters=2)
    assert p_used == ps and k_used == ks
    for i, (W, Q, R) in enumerate(zip(Wh, Qs, Rs)):
        n, m, p, k = SHAPES[i]
        th = Sketch(kind, k, seed=77 + i).materialize(n)
        o = orb.rbgs(W, p, th, "lowsync", "richardson", 2)
        Rg, Qg = to_np(R), to_np(Q)
        assert np.linalg.norm(Rg - o["R"]) <= 1e-12 * np.linalg.norm(o["R"]), i
        assert np.linalg.norm(Qg - o["Q"]) <= 1e-11 * np.linalg.norm(o["Q"]), i
        pc.assert_qrs_entrywise(Qg, Rg, None, o, None, TOL64, TOL64)
        assert factorization_error(W, Qg, Rg) < 1e-14


def test_batched_deterministic_and_graph_replay(gpu_lib):
    import torch
    from paper_2111_14641_amd import binding as B
    say("batched graph replay")
    Wh, Ws = make_batch("f32", decades=6.0, seed0=300)
    ps = [s[2] for s in SHAPES]
    ks = [s[3] for s in SHAPES]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Qe, Re, _, _ = B.rbgs_qr_batched(Ws, ps, ks, seed=5)                 # eager
        Qg, Rg, _, _ = B.rbgs_qr_batched(Ws, ps, ks, seed=5, graph=True)     # eager + record
        snap = [(to_np(Q), to_np(R)) for Q, R in zip(Qg, Rg)]
        for rep in range(3):
            for Q in Qg:
                Q.zero_()
            B.rbgs_qr_batched(Ws, ps, ks, seed=5, Qs=Qg, Rs=Rg, graph=True)  # graph launch
            torch.cuda.synchronize()
            for (Q, R), (q0, r0), Q1, R1 in zip(zip(Qg, Rg), snap, Qe, Re):
                assert np.array_equal(to_np(Q), q0) and np.array_equal(to_np(R), r0), rep
                assert np.array_equal(to_np(Q1), q0) and np.array_equal(to_np(R1), r0)
        # the graph reads W when it runs: new data, same graph
        for W in Ws:
            W.mul_(2.0)
        B.rbgs_qr_batched(Ws, ps, ks, seed=5, Qs=Qg, Rs=Rg, graph=True)
        Qn, Rn, _, _ = B.rbgs_qr_batched(Ws, ps, ks, seed=5)
        torch.cuda.synchronize()
    for Q, R, Q1, R1 in zip(Qg, Rg, Qn, Rn):
        assert np.array_equal(to_np(Q), to_np(Q1)) and np.array_equal(to_np(R), to_np(R1))
    for (q0, r0), R in zip(snap, Rg):
        assert np.allclose(to_np(R), 2.0 * r0, rtol=1e-12, atol=0)


def test_autotuned_batch_fp32_metrics(gpu_lib):
    """p and k left to the autotuner: its choices are admissible and every
    problem meets the accuracy targets (FP32 storage, cond(W) = 1e6)."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("autotuned batch")
    Wh, Ws = make_batch("f32", decades=6.0, seed0=500)
    Qs, Rs, ps, ks = B.rbgs_qr_batched(Ws, seed=9)
    torch.cuda.synchronize()
    for i, (W, Q, R) in enumerate(zip(Wh, Qs, Rs)):
        n, m = W.shape
        assert ps[i] in ([16, 32] if m >= 32 else [16, m] if m >= 16 else [m]), (i, ps[i])
        assert 2 * m <= ks[i] <= min(n, 4 * m + 32) and ks[i] % 8 == 0, (i, ks[i])
        Qg, Rg = to_np(Q), to_np(R)
        assert factorization_error(W, Qg, Rg) <= 1e-6
        assert cond2(Qg) <= 10
    # cached: the same classes give the same answers
    assert B.autotune(Wh[2].shape[0], Wh[2].shape[1]) == (ps[2], ks[2])


LOCK = [  # n, m, p, k: four lock-step groups (same m, p, k) and one problem on the streams
    (3000, 48, 16, 128), (20001, 48, 16, 128), (1025, 48, 16, 128), (70000, 48, 16, 128),
    (4096, 40, 8, 96), (9999, 40, 8, 96), (2500, 40, 8, 96),
    (6000, 48, 32, 128), (8000, 48, 32, 128),      # 32-wide blocks: Householder tree, 2 x 16 update
    (4000, 40, 16, 1104), (4500, 40, 16, 1104),    # k > 1024: two sketch rows per thread, tree
    (5000, 40, 16, 96),
]


def make_lock_batch(store, decades, seed0):
    import torch
    from paper_2111_14641_amd import binding as B
    dt = torch.float64 if store == "f64" else torch.float32
    Wh, Ws = [], []
    for i, (n, m, p, k) in enumerate(LOCK):
        W = svd_matrix(n, m, np.logspace(0, -decades, m), seed=seed0 + i)
        if store == "f32":
            W = W.astype(np.float32).astype(np.float64)
        Wt = B.colmajor(n, m, dt)
        Wt.copy_(torch.from_numpy(W))
        Wh.append(W)
        Ws.append(Wt)
    return Wh, Ws


@pytest.mark.parametrize("store,ls", [("f64", 2), ("f64", 4), ("f64", 1), ("f32", 4)])
def test_lockstep_groups_match_oracle(gpu_lib, store, ls):
    """Problems that share m, p and k run block by block together (one launch
    per kernel and step for the group); each must equal the oracle's RBGS of
    its own W with its own sketch, as the problems run on the streams do.
    Ragged row counts (1025, 20001, 9999) cover partial plan and update tiles."""
    from paper_2111_14641_amd import binding as B
    say("lock-step batch", store, ls)
    decades = 2.0
    Wh, Ws = make_lock_batch(store, decades, 700)
    ps = [s[2] for s in LOCK]
    ks = [s[3] for s in LOCK]
    Qs, Rs, _, _ = B.rbgs_qr_batched(Ws, ps, ks, kind="sparse", seed=41, variant="lowsync",
                                     ls_iters=ls)
    for i, (W, Q, R) in enumerate(zip(Wh, Qs, Rs)):
        n, m, p, k = LOCK[i]
        th = Sketch("sparse", k, seed=41 + i).materialize(n)
        o = orb.rbgs(W, p, th, "lowsync", "richardson", ls)
        Rg, Qg = to_np(R), to_np(Q)
        assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0), i
        if store == "f64":
            assert np.linalg.norm(Rg - o["R"]) <= 1e-12 * np.linalg.norm(o["R"]), i
            assert np.linalg.norm(Qg - o["Q"]) <= 1e-11 * np.linalg.norm(o["Q"]), i
            pc.assert_qrs_entrywise(Qg, Rg, None, o, None, TOL64, TOL64)
            assert factorization_error(W, Qg, Rg) < 1e-14, i
        else:
            assert np.linalg.norm(Rg - o["R"]) <= 64 * 2.0**-24 * 10**decades * np.linalg.norm(o["R"]), i
            tol32 = 64 * 2.0**-24 * 10**decades
            pc.assert_qrs_entrywise(Qg, Rg, None, o, None, tol32, tol32)
            assert factorization_error(W, Qg, Rg) <= 1e-6, i
            assert cond2(Qg) <= 10, i


def test_lockstep_in_place_and_graph_replay(gpu_lib):
    """Lock-step groups in place (Q = W) and under graph record/replay: the
    replays give the eager result bit for bit."""
    import torch
    from paper_2111_14641_amd import binding as B
    say("lock-step in place and graph")
    Wh, Ws = make_lock_batch("f32", 4.0, 800)
    ps = [s[2] for s in LOCK]
    ks = [s[3] for s in LOCK]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Qe, Re, _, _ = B.rbgs_qr_batched(Ws, ps, ks, seed=3)
        Qg, Rg, _, _ = B.rbgs_qr_batched(Ws, ps, ks, seed=3, graph=True)
        for rep in range(2):
            for Q in Qg:
                Q.zero_()
            B.rbgs_qr_batched(Ws, ps, ks, seed=3, Qs=Qg, Rs=Rg, graph=True)
            torch.cuda.synchronize()
            for Q, R, Q1, R1 in zip(Qg, Rg, Qe, Re):
                assert np.array_equal(to_np(Q), to_np(Q1)) and np.array_equal(to_np(R), to_np(R1)), rep
        Wc = [W.clone() for W in Ws]
        Ri = [torch.zeros_like(R) for R in Re]
        B.rbgs_qr_batched(Wc, ps, ks, seed=3, Qs=Wc, Rs=Ri)
        torch.cuda.synchronize()
    for Q, R, Q1, R1 in zip(Wc, Ri, Qe, Re):
        assert np.array_equal(to_np(Q), to_np(Q1)) and np.array_equal(to_np(R), to_np(R1))
