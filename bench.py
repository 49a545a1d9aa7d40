#!/usr/bin/env python3
"""Benchmark of RBGS QR on one MI355X.

Workload (the large single-QR case): W is n = 10^6 x m = 256 with
w_ij = sin(10 (mu_j x_i + 1)) / (cos(100 mu_j x_i - 100 mu_j) + 1.1), block
width p = 16, sketch dimension k = 1024.  One step is one complete RBGS QR
(all blocks: sketches, least squares, update, QR of the sketch, substitution,
re-sketch) with W already resident in HBM.

The headline form stores W and Q in FP32 (step 3 runs on FP64 matrix cores
from the FP32 data, rounding only its result to FP32; all small factors and
sketch accumulation are FP64) with the sparse-sign sketch and the
low-synchronization variant.  The FP64 form and the Gaussian-sketch forms
are timed on the same matrix and reported beside it, each with its accuracy
(||W - QR||_F / ||W||_F, cond2(Q), Delta, Delta~).

`value` is algorithmic HBM throughput in GB/s: n s m ((N-1)/2 + 2) bytes per
QR (N = m/p blocks, s = bytes per element; each block reads Q_(1:i-1) and W_(i)
once and writes Q_(i) once) divided by the measured time per QR.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RBGS QR time & HBM GB/s at n=1e6 m=256: FP32/BF16x3 vs FP64 at equal error"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix-core peak
LS_ITERS = 4   # Richardson sweeps of the least-squares step


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "update_kernel_hbm_traffic_n1e6_m256_p16_k1024_f32.md")
# the update kernel's source: its launcher file and the header with its device bodies
UPDATE_SRC = [os.path.join(ROOT, "paper_2111_14641_amd", "csrc", f)
              for f in ("update_kernels.hip", "update_device.h")]


def measured_traffic(n, m, p, k):
    """HBM bytes per update launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None if it covers another workload or an older kernel source."""
    if (n, m, p, k) != (1_000_000, 256, 16, 1024):
        return None
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(b"".join(open(f, "rb").read() for f in UPDATE_SRC)).hexdigest()
    except OSError:
        return None
    mt = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    mh = re.search(r"source_sha256 \([^)]*\):\s*([0-9a-f]{64})", text)
    if not mt or not mh or mh.group(1) != src:
        return None
    return int(mt.group(1))


def alg_bytes(n, m, p, s):
    N = -(-m // p)
    # sum over blocks of (K + 2 bw) n s with K = i*p
    tot = 0
    for c0 in range(0, m, p):
        bw = min(p, m - c0)
        tot += (c0 + 2 * bw) * n * s
    return float(tot)


def accuracy(W, Q, R, cert):
    import torch
    Wd = W.double()
    Qd = Q.double()
    E = Wd - Qd @ R
    err = (torch.linalg.norm(E) / torch.linalg.norm(Wd)).item()
    G = (Qd.t() @ Qd).cpu().numpy()
    import numpy as np
    ev = np.linalg.eigvalsh(G)
    cond = float(np.sqrt(ev[-1] / ev[0])) if ev[0] > 0 else float("inf")
    return dict(rel_err=err, cond2_Q=cond, delta=cert["delta"], delta_tilde=cert["delta_tilde"])


def accuracy_chunked(W, Q, R, cert, chunk=1 << 20):
    """As `accuracy`, with the FP64 products formed over row chunks (for
    matrices whose FP64 copies would be large)."""
    import numpy as np
    import torch
    n, m = W.shape
    num = torch.zeros((), dtype=torch.float64, device=W.device)
    den = torch.zeros((), dtype=torch.float64, device=W.device)
    G = torch.zeros((m, m), dtype=torch.float64, device=W.device)
    for r0 in range(0, n, chunk):
        Wc = W[r0:r0 + chunk].double()
        Qc = Q[r0:r0 + chunk].double()
        num += ((Wc - Qc @ R) ** 2).sum()
        den += (Wc ** 2).sum()
        G += Qc.t() @ Qc
    ev = np.linalg.eigvalsh(G.cpu().numpy())
    cond = float(np.sqrt(ev[-1] / ev[0])) if ev[0] > 0 else float("inf")
    return dict(rel_err=float(torch.sqrt(num / den)), cond2_Q=cond, delta=cert["delta"],
                delta_tilde=cert["delta_tilde"])


def time_form(W, p, kind, k, seed, variant, steps, warmup, profile_update=False, math="f64",
              profile_sketch=False, chunked_metrics=False, keep_R=False, ls_iters=LS_ITERS):
    """Times `steps` QRs on a dedicated stream.  With profile_update, a second
    timed region of `steps` QRs follows in which HIP events bracket every
    update launch on its stream (the roofline figure); the events themselves
    add a few microseconds around each launch, so the step time is taken from
    the first region.  With profile_sketch (dense operators), events bracket
    every sketch launch in a further region and the sketch's matrix-core rate
    is reported: 2 k n c flops per launch over c sketched columns, against the
    FP64 dense matrix-core peak."""
    import torch
    from paper_2111_14641_amd import binding as B
    n, m = W.shape
    Q = B.colmajor(n, m, W.dtype, W.device)
    R = B.colmajor(m, m, torch.float64, W.device)
    run = lambda **kw: B.rbgs_qr(W, p, kind, k, seed, None, variant, ls_iters, Q=Q, R=R, math=math,
                                 **kw)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # accuracy run (with certificate) outside the timed region
        _, _, _, cert = run(want_cert=True)
        acc = (accuracy_chunked if chunked_metrics else accuracy)(W, Q, R, cert)
        R_acc = R.clone() if keep_R else None
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(steps):
            run()
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        upd = None
        if profile_update:
            B.profile_enable(True, classes=["update"])
            t0.record(stream)
            for _ in range(steps):
                run()
            t1.record(stream)
            torch.cuda.synchronize()
            upd = B.profile_get("update") + (t0.elapsed_time(t1) / steps,)
            B.profile_enable(False)
        sk = {}
        if profile_sketch:
            B.profile_enable(True, classes=["sketch"])
            for _ in range(steps):
                run()
            torch.cuda.synchronize()
            sk_ms, sk_cnt, sk_bytes = B.profile_get("sketch")
            B.profile_enable(False)
            es = 4 if W.dtype == torch.float32 else 8
            tflops = 2.0 * k * (sk_bytes / es) / (sk_ms * 1e-3) / 1e12 if sk_ms > 0 else 0.0
            sk = dict(sketch_ms_per_step=sk_ms / steps, sketch_launches_per_step=sk_cnt // steps,
                      sketch_TFLOPs=tflops, sketch_mfma_frac=tflops / FP64_MFMA_PEAK_TFLOPS)
    s = 4 if W.dtype == torch.float32 else 8
    gbs = alg_bytes(n, m, p, s) / (ms * 1e-3) / 1e9
    res = dict(ms=ms, alg_GBps=gbs, **acc, **sk)
    if keep_R:
        res["_R"] = R_acc
    return res, upd


def post_form(W, p, kind, k, seed, reps=3):
    """Cholesky-QR post-processing of the headline factorization: ms per call
    (HIP events on the call's stream) and the l2 orthogonality of Q before
    and after."""
    import torch
    from paper_2111_14641_amd import binding as B
    n, m = W.shape
    Q0 = B.colmajor(n, m, W.dtype, W.device)
    R0 = B.colmajor(m, m, torch.float64, W.device)
    B.rbgs_qr(W, p, kind, k, seed, None, "lowsync", LS_ITERS, Q=Q0, R=R0)
    Q = B.colmajor(n, m, W.dtype, W.device)
    R = B.colmajor(m, m, torch.float64, W.device)
    torch.cuda.synchronize()

    def orth(X):
        Xd = X.double()
        return float(torch.linalg.matrix_norm(torch.eye(m, dtype=torch.float64, device=X.device)
                                              - Xd.t() @ Xd))
    before = orth(Q0)
    stream = torch.cuda.Stream()
    times = []
    with torch.cuda.stream(stream):
        for _ in range(reps + 1):
            Q.copy_(Q0)
            R.copy_(R0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            B.cholqr_post(Q, R, check=False)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
    after = orth(Q)
    err = float(torch.linalg.matrix_norm(W.double() - Q.double() @ R) / torch.linalg.matrix_norm(W.double()))
    return dict(ms=sorted(times[1:])[len(times[1:]) // 2], orth_before=before, orth_after=after,
                rel_err_after=err)


def kernel_breakdown(W, p, kind, k, seed, variant, reps=2, math="f64"):
    """Per-class kernel milliseconds per QR (events around every launch; run
    after the timed region because the events themselves cost time)."""
    import torch
    from paper_2111_14641_amd import binding as B
    n, m = W.shape
    Q = B.colmajor(n, m, W.dtype, W.device)
    R = B.colmajor(m, m, torch.float64, W.device)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B.rbgs_qr(W, p, kind, k, seed, None, variant, LS_ITERS, Q=Q, R=R, math=math)
        torch.cuda.synchronize()
        B.profile_enable(True)
        for _ in range(reps):
            B.rbgs_qr(W, p, kind, k, seed, None, variant, LS_ITERS, Q=Q, R=R, math=math)
        torch.cuda.synchronize()
        out = {name: round(B.profile_get(name)[0] / reps, 4)
               for name in ("update", "sketch", "reduce", "small", "trsm")}
        B.profile_enable(False)
    return out


def targets(roofline, speedup, forms):
    """The workload's targets beside what this run measured (met or missed)."""
    out = {"update_hbm_frac": dict(target=0.70, measured=roofline["frac"],
                                   met=roofline["frac"] >= 0.70)}
    if speedup is not None:
        out["f32_storage_speedup_vs_f64"] = dict(target=2.0, measured=round(speedup, 3),
                                                 met=speedup >= 2.0)
    g = forms.get("gmres_convdiff_1024_f32basis")
    if g is not None:
        out["gmres_relres"] = dict(target=1e-8, measured=g["relres"], met=bool(g["converged"]))
    b = forms.get("batched_512_f32")
    if b is not None:
        out["batched_persistent_vs_lockstep_graph"] = dict(
            target=1.0, measured=b["persistent_speedup_vs_graph"],
            met=b["persistent_speedup_vs_graph"] > 1.0)
    return out


def batched_form(count=512, reps=3):
    """The batched workload: `count` FP32 problems of uneven n and m, tuned p
    and k: the lock-step groups replayed as one graph per batch, the same QRs
    in one persistent launch (a device queue of the problems' stages), and the
    same QRs launched one by one.  Aggregate algorithmic GB/s over all
    problems."""
    import numpy as np
    import torch
    from paper_2111_14641_amd import binding as B
    from paper_2111_14641_amd.workloads import batched_problems
    probs = batched_problems(count)
    Ws = [w for w, _, _, _ in probs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t = time.perf_counter()
        Qs, Rs, ps, ks = B.rbgs_qr_batched(Ws, seed=0x2111146414, graph=True)  # tune, run, record
        torch.cuda.synchronize()
        first_s = time.perf_counter() - t
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            B.rbgs_qr_batched(Ws, ps, ks, seed=0x2111146414, Qs=Qs, Rs=Rs, graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / reps
        # the same factorizations, one rbgs_qr call after another
        Q1 = [B.colmajor(W.shape[0], W.shape[1], torch.float32) for W in Ws]
        R1 = [B.colmajor(W.shape[1], W.shape[1], torch.float64) for W in Ws]
        e0.record(stream)
        for i, W in enumerate(Ws):
            B.rbgs_qr(W, ps[i], "sparse", ks[i], 0x2111146414 + i, 8, "lowsync", LS_ITERS,
                      Q=Q1[i], R=R1[i])
        e1.record(stream)
        torch.cuda.synchronize()
        ms_single = e0.elapsed_time(e1)
    del Q1, R1
    # the same factorizations in one persistent launch (device queue of stages),
    # recorded as a graph by the first call; each call waits for the device
    Qp = [B.colmajor(W.shape[0], W.shape[1], torch.float32) for W in Ws]
    Rp = [B.colmajor(W.shape[1], W.shape[1], torch.float64) for W in Ws]
    with torch.cuda.stream(stream):
        B.rbgs_qr_batched(Ws, ps, ks, seed=0x2111146414, Qs=Qp, Rs=Rp, graph=True, persistent=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            B.rbgs_qr_batched(Ws, ps, ks, seed=0x2111146414, Qs=Qp, Rs=Rp, graph=True,
                              persistent=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_pers = e0.elapsed_time(e1) / reps
    tot = sum(alg_bytes(W.shape[0], W.shape[1], ps[i], 4) for i, W in enumerate(Ws))

    def metrics(Qs_, Rs_):
        errs, conds = [], []
        for W, Q, R in zip(Ws, Qs_, Rs_):
            Wd, Qd = W.double(), Q.double()
            errs.append((torch.linalg.norm(Wd - Qd @ R) / torch.linalg.norm(Wd)).item())
            ev = np.linalg.eigvalsh((Qd.t() @ Qd).cpu().numpy())
            conds.append(float(np.sqrt(ev[-1] / ev[0])))
        return float(f"{max(errs):.3g}"), float(f"{max(conds):.4g}")

    err_l, cond_l = metrics(Qs, Rs)
    err_p, cond_p = metrics(Qp, Rp)
    # persistent vs lock-step R (the sketches' partial sums are grouped differently)
    dR = max((torch.linalg.norm(R1 - R0) / torch.linalg.norm(R0)).item() for R0, R1 in zip(Rs, Rp))
    return dict(problems=count, alg_GB=round(tot / 1e9, 3), ms_graph=round(ms_graph, 3),
                GBps_graph=round(tot / (ms_graph * 1e-3) / 1e9, 1),
                ms_persistent=round(ms_pers, 3), GBps_persistent=round(tot / (ms_pers * 1e-3) / 1e9, 1),
                persistent_speedup_vs_graph=round(ms_graph / ms_pers, 3),
                ms_one_by_one=round(ms_single, 3),
                GBps_one_by_one=round(tot / (ms_single * 1e-3) / 1e9, 1),
                speedup=round(ms_single / ms_graph, 3), first_call_s=round(first_s, 3),
                max_rel_err=err_l, max_cond2_Q=cond_l, max_rel_err_persistent=err_p,
                max_cond2_Q_persistent=cond_p, max_rel_dR_persistent_vs_lockstep=float(f"{dR:.3g}"),
                p_used=sorted(set(ps)), k_over_m=sorted(set(round(k / W.shape[1], 2)
                                                          for k, W in zip(ks, Ws))))


def mixed_form(steps, warmup, maths=("f64", "f32", "bf16x3")):
    """The mixed-precision workload: W is n = 4e6 x m = 512, cond 1e10
    (U diag(logspace(0, -10, 512)) V^T), p = 32, k = 2048, sparse sign,
    low-sync; FP32 storage with each product arithmetic in `maths` against
    FP64 storage.  Each form reports ms per QR, algorithmic GB/s,
    ||W - QR||_F / ||W||_F against its stored input, cond2(Q), Delta,
    Delta~ and ||R - R_64||_F / ||R_64||_F against the FP64 form's R."""
    import torch
    from paper_2111_14641_amd.workloads import mixed_single_qr_gpu, THETA_SEED_MIXED
    p, k = 32, 2048
    W64, W32 = mixed_single_qr_gpu(dtypes=("float64", "float32"))
    torch.cuda.synchronize()
    out = {}
    print("[bench] mixed workload: fp64", file=sys.stderr, flush=True)
    f64, _ = time_form(W64, p, "sparse", k, THETA_SEED_MIXED, "lowsync", steps, warmup,
                       chunked_metrics=True, keep_R=True)
    f64["kernel_ms_per_step"] = kernel_breakdown(W64, p, "sparse", k, THETA_SEED_MIXED, "lowsync")
    del W64
    R64 = f64.pop("_R")
    for mth in maths:
        print(f"[bench] mixed workload: fp32 storage, {mth} arithmetic", file=sys.stderr, flush=True)
        f, _ = time_form(W32, p, "sparse", k, THETA_SEED_MIXED, "lowsync", steps, warmup,
                         math=mth, chunked_metrics=True, keep_R=True)
        R = f.pop("_R")
        f["rel_diff_R_vs_f64"] = float(torch.linalg.matrix_norm(R - R64) / torch.linalg.matrix_norm(R64))
        f["speedup_vs_f64"] = f64["ms"] / f["ms"]
        f["kernel_ms_per_step"] = kernel_breakdown(W32, p, "sparse", k, THETA_SEED_MIXED, "lowsync",
                                                   math=mth)
        out[f"mixed_f32_{mth}math"] = f
    out["mixed_f64"] = f64
    return out


def gmres_form(N=1024, bs=8, blocks=40, k=1280, max_cycles=60, tol=1e-8):
    """Restarted randomized block GMRES on the N x N convection-diffusion
    operator (n = N^2, FP64 CSR), bs Gaussian right-hand sides, `blocks` blocks
    per cycle (basis m = blocks bs), sparse-sign sketch with k rows, FP32 basis,
    FP64 Hessenberg least squares; plus the CSR SpMM rate."""
    import torch
    from paper_2111_14641_amd import binding as B
    from paper_2111_14641_amd.workloads import convection_diffusion_csr, gmres_rhs
    indptr, indices, data = convection_diffusion_csr(N)
    A = B.CSR(indptr, indices, data)
    n = N * N
    Bh = gmres_rhs(n, bs)
    Bt = B.colmajor(n, bs, torch.float64)
    Bt.copy_(torch.from_numpy(Bh))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        X32 = B.colmajor(n, bs, torch.float32)
        X32.copy_(Bt)
        B.spmm(A, X32)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            B.spmm(A, X32)
        e1.record(stream)
        torch.cuda.synchronize()
        spmm_us = e0.elapsed_time(e1) / 20 * 1e3
        spmm_bytes = 8 * (n + 1) + 12 * len(data) + 2 * 4 * n * bs  # CSR + X once + Y
        t = time.perf_counter()
        X, iters, rel, hist, ok = B.block_gmres(A, Bt, None, blocks, max_cycles, tol, kind="sparse",
                                                k=k, seed=0x2111146413, store="f32")
        torch.cuda.synchronize()
        secs = time.perf_counter() - t
    return dict(n=n, nnz=len(data), bs=bs, blocks_per_cycle=blocks, k=k, converged=bool(ok),
                cycles=len(hist) - (0 if ok else 1), block_iters=iters, relres=float(f"{rel:.3g}"),
                seconds=round(secs, 3), ms_per_block_iter=round(secs * 1e3 / max(iters, 1), 4),
                history_head=[float(f"{v:.3g}") for v in hist[:4]],
                history_tail=[float(f"{v:.3g}") for v in hist[-3:]],
                spmm_us=round(spmm_us, 2), spmm_GBps=round(spmm_bytes / (spmm_us * 1e-6) / 1e9, 1))


def copy_bandwidth():
    """Measured rate of a plain streaming kernel, y = x + 1 over 1 GiB of FP32
    (1 GiB read + 1 GiB written): a practical ceiling beside the nominal
    8 TB/s, and the known-size dispatch that calibrates the FETCH_SIZE /
    WRITE_SIZE counters."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, 1.0, out=b)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(10):
        torch.add(a, 1.0, out=b)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 10
    del a, b
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def cpu_baseline(W64_host, p, k, seed, target_s=15.0):
    """The FP64 oracle timed on a row sample of the same workload (sparse sign,
    low-sync), scaled to GB/s with the same algorithmic byte count (FP64)."""
    import numpy as np
    import oracle.rbgs as orb
    from oracle.theta import Sketch
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    n_full, m = W64_host.shape
    n_s = 62_500
    while True:
        Ws = np.asfortranarray(W64_host[:n_s])
        th = Sketch("sparse", k, seed=seed).materialize(n_s)
        t = time.perf_counter()
        orb.rbgs(Ws, p, th, "lowsync", "householder")
        dt = time.perf_counter() - t
        if dt * 2 > target_s or n_s * 2 > n_full:
            break
        n_s *= 2
    gbs = alg_bytes(n_s, m, p, 8) / dt / 1e9
    return dict(value=gbs, unit="GB/s", cores=int(threads), kind="oracle",
                blas_threads=int(threads), host_cpus=os.cpu_count(),
                sample=f"FP64 oracle, low-sync sparse-sign RBGS on the first {n_s} rows of the "
                       f"workload (m={m}, p={p}, k={k}); one run, {dt:.2f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=256)
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--k", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gaussian", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--forms", default="all",
                    choices=["all", "headline", "srht", "batched", "gaussian", "mixed"],
                    help="'headline': only the headline form; 'srht' / 'batched' / 'mixed': the "
                         "headline and that form; 'gaussian': the headline and the FP32 Gaussian "
                         "and Rademacher forms (for profiling one form)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2111_14641_amd import binding as B
    from paper_2111_14641_amd.workloads import large_single_qr, THETA_SEED_LARGE

    torch.cuda.set_device(0)
    n, m, p, k = args.n, args.m, args.p, args.k
    print(f"[bench] generating W {n}x{m}", file=sys.stderr, flush=True)
    W64h = large_single_qr(n=n, m=m)
    W64 = B.colmajor(n, m, torch.float64)
    W64.copy_(torch.from_numpy(W64h))
    W32 = B.colmajor(n, m, torch.float32)
    W32.copy_(W64)
    torch.cuda.synchronize()

    forms = {}
    print("[bench] fp32 sparse lowsync (headline)", file=sys.stderr, flush=True)
    head, upd = time_form(W32, p, "sparse", k, THETA_SEED_LARGE, "lowsync", args.steps,
                          args.warmup, profile_update=True)
    forms["f32_sparse_lowsync"] = head
    print("[bench] kernel breakdown", file=sys.stderr, flush=True)
    kernel_ms = kernel_breakdown(W32, p, "sparse", k, THETA_SEED_LARGE, "lowsync")
    if args.forms == "gaussian":
        print("[bench] gaussian sketch", file=sys.stderr, flush=True)
        forms["f32_gauss_lowsync"], _ = time_form(W32, p, "gaussian", k, THETA_SEED_LARGE,
                                                  "lowsync", max(2, args.steps // 10), 1,
                                                  profile_sketch=True)
        forms["f32_rademacher_lowsync"], _ = time_form(W32, p, "rademacher", k, THETA_SEED_LARGE,
                                                       "lowsync", max(2, args.steps // 10), 1,
                                                       profile_sketch=True)
    if args.forms == "all":
        print("[bench] fp64 sparse lowsync", file=sys.stderr, flush=True)
        forms["f64_sparse_lowsync"], _ = time_form(W64, p, "sparse", k, THETA_SEED_LARGE, "lowsync",
                                                   args.steps, args.warmup)
        print("[bench] fp32 storage with fp32 arithmetic", file=sys.stderr, flush=True)
        forms["f32_f32math_sparse_lowsync"], _ = time_form(W32, p, "sparse", k, THETA_SEED_LARGE,
                                                           "lowsync", args.steps, args.warmup,
                                                           math="f32")
        print("[bench] fp32 storage with bf16x3 products", file=sys.stderr, flush=True)
        forms["f32_bf16x3math_sparse_lowsync"], _ = time_form(W32, p, "sparse", k, THETA_SEED_LARGE,
                                                              "lowsync", args.steps, args.warmup,
                                                              math="bf16x3")
        print("[bench] fp32/fp64 sparse plain", file=sys.stderr, flush=True)
        forms["f32_sparse_plain"], _ = time_form(W32, p, "sparse", k, THETA_SEED_LARGE, "plain",
                                                 max(3, args.steps // 4), 1)
        forms["f64_sparse_plain"], _ = time_form(W64, p, "sparse", k, THETA_SEED_LARGE, "plain",
                                                 max(3, args.steps // 4), 1)
        print("[bench] Cholesky-QR post-processing", file=sys.stderr, flush=True)
        forms["post_cholqr_f32"] = post_form(W32, p, "sparse", k, THETA_SEED_LARGE)
        print("[bench] two-pass inter-block forms", file=sys.stderr, flush=True)
        forms["f32_sparse_twice"], _ = time_form(W32, p, "sparse", k, THETA_SEED_LARGE, "twice",
                                                 max(3, args.steps // 4), 1)
        forms["f32_sparse_l2qr"], _ = time_form(W32, p, "sparse", k, THETA_SEED_LARGE, "l2qr",
                                                max(3, args.steps // 4), 1)
        # the direct (Householder) least squares in place of the sweeps
        forms["f32_sparse_lowsync_householder_ls"], _ = time_form(
            W32, p, "sparse", k, THETA_SEED_LARGE, "lowsync", max(3, args.steps // 4), 1, ls_iters=0)
        if not args.no_gaussian:
            print("[bench] gaussian forms", file=sys.stderr, flush=True)
            forms["f32_gauss_lowsync"], _ = time_form(W32, p, "gaussian", k, THETA_SEED_LARGE,
                                                      "lowsync", max(2, args.steps // 10), 1,
                                                      profile_sketch=True)
            forms["f64_gauss_lowsync"], _ = time_form(W64, p, "gaussian", k, THETA_SEED_LARGE,
                                                      "lowsync", max(2, args.steps // 10), 1,
                                                      profile_sketch=True)
            forms["f32_rademacher_lowsync"], _ = time_form(W32, p, "rademacher", k,
                                                           THETA_SEED_LARGE, "lowsync",
                                                           max(2, args.steps // 10), 1,
                                                           profile_sketch=True)
    if args.forms in ("all", "srht"):
        print("[bench] SRHT sketch", file=sys.stderr, flush=True)
        forms["f32_srht_lowsync"], _ = time_form(W32, p, "srht", k, THETA_SEED_LARGE, "lowsync",
                                                 max(3, args.steps // 4), 1)
        forms["f64_srht_lowsync"], _ = time_form(W64, p, "srht", k, THETA_SEED_LARGE, "lowsync",
                                                 max(3, args.steps // 4), 1)
    del W64
    if args.forms in ("all", "mixed") and not args.no_mixed:
        forms.update(mixed_form(max(3, args.steps // 4), 1))
    if args.forms in ("all", "batched") and not args.no_batched:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        forms["batched_512_f32"] = batched_form()
    if args.forms == "all" and not args.no_gmres:
        print("[bench] block GMRES", file=sys.stderr, flush=True)
        forms["gmres_convdiff_1024_f32basis"] = gmres_form()
    copy_gbs = copy_bandwidth()
    upd_ms, upd_cnt, upd_bytes, upd_step_ms = upd
    achieved = upd_bytes / (upd_ms * 1e-3) / 1e9 if upd_ms > 0 else 0.0
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(n, m, p, k),
                    traffic_unit="bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    alg_bytes_per_launch=round(upd_bytes / max(upd_cnt, 1)),
                    kernel="update_p_kernel<float> / update_fused_kernel<float> (persistent; "
                           "step 3 + substitution, low-sync; in the fused launches the first "
                           "workgroup also factors the sketch of the block)",
                    launches=upd_cnt, avg_launch_us=round(upd_ms / max(upd_cnt, 1) * 1e3, 2),
                    share_of_step=round(upd_ms / args.steps / upd_step_ms, 3),
                    events_region_ms_per_step=round(upd_step_ms, 4),
                    copy_GBps=round(copy_gbs, 1), frac_of_copy=round(achieved / copy_gbs, 4))
    speedup = None
    if "f64_sparse_lowsync" in forms:
        speedup = forms["f64_sparse_lowsync"]["ms"] / head["ms"]
    out = {
        "metric": METRIC,
        "value": round(head["alg_GBps"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"oscillatory W n={n} m={m}, p={p}, k={k}, sparse-sign zeta=8, "
                               "low-sync RBGS, FP32 storage with FP64 arithmetic",
                   "n": n, "m": m, "p": p, "k": k, "parallelism": "single GPU"},
        "speedup_f32_vs_f64": None if speedup is None else round(speedup, 3),
        "forms": {name: {kk: (float(f"{v:.4g}") if isinstance(v, float) else v)
                         for kk, v in f.items()}
                  for name, f in forms.items()},
        "kernel_ms_per_step": kernel_ms,
        "roofline": roofline,
        "targets": targets(roofline, speedup, forms),
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W64h, p, k, THETA_SEED_LARGE)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
