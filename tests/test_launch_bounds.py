"""Host-side bounds check of every kernel launch of rbgs_qr (CPU, no GPU).

The library's object files are linked with a recording stand-in for the HIP
runtime (tests/launch_bounds/mock_hip.cpp) and driven through the C ABI
(tests/launch_bounds/driver.cpp), so the real host code chooses every grid,
workspace offset and argument.  tests/launch_bounds/check_launches.py restates
each kernel's index expressions and checks that every global-memory access of
every launch stays inside a live allocation.  The shapes include the full-size
workloads (n = 10^6, m = 256, p = 16, k = 1024 and n = 4 10^6, m = 512,
p = 32, k = 2048) with every sketch, storage and inter-block variant they use,
and the small shapes the GPU parity tests run."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "launch_bounds")
CLANG = "/opt/rocm/llvm/bin/clang++"

GAUSS, SPARSE, RADEM, SRHT = 0, 1, 3, 4
F64, F32 = 0, 1
PLAIN, LOWSYNC, TWICE, L2QR = 0, 1, 2, 3

CASES = [
    # n, m, p, k, kind, store, math, variant, ls, want_S, want_cert
    (4_000_000, 512, 32, 2048, GAUSS, F32, 0, LOWSYNC, 4, 0, 1),
    (4_000_000, 512, 32, 2048, SPARSE, F32, 0, LOWSYNC, 4, 0, 1),
    (4_000_000, 512, 32, 2048, SPARSE, F32, 0, LOWSYNC, 4, 1, 1),
    (4_000_000, 512, 32, 2048, SPARSE, F64, 0, LOWSYNC, 4, 0, 1),
    (4_000_000, 512, 32, 2048, SPARSE, F64, 0, LOWSYNC, 4, 1, 1),
    (4_000_000, 512, 32, 2048, SPARSE, F32, 1, LOWSYNC, 4, 0, 1),
    (4_000_000, 512, 32, 2048, SPARSE, F32, 2, LOWSYNC, 4, 0, 1),
    (1_000_000, 256, 16, 1024, SPARSE, F32, 2, LOWSYNC, 4, 1, 1),
    (10_000, 64, 8, 256, GAUSS, F32, 2, PLAIN, 2, 1, 1),
    (4097, 70, 32, 256, SPARSE, F32, 2, LOWSYNC, 2, 1, 1),
    (4_000_000, 512, 32, 2048, GAUSS, F64, 0, LOWSYNC, 4, 1, 1),
    (1_000_000, 256, 16, 1024, SPARSE, F32, 0, LOWSYNC, 4, 1, 1),
    (1_000_000, 256, 16, 1024, SPARSE, F64, 0, LOWSYNC, 4, 1, 1),
    (1_000_000, 256, 16, 1024, GAUSS, F32, 0, LOWSYNC, 4, 0, 1),
    (1_000_000, 256, 16, 1024, SPARSE, F32, 0, PLAIN, 4, 0, 1),
    (1_000_000, 256, 16, 1024, SRHT, F32, 0, LOWSYNC, 4, 0, 1),
    (10_000, 64, 8, 256, GAUSS, F64, 0, PLAIN, 2, 1, 1),
    (4097, 30, 8, 128, SPARSE, F64, 0, LOWSYNC, 2, 1, 1),
    (3000, 70, 32, 512, SPARSE, F64, 0, LOWSYNC, 2, 1, 1),
    (5000, 96, 32, 256, GAUSS, F64, 0, LOWSYNC, 2, 1, 1),
    (9000, 40, 16, 2048, SPARSE, F64, 0, LOWSYNC, 2, 1, 1),
    (3000, 560, 16, 576, SPARSE, F64, 0, LOWSYNC, 2, 1, 1),
    (6000, 64, 32, 2048, SPARSE, F64, 0, LOWSYNC, 2, 1, 1),
    (5000, 72, 24, 1536, GAUSS, F64, 0, LOWSYNC, 2, 1, 1),
    (8192, 40, 32, 8192, 2, F64, 0, PLAIN, 2, 1, 1),
    (4097, 30, 8, 132, RADEM, F64, 0, LOWSYNC, 2, 1, 1),
    (10_000, 64, 8, 256, GAUSS, F32, 1, PLAIN, 2, 1, 1),
    # Householder least squares (ls_iters = 0)
    (1_000_000, 256, 16, 1024, SPARSE, F32, 0, LOWSYNC, 0, 1, 1),
    (10_000, 64, 8, 256, GAUSS, F64, 0, PLAIN, 0, 1, 1),
    (5000, 96, 32, 512, SPARSE, F64, 0, LOWSYNC, 0, 1, 1),
    (4097, 70, 32, 256, GAUSS, F64, 0, TWICE, 0, 1, 1),
    (3000, 150, 16, 1024, RADEM, F64, 0, LOWSYNC, 0, 0, 0),
]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    objs = sorted(glob.glob(os.path.join(ROOT, "paper_2111_14641_amd", "_build", "*.o")))
    if len(objs) < 6:
        from paper_2111_14641_amd import build
        build.build()
        objs = sorted(glob.glob(os.path.join(ROOT, "paper_2111_14641_amd", "_build", "*.o")))
    out = tmp_path_factory.mktemp("lb")
    flags = ["-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I" + os.path.join(ROOT, "include"), "-w"]
    for src in ("mock_hip.cpp", "driver.cpp"):
        subprocess.run([CLANG, *flags, "-c", os.path.join(HERE, src), "-o",
                        str(out / (src + ".o"))], check=True)
    exe = str(out / "driver")
    subprocess.run([CLANG, "-o", exe, str(out / "mock_hip.cpp.o"), str(out / "driver.cpp.o"), *objs],
                   check=True)
    return exe, out


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(str(v) for v in c[:4]) +
                         f"-kind{c[4]}-store{c[5]}-math{c[6]}-var{c[7]}")
def test_every_launch_stays_in_bounds(driver, case):
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    exe, out = driver
    log = str(out / ("log_" + "_".join(str(v) for v in case) + ".txt"))
    r = subprocess.run([exe, *[str(v) for v in case]], env={**os.environ, "RBGS_LAUNCH_LOG": log},
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    violations, n, seen = cl.check_events(cl.parse_log(log))
    assert n > 0
    assert not violations, "\n".join(violations[:20])


FUSED_CASES = [
    # case as above, then the blocks whose update launch also factors the sketch
    ((20_000, 128, 16, 256, SPARSE, F32, 0, LOWSYNC, 4, 0, 0), [48, 64, 80, 96, 112]),
    ((20_000, 128, 16, 256, SPARSE, F64, 0, LOWSYNC, 0, 0, 0), [48, 64, 80, 96, 112]),
    ((3000, 600, 16, 1024, SPARSE, F64, 0, LOWSYNC, 2, 0, 0), list(range(48, 513, 16))),
    ((20_000, 128, 16, 256, SPARSE, F32, 1, LOWSYNC, 4, 0, 0), []),     # FP32 arithmetic
    ((20_000, 128, 16, 256, SPARSE, F32, 0, PLAIN, 4, 0, 0), []),       # plain variant
    ((20_000, 128, 32, 256, SPARSE, F32, 0, LOWSYNC, 4, 0, 0), []),     # 32-column blocks
    ((20_000, 128, 16, 2048, SPARSE, F32, 0, LOWSYNC, 4, 0, 0), []),    # k > 1024
]


@pytest.mark.parametrize("case,fused_K", FUSED_CASES,
                         ids=lambda c: "x".join(str(v) for v in c[:4]) + "-math%d-var%d" % (c[6], c[7])
                         if isinstance(c, tuple) else None)
def test_fused_update_takes_exactly_the_eligible_blocks(driver, case, fused_K):
    """Host dispatch of the update that also factors the sketch: low-sync, FP64
    arithmetic, 16-column blocks with 48 <= K <= 512 and k <= 1024, and for
    those blocks no separate QR launch; every other block keeps the QR launch
    and the plain update."""
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    exe, out = driver
    log = str(out / ("fused_" + "_".join(str(v) for v in case) + ".txt"))
    r = subprocess.run([exe, *[str(v) for v in case]], env={**os.environ, "RBGS_LAUNCH_LOG": log},
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    launches = [e[1] for e in cl.parse_log(log) if e[0] == "launch"]
    fused = [L for L in launches if cl.kernel_base(L.name) == "update_fused_kernel"]
    assert sorted(L.i(12) for L in fused) == fused_K          # argument 12: K
    n, m, p, k = case[:4]
    blocks = -(-m // p)
    updates = [L for L in launches if cl.kernel_base(L.name) in ("update_p_kernel", "update_kernel")]
    assert len(updates) + len(fused) == blocks
    if case[7] == LOWSYNC:
        qrs = [L for L in launches if cl.kernel_base(L.name) in ("qr_wave_kernel", "qr_fused_kernel")]
        assert len(qrs) == blocks - len(fused)


NOALLOC_CASES = [
    # the no-allocation entry point (two calls, the second on half the rows)
    (1_000_000, 256, 16, 1024, SPARSE, F32, 0, LOWSYNC, 4, 1, 0),
    (10_000, 64, 8, 256, GAUSS, F64, 0, PLAIN, 2, 1, 0),
    (4097, 30, 8, 128, SPARSE, F64, 0, LOWSYNC, 2, 0, 0),
    (5000, 96, 32, 256, GAUSS, F32, 0, LOWSYNC, 2, 1, 0),
]


@pytest.mark.parametrize("case", NOALLOC_CASES, ids=lambda c: "noalloc-" + "x".join(str(v) for v in c[:4]))
def test_noalloc_launches_stay_in_the_scratch_array(driver, case):
    """Every launch of rbgs_qr_noalloc stays inside the caller's arrays and
    the library's scratch array (logged as one allocation of its size), and
    the call allocates nothing else."""
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    exe, out = driver
    log = str(out / ("noalloc_" + "_".join(str(v) for v in case) + ".txt"))
    r = subprocess.run([exe, *[str(v) for v in case], "1"],
                       env={**os.environ, "RBGS_LAUNCH_LOG": log}, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    events = cl.parse_log(log)
    allocs = [e for e in events if e[0] == "alloc"]
    # W, Q, R, (S), then the scratch array on the first call, nothing more
    assert len(allocs) == (5 if case[9] else 4)
    assert allocs[-1][2] == 64 << 20
    violations, n, seen = cl.check_events(events)
    assert n > 0
    assert not violations, "\n".join(violations[:20])


BATCH_CASES = [
    # count, p, k / m, ragged leading dimensions
    (24, 16, 4, 0),
    (24, 32, 2, 1),
    (9, 32, 4, 0),
    (16, 8, 3, 1),
]


@pytest.mark.parametrize("case", BATCH_CASES, ids=lambda c: "batch-%d-p%d-k%d-ld%d" % c)
def test_persistent_batch_launches_stay_in_bounds(driver, case):
    """rbgs_qr_batched with the persistent queue: the descriptors the host
    uploads are read back from the log, and every stage of every problem
    (restated from the kernel) stays inside its arrays; the queue holds
    exactly the stages the problems' chains need."""
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    exe, out = driver
    log = str(out / ("batch_%d_%d_%d_%d.txt" % case))
    r = subprocess.run([exe, "batch", *[str(v) for v in case]],
                       env={**os.environ, "RBGS_LAUNCH_LOG": log},
                       capture_output=True, text=True)
    # no kernel runs here: the host's read-back of the queue's control words
    # (filled with 0xFF bytes by the stand-in) is reported as an error
    assert r.returncode == 0 or "persistent batch:" in r.stdout, r.stdout + r.stderr
    events = cl.parse_log(log)
    names = [cl.kernel_base(e[1].name) for e in events if e[0] == "launch"]
    assert names.count("persistent_batch_kernel") == 1 and names.count("persistent_init_kernel") == 1
    violations, n, seen = cl.check_events(events)
    assert n > 0
    assert not violations, "\n".join(violations[:20])


def test_persistent_batch_gpu_test_shapes_stay_in_bounds(driver):
    """The shapes the GPU tests of the persistent batch run."""
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_gpu_persistent as tp
    exe, out = driver
    for name, shapes in (("oracle", tp.SHAPES), ("streams", tp.STREAM_SHAPES),
                         ("random", tp.RANDOM_SHAPES)):
        spec = ";".join(",".join(str(v) for v in s) for s in shapes)
        log = str(out / ("batchs_%s.txt" % name))
        r = subprocess.run([exe, "batchs", spec], capture_output=True, text=True,
                           env={**os.environ, "RBGS_LAUNCH_LOG": log})
        assert r.returncode == 0 or "persistent batch:" in r.stdout, r.stdout + r.stderr
        events = cl.parse_log(log)
        names = [cl.kernel_base(e[1].name) for e in events if e[0] == "launch"]
        assert names.count("persistent_batch_kernel") == 1, name
        violations, n, seen = cl.check_events(events)
        assert n > 0 and not violations, "\n".join(violations[:20])


def test_persistent_batch_checker_catches_a_short_array(driver):
    """A problem's R one row short (leading dimension m - 1) must be flagged."""
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    exe, out = driver
    log = str(out / "batch_planted.txt")
    subprocess.run([exe, "batch", "9", "32", "4", "0"], capture_output=True,
                   env={**os.environ, "RBGS_LAUNCH_LOG": log})
    events = cl.parse_log(log)
    assert not cl.check_events(events)[0]
    il = next(i for i, e in enumerate(events) if e[0] == "launch" and
              cl.kernel_base(e[1].name) == "persistent_batch_kernel")
    pa = events[il][1].u(0)
    idx = next(i for i, e in enumerate(events) if e[0] == "data" and e[1] == pa)
    raw = bytearray(events[idx][2])
    off = cl.PB_FIELDS.index("ldr")
    # ldr is the 17th 8-byte field; make it one larger for problem 3
    pos = 3 * cl.PB_SIZE + 8 * off
    ldr = int.from_bytes(raw[pos:pos + 8], "little")
    raw[pos:pos + 8] = (ldr + 1).to_bytes(8, "little")
    bad = list(events)
    bad[idx] = ("data", pa, bytes(raw))
    assert any("descriptor" in v for v in cl.check_events(bad)[0])


def test_noalloc_rejects_a_workspace_beyond_the_scratch_array(driver):
    exe, out = driver
    log = str(out / "noalloc_big.txt")
    r = subprocess.run([exe, "4000000", "512", "32", "2048", str(SPARSE), str(F32), "0",
                        str(LOWSYNC), "4", "0", "0", "1"],
                       env={**os.environ, "RBGS_LAUNCH_LOG": log}, capture_output=True, text=True)
    assert r.returncode == 1
    assert "status -2" in r.stdout and "no-allocation entry point has 67108864" in r.stdout
    assert "launch" not in open(log).read()


def test_checker_catches_planted_out_of_bounds(driver):
    """The checker must flag accesses past an allocation: on a recorded
    4e6 x 512 Gaussian factorization, (a) the workspace shortened by one
    element, (b) the last update launch given an output leading dimension one larger,
    (c) one sketch reduction given one partial sum more, (d) a kernel without
    a mirror."""
    import sys
    sys.path.insert(0, HERE)
    import check_launches as cl
    exe, out = driver
    log = str(out / "planted.txt")
    case = CASES[0]
    subprocess.run([exe, *[str(v) for v in case]], env={**os.environ, "RBGS_LAUNCH_LOG": log},
                   check=True, capture_output=True)
    events = cl.parse_log(log)
    assert not cl.check_events(events)[0]

    def first(pred):
        return next(i for i, e in enumerate(events) if pred(e))

    # (a) the largest allocation (the workspace or W) one element shorter
    ia = max((i for i, e in enumerate(events) if e[0] == "alloc"), key=lambda i: events[i][2])
    bad = list(events)
    bad[ia] = ("alloc", events[ia][1], events[ia][2] - 8)
    assert cl.check_events(bad)[0]
    # (b) the last update launch with an output leading dimension one larger
    # (its last block of Q then ends 31 elements past the end of Q)
    iu = max(i for i, e in enumerate(events)
             if e[0] == "launch" and cl.kernel_base(e[1].name) in ("update_kernel", "update_p_kernel"))
    L = events[iu][1]
    raw = list(L.raw)
    raw[5] = (L.i(5) + 1).to_bytes(8, "little", signed=True)
    bad = list(events)
    bad[iu] = ("launch", cl.Launch(L.name, L.grid, L.block, L.shmem, raw))
    assert any("update_" in v for v in cl.check_events(bad)[0])
    # (c) a reduction over one more partial sum than were written
    ir = first(lambda e: e[0] == "launch" and cl.kernel_base(e[1].name) == "sketch_reduce_kernel")
    L = events[ir][1]
    raw = list(L.raw)
    raw[1] = (L.i(1) + 4000).to_bytes(4, "little", signed=True)
    bad = list(events)
    bad[ir] = ("launch", cl.Launch(L.name, L.grid, L.block, L.shmem, raw))
    assert any("sketch_reduce_kernel" in v for v in cl.check_events(bad)[0])
    # (d) an unknown kernel
    L = events[ir][1]
    bad = list(events) + [("launch", cl.Launch("_ZN4rbgs9new_thingEv", (1, 1, 1), (64, 1, 1), 0, []))]
    assert any("no bounds mirror" in v for v in cl.check_events(bad)[0])
