"""rbgs_qr_noalloc (the entry point that allocates nothing: its workspace is
the library's fixed device scratch array) against rbgs_qr, through the C ABI,
on the GPU.

Both entry points run the same kernels with the same launch configurations on
the same inputs, so Q, R and S must be bitwise identical.  Two no-allocation
calls in a row, the second with a smaller input, check that the contents the
first call leaves in the shared scratch array do not leak into the second.  A
factorization whose workspace exceeds the array is rejected before anything is
enqueued."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _input(n, m, dtype, seed):
    import torch
    from paper_2111_14641_amd import binding as B
    from paper_2111_14641_amd.workloads import svd_matrix
    W = B.colmajor(n, m, dtype)
    W.copy_(torch.from_numpy(svd_matrix(n, m, np.logspace(0, -5, m), seed)))
    return W


def _bits_equal(X, Y):
    import torch
    return torch.equal(X.cpu(), Y.cpu())


# (n, m, p, k, kind, dtype, variant): each pair is run large then small
PAIRS = [
    ((200_000, 96, 16, 512, "sparse", "float32", "lowsync"),
     (30_011, 40, 8, 256, "sparse", "float32", "lowsync")),
    ((50_000, 64, 16, 256, "gaussian", "float64", "plain"),
     (9_001, 24, 8, 128, "gaussian", "float64", "plain")),
    ((120_000, 70, 32, 512, "sparse", "float64", "lowsync"),
     (7_000, 33, 32, 256, "sparse", "float64", "lowsync")),
]


@pytest.mark.parametrize("pair", PAIRS, ids=lambda pr: f"{pr[0][4]}-{pr[0][5]}-{pr[0][6]}")
def test_noalloc_matches_rbgs_qr_bitwise(gpu_lib, pair):
    import torch
    from paper_2111_14641_amd import binding as B
    outs = []
    for i, (n, m, p, k, kind, dt, variant) in enumerate(pair):
        say("noalloc vs rbgs_qr", n, m, p, k, kind, dt, variant)
        W = _input(n, m, getattr(torch, dt), seed=100 + i)
        seed = 0x5EED + i
        Qn, Rn, Sn, _ = B.rbgs_qr(W, p, kind, k, seed, None, variant, 2, want_S=True, noalloc=True)
        torch.cuda.synchronize()
        outs.append((W, Qn, Rn, Sn, (n, m, p, k, kind, variant, seed)))
    # the reference calls run after both no-allocation calls, so the second
    # no-allocation call saw the scratch contents of the first
    for W, Qn, Rn, Sn, (n, m, p, k, kind, variant, seed) in outs:
        Q, R, S, cert = B.rbgs_qr(W, p, kind, k, seed, None, variant, 2, want_S=True, want_cert=True)
        torch.cuda.synchronize()
        assert cert["breakdown_col"] == -1
        assert _bits_equal(Qn, Q), (n, m)
        assert _bits_equal(Rn, R), (n, m)
        assert _bits_equal(Sn, S), (n, m)
        say("bitwise equal", n, m, "delta", cert["delta"])


def test_noalloc_rejects_a_workspace_beyond_the_scratch_array(gpu_lib):
    import torch
    from paper_2111_14641_amd import binding as B
    n, m = 3_000_000, 32
    W = B.colmajor(n, m, torch.float32)
    W.zero_()
    with pytest.raises(B.RbgsError) as ei:
        B.rbgs_qr(W, 16, "sparse", 2048, 1, 8, "lowsync", 4, noalloc=True)
    assert ei.value.status == B.RBGS_ENOMEM
    assert "67108864" in str(ei.value)
