"""The seeded input generators (CPU): the constructions deliver what they
promise, so the parity cases test what they claim to test."""
import numpy as np

from paper_2111_14641_amd import workloads as wl


def test_svd_matrix_has_the_prescribed_singular_values():
    s = np.logspace(0, -8, 24)
    W = wl.svd_matrix(2000, 24, s, seed=3)
    assert W.flags.f_contiguous
    assert np.allclose(np.linalg.svd(W, compute_uv=False), s, rtol=1e-7, atol=0)


def test_gpu_construction_on_the_cpu_device():
    """The row-chunked torch construction used for the 4e6 x 512 workload, run
    on the CPU device at a small size with several chunks and a ragged last
    chunk: column-major, prescribed singular values (cond 1e10 as in the
    workload), deterministic for a seed, the FP32 output the rounded FP64 one."""
    s = np.logspace(0, -10, 16)
    W, W32 = wl.svd_matrix_gpu(3000, 16, s, 7, device="cpu", dtypes=("float64", "float32"),
                               chunk=1024)
    assert W.stride() == (1, 3000) and W32.stride() == (1, 3000)
    sv = np.linalg.svd(W.numpy(), compute_uv=False)
    assert np.allclose(sv, s, rtol=1e-5, atol=0)
    assert np.allclose(sv[:8], s[:8], rtol=1e-12, atol=0)
    assert np.array_equal(W32.numpy(), W.numpy().astype(np.float32))
    W2 = wl.svd_matrix_gpu(3000, 16, s, 7, device="cpu", chunk=1024)
    assert np.array_equal(W.numpy(), W2.numpy())
    # the chunks are independent draws (no chunk repeats another)
    assert not np.allclose(W.numpy()[:952], W.numpy()[1024:1976])


def test_oscillatory_matrix_formula_and_chunking():
    n, m = 1001, 5
    W = wl.oscillatory_matrix(n, m, seed=11, chunk=64)
    mu = np.random.default_rng(11).random(m)
    x = np.arange(n) / (n - 1)
    for j in range(m):
        ref = np.sin(10 * (mu[j] * x + 1)) / (np.cos(100 * mu[j] * x - 100 * mu[j]) + 1.1)
        # (another rounding order of the arguments: the denominator can be 0.1)
        assert np.allclose(W[:, j], ref, rtol=1e-11, atol=1e-12)
    assert np.all(np.abs(W) <= 10 / 0.1 + 1e-9)


def test_batched_problems_on_the_cpu_device():
    probs = wl.batched_problems(count=4, seed=3, device="cpu")
    for W, n, m, c in probs:
        assert 2 ** 14 - 1 <= n <= 2 ** 18 + 1 and m in (32, 64, 128, 256)
        assert W.dtype.is_floating_point and W.element_size() == 4 and W.stride() == (1, n)
        s = np.linalg.svd(W.double().numpy(), compute_uv=False)
        ratio = s[0] / s[-1]
        # FP32 rounding (about 6e-8 relative) hides singular values below it
        assert min(10 ** c / 1.5, 1e6) <= ratio <= 10 ** c * 1.5
