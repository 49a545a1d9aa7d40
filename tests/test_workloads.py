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
    """The torch construction used for the 4e6 x 512 workload, run on the CPU
    device at a small size: column-major, prescribed singular values,
    deterministic for a seed."""
    s = np.logspace(0, -6, 16)
    W = wl.svd_matrix_gpu(3000, 16, s, 7, device="cpu")
    assert W.stride() == (1, 3000)
    assert np.allclose(np.linalg.svd(W.numpy(), compute_uv=False), s, rtol=1e-10, atol=0)
    W2 = wl.svd_matrix_gpu(3000, 16, s, 7, device="cpu")
    assert np.array_equal(W.numpy(), W2.numpy())


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
