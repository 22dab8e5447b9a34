"""The low-rank generator for d >> n keeps its promise, on the CPU: the stored
bf16 data has covariance B diag(lam) B^T up to its own rounding, B has
orthonormal columns, and X is centred.  (A mistake in the whitening, the
scaling by sqrt(lam) or the orthonormal block fails one of these.)"""
import numpy as np
import torch

from synthdata import make_lowrank_device, spectrum


def test_lowrank_generator_exact_covariance():
    n, d, r = 96, 4096, 8
    x, lam, b = make_lowrank_device(n, d, r, "exp0.9", seed=5, device="cpu")
    assert x.dtype == torch.bfloat16 and x.shape == (n, d)
    np.testing.assert_array_equal(lam, spectrum("exp0.9", r))
    bh = b.double().numpy()
    np.testing.assert_allclose(bh.T @ bh, np.eye(r), atol=1e-6)
    xs = x.double().numpy()
    # rounding of the stored data: 2^-9 relative per element
    cov = xs.T @ xs / n
    ref = (bh * lam[None, :]) @ bh.T
    assert np.max(np.abs(cov - ref)) < 2e-2 * lam[0] / np.sqrt(d) + 1e-3 * np.max(np.abs(ref))
    # eigenpairs: B's columns carry the spectrum
    rq = np.einsum("ji,jk,ki->i", bh, cov, bh)
    np.testing.assert_allclose(rq, lam, rtol=1e-2)
    assert np.max(np.abs(xs.mean(axis=0))) < 1e-2 * np.sqrt(lam[0] / d)
