"""Pins for the oracle's exact PCA: covariance + cyclic Jacobi (O1/O2)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ppca_oracle as O
from synthdata import make_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_jacobi_2x2_closed_form():
    for a, b, c in [(2.0, 1.0, 3.0), (1.0, -4.0, 1.0), (5.0, 1e-9, 5.0), (0.0, 2.0, -3.0)]:
        lam, u = O.jacobi_eigh(np.array([[a, b], [b, c]]))
        mid = (a + c) / 2
        rad = math.sqrt(((a - c) / 2) ** 2 + b * b)
        assert lam[0] == pytest.approx(mid + rad, rel=1e-14, abs=1e-14)
        assert lam[1] == pytest.approx(mid - rad, rel=1e-14, abs=1e-14)
        a2 = np.array([[a, b], [b, c]])
        assert np.allclose(a2 @ u, u * lam[None, :], atol=1e-13)


def test_counterexample_covariance_eigenpairs():
    """Sec. 4.1 worked example: eigenvalues 3, 4/3, 1/3 with e1, e2 = axes."""
    g = json.load(open(os.path.join(GOLD, "counterexample.json")))
    x = np.array(g["points"], np.float64)
    lam, u = O.exact_pca(x)
    assert np.allclose(lam, g["covariance_eigenvalues"], rtol=1e-15, atol=1e-15)
    assert np.allclose(u[:, 0], g["e1"], atol=1e-15)
    assert np.allclose(u[:, 1], g["e2"], atol=1e-15)


def test_jacobi_vs_numpy_eigh():
    rng = np.random.default_rng(4)
    for m in (1, 3, 17, 40):
        a = rng.standard_normal((m, m))
        a = a + a.T
        lam, u = O.jacobi_eigh(a)
        ref, uref = np.linalg.eigh(a)
        ref = ref[::-1]
        uref = uref[:, ::-1]
        assert np.allclose(lam, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        # eigenvectors up to sign
        dots = np.abs(np.sum(u * uref, axis=0))
        assert np.allclose(dots, 1.0, atol=1e-10)


def test_jacobi_invariants():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((30, 30))
    a = a @ a.T
    lam, u = O.jacobi_eigh(a)
    assert abs(lam.sum() - np.trace(a)) <= 1e-12 * abs(np.trace(a))
    assert np.linalg.norm(a @ u - u * lam[None, :]) <= 1e-12 * np.linalg.norm(a)
    assert np.linalg.norm(u.T @ u - np.eye(30)) <= 1e-13
    assert np.all(np.diff(lam) <= 0)
    # sign rule: largest-magnitude entry of every column is positive
    piv = np.argmax(np.abs(u), axis=0)
    assert np.all(u[piv, np.arange(30)] > 0)


def test_jacobi_repeated_and_diagonal():
    lam, u = O.jacobi_eigh(np.eye(5) * 2.0)
    assert np.all(lam == 2.0) and np.allclose(u, np.eye(5))
    lam, _ = O.jacobi_eigh(np.diag([1.0, 5.0, 3.0]))
    assert list(lam) == [5.0, 3.0, 1.0]


def test_jacobi_sweep_cap():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((12, 12))
    with pytest.raises(O.NoConvergence):
        O.jacobi_eigh(a + a.T, max_sweeps=1)


def test_covariance_brute_force():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((9, 4))
    c = O.covariance(x)
    for i in range(4):
        for j in range(4):
            s = 0.0
            for r in range(9):
                s += x[r, i] * x[r, j]
            assert c[i, j] == pytest.approx(s / 9, rel=1e-14, abs=1e-15)


def test_exact_spectrum_generator_closed_form():
    """X = Z_w diag(sqrt(lam)) Q^T with whitened Z_w has covariance exactly
    Q diag(lam) Q^T: the oracle's exact PCA must return lam and +-q_i."""
    p = make_problem(3000, 24, "exp0.9", seed=11, mode="exact", dtype=np.float64)
    xc = p.x - O.column_means(p.x)[None, :]
    lam, u = O.exact_pca(xc, 10)
    assert np.allclose(lam, p.lam[:10], rtol=1e-11)
    dots = np.abs(np.sum(u * p.q[:, :10], axis=0))
    assert np.allclose(dots, 1.0, atol=1e-9)
