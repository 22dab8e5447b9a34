"""Pins for the oracle's pPCA step (O7) and metrics (O8)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ppca_oracle as O
from synthdata import make_problem, gaussian_block

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLD, "counterexample.json")))["cases"])
def test_counterexample_order_swap(case):
    """Sec. 4.1: full PCA on the span of the priming vectors swaps the order."""
    g = json.load(open(os.path.join(GOLD, "counterexample.json")))
    x = np.array(g["points"], np.float64)
    eps = case["eps"]
    v = np.array([[eps, 0.0], [0.0, 1.0], [math.sqrt(1 - eps ** 2), 0.0]])
    gram, b = O.project_gram(x, v)
    cov = gram / 6.0
    assert cov[0, 0] == pytest.approx(case["projected_cov_11"], rel=1e-12)
    assert cov[1, 1] == pytest.approx(case["projected_cov_22"], rel=1e-12)
    assert abs(cov[0, 1]) < 1e-15
    th, e = O.ppca(x, v, 2)
    assert th[0] == pytest.approx(4.0 / 3.0, rel=1e-14)
    e1 = np.array(g["e1"], np.float64)
    assert (e[:, 0] @ e1) ** 2 == pytest.approx(case["cos2_ppca_e1"], abs=1e-28)
    assert (v[:, 0] @ e1) ** 2 == pytest.approx(case["cos2_prime_e1"], rel=1e-12)


def _data(n=2000, d=20, seed=21):
    p = make_problem(n, d, "exp0.9", seed=seed, mode="exact", dtype=np.float64)
    return p, p.x - O.column_means(p.x)[None, :]


def test_variance_identity():
    """Sec. 4.2: Var_v of the projected data equals v^T X^T X v on S."""
    p, x = _data()
    v = O.cholqr2(gaussian_block(20, 5, 3, np.float64))[0]
    gram, b = O.project_gram(x, v)
    assert np.allclose(gram / x.shape[0], v.T @ O.covariance(x) @ v, rtol=1e-13, atol=1e-16)
    # and through the explicit projection P_S = V V^T
    xt = x @ (v @ v.T)
    assert np.allclose(v.T @ O.covariance(xt) @ v, gram / x.shape[0], rtol=1e-12, atol=1e-16)


def test_interlacing_and_ky_fan():
    p, x = _data()
    lam = p.lam
    d = 20
    for kk, k in ((6, 6), (6, 3), (9, 4)):
        v = O.cholqr2(gaussian_block(d, kk, 40 + kk, np.float64) + 0.3 * p.q[:, :kk])[0]
        gram, b = O.project_gram(x, v)
        th, e, th_all = O.rayleigh_ritz(gram, b, v, x.shape[0], k)
        for i in range(kk):
            assert lam[d - kk + i] * (1 - 1e-12) <= th_all[i] <= lam[i] * (1 + 1e-12)
        rq = np.diag(v.T @ O.covariance(x) @ v)
        if k == kk:
            assert th.sum() == pytest.approx(rq.sum(), rel=1e-12)
        else:
            assert th.sum() >= rq[:k].sum() * (1 - 1e-13)
        assert np.allclose(e.T @ e, np.eye(k), atol=1e-12)


def test_span_containing_top_k_is_exact():
    p, x = _data()
    rng = np.random.default_rng(1)
    v = np.hstack([p.q[:, :4], rng.standard_normal((20, 3))]) @ rng.standard_normal((7, 7))
    gram, b = O.project_gram(x, v)
    th, e, _ = O.rayleigh_ritz(gram, b, v, x.shape[0], 4)
    assert np.allclose(th, p.lam[:4], rtol=1e-10)
    assert np.allclose(np.abs(np.sum(e * p.q[:, :4], axis=0)), 1.0, atol=1e-9)


def test_basis_invariance():
    p, x = _data()
    rng = np.random.default_rng(2)
    v = rng.standard_normal((20, 6))
    a = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    t1, e1 = O.ppca(x, v, 4)
    t2, e2 = O.ppca(x, v @ a, 4)
    assert np.allclose(t1, t2, rtol=1e-12)
    assert np.allclose(e1, e2, atol=1e-10)


def test_prop_3_1_first_component():
    """Prop. 3.1: if pi_S(e1) maximises the variance on S, the full-PCA step
    returns pi_S(e1), so it cannot be worse than any priming direction in S.
    S = span(e1 + 0.3 e5, e2, e3, e4): the restricted quadratic form is
    diagonal in that basis and (lam1 + 0.09 lam5)/1.09 > lam2, so the
    hypothesis holds exactly."""
    p, x = _data(d=12, seed=22)
    q = p.q
    u = (q[:, 0] + 0.3 * q[:, 4]) / math.sqrt(1.09)
    s_basis = np.stack([u, q[:, 1], q[:, 2], q[:, 3]], axis=1)
    assert (p.lam[0] + 0.09 * p.lam[4]) / 1.09 > p.lam[1]
    rng = np.random.default_rng(3)
    mix = O.cholqr2(rng.standard_normal((4, 4)))[0]
    v = s_basis @ mix                  # priming directions: rotated inside S
    th, e = O.ppca(x, v, 1)
    e1 = q[:, 0]
    assert abs(u @ e[:, 0]) == pytest.approx(1.0, abs=1e-12)
    a_ppca = O.angles(e[:, :1], e1[:, None])[0]
    assert a_ppca == pytest.approx(math.atan(0.3), abs=1e-9)
    for j in range(4):
        assert a_ppca <= O.angles(v[:, j:j + 1], e1[:, None])[0] + 1e-12


def test_streak_example():
    g = json.load(open(os.path.join(GOLD, "streak_example.json")))
    thr = math.pi / 8
    assert O.streak(np.array(g["angles_over_V"]) * thr, thr) == g["streak"]


def test_sin_theta_max_limits():
    rng = np.random.default_rng(4)
    u = O.cholqr2(rng.standard_normal((10, 3)))[0]
    assert O.sin_theta_max(u @ rng.standard_normal((3, 3)), u) < 1e-7
    w = np.eye(10)
    assert O.sin_theta_max(w[:, 3:5], w[:, :3]) == pytest.approx(1.0, abs=1e-15)
    # a known angle: rotate one column by phi out of the span
    phi = 0.3
    e = w[:, :2].copy()
    e[:, 1] = math.cos(phi) * w[:, 1] + math.sin(phi) * w[:, 5]
    assert O.sin_theta_max(e, w[:, :2]) == pytest.approx(math.sin(phi), rel=1e-12)


def test_rel_eig_error():
    assert np.allclose(O.rel_eig_error([1.1, 2.0], [1.0, 2.0, 3.0]), [0.1, 0.0])


def test_rr_not_spd_for_rank_deficient_basis():
    p, x = _data()
    v = gaussian_block(20, 3, 5, np.float64)
    v[:, 2] = v[:, 0]
    gram, b = O.project_gram(x, v)
    with pytest.raises(O.NotSPD):
        O.rayleigh_ritz(gram, b, v, x.shape[0], 2)
