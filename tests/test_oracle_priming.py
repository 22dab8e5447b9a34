"""Pins for the oracle's Cholesky/CholeskyQR2 (O3) and priming loops (O4-O6)."""
import math

import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O
from synthdata import make_problem, gaussian_block


def _householder_q(a):
    q, r = np.linalg.qr(a)
    s = np.sign(np.diag(r))
    s[s == 0] = 1
    return q * s[None, :], r * s[:, None]


def test_cholesky_vs_numpy():
    rng = np.random.default_rng(10)
    a = rng.standard_normal((20, 20))
    a = a @ a.T + 0.1 * np.eye(20)
    r = O.cholesky_upper(a)
    assert np.allclose(r, np.triu(r))
    assert np.allclose(r.T, np.linalg.cholesky(a), rtol=1e-12, atol=1e-12)


def test_cholesky_not_spd():
    v = np.random.default_rng(11).standard_normal((10, 3))
    v[:, 2] = v[:, 1]
    with pytest.raises(O.NotSPD):
        O.cholesky_upper(v.T @ v - 1e-12 * np.eye(3))
    with pytest.raises(O.NotSPD):
        O.cholesky_upper(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(O.NotSPD):
        O.cholesky_upper(np.array([[np.nan]]))


def test_solve_right_upper():
    rng = np.random.default_rng(12)
    r = np.triu(rng.standard_normal((6, 6))) + 4 * np.eye(6)
    z = rng.standard_normal((15, 6))
    q = O.solve_right_upper(z, r)
    assert np.allclose(q @ r, z, atol=1e-13)


def test_cholqr2_vs_householder():
    rng = np.random.default_rng(13)
    a = rng.standard_normal((200, 12)) @ np.diag(np.logspace(0, -6, 12))
    q, r = O.cholqr2(a)
    qh, rh = _householder_q(a)
    assert np.linalg.norm(q.T @ q - np.eye(12)) < 1e-14 * 12
    assert np.allclose(q @ r, a, atol=1e-13)
    assert np.allclose(q, qh, atol=1e-9)
    assert np.allclose(r, rh, rtol=1e-9, atol=1e-15)


def test_power_equals_qr_of_matrix_power():
    """V_t is the Q factor (positive diagonal) of (X^T X)^t V_0, column by
    column, because products of upper-triangular factors stay triangular."""
    p = make_problem(400, 10, "exp0.9", seed=3, mode="gaussian", dtype=np.float64)
    x = p.x - p.x.mean(axis=0)
    v0 = gaussian_block(10, 4, 99, np.float64)
    m = x.T @ x
    for t in (1, 2, 3):
        vt, grams = O.prime_power(x, v0, t)
        ref, _ = _householder_q(np.linalg.matrix_power(m, t) @ _householder_q(v0)[0])
        assert np.allclose(vt, ref, atol=1e-10)
        assert len(grams) == t


def test_power_fixed_point_and_gram():
    p = make_problem(500, 12, "exp0.9", seed=4, mode="exact", dtype=np.float64)
    x = p.x - O.column_means(p.x)[None, :]
    u = p.q[:, :3]
    vt, grams = O.prime_power(x, u, 4)
    assert np.allclose(np.abs(np.sum(vt * u, axis=0)), 1.0, atol=1e-12)
    # G_{t-1} = V^T X^T X V: the Rayleigh quotients times n
    assert np.allclose(np.diag(grams[-1]) / 500, p.lam[:3], rtol=1e-10)


def test_power_rate_bound():
    p = make_problem(800, 16, "exp0.9", seed=5, mode="exact", dtype=np.float64)
    x = p.x - O.column_means(p.x)[None, :]
    kk = 4
    v0 = gaussian_block(16, kk, 5, np.float64)
    u = p.q[:, :kk]
    q0 = O.cholqr2(v0)[0]
    c0 = np.linalg.svd(u.T @ q0, compute_uv=False).min()
    tan0 = math.sqrt(1 - c0 ** 2) / c0
    ratio = p.lam[kk] / p.lam[kk - 1]
    for t in (1, 3, 6):
        vt, _ = O.prime_power(x, v0, t)
        assert O.sin_theta_max(vt, u) <= ratio ** t * tan0 * (1 + 1e-9) + 1e-13


def test_sanger_matrix_form_equals_printed_rule():
    rng = np.random.default_rng(14)
    xb = rng.standard_normal((7, 5))
    v = rng.standard_normal((5, 3))
    z, g = O.stream_pass(xb, v)
    assert np.allclose(O.sanger_direction(z, g, v, 7), O.sanger_per_sample(xb, v), atol=1e-13)


def test_sanger_fixed_point_full_batch():
    p = make_problem(300, 8, "exp0.9", seed=6, mode="exact", dtype=np.float64)
    x = p.x - O.column_means(p.x)[None, :]
    u = p.q[:, :3]
    z, g = O.stream_pass(x, u)
    assert np.max(np.abs(O.sanger_direction(z, g, u, 300))) < 1e-12


def test_eigengame_grad_finite_differences():
    rng = np.random.default_rng(15)
    b, d, kk = 11, 6, 4
    xb = rng.standard_normal((b, d))
    v = rng.standard_normal((d, kk))
    m = xb.T @ xb / b
    z, g = O.stream_pass(xb, v)
    grad = O.eigengame_grad(z, g, b)
    h = 1e-6
    for j in range(kk):
        for i in range(d):
            vp = v.copy(); vp[i, j] += h
            vm = v.copy(); vm[i, j] -= h
            fd = (O.eigengame_utility(m, vp, j) - O.eigengame_utility(m, vm, j)) / (2 * h)
            assert fd == pytest.approx(grad[i, j], rel=1e-6, abs=1e-8)


def test_eigengame_fixed_point():
    p = make_problem(300, 8, "exp0.9", seed=7, mode="exact", dtype=np.float64)
    x = p.x - O.column_means(p.x)[None, :]
    u = p.q[:, :3]
    z, g = O.stream_pass(x, u)
    grad = O.eigengame_grad(z, g, 300)
    riem = grad - u * np.sum(u * grad, axis=0)[None, :]
    assert np.max(np.abs(riem)) < 1e-12
    v, _ = O.prime_eigengame(x, u, batch=300, steps=3, eta0=0.5, orthonormalise_start=False)
    assert np.allclose(np.abs(np.sum(v * u, axis=0)), 1.0, atol=1e-12)


def _sphere_fd_gradient(m, v, j, h=1e-5):
    """Riemannian gradient of U_j (Sec. 2.3, eq. (3)) at the unit vector v_j
    by central differences of U_j(normalise(v_j + h t)) along an orthonormal
    basis t of the tangent space {t : t . v_j = 0}; the other players fixed."""
    d = v.shape[0]
    vj = v[:, j]
    q, _ = np.linalg.qr(np.column_stack([vj, np.eye(d)]))
    tangents = q[:, 1:d]
    g = np.zeros(d)
    for t in tangents.T:
        vp = v.copy()
        vp[:, j] = (vj + h * t) / np.linalg.norm(vj + h * t)
        vm = v.copy()
        vm[:, j] = (vj - h * t) / np.linalg.norm(vj - h * t)
        g += (O.eigengame_utility(m, vp, j) - O.eigengame_utility(m, vm, j)) / (2 * h) * t
    return g


def _eigengame_step_error(step_fn, seed):
    """One step V1 = step_fn(V0) with unit columns, full batch, constant rate
    eta.  A step normalise(v + eta g) with g tangent to the sphere at v has
    (I - v v^T) v1 / (eta (v1 . v)) = g exactly; the result is compared with
    the finite-difference Riemannian gradient.  Returns the largest relative
    deviation over the players and whether every player's own utility rose
    (the others held at V0) and every column stayed on the unit sphere."""
    rng = np.random.default_rng(seed)
    b, d, kk, eta = 13, 7, 4, 0.05
    xb = rng.standard_normal((b, d)) * np.sqrt(np.linspace(3.0, 0.2, d))[None, :]
    v0 = rng.standard_normal((d, kk))
    v0 /= np.linalg.norm(v0, axis=0)[None, :]
    m = xb.T @ xb / b
    v1 = step_fn(xb, v0, batch=b, steps=1, eta0=eta, t0=0.0, orthonormalise_start=False)[0]
    worst, rises = 0.0, True
    for j in range(kk):
        vj, wj = v0[:, j], v1[:, j]
        g_step = (wj - vj * (vj @ wj)) / (eta * (vj @ wj))
        g_fd = _sphere_fd_gradient(m, v0, j)
        worst = max(worst, float(np.linalg.norm(g_step - g_fd) / np.linalg.norm(g_fd)))
        vt = v0.copy()
        vt[:, j] = wj
        rises &= O.eigengame_utility(m, vt, j) > O.eigengame_utility(m, v0, j)
    on_sphere = bool(np.allclose(np.linalg.norm(v1, axis=0), 1.0, atol=1e-14))
    return worst, rises, on_sphere


def _eigengame_mutant_without_projection():
    """The oracle's EigenGame loop with the tangent projection deleted (a
    plausible bug: stepping along the Euclidean gradient, then renormalising)."""
    import inspect
    src = inspect.getsource(O.prime_eigengame).splitlines()
    kept = [line for line in src if "grad - v * np.sum(v * grad" not in line]
    assert len(kept) == len(src) - 1
    ns = dict(vars(O))
    exec("\n".join(kept), ns)
    return ns["prime_eigengame"]


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_eigengame_step_on_the_sphere(seed):
    """Sec. 2.3: each player ascends its utility on the unit sphere.  One
    oracle step moves every v_j along the finite-difference Riemannian
    gradient of eq. (3) (rel 1e-6), raises every U_j and keeps |v_j| = 1.
    The same check run on a copy without the tangent projection fails: the
    radial part of the Euclidean gradient shrinks every step by a factor
    1 / (1 + eta v_j . grad_j)."""
    worst, rises, on_sphere = _eigengame_step_error(O.prime_eigengame, seed)
    assert worst < 1e-6 and rises and on_sphere
    worst_m, _, _ = _eigengame_step_error(_eigengame_mutant_without_projection(), seed)
    assert worst_m > 1e-3


def test_momentum_matches_torch_sgd_nesterov():
    """Sec. 5 trains with SGD + Nesterov momentum 0.9; the oracle's update is
    pinned to torch.optim.SGD (ascent: the gradient handed to torch is -g)."""
    rng = np.random.default_rng(16)
    x = rng.standard_normal((64, 6))
    v0 = rng.standard_normal((6, 3))
    eta, mu = 0.01, 0.9
    v_or, _ = O.prime_oja(x, v0, batch=16, steps=5, eta0=eta, t0=0.0, momentum=mu,
                          nesterov=True, orthonormalise_start=False)
    p = torch.tensor(v0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SGD([p], lr=eta, momentum=mu, nesterov=True)
    for t in range(5):
        xb = x[O.minibatch_rows(64, 16, t)]
        vv = p.detach().numpy()
        z, g = O.stream_pass(xb, vv)
        p.grad = torch.from_numpy(-O.sanger_direction(z, g, vv, 16))
        opt.step()
    assert np.allclose(v_or, p.detach().numpy(), atol=1e-13)


def test_schedule_and_rows():
    assert O.learning_rate(0.1, 1000, 0) == 0.1
    assert O.learning_rate(0.1, 1000, 1000) == pytest.approx(0.05)
    assert O.learning_rate(0.1, 0, 5000) == 0.1
    assert list(O.minibatch_rows(10, 4, 2)) == [8, 9, 0, 1]


def test_oja_converges_on_easy_problem():
    p = make_problem(4000, 10, "paper-exp", seed=8, mode="exact", dtype=np.float64)
    x = p.x - O.column_means(p.x)[None, :]
    x = x / math.sqrt(p.lam[0])
    v, _ = O.prime_oja(x, gaussian_block(10, 3, 1, np.float64), batch=100, steps=1500, eta0=0.2, t0=0)
    ang = O.angles(v, p.q[:, :3])
    assert np.all(ang < 0.05)


# ------------------------------------------------ termination rule (Sec. 2.1)
def _data(n, d, seed):
    """Centred Gaussian rows with a decaying column scale (distinct eigenvalues)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)) * (0.8 ** np.arange(d))[None, :]
    return x - x.mean(axis=0, keepdims=True)

def test_power_eps_stops_where_the_iterates_stop_moving():
    """The eps-terminated block power iteration is the plain iteration cut at
    the first t where the new span lies within eps of the previous one: its
    changes equal the largest principal-angle sines between successive plain
    iterates (brute force through an SVD; equal to the largest column
    residual up to the factor sqrt(K) at most, here compared as bounds), and
    it stops at the first one below eps."""
    x = _data(300, 12, seed=41)
    v0 = np.random.default_rng(42).standard_normal((12, 4))
    eps = 1e-6
    v, t, changes = O.prime_power_eps(x, v0, 200, eps)
    prev = O.cholqr2(v0)[0]
    for s in range(1, t + 1):
        cur, _ = O.prime_power(x, v0, s)
        res = cur - prev @ (prev.T @ cur)
        ch = np.max(np.linalg.norm(res, axis=0))
        assert abs(ch - changes[s - 1]) < 1e-12
        # the largest principal-angle sine (SVD) bounds it from both sides
        sin_max = np.linalg.svd(res, compute_uv=False)[0]
        assert sin_max / 2.0 - 1e-12 <= ch <= sin_max + 1e-12
        assert (ch < eps) == (s == t)
        prev = cur
    assert np.allclose(v, prev, atol=1e-14)


def test_span_change_of_one_vector_is_the_printed_quantity():
    """For one unit vector the span change is the sine of the turn, equal to
    the printed |x_i - x_{i+1}| to first order in the angle."""
    a = np.array([[1.0], [0.0], [0.0]])
    for th in (1e-2, 1e-4, 1e-6):
        b = np.array([[math.cos(th)], [math.sin(th)], [0.0]])
        assert abs(O.span_change(b, a) - math.sin(th)) < 1e-15
        assert abs(O.span_change(b, a) - np.linalg.norm(b - a)) < th * th


def test_power_eps_fixed_point():
    """Started on the top-K eigenvectors the iterates do not move: one step."""
    p = make_problem(400, 10, "exp0.9", seed=43, mode="exact")
    x = O.center_fp32(p.x, O.column_means(p.x)).astype(np.float64)
    u = O.exact_pca(x, 3)[1]
    v, t, ch = O.prime_power_eps(x, u, 50, 1e-9)
    assert t == 1 and ch[0] < 1e-9


def test_sequential_power_first_direction_is_the_printed_recurrence():
    """Direction 0 of the sequential method is x_{t+1} = M x_t / |M x_t|
    (Sec. 2.1) run until |x_t - x_{t+1}| < eps: the same vector as
    M^T x_0 / |M^T x_0| for the step count it reports (matrix powers)."""
    x = _data(200, 8, seed=44)
    m = x.T @ x
    v0 = np.random.default_rng(45).standard_normal((8, 3))
    v, steps = O.prime_power_sequential(x, v0, 1e-8, 5000)
    t = steps[0]
    u0 = v0[:, 0] / np.linalg.norm(v0[:, 0])
    mp = np.linalg.matrix_power(m / np.linalg.norm(m, 2), t)
    ref = mp @ u0
    ref /= np.linalg.norm(ref)
    assert np.allclose(v[:, 0], ref, atol=1e-10)
    # the rule: the last step moved less than eps, the one before did not
    mp1 = np.linalg.matrix_power(m / np.linalg.norm(m, 2), t - 1) @ u0
    mp1 /= np.linalg.norm(mp1)
    assert np.linalg.norm(ref - mp1) < 1e-8
    if t >= 2:
        mp2 = np.linalg.matrix_power(m / np.linalg.norm(m, 2), t - 2) @ u0
        mp2 /= np.linalg.norm(mp2)
        assert np.linalg.norm(mp1 - mp2) >= 1e-8


def test_sequential_power_finds_the_eigenvectors_in_order():
    """On exact-spectrum data with separated eigenvalues every direction
    converges to +-q_i in order, orthonormal (closed form of the generator)."""
    p = make_problem(2000, 12, "exp0.9", seed=46, mode="exact")
    x = O.center_fp32(p.x, O.column_means(p.x)).astype(np.float64)
    v0 = np.random.default_rng(47).standard_normal((12, 5))
    v, steps = O.prime_power_sequential(x, v0, 1e-11, 20000)
    cos = np.abs(np.sum(v * p.q[:, :5], axis=0))
    assert np.min(cos) > 1 - 1e-8
    assert np.linalg.norm(v.T @ v - np.eye(5)) < 1e-10
    assert all(s < 20000 for s in steps)
