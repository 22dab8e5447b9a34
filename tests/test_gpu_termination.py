"""Termination rule of the power method, the sequential power method
(Sec. 2.1) and the projection of a row window (Sec. 5.2 projects a tenth of
the rows), through the C ABI, against the oracle on the same stored data."""
import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O
from synthdata import gaussian_block, make_problem

from ._gpu_util import BF16, F32, device_data, gram_err, projection_basis, sin_theta

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as P
    P.lib()
    P.set_chunk_rows(0)
    yield


def P():
    import paper_2109_03709_amd as mod
    return mod


def test_power_eps_matches_oracle():
    """Changes per iteration equal the oracle's (float32 iterates: 1e-3
    relative), and the run stops at the same iteration, eps being chosen
    between two of the oracle's changes so that rounding cannot move it."""
    n, d, k, l = 4000, 200, 8, 8
    p = make_problem(n, d, "exp0.9", seed=71, mode="exact")
    data, xs, _ = device_data(p.x, F32)
    v0 = gaussian_block(d, k + l, 72, np.float32)
    _, t_ref, ch_ref = O.prime_power_eps(xs, v0.astype(np.float64), 60, 0.0)
    ch_ref = np.array(ch_ref)
    # eps between the changes of iterations 11 and 12 (geometric mean); the
    # oracle's changes before the stop stay at least 1 % away from it
    eps = float(np.sqrt(ch_ref[10] * ch_ref[11]))
    v_or, t_or, _ = O.prime_power_eps(xs, v0.astype(np.float64), 60, eps)
    assert np.all(np.abs(ch_ref[:t_or] - eps) > 1e-2 * eps)
    V = torch.from_numpy(v0.copy()).cuda()
    V, t, ch = P().prime_power_eps(data, k, l, 60, eps, V)
    torch.cuda.synchronize()
    assert t == t_or
    assert np.all(np.abs(np.array(ch) - ch_ref[:t]) <= 1e-6 + 1e-3 * ch_ref[:t])
    assert sin_theta(V.cpu().numpy(), v_or) < 1e-4


def test_power_eps_fixed_point_stops_at_once():
    n, d, K = 3000, 64, 6
    p = make_problem(n, d, "exp0.9", seed=73, mode="exact")
    data, xs, _ = device_data(p.x, F32)
    V = torch.from_numpy(np.ascontiguousarray(p.q[:, :K].astype(np.float32))).cuda()
    _, t, ch = P().prime_power_eps(data, 3, 3, 30, 1e-4, V)
    torch.cuda.synchronize()
    assert t == 1 and ch[0] < 1e-4


@pytest.mark.parametrize("spec", ["paper-exp", "paper-lin"])
def test_sequential_power_matches_oracle(spec):
    """The paper's small-scale synthetic shape (5000 x 50, spectrum from 1000
    to 1), 16 directions one after the other with eps = 1e-5: every direction
    takes the oracle's number of steps (to one step: float32 iterates near the
    threshold) and points the same way; columns orthonormal."""
    n, d, k = 5000, 50, 16
    p = make_problem(n, d, spec, seed=74, mode="exact")
    data, xs, _ = device_data(p.x, F32)
    v0 = gaussian_block(d, k, 75, np.float32)
    v_or, steps_or = O.prime_power_sequential(xs, v0.astype(np.float64), 1e-5, 20000)
    V = torch.from_numpy(v0.copy()).cuda()
    V, steps = P().prime_power_seq(data, k, 0, 1e-5, 20000, V)
    torch.cuda.synchronize()
    v = V.cpu().numpy().astype(np.float64)
    print(f"{spec}: steps {steps}\noracle {steps_or}")
    assert np.all(np.abs(np.array(steps) - np.array(steps_or)) <= 1)
    cos = np.abs(np.sum(v * v_or, axis=0))
    assert np.min(cos) > 1 - 1e-6
    assert np.linalg.norm(v.T @ v - np.eye(k)) < 1e-5


@pytest.mark.parametrize("dtype", [F32, BF16])
def test_projection_of_a_row_window(dtype):
    """G over rows r0 .. r0 + nrows - 1 (wrapping) against the oracle's Gram of
    those rows; Rayleigh-Ritz with n = nrows against the oracle's."""
    n, d, K, k, r0, nrows = 20_011, 300, 32, 16, 15_000, 9_000
    p = make_problem(n, d, "exp0.9", seed=76, mode="exact")
    data, xs, scale = device_data(p.x, dtype)
    v = gaussian_block(d, K, 77, np.float32) + p.q[:, :K].astype(np.float32)
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram_rows(data, K, vd, r0, nrows)
    ev, E = P().ppca(data, vd, k, rows=(r0, nrows))
    torch.cuda.synchronize()
    rows = (r0 + np.arange(nrows)) % n
    veff = projection_basis(v, dtype, scale)
    g_ref, b_ref = O.project_gram(xs[rows], veff)
    assert gram_err(G.cpu().numpy(), g_ref) < (2e-5 if dtype == F32 else 4e-3)
    assert np.allclose(B.cpu().numpy(), b_ref, rtol=1e-12, atol=1e-12 * np.abs(b_ref).max())
    th, e_ref, _ = O.rayleigh_ritz(G.cpu().numpy(), B.cpu().numpy(), veff, nrows, k)
    assert np.max(O.rel_eig_error(ev.cpu().numpy(), th)) < 1e-8
    assert sin_theta(E.cpu().numpy(), e_ref) < 1e-6
