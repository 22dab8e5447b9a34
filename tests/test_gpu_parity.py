"""GPU parity: the HIP path (through the C ABI) against the float64 oracle on
the same seeded inputs.  Sizes span several tiles and ragged tails.

Tolerances (each derived from the arithmetic of the step it bounds):
* centring / storage codes: bit-exact (integer results);
* Gram of the projected data: f32 data 2e-5, bf16/fp8 data 4e-3 of
  sqrt(G_ii G_jj) (the bf16 rounding of Y before the Gram bounds it by 2^-8);
  the operand Gram B: 1e-12;
* pPCA results: 1e-4 (f32 path) and 2e-3 (bf16/fp8 path after
  Rayleigh-Ritz) in eigenvalue relative error and largest principal-angle sine.
"""
import math

import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O
from synthdata import gaussian_block, make_problem

from ._gpu_util import (BF16, F32, FP8, TRAJ_REL, col_cos, device_data, gram_err, host,
                        operand_basis, oracle_replay, projection_basis, sin_theta,
                        trajectory_error)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as P
    P.lib()        # fails loudly if the library is missing
    P.set_chunk_rows(0)
    yield


def P():
    import paper_2109_03709_amd as mod
    return mod


# ----------------------------------------------------------------- a0 parity
@pytest.mark.parametrize("dtype", [F32, BF16, FP8])
@pytest.mark.parametrize("shape", [(3001, 77), (64, 16), (1, 5)])
def test_center_quantize_bit_exact(dtype, shape):
    n, d = shape
    rng = np.random.default_rng(n + d)
    x = (rng.standard_normal((n, d)) * rng.uniform(0.01, 100, d) + rng.uniform(-5, 5, d))
    x = x.astype(np.float32)
    x[:, -1] = 0.0 if d > 1 else x[:, -1]          # an all-zero column
    xd = torch.from_numpy(x).cuda()
    data, mean = P().center_quantize(xd, dtype)
    torch.cuda.synchronize()
    mu = O.column_means(x)
    assert np.array_equal(mean.cpu().numpy(), mu)
    c = O.center_fp32(x, mu)
    if dtype == F32:
        assert np.array_equal(data.x.cpu().numpy().view(np.uint32), c.view(np.uint32))
    elif dtype == BF16:
        assert np.array_equal(host(data.x), O.bf16_round(c))
    else:
        s = O.fp8_column_scales(c)
        assert np.array_equal(data.col_scale.cpu().numpy(), s)
        assert np.array_equal(data.x.cpu().numpy(), O.fp8_quantize(c, s))


# --------------------------------------------------------- projection + Gram
@pytest.mark.parametrize("dtype", [F32, BF16, FP8])
@pytest.mark.parametrize("n,d,K,pad", [(5003, 200, 24, 0), (3000, 256, 128, 0),
                                        (777, 64, 1, 16), (4096, 600, 40, 32), (9, 33, 3, 15)])
def test_project_gram(dtype, n, d, K, pad):
    p = make_problem(n, d, "exp0.9", seed=n + K, mode="gaussian")
    ld = d + pad
    data, xs, scale = device_data(p.x, dtype, ld)
    v = gaussian_block(d, K, 7, np.float32)
    G, B = P().project_gram(data, K, torch.from_numpy(v).cuda())
    torch.cuda.synchronize()
    veff = projection_basis(v, dtype, scale)
    g_ref, b_ref = O.project_gram(xs, veff)
    tol = 2e-5 if dtype == F32 else 4e-3
    assert gram_err(G.cpu().numpy(), g_ref) < tol
    assert np.allclose(B.cpu().numpy(), b_ref, rtol=1e-12, atol=1e-12 * np.abs(b_ref).max())
    assert np.array_equal(G.cpu().numpy(), G.cpu().numpy().T)


# ------------------------------------------------------- the streaming pass
@pytest.mark.parametrize("dtype", [F32, BF16, FP8])
@pytest.mark.parametrize("n,d,K,r0,rows", [(5003, 300, 64, 0, 5003), (4000, 1024, 128, 3900, 1024),
                                            (1500, 77, 5, 17, 999), (20000, 512, 32, 123, 20000),
                                            (3000, 200, 70, 11, 2500)])
def test_stream_pass_elementwise_bound(dtype, n, d, K, r0, rows):
    """Z = X^T (X V') and G on a (wrapping) row range.  Elementwise bound:
    |Z - Z_ref| <= c |X|^T |Y| with c = 2^-8 when Y is rounded to bf16 before
    the second product (bf16 / fp8 data) and c = 1e-5 for float32 data."""
    p = make_problem(n, d, "pow1.5", seed=n + d + K, mode="gaussian")
    data, xs, scale = device_data(p.x, dtype)
    v = gaussian_block(d, K, 17, np.float32)
    Z, G = P().stream_pass(data, K, torch.from_numpy(v).cuda(), r0=r0, nrows=rows)
    torch.cuda.synchronize()
    xb = xs[(r0 + np.arange(rows)) % n]
    veff = operand_basis(v, dtype, scale)
    y = xb @ veff
    z_ref, g_ref = xb.T @ y, y.T @ y
    bound = np.abs(xb).T @ np.abs(y)
    c = 1e-5 if dtype == F32 else 2.0 ** -8
    assert np.all(np.abs(Z.cpu().numpy() - z_ref) <= c * bound + 1e-30)
    assert gram_err(G.cpu().numpy(), g_ref) < (2e-5 if dtype == F32 else 4e-3)


@pytest.mark.parametrize("dtype,K,want_g", [(BF16, 32, False), (BF16, 64, False), (BF16, 48, False),
                                             (BF16, 64, True), (F32, 64, False), (FP8, 64, False),
                                             (F32, 32, True), (BF16, 16, True), (F32, 80, False)])
def test_stream_pass_wide_tiles(dtype, K, want_g):
    """Passes of at least 65,536 rows run on 256-row tiles (Y = X V' of the
    power step: one DMA pipeline over all tiles of a workgroup, Y stored from
    the accumulators; bf16 with K a multiple of 32 on 32x32x16 MFMAs).
    n = 140,001 gives every workgroup two or three tiles and a partial last
    tile; d = 300 ends inside a k-step and inside a 16-byte chunk; the row
    range wraps.  Small K with G and f32 data with K > 64 (128-row tiles)
    are covered too.  Same elementwise bound as the shorter passes."""
    n, d, r0 = 140_001, 300, 70_123
    p = make_problem(n, d, "pow1.5", seed=7 * K + 1, mode="gaussian")
    data, xs, scale = device_data(p.x, dtype)
    v = gaussian_block(d, K, 29, np.float32)
    Z, G = P().stream_pass(data, K, torch.from_numpy(v).cuda(), r0=r0, nrows=n, want_g=want_g)
    torch.cuda.synchronize()
    assert (G is None) == (not want_g)
    xb = np.roll(xs, -r0, axis=0)
    veff = operand_basis(v, dtype, scale)
    y = xb @ veff
    z_ref = xb.T @ y
    bound = np.abs(xb).T @ np.abs(y)
    c = 1e-5 if dtype == F32 else 2.0 ** -8
    assert np.all(np.abs(Z.cpu().numpy() - z_ref) <= c * bound + 1e-30)
    if want_g:
        assert gram_err(G.cpu().numpy(), y.T @ y) < (2e-5 if dtype == F32 else 4e-3)


# ---------------------------------------------------------------- power pass
@pytest.mark.parametrize("dtype", [F32, BF16, FP8])
@pytest.mark.parametrize("n,d,k,l,spec", [(6007, 300, 8, 8, "exp0.9"),
                                           (2048, 512, 16, 16, "exp0.97+1e-5"),
                                           (500, 40, 3, 0, "exp0.9")])
def test_power_iterates(dtype, n, d, k, l, spec):
    """V_t of block power (CholeskyQR2 of Z = X^T X V') against the oracle's
    iteration on the stored data, for t = 1 and 3."""
    K = k + l
    p = make_problem(n, d, spec, seed=3 * n + d, mode="exact")
    data, xs, scale = device_data(p.x, dtype)
    v0 = gaussian_block(d, K, 11, np.float32)
    for iters in (1, 3):
        V = torch.from_numpy(v0.copy()).cuda()
        gh = torch.zeros((iters, K, K), dtype=torch.float64, device="cuda")
        P().prime_power(data, k, l, iters, V, gram_hist=gh)
        torch.cuda.synchronize()
        v_gpu = V.cpu().numpy().astype(np.float64)
        # oracle: same loop, operand of every pass built from the current V
        v = O.cholqr2(v0.astype(np.float64))[0]
        for t in range(iters):
            veff = operand_basis(v.astype(np.float32), dtype, scale)
            z, g = O.stream_pass(xs, veff)
            v = O.cholqr2(z)[0]
        tol = 1e-4 if dtype == F32 else 2e-2
        assert np.linalg.norm(v_gpu.T @ v_gpu - np.eye(K)) < 1e-5 * K
        assert sin_theta(v_gpu, v) < tol
        if dtype == F32:     # columns match one by one (CholeskyQR keeps the nested spans)
            assert np.min(col_cos(v_gpu, v)) > 1 - 1e-6
        assert gram_err(gh[iters - 1].cpu().numpy(), g) < (2e-5 if dtype == F32 else 4e-3)


def test_power_deterministic():
    p = make_problem(5000, 256, "exp0.9", seed=5, mode="exact")
    data, _, _ = device_data(p.x, BF16)
    v0 = torch.from_numpy(gaussian_block(256, 32, 1, np.float32)).cuda()
    a = P().prime_power(data, 16, 16, 4, v0.clone())
    b = P().prime_power(data, 16, 16, 4, v0.clone())
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_chunked_pass_matches_single_pass():
    p = make_problem(9000, 128, "exp0.9", seed=6, mode="exact")
    data, _, _ = device_data(p.x, BF16)
    v = torch.from_numpy(gaussian_block(128, 32, 2, np.float32)).cuda()
    g1, _ = P().project_gram(data, 32, v)
    P().set_chunk_rows(1000)
    try:
        g2, _ = P().project_gram(data, 32, v)
    finally:
        P().set_chunk_rows(0)
    torch.cuda.synchronize()
    assert gram_err(g2.cpu().numpy(), g1.cpu().numpy()) < 1e-6


# ------------------------------------------------------------- Rayleigh-Ritz
@pytest.mark.parametrize("K,k", [(32, 16), (128, 64), (7, 7), (1, 1), (65, 20)])
def test_rayleigh_ritz_vs_oracle(K, k):
    d = max(200, K)
    p = make_problem(4000, d, "exp0.9", seed=K, mode="exact")
    data, xs, _ = device_data(p.x, F32)
    v = gaussian_block(d, K, 3, np.float32) + p.q[:, :K].astype(np.float32)
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram(data, K, vd)
    ev, E = P().rayleigh_ritz(data, K, k, G, B, vd)
    torch.cuda.synchronize()
    th, e_ref, _ = O.rayleigh_ritz(G.cpu().numpy(), B.cpu().numpy(), v.astype(np.float64),
                                   data.n, k)
    assert np.max(O.rel_eig_error(ev.cpu().numpy(), th)) < 1e-8
    e = E.cpu().numpy().astype(np.float64)
    assert np.min(col_cos(e, e_ref)) > 1 - 1e-9
    # sign rule: largest-magnitude entry of each column positive
    piv = np.argmax(np.abs(e), axis=0)
    assert np.all(e[piv, np.arange(k)] > 0)
    assert np.linalg.norm(e.T @ e - np.eye(k)) < 1e-5


@pytest.mark.parametrize("d,K,k", [(1000, 32, 16), (4099, 64, 64), (513, 8, 3)])
def test_rayleigh_ritz_sign_rule_wide(d, K, k):
    """Ritz vectors with more rows than the sign-fix workgroup has threads:
    every column must equal the oracle's sign-normalised column with the same
    sign in every row (a column negated only in part would fail), and its
    largest-magnitude entry must be positive."""
    # the Ritz values only need the projected Gram: Gaussian rows suffice at n < d
    p = make_problem(3000, d, "exp0.9", seed=d + K, mode="gaussian")
    data, xs, _ = device_data(p.x, F32)
    v = gaussian_block(d, K, 5, np.float32) + p.q[:, :K].astype(np.float32)
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram(data, K, vd)
    for _ in range(3):
        ev, E = P().rayleigh_ritz(data, K, k, G, B, vd)
        torch.cuda.synchronize()
        _, e_ref, _ = O.rayleigh_ritz(G.cpu().numpy(), B.cpu().numpy(), v.astype(np.float64),
                                      data.n, k)
        e = E.cpu().numpy().astype(np.float64)
        signed = np.sum(e * e_ref, axis=0) / (np.linalg.norm(e, axis=0) *
                                              np.linalg.norm(e_ref, axis=0))
        assert np.min(signed) > 1 - 1e-9
        piv = np.argmax(np.abs(e), axis=0)
        assert np.all(e[piv, np.arange(k)] > 0)


def test_counterexample_on_gpu():
    """Sec. 4.1 worked example through the GPU Rayleigh-Ritz: the order swap."""
    eps = 0.1
    pts = np.array([[3, 0, 0], [-3, 0, 0], [0, 2, 0], [0, -2, 0], [0, 0, 1], [0, 0, -1]],
                   np.float32)
    x = np.zeros((6, 4), np.float32)       # pad d to a multiple of 4 with a zero column
    x[:, :3] = pts
    data, _ = P().center_quantize(torch.from_numpy(x).cuda(), F32)
    v = np.zeros((4, 2), np.float32)
    v[:3, 0] = [eps, 0, math.sqrt(1 - eps ** 2)]
    v[:3, 1] = [0, 1, 0]
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram(data, 2, vd)
    ev, E = P().rayleigh_ritz(data, 2, 2, G, B, vd)
    torch.cuda.synchronize()
    assert ev.cpu().numpy() == pytest.approx([4.0 / 3.0, (1 + 8 * eps ** 2) / 3], rel=1e-6)
    assert abs(E.cpu().numpy()[0, 0]) < 1e-7          # e1_pPCA is orthogonal to e1


# --------------------------------------------------- end-to-end pPCA results
def _ppca_gpu(data, k, l, iters, v0):
    V = torch.from_numpy(v0.copy()).cuda()
    P().prime_power(data, k, l, iters, V)
    ev, E = P().ppca(data, V, k)
    torch.cuda.synchronize()
    return ev.cpu().numpy(), E.cpu().numpy().astype(np.float64)


def test_small_config_full_size_f32():
    """n=10,000, d=256, lambda_i = 0.9^i, k=16, l=16, 10 power iterations,
    pPCA with a 32 x 32 eigensolve; f32 path tolerance 1e-4."""
    n, d, k, l = 10000, 256, 16, 16
    p = make_problem(n, d, "exp0.9", seed=1001, mode="exact")
    data, xs, _ = device_data(p.x, F32)
    v0 = gaussian_block(d, k + l, 2001, np.float32)
    ev, E = _ppca_gpu(data, k, l, 10, v0)
    v_or, _ = O.prime_power(xs, v0.astype(np.float64), 10)
    th, e_or = O.ppca(xs, v_or, k)
    assert np.max(O.rel_eig_error(ev, th)) < 1e-4
    assert sin_theta(E, e_or) < 1e-4
    # against the exact spectrum (priming has converged: rate 0.9^(17*10))
    assert np.max(O.rel_eig_error(ev, p.lam[:k])) < 1e-4
    assert sin_theta(E, p.q[:, :k]) < 1e-4
    # Ky Fan: the pPCA Rayleigh-quotient sum is at least the priming one
    vq = O.cholqr2(v_or)[0]
    rq = np.sort(np.diag(vq.T @ O.covariance(xs) @ vq))[::-1]
    assert ev.sum() >= rq[:k].sum() * (1 - 1e-6)


@pytest.mark.parametrize("dtype,spec,k,iters", [(BF16, "exp0.9", 64, 6),
                                                 (FP8, "exp0.97+1e-5", 32, 15)])
def test_low_precision_ppca_scaled(dtype, spec, k, iters):
    """bf16 (K = 128) and fp8 (K = 64) storage on d = 2048 with a ragged row
    count.  Parity: after Rayleigh-Ritz the GPU result matches the oracle's
    own run on the same stored data within 2e-3 (eigenvalue relative error
    and largest principal-angle sine).  Against the exact spectrum of the
    float32 data the eigenvalues stay within 2e-3.  The bf16 subspace is held
    to 2e-3 as well: the projection multiplies by the two-term operand
    hi + lo, whose span is that of V to about 2^-16 (a single bf16 operand
    alone puts a floor of about 2e-3 under the largest principal-angle sine,
    whatever n).  fp8 storage (3 mantissa bits, per-column scales) moves the
    stored data's own eigenvectors by about 4e-3 at this n, and its projection
    uses the single operand: 1e-2 there."""
    n, d, l = 20011, 2048, k
    p = make_problem(n, d, spec, seed=1003, mode="exact")
    data, xs, scale = device_data(p.x, dtype)
    v0 = gaussian_block(d, k + l, 2003, np.float32)
    ev, E = _ppca_gpu(data, k, l, iters, v0)
    v_or, _ = O.prime_power(xs, v0.astype(np.float64), iters)
    th, e_or = O.ppca(xs, v_or, k)
    assert np.max(O.rel_eig_error(ev, th)) < 2e-3
    assert sin_theta(E, e_or) < 2e-3
    assert np.max(O.rel_eig_error(ev, p.lam[:k])) < 2e-3
    s_exact = sin_theta(E, p.q[:, :k])
    print(f"sin theta vs exact subspace: {s_exact:.3e}")
    assert s_exact < (2e-3 if dtype == BF16 else 1e-2)


# ----------------------------------------------------- minibatch primings
@pytest.mark.parametrize("dtype", [F32, BF16])
def test_oja_trajectory(dtype):
    n, d, k, l, b = 20000, 256, 16, 16, 1024
    p = make_problem(n, d, "pow1.2+1e-4", seed=1002, mode="exact")
    data, xs, scale = device_data(p.x, dtype)
    v0 = gaussian_block(d, k + l, 2002, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    steps, eta0 = 5, 0.5
    P().prime_oja(data, k, l, V, batch=b, steps=steps, eta0=eta0, t0=1000.0)
    torch.cuda.synchronize()
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    v = oracle_replay("oja", lambda t: xs[O.minibatch_rows(n, b, t)], v_start, range(steps), b,
                      eta0, 1000.0, lambda u: operand_basis(u.astype(np.float32), dtype, scale))
    vg = V.cpu().numpy()
    if dtype == F32:
        assert np.max(np.abs(vg - v)) / np.max(np.abs(v)) < 1e-4
    else:
        assert trajectory_error(vg, v, v_start) < TRAJ_REL


@pytest.mark.parametrize("dtype", [F32, FP8])
def test_eigengame_trajectory(dtype):
    n, d, k, l, b = 12000, 512, 8, 8, 4096
    p = make_problem(n, d, "exp0.97+1e-5", seed=1004, mode="exact")
    data, xs, scale = device_data(p.x, dtype)
    v0 = gaussian_block(d, k + l, 2004, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    steps, eta0 = 4, 0.5
    P().prime_eigengame(data, k, l, V, batch=b, steps=steps, eta0=eta0)
    torch.cuda.synchronize()
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    v = oracle_replay("eigengame", lambda t: xs[O.minibatch_rows(n, b, t)], v_start, range(steps),
                      b, eta0, 0.0, lambda u: operand_basis(u.astype(np.float32), dtype, scale))
    vg = V.cpu().numpy()
    if dtype == F32:
        assert np.max(np.abs(vg - v)) < 1e-4
    else:
        assert trajectory_error(vg, v, v_start) < TRAJ_REL


def test_momentum_and_resume():
    """Nesterov momentum 0.9 (Sec. 5) and resuming from (V, step, buffer):
    two calls of 3 steps equal one call of 6."""
    n, d, k, l, b = 8000, 128, 8, 0, 1000
    p = make_problem(n, d, "paper-exp", seed=9, mode="exact")
    data, xs, _ = device_data((p.x / math.sqrt(1000.0)).astype(np.float32), F32)
    v0 = torch.from_numpy(gaussian_block(d, k, 3, np.float32)).cuda()
    kw = dict(batch=b, eta0=1e-3, t0=0.0, momentum=0.9, nesterov=True)
    va, ma = v0.clone(), torch.zeros_like(v0)
    P().prime_oja(data, k, l, va, steps=6, mom_buf=ma, **kw)
    vb, mb = v0.clone(), torch.zeros_like(v0)
    P().prime_oja(data, k, l, vb, steps=3, mom_buf=mb, **kw)
    P().prime_oja(data, k, l, vb, steps=3, mom_buf=mb, start_step=3, orthonormalise_start=False,
                  **kw)
    torch.cuda.synchronize()
    assert torch.equal(va, vb) and torch.equal(ma, mb)
    v_or, _ = O.prime_oja(xs, v0.cpu().numpy().astype(np.float64), batch=b, steps=6, eta0=1e-3,
                          t0=0.0, momentum=0.9, nesterov=True)
    assert np.max(np.abs(va.cpu().numpy() - v_or)) < 1e-4 * np.max(np.abs(v_or))


@pytest.mark.parametrize("nesterov", [True, False])
def test_eigengame_momentum_and_resume(nesterov):
    """EigenGame with momentum 0.9 (Nesterov and heavy ball): six steps match
    the oracle's, two calls of three equal one of six (V and the buffer
    bitwise), and the run without momentum lies well outside the tolerance
    (so a dropped or mis-weighted momentum term would fail)."""
    n, d, k, l, b = 8000, 128, 4, 4, 1000
    p = make_problem(n, d, "paper-exp", seed=19, mode="exact")
    data, xs, _ = device_data((p.x / math.sqrt(1000.0)).astype(np.float32), F32)
    v0 = torch.from_numpy(gaussian_block(d, k + l, 13, np.float32)).cuda()
    kw = dict(batch=b, eta0=0.05, t0=0.0, momentum=0.9, nesterov=nesterov)
    va, ma = v0.clone(), torch.zeros_like(v0)
    P().prime_eigengame(data, k, l, va, steps=6, mom_buf=ma, **kw)
    vb, mb = v0.clone(), torch.zeros_like(v0)
    P().prime_eigengame(data, k, l, vb, steps=3, mom_buf=mb, **kw)
    P().prime_eigengame(data, k, l, vb, steps=3, mom_buf=mb, start_step=3,
                        orthonormalise_start=False, **kw)
    vc = v0.clone()
    P().prime_eigengame(data, k, l, vc, steps=6, batch=b, eta0=0.05, t0=0.0)
    torch.cuda.synchronize()
    assert torch.equal(va, vb) and torch.equal(ma, mb)
    v_or, m_or = O.prime_eigengame(xs, v0.cpu().numpy().astype(np.float64), batch=b, steps=6,
                                   eta0=0.05, t0=0.0, momentum=0.9, nesterov=nesterov)
    err = np.max(np.abs(va.cpu().numpy() - v_or))
    assert err < 1e-4
    assert np.max(np.abs(ma.cpu().numpy() - m_or)) < 1e-4 * max(1.0, np.max(np.abs(m_or)))
    assert np.max(np.abs(vc.cpu().numpy() - v_or)) > 100 * 1e-4


@pytest.mark.parametrize("method", ["oja", "eigengame"])
def test_minibatch_at_the_largest_k(method):
    """K = PPCA_MAX_K = 128 (k = l = 64): the update kernels then hold the K x K
    matrix built from G in 128 KB of LDS; two steps against the oracle."""
    n, d, k, l, b = 4096, 256, 64, 64, 1024
    p = make_problem(n, d, "exp0.9", seed=31, mode="exact")
    data, xs, _ = device_data(p.x, F32)
    v0 = gaussian_block(d, k + l, 32, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    fn, ofn = ((P().prime_oja, O.prime_oja) if method == "oja"
               else (P().prime_eigengame, O.prime_eigengame))
    fn(data, k, l, V, batch=b, steps=2, eta0=0.2, t0=0.0)
    torch.cuda.synchronize()
    v, _ = ofn(xs, v0.astype(np.float64), batch=b, steps=2, eta0=0.2, t0=0.0)
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    err = trajectory_error(V.cpu().numpy(), v, v_start)
    print(f"{method} K = 128: trajectory error {err:.2e}", flush=True)
    assert err < 1e-4


def test_snapshots():
    n, d, K, b = 4000, 64, 8, 500
    p = make_problem(n, d, "exp0.9", seed=10, mode="exact")
    data, _, _ = device_data(p.x, F32)
    v = torch.from_numpy(gaussian_block(d, K, 4, np.float32)).cuda()
    snaps = torch.zeros((3, d, K), dtype=torch.float32, device="cuda")
    P().prime_eigengame(data, 4, 4, v, batch=b, steps=7, eta0=0.1, snapshot_every=2,
                        snapshots=snaps)
    v6 = torch.from_numpy(gaussian_block(d, K, 4, np.float32)).cuda()
    P().prime_eigengame(data, 4, 4, v6, batch=b, steps=6, eta0=0.1)
    torch.cuda.synchronize()
    assert torch.equal(snaps[2], v6)


# ------------------------------------------------------------- error paths
def test_error_not_spd():
    p = make_problem(1000, 64, "exp0.9", seed=12, mode="exact")
    data, _, _ = device_data(p.x, F32)
    v = gaussian_block(64, 6, 5, np.float32)
    v[:, 5] = v[:, 1]
    with pytest.raises(P().PPCAError) as ei:
        P().prime_power(data, 3, 3, 2, torch.from_numpy(v).cuda())
    assert ei.value.code == -3
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram(data, 6, vd)
    with pytest.raises(P().PPCAError) as ei:
        P().rayleigh_ritz(data, 6, 3, G, B, vd)
    assert ei.value.code == -3


def test_error_not_spd_late_block():
    """K = 128 with a zero column 100: the zero pivot comes in the seventh
    16-column block, which the Cholesky factors while the other wavefronts
    still update the trailing blocks; the call reports NOT_SPD, and the next
    call on a full-rank basis runs normally (matching the oracle)."""
    d, K, k = 300, 128, 64
    p = make_problem(1000, d, "exp0.9", seed=15, mode="exact")
    data, _, _ = device_data(p.x, F32)
    v = gaussian_block(d, K, 7, np.float32)
    bad = v.copy()
    bad[:, 100] = 0.0
    with pytest.raises(P().PPCAError) as ei:
        P().prime_power(data, k, K - k, 2, torch.from_numpy(bad).cuda())
    assert ei.value.code == -3
    bd = torch.from_numpy(bad).cuda()
    G, B = P().project_gram(data, K, bd)
    with pytest.raises(P().PPCAError) as ei:
        P().rayleigh_ritz(data, K, k, G, B, bd)
    assert ei.value.code == -3
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram(data, K, vd)
    ev, _ = P().rayleigh_ritz(data, K, k, G, B, vd)
    torch.cuda.synchronize()
    th, _, _ = O.rayleigh_ritz(G.cpu().numpy(), B.cpu().numpy(), v.astype(np.float64), data.n, k)
    assert np.max(O.rel_eig_error(ev.cpu().numpy(), th)) < 1e-8


def test_error_nonfinite():
    p = make_problem(1000, 64, "exp0.9", seed=13, mode="exact")
    data, _, _ = device_data(p.x, F32)
    data.x[17, 5] = float("nan")
    with pytest.raises(P().PPCAError) as ei:
        P().project_gram(data, 4, torch.from_numpy(gaussian_block(64, 4, 6, np.float32)).cuda())
    assert ei.value.code == -4


def test_error_workspace_and_args():
    p = make_problem(1000, 64, "exp0.9", seed=14, mode="exact")
    data, _, _ = device_data(p.x, F32)
    v = torch.from_numpy(gaussian_block(64, 8, 6, np.float32)).cuda()
    need = P().workspace_bytes(P().OP_POWER, data, 8)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(P().PPCAError) as ei:
        P().prime_power(data, 4, 4, 1, v, ws=ws)
    assert ei.value.code == -6
    with pytest.raises(P().PPCAError) as ei:
        P().prime_oja(data, 4, 4, v, batch=2000, steps=1, eta0=0.1)
    assert ei.value.code == -1
