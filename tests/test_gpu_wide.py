"""The d >> n regime (the large-scale runs of Sec. 5.2: ~15M dimensions, a few
thousand rows, minibatch EigenGame then pPCA, a tenth of the rows projected),
at a shape the float64 oracle can follow: n = 1024, d = 262,144, bf16 data
with an exact low-rank covariance (make_lowrank_device).  At this shape the
EigenGame update sums its column partials in two levels (1024 blocks) and the
two-term projection splits its columns over workgroups (16 row tiles)."""
import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O
from synthdata import gaussian_block, make_lowrank_device

from ._gpu_util import (BF16, TRAJ_REL, gram_err, host, operand_basis, oracle_replay,
                        projection_basis, sin_theta, stored_values, trajectory_error)

pytestmark = pytest.mark.gpu

N, D, R, K, B = 1024, 262_144, 32, 8, 256


@pytest.fixture(scope="module")
def wide():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as P
    P.lib()
    P.set_chunk_rows(0)
    print(f"[wide] generating {N} x {D} bf16, rank {R}", flush=True)
    torch.backends.cuda.matmul.allow_tf32 = False
    x, lam, b = make_lowrank_device(N, D, R, "exp0.9", seed=91)
    data = P.Data(x, P.BF16)
    xs = stored_values(host(x), BF16, None)          # float64 copy of the stored data
    yield P, data, xs, lam, b.cpu().numpy().astype(np.float64)


def test_wide_generator_covariance(wide):
    """The stored data's covariance is B diag(lam) B^T up to the bf16 rounding
    of X (relative 2^-9 per element)."""
    P, data, xs, lam, b = wide
    # C b_i = lam_i b_i for the leading directions, through two thin products
    cb = xs.T @ (xs @ b[:, :8]) / N
    assert np.max(np.abs(cb - b[:, :8] * lam[:8][None, :])) < 1e-2 * lam[0]
    assert np.max(np.abs(xs.mean(axis=0))) < 1e-3 * np.sqrt(lam[0])


def test_wide_eigengame_steps_match_oracle(wide):
    """One epoch of minibatch EigenGame (4 steps of 256 rows) from the same
    start, against the oracle's loop replayed on the same rows with the same
    bf16 operand: the motion-relative bound of the minibatch tests."""
    P, data, xs, lam, b = wide
    v0 = gaussian_block(D, K, 92, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    steps, eta0 = 4, 0.2
    P.prime_eigengame(data, 4, 4, V, batch=B, steps=steps, eta0=eta0)
    torch.cuda.synchronize()
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    v = oracle_replay("eigengame", lambda t: xs[O.minibatch_rows(N, B, t)], v_start,
                      range(steps), B, eta0, 0.0,
                      lambda u: operand_basis(u.astype(np.float32), BF16, None))
    err = trajectory_error(V.cpu().numpy(), v, v_start)
    print(f"[wide] EigenGame trajectory error {err:.2e} of the motion", flush=True)
    assert err < TRAJ_REL


def test_wide_projection_and_rayleigh_ritz(wide):
    """Projection of all rows and of a tenth (two-term operand, column-split
    pass) against the oracle's Gram; Rayleigh-Ritz against the oracle's on the
    same G and B; a basis holding the top eigenvectors returns them."""
    P, data, xs, lam, b = wide
    # unit-norm eigenvectors plus a perturbation of norm about 1e-3 per column:
    # the span then lies within ~1e-3 of the top eigenvectors and the Ritz
    # values within ~1e-6 of lam plus the bf16 rounding of the stored X
    v = (b[:, :K] + 1e-3 / np.sqrt(D) * gaussian_block(D, K, 93, np.float64)).astype(np.float32)
    vd = torch.from_numpy(v).cuda()
    veff = projection_basis(v, BF16, None)
    for r0, nrows in ((0, N), (300, N // 10)):
        if nrows == N:
            G, Bm = P.project_gram(data, K, vd)
        else:
            G, Bm = P.project_gram_rows(data, K, vd, r0, nrows)
        torch.cuda.synchronize()
        rows = (r0 + np.arange(nrows)) % N
        g_ref, b_ref = O.project_gram(xs[rows], veff)
        assert gram_err(G.cpu().numpy(), g_ref) < 4e-3
        assert np.allclose(Bm.cpu().numpy(), b_ref, rtol=1e-12, atol=1e-12 * np.abs(b_ref).max())
    ev, E = P.ppca(data, vd, 4)
    torch.cuda.synchronize()
    G, Bm = P.project_gram(data, K, vd)
    th, e_ref, _ = O.rayleigh_ritz(G.cpu().numpy(), Bm.cpu().numpy(), veff, N, 4)
    assert np.max(O.rel_eig_error(ev.cpu().numpy(), th)) < 1e-8
    # Ritz vectors with their signs: the rotation spans 1024 workgroups here,
    # so the sign rule's column maxima are merged across workgroups; every
    # column must match the oracle's sign-normalised one in every row
    e = E.cpu().numpy().astype(np.float64)
    signed = np.sum(e * e_ref, axis=0) / (np.linalg.norm(e, axis=0) *
                                          np.linalg.norm(e_ref, axis=0))
    assert np.min(signed) > 1 - 1e-9
    piv = np.argmax(np.abs(e), axis=0)
    assert np.all(e[piv, np.arange(4)] > 0)
    e_lam = np.max(O.rel_eig_error(ev.cpu().numpy(), lam[:4]))
    s_b = sin_theta(E.cpu().numpy(), b[:, :4])
    print(f"[wide] Ritz values vs lam {e_lam:.2e}, Ritz vectors vs B {s_b:.2e}", flush=True)
    assert e_lam < 1e-3
    assert s_b < 5e-3


def test_wide_eigengame_momentum_matches_oracle(wide):
    """Nesterov momentum at d = 262,144: the update's six column sums (with the
    momentum buffer) go through the two-level reduction over 1024 blocks; four
    steps against the oracle's own loop on the same rows and operand."""
    P, data, xs, lam, b = wide
    v0 = gaussian_block(D, K, 94, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    mom = torch.zeros_like(V)
    P.prime_eigengame(data, 4, 4, V, batch=B, steps=4, eta0=0.2, momentum=0.9, nesterov=True,
                      mom_buf=mom)
    torch.cuda.synchronize()
    hook = lambda u: operand_basis(u.astype(np.float32), BF16, None)
    v, m = O.prime_eigengame(xs, v0.astype(np.float64), batch=B, steps=4, eta0=0.2, t0=0.0,
                             momentum=0.9, nesterov=True, operand=hook)
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    err = trajectory_error(V.cpu().numpy(), v, v_start)
    merr = float(np.linalg.norm(mom.cpu().numpy() - m) / np.linalg.norm(m))
    print(f"[wide] EigenGame + Nesterov trajectory error {err:.2e}, buffer {merr:.2e}", flush=True)
    assert err < TRAJ_REL
    assert merr < TRAJ_REL


def test_wide_oja_matches_oracle(wide):
    """Minibatch Sanger/Oja at d = 262,144 (eight rows per thread in the
    update, the operand written by the update): four steps against the
    oracle's loop on the same rows and operand."""
    P, data, xs, lam, b = wide
    v0 = gaussian_block(D, K, 95, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    P.prime_oja(data, 4, 4, V, batch=B, steps=4, eta0=0.5, t0=1000.0)
    torch.cuda.synchronize()
    hook = lambda u: operand_basis(u.astype(np.float32), BF16, None)
    v, _ = O.prime_oja(xs, v0.astype(np.float64), batch=B, steps=4, eta0=0.5, t0=1000.0,
                       operand=hook)
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    err = trajectory_error(V.cpu().numpy(), v, v_start)
    print(f"[wide] Oja trajectory error {err:.2e}", flush=True)
    assert err < TRAJ_REL


def test_wide_ragged_width():
    """Long rows that end inside a 16-byte chunk (d = 262,150 in rows of
    262,152): the column-split minibatch pass and the two-term projection mask
    the tail; one EigenGame step and the Gram against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as P
    n, d, ld, k = 512, 262_150, 262_152, 8
    # structured rows (a low-rank matrix, viewed at the ragged width): on
    # isotropic rows the bf16 rounding of Y adds up like the signal and alone
    # reaches the 2^-9 bound
    buf, _, _ = make_lowrank_device(n, ld, 16, "exp0.9", seed=96)
    data = P.Data(buf[:, :d], P.BF16)
    xs = stored_values(host(buf[:, :d].contiguous()), BF16, None)
    v0 = gaussian_block(d, k, 97, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    P.prime_eigengame(data, 4, 4, V, batch=256, steps=2, eta0=0.5)
    G, Bm = P.project_gram(data, k, V)
    torch.cuda.synchronize()
    hook = lambda u: operand_basis(u.astype(np.float32), BF16, None)
    v_start = O.cholqr2(v0.astype(np.float64))[0]
    v = oracle_replay("eigengame", lambda t: xs[O.minibatch_rows(n, 256, t)], v_start, range(2),
                      256, 0.5, 0.0, hook)
    err = trajectory_error(V.cpu().numpy(), v, v_start)
    vg = V.cpu().numpy()
    g_ref, b_ref = O.project_gram(xs, projection_basis(vg, BF16, None))
    print(f"[wide] ragged d: EigenGame {err:.2e} of the motion, Gram {gram_err(G.cpu().numpy(), g_ref):.2e}",
          flush=True)
    assert err < TRAJ_REL
    assert gram_err(G.cpu().numpy(), g_ref) < 4e-3
    assert np.allclose(Bm.cpu().numpy(), b_ref, rtol=1e-12, atol=1e-12 * np.abs(b_ref).max())
