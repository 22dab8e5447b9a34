"""Parity at the full size of the streaming workload: n = 2,000,000 rows,
d = 2048, bf16 storage, K = 128 (k = l = 64), 15 power iterations, the same
seeded data recipe and launch configuration as the benchmark's default run.

The oracle cannot run the whole path at this size, so the test checks
sampled outputs against their definition, in float64 on the CPU, with X
brought to the host in row chunks:
* four whole columns of Z = X^T (X V') from the power step's kernels, against
  the same elementwise bound as the smaller stream-pass cases;
* the 4 x 4 block of G = (X V')^T (X V') of those columns from the projection
  pass (two-term operand V' = hi + lo), and B = V'^T V' in full;
* the end-to-end result (priming, projection, Rayleigh-Ritz) against the
  exact spectrum of the data: eigenvalue relative error and largest
  principal-angle sine within 2e-3, orthonormal Ritz vectors.
The minibatch workloads (Oja on f32 data, EigenGame on fp8 data) are checked
at their full sizes on the steps whose rows wrap past the end of the data, and
the 512-problem grouped workload on one step of sampled problems and on every
problem's result against its exact spectrum.
"""
import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O
from synthdata import gaussian_block, make_problem_device

from ._gpu_util import (BF16, F32, FP8, TRAJ_REL, gram_err, operand_basis, oracle_replay,
                        projection_basis, sin_theta, stored_values, trajectory_error)

pytestmark = pytest.mark.gpu

N, D, KK, LL, ITERS = 2_000_000, 2048, 64, 64, 15
SEED = 1003
COLS = [0, 37, 64, 127]        # sampled columns of Z and G: both MFMA N-blocks, both halves
CHUNK = 1 << 16


@pytest.fixture(scope="module")
def workload():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as P
    P.lib()        # fails loudly if the library is missing
    P.set_chunk_rows(0)
    dev = torch.device("cuda:0")
    print(f"[fullsize] generating X {N} x {D}", flush=True)
    xraw, lam, q = make_problem_device(N, D, "exp0.9", SEED, device=dev)
    X, _ = P.center_quantize(xraw, BF16)
    del xraw
    torch.cuda.synchronize()
    yield P, X, lam, q
    del X
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_full_size_stream_and_projection_sampled(workload):
    P, X, _, _ = workload
    K = KK + LL
    v = gaussian_block(D, K, SEED + 1000, np.float32)
    V = torch.from_numpy(v).cuda()
    Z, _ = P.stream_pass(X, K, V, want_g=False)     # the power step's kernels
    G, B = P.project_gram(X, K, V)                   # the projection pass
    torch.cuda.synchronize()
    zs = Z.cpu().numpy().astype(np.float64)[:, COLS]
    gs = G.cpu().numpy()[np.ix_(COLS, COLS)]
    bh = B.cpu().numpy()

    veff = operand_basis(v, BF16, None)              # bf16(V), float64: power step
    vpro = projection_basis(v, BF16, None)           # hi + lo: projection
    vc = torch.from_numpy(np.ascontiguousarray(veff[:, COLS]))
    vp = torch.from_numpy(np.ascontiguousarray(vpro[:, COLS]))
    z_ref = torch.zeros((D, len(COLS)), dtype=torch.float64)
    z_bnd = torch.zeros((D, len(COLS)), dtype=torch.float64)
    g_ref = torch.zeros((len(COLS), len(COLS)), dtype=torch.float64)
    print("[fullsize] host reference over row chunks", flush=True)
    for r0 in range(0, N, CHUNK):
        xc = X.x[r0:r0 + CHUNK].cpu().double()       # bf16 -> float64 is exact
        y = xc @ vc
        z_ref += xc.T @ y
        z_bnd += xc.abs().T @ y.abs()
        yp = xc @ vp
        g_ref += yp.T @ yp
    z_ref, z_bnd, g_ref = z_ref.numpy(), z_bnd.numpy(), g_ref.numpy()

    # Y' = bf16(Y) feeds Z: each term is off by at most 2^-8 of |x||y|
    assert np.all(np.abs(zs - z_ref) <= 2.0 ** -8 * z_bnd + 1e-30)
    assert gram_err(gs, g_ref) < 4e-3
    assert gram_err(bh, vpro.T @ vpro) < 1e-12


@pytest.mark.timeout(600)
def test_full_size_ppca_against_exact_spectrum(workload):
    P, X, lam, q = workload
    K = KK + LL
    v0 = torch.from_numpy(gaussian_block(D, K, SEED + 1000, np.float32)).cuda()
    V = v0.clone()
    P.prime_power(X, KK, LL, ITERS, V)
    G, B = P.project_gram(X, K, V)
    ev, E = P.rayleigh_ritz(X, K, KK, G, B, V)
    torch.cuda.synchronize()
    evh = ev.cpu().numpy()
    Eh = E.cpu().numpy().astype(np.float64)
    assert np.all(np.diff(evh) <= 0)
    assert np.max(O.rel_eig_error(evh, lam[:KK])) < 2e-3
    assert np.max(np.abs(Eh.T @ Eh - np.eye(KK))) < 1e-5
    s_exact = sin_theta(Eh, q[:, :KK])
    print(f"[fullsize] sin theta vs exact subspace: {s_exact:.3e}", flush=True)
    assert s_exact < 2e-3


# ------------------------------------------------ minibatch primings, full size
def _stored_rows(X, rows: np.ndarray, dtype: int) -> np.ndarray:
    """float64 values of the given rows of the device data (codes x scales)."""
    codes = X.x[torch.from_numpy(rows).cuda()].cpu()
    if codes.dtype == torch.bfloat16:
        codes = codes.view(torch.int16)
    scale = None if X.col_scale is None else X.col_scale.cpu().numpy()
    return stored_values(codes.numpy(), dtype, scale)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["eigengame-fp8", "oja-f32"])
def test_full_size_minibatch_steps_across_the_wrap(name):
    """The minibatch workloads at their full size (EigenGame: 8,000,000 x 2048
    fp8, batch 4096, K = 64; Oja: 1,000,000 x 1024 f32, batch 1024, K = 64),
    three steps resumed from the step whose rows wrap past the end of the
    data.  The oracle replays the same steps on the rows the schedule names
    (fetched from the device as stored), with the same bounds as the
    trajectory tests."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as P
    P.lib()
    cfg = {"eigengame-fp8": dict(n=8_000_000, d=2048, spec="exp0.97+1e-5", dtype=FP8, k=32,
                                 l=32, b=4096, eta0=0.2, t0=0.0, seed=1004),
           "oja-f32": dict(n=1_000_000, d=1024, spec="pow1.2+1e-4", dtype=F32, k=32, l=32,
                           b=1024, eta0=0.5, t0=1000.0, seed=1002)}[name]
    n, d, b, dtype = cfg["n"], cfg["d"], cfg["b"], cfg["dtype"]
    K = cfg["k"] + cfg["l"]
    t_first = n // b - 1                  # the next step's rows wrap past row n - 1
    assert (t_first + 1) * b < n < (t_first + 2) * b
    steps = 3
    print(f"[fullsize] {name}: generating X {n} x {d}", flush=True)
    xraw, _, _ = make_problem_device(n, d, cfg["spec"], cfg["seed"], device=torch.device("cuda:0"))
    X, _ = P.center_quantize(xraw, dtype, out=xraw if dtype == F32 else None)
    if dtype != F32:
        del xraw
    v0 = gaussian_block(d, K, cfg["seed"] + 1000, np.float32)
    V = torch.from_numpy(v0.copy()).cuda()
    fn = P.prime_eigengame if dtype == FP8 else P.prime_oja
    fn(X, cfg["k"], cfg["l"], V, batch=b, steps=steps, eta0=cfg["eta0"], t0=cfg["t0"],
       start_step=t_first)
    torch.cuda.synchronize()
    scale = None if X.col_scale is None else X.col_scale.cpu().numpy()

    v_start = O.cholqr2(v0.astype(np.float64))[0]
    v = oracle_replay("eigengame" if dtype == FP8 else "oja",
                      lambda t: _stored_rows(X, O.minibatch_rows(n, b, t), dtype), v_start,
                      range(t_first, t_first + steps), b, cfg["eta0"], cfg["t0"],
                      lambda u: operand_basis(u.astype(np.float32), dtype, scale))
    vg = V.cpu().numpy()
    del X
    torch.cuda.empty_cache()
    if dtype == FP8:
        assert trajectory_error(vg, v, v_start) < TRAJ_REL
    else:
        assert np.max(np.abs(vg - v)) / np.max(np.abs(v)) < 1e-4


# ---------------------------------------------- grouped problems, full size
@pytest.fixture(scope="module")
def grouped_workload():
    """The 512-problem grouped workload of the benchmark (15.4 GB of bf16
    data: n from 2,000 to 200,000, d in {64, ..., 768}, k = l in 4..32), same
    shape, data and start seeds."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    import paper_2109_03709_amd as P
    P.lib()
    c = bench.GROUPED
    shapes = bench.grouped_shapes(c)
    print(f"[fullsize] generating {len(shapes)} grouped problems", flush=True)
    data, refs, v0s = [], [], []
    for p, (n, d, k, l, spec) in enumerate(shapes):
        xraw, lam, q = make_problem_device(n, d, spec, c["data_seed"] + p,
                                           device=torch.device("cuda:0"))
        X, _ = P.center_quantize(xraw, BF16)
        del xraw
        data.append(X)
        refs.append((lam[:k].copy(), q[:, :k].copy()))
        v0s.append(gaussian_block(d, k + l, c["v0_seed"] + p, np.float32))
    torch.cuda.synchronize()
    yield P, c, shapes, data, refs, v0s
    P.set_group_item_bytes(0)
    del data
    torch.cuda.empty_cache()


def _grouped_problems(P, shapes, data, v0s):
    return [P.Problem(X, k, l, torch.from_numpy(v0.copy()).cuda()).alloc()
            for X, (n, d, k, l, _), v0 in zip(data, shapes, v0s)]


@pytest.mark.timeout(600)
def test_full_size_grouped_one_step_sampled(grouped_workload):
    """One fused power step over all 512 problems; the smallest, the tallest
    and the widest-and-deepest problems against the oracle's step on their
    stored data (sin theta 2e-2, the bound of the small grouped cases)."""
    P, _, shapes, data, _, v0s = grouped_workload
    probs = _grouped_problems(P, shapes, data, v0s)
    P.prime_power_grouped(probs, 1)
    torch.cuda.synchronize()
    dims = np.array([(n, d, k + l) for (n, d, k, l, _) in shapes], dtype=np.int64)
    picks = sorted({int(np.argmin(dims[:, 0] * dims[:, 1])), int(np.argmax(dims[:, 0])),
                    int(np.argmax(dims[:, 1] * 1000 + dims[:, 2]))})
    for i in picks:
        n, d, k, l, _ = shapes[i]
        xs = stored_values(data[i].x.cpu().view(torch.int16).numpy(), BF16, None)
        v = O.cholqr2(v0s[i].astype(np.float64))[0]
        z, _ = O.stream_pass(xs, operand_basis(v.astype(np.float32), BF16, None))
        v1 = O.cholqr2(z)[0]
        s1 = sin_theta(probs[i].V.cpu().numpy(), v1)
        assert s1 < 2e-2, f"problem {i}: n={n} d={d} K={k + l}: {s1:.2e}"


@pytest.mark.timeout(600)
def test_full_size_grouped_against_exact_spectra(grouped_workload):
    """The benchmark's whole grouped step (work split from the autotuner, 12
    iterations, projection, Rayleigh-Ritz): every problem's eigenvalues within
    2e-3 of its exact spectrum, orthonormal Ritz vectors, and subspaces within
    the 1e-2 quantisation bound."""
    P, c, shapes, data, refs, v0s = grouped_workload
    probs = _grouped_problems(P, shapes, data, v0s)
    best, _ = P.tune_group_items(probs)
    P.set_group_item_bytes(best)
    P.prime_power_grouped(probs, c["iters"])
    P.rayleigh_ritz_grouped(probs)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (p, (lam_k, q_k)) in enumerate(zip(probs, refs)):
        ev = p.evals.cpu().numpy()
        E = p.E.cpu().numpy().astype(np.float64)
        k = lam_k.size
        assert np.max(O.rel_eig_error(ev, lam_k)) < 2e-3, f"problem {i}"
        assert np.max(np.abs(E.T @ E - np.eye(k))) < 1e-5, f"problem {i}"
        s_i = sin_theta(E, q_k)
        worst = max(worst, s_i)
        assert s_i < 1e-2, f"problem {i}"
    print(f"[grouped] largest sin theta vs exact subspace over 512 problems: {worst:.2e}", flush=True)
