"""Parity at the full size of the streaming workload: n = 2,000,000 rows,
d = 2048, bf16 storage, K = 128 (k = l = 64), 15 power iterations, the same
seeded data recipe and launch configuration as the benchmark's default run.

The oracle cannot run the whole path at this size, so the test checks
sampled outputs against their definition, in float64 on the CPU, with X
brought to the host in row chunks:
* four whole columns of Z = X^T (X V') from the power step's kernels, against
  the same elementwise bound as the smaller stream-pass cases;
* the 4 x 4 block of G = (X V')^T (X V') of those columns from the projection
  pass, and the operand Gram B = V'^T V' in full;
* the end-to-end result (priming, projection, Rayleigh-Ritz) against the
  exact spectrum of the data: eigenvalue relative error 2e-3, orthonormal
  Ritz vectors, and the subspace within the 1e-2 quantisation bound of the
  scaled bf16 case.
"""
import numpy as np
import pytest
import torch

from oracle import ppca_oracle as O
from synthdata import gaussian_block, make_problem_device

from ._gpu_util import BF16, gram_err, operand_basis, sin_theta

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

    veff = operand_basis(v, BF16, None)              # bf16(V), float64
    vc = torch.from_numpy(np.ascontiguousarray(veff[:, COLS]))
    z_ref = torch.zeros((D, len(COLS)), dtype=torch.float64)
    z_bnd = torch.zeros((D, len(COLS)), dtype=torch.float64)
    g_ref = torch.zeros((len(COLS), len(COLS)), dtype=torch.float64)
    print("[fullsize] host reference over row chunks", flush=True)
    for r0 in range(0, N, CHUNK):
        xc = X.x[r0:r0 + CHUNK].cpu().double()       # bf16 -> float64 is exact
        y = xc @ vc
        z_ref += xc.T @ y
        z_bnd += xc.abs().T @ y.abs()
        g_ref += y.T @ y
    z_ref, z_bnd, g_ref = z_ref.numpy(), z_bnd.numpy(), g_ref.numpy()

    # Y' = bf16(Y) feeds Z: each term is off by at most 2^-8 of |x||y|
    assert np.all(np.abs(zs - z_ref) <= 2.0 ** -8 * z_bnd + 1e-30)
    assert gram_err(gs, g_ref) < 4e-3
    assert gram_err(bh, veff.T @ veff) < 1e-12


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
    assert sin_theta(Eh, q[:, :KK]) < 1e-2
