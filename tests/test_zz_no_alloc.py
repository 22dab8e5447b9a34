"""The allocation-free Rayleigh-Ritz entry point (fixed device scratch) gives
the same results as ppca_rayleigh_ritz with a caller workspace, on two calls
in a row with the second smaller than the first (the scratch keeps the first
call's contents, which must not leak into the second)."""
import numpy as np
import pytest
import torch

from synthdata import gaussian_block, make_problem
from tests._gpu_util import BF16, F32, FP8, device_data

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03709_amd as mod
    mod.lib()        # fails loudly if the library is missing
    yield


def P():
    import paper_2109_03709_amd as mod
    return mod


def _case(n, d, K, k, dtype, seed):
    p = make_problem(n, d, "exp0.9", seed=seed, mode="gaussian")
    data, _, _ = device_data(p.x, dtype)
    v = gaussian_block(d, K, seed + 1, np.float32) + p.q[:, :K].astype(np.float32)
    vd = torch.from_numpy(v).cuda()
    G, B = P().project_gram(data, K, vd)
    return data, vd, G, B


@pytest.mark.parametrize("dtype", [F32, BF16, FP8])
def test_noalloc_matches_workspace_entry_point(dtype):
    cases = [(6000, 3000, 64, 20), (900, 500, 16, 5)]     # second call smaller
    for i, (n, d, K, k) in enumerate(cases):
        print(f"noalloc RR: dtype {dtype} n {n} d {d} K {K} k {k}", flush=True)
        data, vd, G, B = _case(n, d, K, k, dtype, 300 + 10 * i + dtype)
        ev_ws, E_ws = P().rayleigh_ritz(data, K, k, G, B, vd)
        ev = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
        E = torch.full((d, k), float("nan"), dtype=torch.float32, device="cuda")
        P().rayleigh_ritz_noalloc(data, K, k, G, B, vd, ev, E)
        torch.cuda.synchronize()
        # same kernels on the same inputs: bitwise equal
        assert torch.equal(ev, ev_ws), (ev - ev_ws).abs().max().item()
        assert torch.equal(E, E_ws), (E - E_ws).abs().max().item()
        # eigenvalues only
        ev2 = torch.zeros(k, dtype=torch.float64, device="cuda")
        P().rayleigh_ritz_noalloc(data, K, k, G, B, vd, ev2, None)
        torch.cuda.synchronize()
        assert torch.equal(ev2, ev_ws)


def test_noalloc_wide_problem():
    """A problem far wider than the fixed scratch could hold a d x K buffer of
    (d = 2,000,000, bf16, K = 32): the allocation-free call still runs (its
    workspace does not grow with d) and equals the workspace entry point."""
    n, d, K, k = 64, 2_000_000, 32, 8
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    x = torch.randn((n, d), generator=g, device="cuda").to(torch.bfloat16)
    data = P().Data(x, BF16)
    vd = torch.randn((d, K), generator=g, device="cuda")
    G, B = P().project_gram(data, K, vd)
    ev_ws, E_ws = P().rayleigh_ritz(data, K, k, G, B, vd)
    ev = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
    E = torch.full((d, k), float("nan"), dtype=torch.float32, device="cuda")
    P().rayleigh_ritz_noalloc(data, K, k, G, B, vd, ev, E)
    torch.cuda.synchronize()
    assert torch.equal(ev, ev_ws)
    assert torch.equal(E, E_ws)
