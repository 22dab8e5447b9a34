"""The minibatch trajectory bound of the GPU tests can fail (CPU only).

The GPU parity tests hold low-precision minibatch trajectories (EigenGame on
fp8 data, Sanger on bf16 data) to |V_gpu - V_or|_F <= TRAJ_REL |V_or - V_start|_F
against the oracle's own loop.  Here, on the shapes those tests run (the
full-size EigenGame workload: d = 2048, K = 64, batch 4096, eta = 0.2, three
steps on fp8-e4m3 data with column scales; the Sanger trajectory case: d =
256, K = 32, batch 1024, five steps on bf16 data), a replay of the GPU's
arithmetic (Y rounded to bf16 before the second product, Z and V kept in
float32) stays well inside the bound, while the plausible mistakes all fail
it: a step that does nothing, half the rate, the tangent projection of the
EigenGame step (Sec. 2.3) dropped, the triangular term of the Sanger rule
(Sec. 2.2) dropped.
"""
import numpy as np
import pytest

from oracle import ppca_oracle as O
from synthdata import gaussian_block, make_problem

from ._gpu_util import BF16, FP8, TRAJ_REL, operand_basis, oracle_replay, trajectory_error
from .test_oracle_priming import _eigengame_mutant_without_projection


def _stored(x32, dtype):
    c = O.center_fp32(x32, O.column_means(x32))
    if dtype == BF16:
        return O.bf16_value(O.bf16_round(c)), None
    s = O.fp8_column_scales(c)
    return O.e4m3_value(O.fp8_quantize(c, s)) * s.astype(np.float64)[None, :], s


def _gpu_like_step(method, xb, v, eta, dtype, scale, b):
    """One step with the GPU's roundings: operand V', Y' = bf16(X V'),
    Z = fl32(X^T Y'), G = Y'^T Y', the update in float64, V stored as float32."""
    y = xb @ operand_basis(v.astype(np.float32), dtype, scale)
    y = O.bf16_value(O.bf16_round(y.astype(np.float32)))
    z = (xb.T @ y).astype(np.float32).astype(np.float64)
    g = y.T @ y
    if method == "eigengame":
        grad = O.eigengame_grad(z, g, b)
        grad = grad - v * np.sum(v * grad, axis=0)[None, :]
        vn = v + eta * grad
        vn = vn / np.linalg.norm(vn, axis=0)[None, :]
    else:
        vn = v + eta * O.sanger_direction(z, g, v, b)
    return vn.astype(np.float32).astype(np.float64)


CASES = {
    "eigengame-fp8-full-size": dict(method="eigengame", dtype=FP8, n=None, d=2048, K=64, b=4096,
                                    steps=3, eta0=0.2, t0=0.0, spec="exp0.97+1e-5", mode="gaussian"),
    "oja-bf16-trajectory": dict(method="oja", dtype=BF16, n=20000, d=256, K=32, b=1024, steps=5,
                                eta0=0.5, t0=1000.0, spec="pow1.2+1e-4", mode="exact"),
}


@pytest.mark.slow
@pytest.mark.parametrize("case", list(CASES))
def test_trajectory_bound_discriminates(case):
    c = CASES[case]
    b, steps, dtype = c["b"], c["steps"], c["dtype"]
    n = c["n"] or steps * b
    p = make_problem(n, c["d"], c["spec"], seed=31, mode=c["mode"])
    xs, scale = _stored(p.x.astype(np.float32), dtype)
    v_start = O.cholqr2(gaussian_block(c["d"], c["K"], 32, np.float32).astype(np.float64))[0]
    op = lambda v: operand_basis(v.astype(np.float32), dtype, scale)
    rows = lambda t: xs[O.minibatch_rows(n, b, t)]
    replay = lambda eta0, fn=None: (
        oracle_replay(c["method"], rows, v_start, range(steps), b, eta0, c["t0"], op) if fn is None
        else _replay_with(fn, rows, v_start, steps, b, eta0, c["t0"], op))
    v_or = replay(c["eta0"])

    v = v_start.astype(np.float32).astype(np.float64)
    for t in range(steps):
        v = _gpu_like_step(c["method"], rows(t), v, O.learning_rate(c["eta0"], c["t0"], t), dtype,
                           scale, b)
    assert trajectory_error(v, v_or, v_start) < TRAJ_REL / 4

    assert trajectory_error(v_start, v_or, v_start) > TRAJ_REL           # no step at all
    assert trajectory_error(replay(c["eta0"] / 2), v_or, v_start) > TRAJ_REL
    if c["method"] == "eigengame":
        mutant = _eigengame_mutant_without_projection()
        assert trajectory_error(replay(c["eta0"], mutant), v_or, v_start) > TRAJ_REL
    else:
        v = v_start.copy()
        for t in range(steps):
            xb = rows(t)
            z, g = O.stream_pass(xb, op(v))
            v = v + O.learning_rate(c["eta0"], c["t0"], t) * (z - v @ np.diag(np.diag(g))) / b
        assert trajectory_error(v, v_or, v_start) > TRAJ_REL


def _replay_with(fn, rows, v_start, steps, b, eta0, t0, op):
    v = v_start
    for t in range(steps):
        v = fn(rows(t), v, batch=b, steps=1, eta0=O.learning_rate(eta0, t0, t), t0=0.0,
               orthonormalise_start=False, operand=op)[0]
    return v
