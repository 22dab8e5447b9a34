"""Helpers shared by the GPU parity tests: oracle-side views of the stored
data and of the operand basis (built with the oracle's own encoders), and
subspace/eigenvalue comparisons.  Nothing here calls the HIP library."""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import ppca_oracle as O

F32, BF16, FP8 = 0, 1, 2


def stored_values(xs_codes: np.ndarray, dtype: int, scale: np.ndarray | None) -> np.ndarray:
    """float64 values of the stored matrix (codes as the device holds them)."""
    if dtype == F32:
        return xs_codes.astype(np.float64)
    if dtype == BF16:
        return O.bf16_value(xs_codes.view(np.uint16))
    return O.e4m3_value(xs_codes.view(np.uint8)) * scale.astype(np.float64)[None, :]


def operand_basis(v32: np.ndarray, dtype: int, scale: np.ndarray | None) -> np.ndarray:
    """V_eff: the basis the stored data is multiplied with (f32: V; bf16:
    bf16(V); fp8: bf16(s_j V_jc) / s_j), float64."""
    v32 = np.asarray(v32, np.float32)
    if dtype == F32:
        return v32.astype(np.float64)
    if dtype == BF16:
        return O.bf16_value(O.bf16_round(v32))
    sv = (scale.astype(np.float32)[:, None] * v32).astype(np.float32)
    return O.bf16_value(O.bf16_round(sv)) / scale.astype(np.float64)[:, None]


def projection_basis(v32: np.ndarray, dtype: int, scale: np.ndarray | None) -> np.ndarray:
    """V_eff of the projection pass and of Rayleigh-Ritz: for bf16 data the
    two-term operand hi + lo, hi = bf16(V), lo = bf16(V - hi) (V - hi is exact
    in float32); for f32 and fp8 data the single operand of operand_basis."""
    if dtype != BF16:
        return operand_basis(v32, dtype, scale)
    v32 = np.asarray(v32, np.float32)
    hi = O.bf16_value(O.bf16_round(v32))
    rest = (v32.astype(np.float64) - hi).astype(np.float32)
    return hi + O.bf16_value(O.bf16_round(rest))


def host(t: torch.Tensor) -> np.ndarray:
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def sin_theta(a: np.ndarray, b: np.ndarray) -> float:
    """Largest principal-angle sine between span(a) and span(b)."""
    qa = np.linalg.qr(np.asarray(a, np.float64))[0]
    qb = np.linalg.qr(np.asarray(b, np.float64))[0]
    w = qa - qb @ (qb.T @ qa)
    return float(np.linalg.norm(w, 2))


def col_cos(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(np.sum(a * b, axis=0)) / (np.linalg.norm(a, axis=0) * np.linalg.norm(b, axis=0))


def gram_err(g_gpu: np.ndarray, g_ref: np.ndarray) -> float:
    """max |dG_ij| / sqrt(G_ii G_jj) (scale-free error of a Gram matrix)."""
    dg = np.sqrt(np.abs(np.diag(g_ref)))
    den = np.outer(dg, dg)
    den[den == 0] = 1.0
    return float(np.max(np.abs(g_gpu - g_ref) / den))


def aligned_ld(d: int, dtype: int) -> int:
    """Smallest row stride >= d whose byte size is a multiple of 16."""
    es = {F32: 4, BF16: 2, FP8: 1}[dtype]
    return int(math.ceil(d * es / 16) * 16 // es)


def device_data(x32: np.ndarray, dtype: int, ld: int | None = None):
    """Centre and store host float32 data on the GPU through the library.
    Returns (Data, host float64 values of the stored matrix, host scale)."""
    import paper_2109_03709_amd as P
    n, d = x32.shape
    ld = aligned_ld(max(d, ld or d), dtype)
    xd = torch.from_numpy(np.ascontiguousarray(x32)).cuda()
    if ld == d:
        data, _ = P.center_quantize(xd, dtype)
    else:
        tdt = {F32: torch.float32, BF16: torch.bfloat16, FP8: torch.uint8}[dtype]
        buf = torch.zeros((n, ld), dtype=tdt, device="cuda")
        data, _ = P.center_quantize(xd, dtype, out=buf[:, :d])
    torch.cuda.synchronize()
    scale = None if data.col_scale is None else data.col_scale.cpu().numpy()
    codes = host(data.x.contiguous())
    return data, stored_values(codes, dtype, scale), scale


# ---------------------------------------------------- minibatch trajectories
# On low-precision data the GPU multiplies X by the rounded operand V' (which
# the oracle models through its `operand` hook) and rounds Y = X V' to bf16
# before the second product (which the oracle does not model: it is part of
# the kernel's arithmetic, not of the method).  That rounding, unit roundoff
# 2^-9, perturbs each step's direction to first order, so the distance between
# the two trajectories is bounded relative to how far V moved:
#     |V_gpu - V_or|_F <= TRAJ_REL |V_or - V_start|_F.
# tests/test_trajectory_bounds.py shows on the CPU that a replay of the GPU's
# roundings stays an order of magnitude inside it, while a step that does
# nothing, a halved rate, a dropped tangent projection (EigenGame) or a dropped
# triangular term (Sanger) all fail it, at the full-size fp8 EigenGame shape.
TRAJ_REL = 2.0 ** -9


def trajectory_error(v_gpu, v_or, v_start) -> float:
    """|V_gpu - V_or|_F / |V_or - V_start|_F."""
    v_or = np.asarray(v_or, np.float64)
    return float(np.linalg.norm(np.asarray(v_gpu, np.float64) - v_or) /
                 np.linalg.norm(v_or - np.asarray(v_start, np.float64)))


def oracle_replay(method: str, rows_of_step, v_start, steps, batch: int, eta0: float,
                  t0: float, operand=None):
    """The oracle's own minibatch loop (prime_oja / prime_eigengame), one step
    at a time on the rows the schedule names: rows_of_step(t) returns the
    float64 rows of step t, and the step's rate eta_t = eta0 / (1 + t/t0) is
    passed as a constant rate.  ``steps`` is an iterable of global step
    indices.  Returns V after the last step."""
    fn = {"oja": O.prime_oja, "eigengame": O.prime_eigengame}[method]
    v = np.asarray(v_start, np.float64)
    for t in steps:
        v = fn(rows_of_step(t), v, batch=batch, steps=1, eta0=O.learning_rate(eta0, t0, t),
               t0=0.0, orthonormalise_start=False, operand=operand)[0]
    return v


# ------------------------------------------------------ exact-arithmetic data
# Inputs on which every rounding of the GPU path is exact: codes in {-1, 0, 1}
# (fp8: times a power-of-two column scale), and directions with at most two
# nonzeros per column, each in {+-1, +-1/2}, on a small set of rows.  Then
# V' = bf16(V) (fp8: bf16(s_j V_jc)) equals V, every Y = X V' is a multiple of
# 1/2 of magnitude <= 1 (exact in bf16), and every float32 partial of Z and G
# is a multiple of 1/4 below 2^21 (n <= 2^21 rows), so Z and G must equal
# their float64 values exactly.
E4M3_ONE, E4M3_MINUS_ONE = 0x38, 0xB8


def exact_codes(n: int, d: int, dtype: int, seed: int, device="cuda"):
    """(Data on the device, per-column scale or None).  Codes drawn on the
    device (so that multi-GB cases need no host copy of X)."""
    import paper_2109_03709_amd as P
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    ld = aligned_ld(d, dtype)              # 16-byte row stride; X is the view [:, :d]
    c = torch.randint(-1, 2, (n, ld), generator=g, device=device, dtype=torch.int8)
    if dtype == F32:
        return P.Data(c.float()[:, :d], F32), None
    if dtype == BF16:
        return P.Data(c.to(torch.bfloat16)[:, :d], BF16), None
    codes = torch.where(c > 0, torch.tensor(E4M3_ONE, dtype=torch.uint8, device=device),
                        torch.where(c < 0, torch.tensor(E4M3_MINUS_ONE, dtype=torch.uint8,
                                                        device=device),
                                    torch.tensor(0, dtype=torch.uint8, device=device)))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    scale = np.ldexp(1.0, rng.integers(-3, 1, d)).astype(np.float32)
    return P.Data(codes[:, :d], FP8, torch.from_numpy(scale).to(device)), scale


def exact_directions(d: int, K: int, seed: int, rows_used: int = 48) -> np.ndarray:
    """d x K float32 with at most two nonzeros per column, in {+-1, +-1/2},
    on a set of at most rows_used rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = rng.choice(d, size=min(rows_used, d), replace=False)
    v = np.zeros((d, K), np.float32)
    vals = np.array([1.0, -1.0, 0.5, -0.5], np.float32)
    for c in range(K):
        nz = rng.choice(rows, size=min(2, len(rows)), replace=False)
        v[nz, c] = rng.choice(vals, size=len(nz))
        if not np.any(v[:, c]):
            v[nz[0], c] = 1.0
    return v


def host_columns(data, cols: np.ndarray, scale, chunk: int = 1 << 18) -> np.ndarray:
    """float64 values of the stored matrix at the given columns (all rows)."""
    out = np.empty((data.n, len(cols)), np.float64)
    idx = torch.from_numpy(np.asarray(cols, np.int64)).to(data.x.device)
    for r0 in range(0, data.n, chunk):
        r1 = min(data.n, r0 + chunk)
        sub = data.x[r0:r1].index_select(1, idx)
        out[r0:r1] = stored_values(host(sub.contiguous()), data.dtype,
                                   None if scale is None else scale[cols])
    return out
