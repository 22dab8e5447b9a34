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
