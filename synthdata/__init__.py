"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *draws* data: Gaussian samples, a Haar-orthogonal basis, a
spectrum, a column offset and a starting block V0.  It contains none of the
arithmetic of primed PCA (no power pass, no orthonormalisation of V, no
eigensolve of the data, no Rayleigh-Ritz).  Both sides of every parity check
receive the *same* arrays produced here.

Recipe (the workloads of the paper's synthetic study, Sec. 5 "Synthetic
data", and of the large single-GPU shapes used for measurement):

    X_raw = Z_w . diag(sqrt(lambda)) . Q^T + 1 mu^T

* ``lambda`` is a named spectrum (``spectrum()``), sorted descending.
* ``Q`` is Haar-orthogonal: Householder QR of a seeded d x d Gaussian with the
  sign fix Q <- Q diag(sign(diag R)).
* ``Z_w`` is an n x d Gaussian matrix.  In ``mode="exact"`` it is centred and
  whitened so that Z_w^T Z_w / n = I, which makes the covariance of the
  centred data exactly Q diag(lambda) Q^T (the reference spectrum is then
  known in closed form at any n).  In ``mode="gaussian"`` Z_w is the raw
  centred Gaussian sample (the plain recipe; its sample spectrum differs from
  lambda by O(sqrt(2/n))).
* ``mu`` is a seeded column offset, so that the centring step of the path has
  real work to do; centring removes it again.

Host generation uses numpy's PCG64 in float64; device generation (for the
multi-GB shapes) uses torch's CUDA generator and float64 GEMMs on the device.
Host and device data for the same seed are *different* samples: a test always
hands one array to both sides.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "spectrum",
    "haar",
    "make_problem",
    "make_problem_device",
    "gaussian_block",
    "Problem",
]


def spectrum(name: str, d: int) -> np.ndarray:
    """Named eigenvalue profiles (descending, float64, index i = 1..d).

    ``exp0.9``         lambda_i = 0.9**i
    ``exp0.97+1e-5``   lambda_i = 0.97**i + 1e-5
    ``pow1.2+1e-4``    lambda_i = i**-1.2 + 1e-4
    ``pow1.5``         lambda_i = i**-1.5
    ``paper-exp``      exponential decay from 1000 to 1 over d entries
    ``paper-lin``      linear decay from 1000 to 1 over d entries
    """
    i = np.arange(1, d + 1, dtype=np.float64)
    if name == "exp0.9":
        lam = 0.9 ** i
    elif name == "exp0.97+1e-5":
        lam = 0.97 ** i + 1e-5
    elif name == "pow1.2+1e-4":
        lam = i ** -1.2 + 1e-4
    elif name == "pow1.5":
        lam = i ** -1.5
    elif name == "paper-exp":
        lam = 1000.0 ** ((d - i) / max(d - 1, 1))
    elif name == "paper-lin":
        lam = 1000.0 - 999.0 * (i - 1) / max(d - 1, 1)
    else:
        raise ValueError(f"unknown spectrum {name!r}")
    return lam


def haar(d: int, seed: int) -> np.ndarray:
    """Haar-distributed orthogonal d x d matrix (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((d, d))
    q, r = np.linalg.qr(a)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def gaussian_block(rows: int, cols: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Seeded N(0,1) block, e.g. the starting directions V0 (d x K)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((rows, cols)).astype(dtype)


@dataclass
class Problem:
    x: np.ndarray          # n x d raw (uncentred) data, float32 or float64
    lam: np.ndarray        # spectrum used to build it (descending)
    q: np.ndarray          # d x d Haar basis; column i spans the i-th direction
    mu: np.ndarray         # column offset that was added (float64)
    mode: str


def _whiten_rows(z: np.ndarray) -> np.ndarray:
    z = z - z.mean(axis=0, keepdims=True)
    s = (z.T @ z) / z.shape[0]
    ell = np.linalg.cholesky(s)
    # z <- z L^{-T}  so that (z^T z)/n = I
    return np.linalg.solve(ell, z.T).T


def make_problem(n: int, d: int, spec: str | np.ndarray, seed: int, *,
                 mode: str = "exact", offset_scale: float = 0.25,
                 dtype=np.float32) -> Problem:
    """Host-side generator (numpy, float64 arithmetic, cast at the end)."""
    lam = spectrum(spec, d) if isinstance(spec, str) else np.asarray(spec, np.float64)
    q = haar(d, seed * 7919 + 17)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n, d))
    if mode == "exact":
        if n <= d:
            raise ValueError("exact mode needs n > d")
        z = _whiten_rows(z)
    elif mode == "gaussian":
        z = z - z.mean(axis=0, keepdims=True)
    else:
        raise ValueError(mode)
    x = (z * np.sqrt(lam)[None, :]) @ q.T
    mu = offset_scale * rng.standard_normal(d)
    x = x + mu[None, :]
    return Problem(x=x.astype(dtype), lam=lam, q=q, mu=mu, mode=mode)


def make_problem_device(n: int, d: int, spec: str, seed: int, *, device="cuda",
                        mode: str = "exact", offset_scale: float = 0.25,
                        chunk: int = 1 << 16):
    """Device-side generator for the multi-GB shapes (torch, float64 GEMMs).

    Returns (x_raw_fp32 [n, d] on ``device``, lam, q).  Rows are produced in
    chunks so that the float64 temporaries stay small.
    """
    import torch

    lam = spectrum(spec, d)
    q = haar(d, seed * 7919 + 17)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.empty((n, d), dtype=torch.float32, device=device)
    # 1. draw Z in chunks straight into x (float32), accumulate column sums
    colsum = torch.zeros(d, dtype=torch.float64, device=device)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        zc = torch.randn((r1 - r0, d), generator=g, device=device, dtype=torch.float32)
        x[r0:r1].copy_(zc)
        colsum += zc.double().sum(dim=0)
        del zc
    zmean = colsum / n
    if mode == "exact":
        s = torch.zeros((d, d), dtype=torch.float64, device=device)
        for r0 in range(0, n, chunk):
            r1 = min(n, r0 + chunk)
            zc = x[r0:r1].double() - zmean[None, :]
            s += zc.T @ zc
            del zc
        s = (s / n).cpu().numpy()
        ell = np.linalg.cholesky(s)
        w = np.linalg.inv(ell).T          # z <- z L^{-T}
    elif mode == "gaussian":
        w = np.eye(d)
    else:
        raise ValueError(mode)
    m = w @ (np.sqrt(lam)[:, None] * q.T)
    m_dev = torch.from_numpy(m).to(device)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    mu = torch.from_numpy(offset_scale * rng.standard_normal(d)).to(device)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        zc = x[r0:r1].double() - zmean[None, :]
        x[r0:r1].copy_((zc @ m_dev + mu[None, :]).float())
        del zc
    return x, lam, q


def make_lowrank_device(n: int, d: int, r: int, spec: str, seed: int, *, device="cuda",
                        chunk_rows: int = 32):
    """Centred data with an exact low-rank covariance, for d >> n (where a
    d x d Haar basis cannot be formed): X = A_w diag(sqrt(lam)) B^T with B a
    d x r block with orthonormal columns (Householder QR of a Gaussian block,
    float64) and A_w an n x r Gaussian block, centred and whitened so that
    A_w^T A_w / n = I.  Then X^T X / n = B diag(lam) B^T exactly: the top r
    eigenpairs are (lam_i, b_i) and the rest are zero.  X is written straight
    to bf16 (round to nearest even) in row chunks; nothing of size n x d is
    kept in float32.  Returns (X bf16 [n, d] on ``device``, lam [r], B float32
    [d, r] on ``device``)."""
    import torch

    lam = spectrum(spec, r)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    # orthonormal columns: Householder QR of a Gaussian block (library routine, float64)
    b = torch.linalg.qr(torch.randn((d, r), generator=g, device=device, dtype=torch.float64),
                        mode="reduced")[0].to(torch.float32)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    a = _whiten_rows(rng.standard_normal((n, r)))   # centred, A^T A / n = I
    a = a * np.sqrt(lam)[None, :]
    a_dev = torch.from_numpy(a).to(device=device, dtype=torch.float32)
    x = torch.empty((n, d), dtype=torch.bfloat16, device=device)
    bt = b.T.contiguous()
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        x[r0:r1] = (a_dev[r0:r1] @ bt).to(torch.bfloat16)
    return x, lam, b
