"""Float64 CPU oracle for primed PCA (pPCA).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  The GPU library never calls it and shares no code with
it.  Everything here is plain numpy in float64 (a matmul is the only library
primitive used for the heavy products); the eigensolver, the Cholesky
factorisation, the triangular solves and the storage-format encoders are
written out below.

Paper references are to "Speeding up PCA with priming" (Mate & Fleuret):
Alg. 1 (Primed PCA), Sec. 2.1 (power method), Sec. 2.2 (Oja / Sanger rule),
Sec. 2.3 eqs. (1)-(3) (EigenGame utilities), Sec. 3.3 (extra components),
Sec. 4.1 (counterexample), Sec. 4.2 (variance restricted to S), Sec. 5
(training setup), Sec. 5.3 (longest correct eigenvector streak).

Pins (what checks this file against something other than itself) live in
tests/test_oracle_*.py.  Every function below has at least one pin.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "NotSPD", "NoConvergence",
    "column_means", "center_fp32", "bf16_round", "bf16_value", "e4m3_table",
    "e4m3_encode", "e4m3_value", "fp8_column_scales",
    "covariance", "jacobi_eigh", "exact_pca", "sign_normalise",
    "cholesky_upper", "solve_right_upper", "cholqr2",
    "stream_pass", "prime_power", "prime_power_eps", "prime_power_sequential",
    "minibatch_rows", "learning_rate",
    "sanger_direction", "sanger_per_sample", "prime_oja",
    "eigengame_utility", "eigengame_grad", "prime_eigengame",
    "project_gram", "rayleigh_ritz", "ppca",
    "rel_eig_error", "sin_theta_max", "streak", "angles",
]


class NotSPD(ArithmeticError):
    """A Cholesky pivot was not positive (rank-deficient or indefinite input)."""


class NoConvergence(ArithmeticError):
    """The Jacobi sweep cap was reached before the off-diagonal norm vanished."""


# --------------------------------------------------------------------------
# a0. Centring (Sec. 1: X is a centred dataset) and storage formats.
# The paper fixes no precision; the reading used here: centre with float64
# column means of the float32 input, keep the centred value in float32, then
# round that float32 value to bf16 or to fp8-e4m3 (with a per-column scale).
# --------------------------------------------------------------------------

def column_means(x32: np.ndarray) -> np.ndarray:
    """mu_j = (correctly rounded sum_r x_rj) / n, in float64.

    ``math.fsum`` returns the correctly rounded float64 of the exact sum, so
    the result does not depend on summation order.
    """
    n = x32.shape[0]
    xt = np.ascontiguousarray(np.asarray(x32, dtype=np.float64).T)
    return np.array([math.fsum(col) / n for col in xt], dtype=np.float64)


def center_fp32(x32: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """c = float32(float64(x) - mu): the centred data in float32."""
    return (np.asarray(x32, np.float64) - mu[None, :]).astype(np.float32)


def bf16_round(c32: np.ndarray) -> np.ndarray:
    """bf16 code (uint16) of the nearest bf16 value to each float32, ties to
    the even code.  Written as the definition: take the two bf16 neighbours
    (truncation toward zero and the next code away from zero), compare the
    exact float64 distances, break ties on the even code."""
    c32 = np.ascontiguousarray(c32, dtype=np.float32)
    bits = c32.view(np.uint32).astype(np.uint64)
    lo = (bits & 0xFFFF0000)
    hi = lo + 0x10000
    v = c32.astype(np.float64)
    vlo = (lo.astype(np.uint32)).view(np.float32).astype(np.float64)
    vhi = (hi.astype(np.uint32)).view(np.float32).astype(np.float64)
    dlo = np.abs(v - vlo)
    dhi = np.abs(vhi - v)
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (((lo >> 16) & 1) == 1))
    out = np.where(pick_hi, hi, lo) >> 16
    return out.astype(np.uint16)


def bf16_value(codes: np.ndarray) -> np.ndarray:
    """float64 value of bf16 codes."""
    b = (np.asarray(codes, np.uint16).astype(np.uint32) << 16)
    return b.view(np.float32).astype(np.float64)


def e4m3_table() -> np.ndarray:
    """Value of every fp8-e4m3 code (OCP "fn" variant: bias 7, no infinity,
    S.1111.111 is NaN, largest finite 448).  float64[256]."""
    vals = np.empty(256, np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * m * 2.0 ** -9
        else:
            vals[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


_E4M3 = e4m3_table()
_E4M3_POS_CODES = np.arange(0, 0x7F)             # 0 .. 126: finite, >= 0
_E4M3_POS_VALS = _E4M3[_E4M3_POS_CODES]          # increasing


def e4m3_encode(v32: np.ndarray) -> np.ndarray:
    """fp8-e4m3 code of the nearest finite e4m3 value, ties to the even code,
    magnitudes above 448 saturate to 448.  The sign bit copies the sign of the
    float32 input (so -0.0 and tiny negatives give 0x80)."""
    v32 = np.asarray(v32, np.float32)
    mag = np.abs(v32.astype(np.float64))
    idx = np.searchsorted(_E4M3_POS_VALS, mag, side="left")
    idx = np.clip(idx, 1, len(_E4M3_POS_VALS) - 1)
    lo = idx - 1
    hi = idx
    vlo = _E4M3_POS_VALS[lo]
    vhi = _E4M3_POS_VALS[hi]
    dlo = mag - vlo
    dhi = vhi - mag
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((_E4M3_POS_CODES[hi] & 1) == 0))
    code = np.where(pick_hi, _E4M3_POS_CODES[hi], _E4M3_POS_CODES[lo])
    code = np.where(mag >= 448.0, 0x7E, code)
    sign = np.signbit(v32).astype(np.int64) << 7
    return (code | sign).astype(np.uint8)


def e4m3_value(codes: np.ndarray) -> np.ndarray:
    return _E4M3[np.asarray(codes, np.uint8)]


def fp8_column_scales(c32: np.ndarray) -> np.ndarray:
    """s_j = float32(max_r |c_rj| / 448); an all-zero column gets s_j = 1."""
    amax = np.max(np.abs(c32), axis=0).astype(np.float32)
    s = (amax / np.float32(448.0)).astype(np.float32)
    return np.where(amax > 0, s, np.float32(1.0)).astype(np.float32)


def fp8_quantize(c32: np.ndarray, s: np.ndarray) -> np.ndarray:
    """q_rj = e4m3(float32(c_rj / s_j)); x_rj is then represented as q_rj * s_j."""
    v = (np.asarray(c32, np.float32) / s[None, :].astype(np.float32)).astype(np.float32)
    return e4m3_encode(v)


# --------------------------------------------------------------------------
# O1/O2. Exact PCA: covariance (Sec. 1: principal directions are the
# eigenvectors of X^T X) and a cyclic Jacobi eigensolver.
# --------------------------------------------------------------------------

def covariance(x: np.ndarray) -> np.ndarray:
    """C = X^T X / n for centred X (float64)."""
    x = np.asarray(x, np.float64)
    return (x.T @ x) / x.shape[0]


def sign_normalise(u: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive
    (ties: the lowest row index).  Eigenvectors are defined up to sign; this
    rule only makes outputs reproducible."""
    u = np.array(u, np.float64, copy=True)
    if u.size == 0:
        return u
    piv = np.argmax(np.abs(u), axis=0)
    s = np.sign(u[piv, np.arange(u.shape[1])])
    s[s == 0] = 1.0
    return u * s[None, :]


def jacobi_eigh(a: np.ndarray, *, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic (row-by-row) Jacobi for a symmetric matrix, float64.

    Each rotation zeroes a_pq with tau = (a_qq - a_pp) / (2 a_pq),
    t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1+t^2), s = t c
    (the classical symmetric Schur step).  Stops when the off-diagonal
    Frobenius norm is <= tol * ||A||_F or a sweep applies no rotation.
    Returns (eigenvalues descending, eigenvectors as columns, sign-normalised).
    """
    a = np.array(a, np.float64, copy=True)
    m = a.shape[0]
    if a.shape != (m, m):
        raise ValueError("square matrix required")
    a = 0.5 * (a + a.T)
    v = np.eye(m)
    fro = math.sqrt(float(np.sum(a * a)))
    eps = np.finfo(np.float64).eps
    converged = m <= 1 or fro == 0.0
    offmask = ~np.eye(m, dtype=bool)
    for _ in range(max_sweeps):
        if converged:
            break
        off = math.sqrt(float(np.sum(a[offmask] ** 2)))
        if off <= tol * fro:
            converged = True
            break
        rotated = False
        for p in range(m - 1):
            for q in range(p + 1, m):
                apq = a[p, q]
                app = a[p, p]
                aqq = a[q, q]
                if abs(apq) <= 1e-300 or abs(apq) < 0.1 * eps * math.sqrt(abs(app * aqq)):
                    continue
                tau = (aqq - app) / (2.0 * apq)
                t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + math.sqrt(1.0 + tau * tau))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                colp = a[:, p].copy()
                colq = a[:, q].copy()
                a[:, p] = c * colp - s * colq
                a[:, q] = s * colp + c * colq
                a[p, :] = a[:, p]
                a[q, :] = a[:, q]
                a[p, p] = app - t * apq
                a[q, q] = aqq + t * apq
                a[p, q] = 0.0
                a[q, p] = 0.0
                vp = v[:, p].copy()
                vq = v[:, q].copy()
                v[:, p] = c * vp - s * vq
                v[:, q] = s * vp + c * vq
                rotated = True
        if not rotated:
            converged = True
    if not converged:
        off = math.sqrt(float(np.sum(a[offmask] ** 2)))
        if off > tol * fro:
            raise NoConvergence(f"Jacobi: off-diagonal {off:.3e} after {max_sweeps} sweeps")
    w = np.diag(a).copy()
    order = np.argsort(-w, kind="stable")
    return w[order], sign_normalise(v[:, order])


def exact_pca(x: np.ndarray, k: int | None = None):
    """Top-k eigenpairs of C = X^T X / n for centred X: (lam desc, U d x k)."""
    lam, u = jacobi_eigh(covariance(x))
    if k is not None:
        lam, u = lam[:k], u[:, :k]
    return lam, u


# --------------------------------------------------------------------------
# O3. Cholesky and CholeskyQR2 (orthonormalisation after every power step,
# Sec. 2.1).  Gram-Schmidt-equivalent: the span of the first j columns is kept.
# --------------------------------------------------------------------------

def cholesky_upper(a: np.ndarray) -> np.ndarray:
    """Upper-triangular R with R^T R = A (column-by-column definition).
    Raises NotSPD when a pivot is not finite or not above m * eps * a_jj
    (a pivot at rounding level means the columns behind A are numerically
    dependent; the paper fixes no threshold, this is the reading used)."""
    a = np.asarray(a, np.float64)
    m = a.shape[0]
    r = np.zeros_like(a)
    eps = np.finfo(np.float64).eps
    for j in range(m):
        piv = a[j, j] - float(r[:j, j] @ r[:j, j])
        if not math.isfinite(piv) or not (piv > m * eps * abs(a[j, j])) or not (piv > 0.0):
            raise NotSPD(f"Cholesky pivot {j} = {piv!r}")
        r[j, j] = math.sqrt(piv)
        if j + 1 < m:
            r[j, j + 1:] = (a[j, j + 1:] - r[:j, j] @ r[:j, j + 1:]) / r[j, j]
    return r


def solve_right_upper(z: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Q = Z R^{-1} for upper-triangular R, by forward column substitution:
    Q[:, j] = (Z[:, j] - Q[:, :j] R[:j, j]) / R[j, j]."""
    z = np.asarray(z, np.float64)
    q = np.zeros_like(z)
    for j in range(r.shape[0]):
        q[:, j] = (z[:, j] - q[:, :j] @ r[:j, j]) / r[j, j]
    return q


def cholqr2(z: np.ndarray):
    """CholeskyQR2: R1 = chol(Z^T Z), Q1 = Z R1^-1, R2 = chol(Q1^T Q1),
    Q = Q1 R2^-1.  Returns (Q, R = R2 R1)."""
    z = np.asarray(z, np.float64)
    r1 = cholesky_upper(z.T @ z)
    q1 = solve_right_upper(z, r1)
    r2 = cholesky_upper(q1.T @ q1)
    q = solve_right_upper(q1, r2)
    return q, r2 @ r1


# --------------------------------------------------------------------------
# O4. Power priming, block form (Sec. 2.1; the cited simultaneous iteration).
# One pass streams X through Y = X V, Z = X^T Y, G = Y^T Y.
# --------------------------------------------------------------------------

def stream_pass(x: np.ndarray, v: np.ndarray):
    """(Z, G) = (X^T X V, V^T X^T X V) for the rows given."""
    x = np.asarray(x, np.float64)
    y = x @ np.asarray(v, np.float64)
    return x.T @ y, y.T @ y


def prime_power(x: np.ndarray, v0: np.ndarray, iters: int, operand=None):
    """V_0 = orth(V0); for t = 1..iters: (Z, G_{t-1}) = pass(X, V_{t-1}),
    V_t = CholQR2(Z).  Returns (V_iters, [G_0 .. G_{iters-1}]).
    ``operand`` as in prime_oja."""
    v, _ = cholqr2(v0)
    grams = []
    for _ in range(iters):
        z, g = stream_pass(x, v if operand is None else operand(v))
        grams.append(g)
        v, _ = cholqr2(z)
    return v, grams


def span_change(v_new: np.ndarray, v_old: np.ndarray) -> float:
    """max_j |v_new[:, j] - V_old (V_old^T v_new[:, j])|_2: how far the new
    iterate's directions lie from the previous iterate's span (V_old with
    orthonormal columns).  This is the termination quantity of the power
    method (Sec. 2.1, |x_i - x_{i+1}| < eps) read for a block: a single unit
    vector gives the sine of the angle it turned, |x_i - x_{i+1}| to first
    order.  Columns of a block keep turning inside the K-dimensional span
    long after the span itself has settled, so a column-by-column change
    would not measure the convergence of block iteration."""
    v_new = np.asarray(v_new, np.float64)
    v_old = np.asarray(v_old, np.float64)
    r = v_new - v_old @ (v_old.T @ v_new)
    return float(np.max(np.linalg.norm(r, axis=0)))


def prime_power_eps(x: np.ndarray, v0: np.ndarray, max_iters: int, eps: float, operand=None):
    """Block power iteration with the termination rule of Sec. 2.1: as
    prime_power, stopping after the first iteration t whose span change
    (span_change of V_t against V_{t-1}) is below eps, or after max_iters.
    Returns (V_t, t, [changes])."""
    v, _ = cholqr2(v0)
    changes = []
    for t in range(1, max_iters + 1):
        z, _ = stream_pass(x, v if operand is None else operand(v))
        vn, _ = cholqr2(z)
        changes.append(span_change(vn, v))
        v = vn
        if changes[-1] < eps:
            return v, t, changes
    return v, max_iters, changes


def prime_power_sequential(x: np.ndarray, v0: np.ndarray, eps: float, max_iters: int):
    """The power method of Sec. 2.1 for several directions, one after the
    other: direction i starts from column i of V0 and iterates
    u <- P M u / |P M u| with M = X^T X and P = I - V_<i V_<i^T (the
    orthogonalisation after every step that keeps it in the complement of the
    directions already found), until |u_t - u_{t+1}| < eps or max_iters
    steps.  Returns (V d x K with orthonormal columns, [steps per direction])."""
    x = np.asarray(x, np.float64)
    v0 = np.asarray(v0, np.float64)
    d, kk = v0.shape
    v = np.zeros((d, kk))
    steps = []
    for i in range(kk):
        prev = v[:, :i]
        u = v0[:, i] - prev @ (prev.T @ v0[:, i])
        u = u / np.linalg.norm(u)
        t = 0
        while t < max_iters:
            w = x.T @ (x @ u)
            w = w - prev @ (prev.T @ w)
            w = w / np.linalg.norm(w)
            t += 1
            delta = np.linalg.norm(w - u)
            u = w
            if delta < eps:
                break
        v[:, i] = u
        steps.append(t)
    return v, steps


# --------------------------------------------------------------------------
# O5. Oja / Sanger (Sec. 2.2), minibatch mean of the per-sample updates.
# --------------------------------------------------------------------------

def minibatch_rows(n: int, b: int, step: int) -> np.ndarray:
    """Rows of minibatch ``step``: (step*b + i) mod n, i < b (no shuffle)."""
    return (step * b + np.arange(b, dtype=np.int64)) % n


def learning_rate(eta0: float, t0: float, step: int) -> float:
    """eta_t = eta0 / (1 + t/t0); t0 <= 0 means a constant rate."""
    return eta0 if t0 <= 0 else eta0 / (1.0 + step / t0)


def sanger_per_sample(xb: np.ndarray, v: np.ndarray) -> np.ndarray:
    """The rule exactly as printed, one sample at a time at fixed weights:
    dw_m = y_m (x - sum_{l<=m} y_l w_l), averaged over the minibatch."""
    xb = np.asarray(xb, np.float64)
    v = np.asarray(v, np.float64)
    d, kk = v.shape
    acc = np.zeros((d, kk))
    for x in xb:
        y = x @ v
        for m in range(kk):
            resid = x - v[:, : m + 1] @ y[: m + 1]
            acc[:, m] += y[m] * resid
    return acc / xb.shape[0]


def sanger_direction(z: np.ndarray, g: np.ndarray, v: np.ndarray, b: int) -> np.ndarray:
    """Matrix form of the averaged rule: (Z - V triu(G)) / b, where
    Z = X_b^T X_b V and G = V^T X_b^T X_b V (triu keeps the diagonal)."""
    return (np.asarray(z, np.float64) - np.asarray(v, np.float64) @ np.triu(g)) / b


def _momentum_step(grad, buf, momentum, nesterov):
    if momentum == 0.0:
        return grad, buf
    buf = momentum * buf + grad
    step = grad + momentum * buf if nesterov else buf
    return step, buf


def prime_oja(x: np.ndarray, v0: np.ndarray, *, batch: int, steps: int,
              eta0: float, t0: float = 1000.0, momentum: float = 0.0,
              nesterov: bool = False, start_step: int = 0, mom_buf=None,
              orthonormalise_start: bool = True, operand=None):
    """Minibatch Sanger priming.  Returns (V, momentum buffer).

    ``operand`` (optional) maps V to the basis the minibatch is multiplied
    with in the pass (default: V itself); a low-precision store multiplies
    with a rounded copy of V while the update acts on V."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    v = cholqr2(v0)[0] if orthonormalise_start else np.asarray(v0, np.float64).copy()
    buf = np.zeros_like(v) if mom_buf is None else np.asarray(mom_buf, np.float64).copy()
    for t in range(start_step, start_step + steps):
        xb = x[minibatch_rows(n, batch, t)]
        z, g = stream_pass(xb, v if operand is None else operand(v))
        step, buf = _momentum_step(sanger_direction(z, g, v, batch), buf, momentum, nesterov)
        v = v + learning_rate(eta0, t0, t) * step
    return v, buf


# --------------------------------------------------------------------------
# O6. EigenGame (Sec. 2.3, eqs. (1)-(3)); M_hat = X_b^T X_b / b.
# --------------------------------------------------------------------------

def eigengame_utility(m: np.ndarray, v: np.ndarray, j: int) -> float:
    """U_j(v_j) = v_j^T M v_j - sum_{i<j} (v_j^T M v_i)^2 / (v_i^T M v_i)."""
    vj = v[:, j]
    u = float(vj @ m @ vj)
    for i in range(j):
        vi = v[:, i]
        u -= float(vj @ m @ vi) ** 2 / float(vi @ m @ vi)
    return u


def eigengame_grad(z: np.ndarray, g: np.ndarray, b: int) -> np.ndarray:
    """Column j is dU_j/dv_j = (2/b) (Z_j - sum_{i<j} (G_ij / G_ii) Z_i)
    = (2/b) (Z R)_j with R = I, R_ij = -G_ij/G_ii for i < j."""
    kk = g.shape[0]
    r = np.eye(kk)
    for j in range(kk):
        for i in range(j):
            if g[i, i] > 1e-300:
                r[i, j] = -g[i, j] / g[i, i]
    return (2.0 / b) * (np.asarray(z, np.float64) @ r)


def prime_eigengame(x: np.ndarray, v0: np.ndarray, *, batch: int, steps: int,
                    eta0: float, t0: float = 0.0, momentum: float = 0.0,
                    nesterov: bool = False, start_step: int = 0, mom_buf=None,
                    orthonormalise_start: bool = True, operand=None):
    """All players step together on the same minibatch: Riemannian gradient
    (grad_j - (v_j . grad_j) v_j), optional momentum, ascent step, then each
    v_j is put back on the unit sphere.  Returns (V, momentum buffer).
    ``operand`` as in prime_oja."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    v = cholqr2(v0)[0] if orthonormalise_start else np.asarray(v0, np.float64).copy()
    buf = np.zeros_like(v) if mom_buf is None else np.asarray(mom_buf, np.float64).copy()
    for t in range(start_step, start_step + steps):
        xb = x[minibatch_rows(n, batch, t)]
        z, g = stream_pass(xb, v if operand is None else operand(v))
        grad = eigengame_grad(z, g, batch)
        grad = grad - v * np.sum(v * grad, axis=0)[None, :]
        step, buf = _momentum_step(grad, buf, momentum, nesterov)
        v = v + learning_rate(eta0, t0, t) * step
        v = v / np.linalg.norm(v, axis=0)[None, :]
    return v, buf


# --------------------------------------------------------------------------
# O7. The pPCA step (Alg. 1 steps 2-4).  Full PCA of the data projected on
# span(V) is Rayleigh-Ritz for X^T X on that span (Sec. 4.2).  V need not be
# orthonormal: with B = V^T V = R^T R the span has orthonormal basis V R^-1.
# --------------------------------------------------------------------------

def project_gram(x: np.ndarray, v: np.ndarray):
    """G = (X V)^T (X V) and B = V^T V (float64)."""
    x = np.asarray(x, np.float64)
    v = np.asarray(v, np.float64)
    y = x @ v
    return y.T @ y, v.T @ v


def rayleigh_ritz(g: np.ndarray, b: np.ndarray, v: np.ndarray, n: int, k: int):
    """Ritz pairs of C = X^T X / n on span(V): R = chol(B),
    H = R^-T G R^-1 / n, H = W Theta W^T, E = V R^-1 W[:, :k].
    Returns (theta[:k] descending, E d x k sign-normalised, theta all)."""
    r = cholesky_upper(b)
    kk = r.shape[0]
    rinv = solve_right_upper(np.eye(kk), r)          # R^-1
    h = rinv.T @ np.asarray(g, np.float64) @ rinv / n
    theta, w = jacobi_eigh(0.5 * (h + h.T))
    e = np.asarray(v, np.float64) @ (rinv @ w[:, :k])
    return theta[:k], sign_normalise(e), theta


def ppca(x: np.ndarray, v_primed: np.ndarray, k: int):
    """Alg. 1 steps 2-4 on already-primed directions: (theta[:k], E)."""
    g, b = project_gram(x, v_primed)
    th, e, _ = rayleigh_ritz(g, b, v_primed, x.shape[0], k)
    return th, e


# --------------------------------------------------------------------------
# O8. Metrics (Sec. 5.3) and the error measures used for parity.
# --------------------------------------------------------------------------

def rel_eig_error(est: np.ndarray, ref: np.ndarray) -> np.ndarray:
    est = np.asarray(est, np.float64)
    ref = np.asarray(ref, np.float64)[: len(est)]
    return np.abs(est - ref) / np.abs(ref)


def sin_theta_max(e: np.ndarray, u: np.ndarray) -> float:
    """Largest principal-angle sine between span(E) and span(U), computed as
    sqrt(lambda_max(W^T W)) with W = Q_E - U (U^T Q_E), which avoids the
    cancellation in 1 - cos^2.  U must have orthonormal columns."""
    qe, _ = cholqr2(np.asarray(e, np.float64))
    u = np.asarray(u, np.float64)
    w = qe - u @ (u.T @ qe)
    s = jacobi_eigh(w.T @ w)[0]
    return float(math.sqrt(max(s[0], 0.0)))


def angles(e: np.ndarray, u: np.ndarray) -> np.ndarray:
    """angle_i = arccos(|<e_i, u_i>| / (|e_i| |u_i|)), column by column."""
    e = np.asarray(e, np.float64)
    u = np.asarray(u, np.float64)
    c = np.abs(np.sum(e * u, axis=0)) / (np.linalg.norm(e, axis=0) * np.linalg.norm(u, axis=0))
    return np.arccos(np.clip(c, 0.0, 1.0))


def streak(ang: np.ndarray, thresh: float) -> int:
    """Longest correct eigenvector streak: the number of leading indices whose
    angle is below the threshold."""
    n = 0
    for a in ang:
        if a < thresh:
            n += 1
        else:
            break
    return n
