"""ctypes binding of libppca (include/ppca.h).

Argument marshalling only: every step of the path runs in the HIP library.
Tensors are torch tensors on the GPU; workspaces are allocated with torch and
passed to the library, which never allocates.  Each call runs on torch's
current HIP stream.  Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppca.so")

F32, BF16, FP8_E4M3 = 0, 1, 2
OP_CENTER, OP_POWER, OP_OJA, OP_EIGENGAME, OP_PROJECT, OP_RR, OP_STREAM, OP_POWER_SEQ = range(8)
MAX_K = 128

EXPORTS = [
    "ppca_center_quantize", "ppca_prime_power", "ppca_prime_oja", "ppca_prime_eigengame",
    "ppca_stream_pass", "ppca_project_gram", "ppca_rayleigh_ritz", "ppca_workspace_bytes", "ppca_strerror",
    "ppca_set_kernel_timing", "ppca_kernel_stats", "ppca_set_chunk_rows",
    "ppca_prime_power_grouped", "ppca_rayleigh_ritz_grouped", "ppca_grouped_workspace_bytes",
    "ppca_grouped_workspace_bytes_for", "ppca_set_group_item_bytes", "ppca_tune_group_items",
    "ppca_rayleigh_ritz_noalloc", "ppca_set_fused_pass", "ppca_prime_power_eps",
    "ppca_prime_power_seq", "ppca_project_gram_rows", "ppca_read_probe",
]
NOALLOC_SCRATCH_BYTES = 4 << 20
GROUP_MAX_D, GROUP_MAX_K, GROUP_GRAPH = 768, 64, 1


class PPCAError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} (status {code})")
        self.code = code


class _Matrix(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("col_scale", ctypes.c_void_p)]


class _Sgd(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("steps", ctypes.c_int64), ("eta0", ctypes.c_double),
                ("t0", ctypes.c_double), ("momentum", ctypes.c_double),
                ("nesterov", ctypes.c_int32), ("start_step", ctypes.c_int64),
                ("mom_buf", ctypes.c_void_p), ("snapshot_every", ctypes.c_int32),
                ("snapshots", ctypes.c_void_p), ("orthonormalise_start", ctypes.c_int32)]


class _Problem(ctypes.Structure):
    _fields_ = [("X", _Matrix), ("k", ctypes.c_int32), ("l", ctypes.c_int32),
                ("V", ctypes.c_void_p), ("G", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("E", ctypes.c_void_p), ("evals", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2109_03709_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_double, ctypes.c_size_t)
        mp = ctypes.POINTER(_Matrix)
        sp = ctypes.POINTER(_Sgd)
        L.ppca_center_quantize.argtypes = [vp, i64, i64, i64, i32, vp, i64, vp, vp, vp, sz, vp]
        L.ppca_prime_power.argtypes = [mp, i32, i32, i32, vp, vp, vp, vp, sz, vp]
        L.ppca_prime_oja.argtypes = [mp, i32, i32, sp, vp, vp, sz, vp]
        L.ppca_prime_power_eps.argtypes = [mp, i32, i32, i32, dbl, vp, ctypes.POINTER(i32),
                                           ctypes.POINTER(dbl), vp, sz, vp]
        L.ppca_prime_power_seq.argtypes = [mp, i32, i32, dbl, i32, vp, ctypes.POINTER(i32), vp,
                                           sz, vp]
        L.ppca_project_gram_rows.argtypes = [mp, i32, vp, i64, i64, vp, vp, vp, sz, vp]
        L.ppca_read_probe.argtypes = [mp, i32, i32, vp, i64, vp]
        L.ppca_prime_eigengame.argtypes = [mp, i32, i32, sp, vp, vp, sz, vp]
        L.ppca_stream_pass.argtypes = [mp, i32, vp, i64, i64, vp, vp, vp, sz, vp]
        L.ppca_project_gram.argtypes = [mp, i32, vp, vp, vp, vp, sz, vp]
        L.ppca_rayleigh_ritz.argtypes = [mp, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
        L.ppca_rayleigh_ritz_noalloc.argtypes = [mp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.ppca_workspace_bytes.argtypes = [i32, mp, i32, i32]
        L.ppca_workspace_bytes.restype = sz
        L.ppca_strerror.argtypes = [ctypes.c_int]
        L.ppca_strerror.restype = ctypes.c_char_p
        L.ppca_set_kernel_timing.argtypes = [i32]
        L.ppca_set_kernel_timing.restype = None
        L.ppca_kernel_stats.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        L.ppca_set_chunk_rows.argtypes = [i64]
        L.ppca_set_chunk_rows.restype = None
        L.ppca_set_fused_pass.argtypes = [i32]
        L.ppca_set_fused_pass.restype = None
        pp = ctypes.POINTER(_Problem)
        L.ppca_prime_power_grouped.argtypes = [pp, i32, i32, i32, vp, sz, vp]
        L.ppca_rayleigh_ritz_grouped.argtypes = [pp, i32, vp, sz, vp]
        L.ppca_grouped_workspace_bytes.argtypes = [pp, i32]
        L.ppca_grouped_workspace_bytes.restype = sz
        L.ppca_grouped_workspace_bytes_for.argtypes = [pp, i32, i64]
        L.ppca_grouped_workspace_bytes_for.restype = sz
        L.ppca_set_group_item_bytes.argtypes = [i64]
        L.ppca_tune_group_items.argtypes = [pp, i32, ctypes.POINTER(i64), i32, vp, sz, vp,
                                            ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().ppca_strerror(int(code)).decode()


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check(code: int, what: str):
    if code != 0:
        raise PPCAError(code, what)


@dataclass
class Data:
    """A centred data matrix X (n x d) stored as f32, bf16 or fp8-e4m3 codes
    with per-column float32 scales (value = code * scale[j])."""
    x: torch.Tensor
    dtype: int
    col_scale: torch.Tensor | None = None

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def d(self) -> int:
        return self.x.shape[1]

    def as_c(self) -> _Matrix:
        if self.x.dim() != 2 or self.x.stride(1) != 1:
            raise ValueError("X must be a 2-D tensor with unit column stride")
        want = {F32: (torch.float32,), BF16: (torch.bfloat16,),
                FP8_E4M3: (torch.uint8, torch.float8_e4m3fn)}[self.dtype]
        if self.x.dtype not in want:
            raise TypeError(f"X dtype {self.x.dtype} does not match storage code {self.dtype}")
        return _Matrix(self.x.data_ptr(), self.x.shape[0], self.x.shape[1], self.x.stride(0),
                       self.dtype, 0 if self.col_scale is None else self.col_scale.data_ptr())


def workspace_bytes(op: int, X: Data, K: int, batch: int = 0) -> int:
    m = X.as_c()
    return int(lib().ppca_workspace_bytes(op, ctypes.byref(m), K, batch))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def center_quantize(x: torch.Tensor, out_dtype: int, out: torch.Tensor | None = None):
    """Centre float32 X (n x d) and store it as out_dtype.  Returns
    (Data, mean[d] float64)."""
    if x.dtype != torch.float32 or x.dim() != 2 or x.stride(1) != 1:
        raise TypeError("x must be a 2-D float32 tensor with unit column stride")
    n, d = x.shape
    tdt = {F32: torch.float32, BF16: torch.bfloat16, FP8_E4M3: torch.uint8}[out_dtype]
    if out is None:
        out = torch.empty((n, d), dtype=tdt, device=x.device)
    scale = torch.empty(d, dtype=torch.float32, device=x.device) if out_dtype == FP8_E4M3 else None
    mean = torch.empty(d, dtype=torch.float64, device=x.device)
    probe = Data(out, out_dtype, scale)
    ws = _workspace(workspace_bytes(OP_CENTER, probe, 1), x.device)
    code = lib().ppca_center_quantize(_ptr(x), n, d, x.stride(0), out_dtype, _ptr(out),
                                      out.stride(0), _ptr(scale), _ptr(mean), _ptr(ws),
                                      ws.numel(), _stream())
    _check(code, "ppca_center_quantize")
    return Data(out, out_dtype, scale), mean


def prime_power(X: Data, k: int, l: int, iters: int, V: torch.Tensor,
                gram_hist: torch.Tensor | None = None, b_hist: torch.Tensor | None = None,
                ws: torch.Tensor | None = None) -> torch.Tensor:
    """Block power priming; V (d x K float32) is updated in place and returned."""
    K = k + l
    _check_v(V, X.d, K)
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_POWER, X, K), V.device)
    code = lib().ppca_prime_power(ctypes.byref(m), k, l, iters, _ptr(V), _ptr(gram_hist),
                                  _ptr(b_hist), _ptr(ws), ws.numel(), _stream())
    _check(code, "ppca_prime_power")
    return V


def prime_power_eps(X: Data, k: int, l: int, max_iters: int, eps: float, V: torch.Tensor,
                    ws: torch.Tensor | None = None):
    """Block power priming stopped by the Sec. 2.1 rule (every new direction
    within eps of the previous span); V updated in place.  Returns (V,
    iterations run, [span changes])."""
    K = k + l
    _check_v(V, X.d, K)
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_POWER, X, K), V.device)
    it = ctypes.c_int32(0)
    ch = (ctypes.c_double * max_iters)()
    code = lib().ppca_prime_power_eps(ctypes.byref(m), k, l, max_iters, float(eps), _ptr(V),
                                      ctypes.byref(it), ch, _ptr(ws), ws.numel(), _stream())
    _check(code, "ppca_prime_power_eps")
    return V, it.value, list(ch[:it.value])


def prime_power_seq(X: Data, k: int, l: int, eps: float, max_steps: int, V: torch.Tensor,
                    ws: torch.Tensor | None = None):
    """Sequential power method (one direction after the other, Sec. 2.1); V
    updated in place.  Returns (V, [steps per direction])."""
    K = k + l
    _check_v(V, X.d, K)
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_POWER_SEQ, X, K), V.device)
    steps = (ctypes.c_int32 * K)()
    code = lib().ppca_prime_power_seq(ctypes.byref(m), k, l, float(eps), max_steps, _ptr(V),
                                      steps, _ptr(ws), ws.numel(), _stream())
    _check(code, "ppca_prime_power_seq")
    return V, list(steps)


def _sgd(X: Data, K: int, V: torch.Tensor, batch: int, steps: int | None, epochs: float | None,
         eta0: float, t0: float, momentum: float, nesterov: bool, start_step: int,
         mom_buf, snapshot_every: int, snapshots, orthonormalise_start: bool) -> _Sgd:
    if steps is None:
        if epochs is None:
            raise ValueError("give steps or epochs")
        steps = math.ceil(epochs * X.n / batch)
    return _Sgd(batch, steps, eta0, t0, momentum, 1 if nesterov else 0, start_step,
                0 if mom_buf is None else mom_buf.data_ptr(), snapshot_every,
                0 if snapshots is None else snapshots.data_ptr(),
                1 if orthonormalise_start else 0)


def _prime_sgd(fn_name: str, op: int, X: Data, k: int, l: int, V: torch.Tensor, *, batch: int,
               steps: int | None = None, epochs: float | None = None, eta0: float,
               t0: float = 0.0, momentum: float = 0.0, nesterov: bool = False,
               start_step: int = 0, mom_buf=None, snapshot_every: int = 0, snapshots=None,
               orthonormalise_start: bool = True, ws=None):
    K = k + l
    _check_v(V, X.d, K)
    p = _sgd(X, K, V, batch, steps, epochs, eta0, t0, momentum, nesterov, start_step, mom_buf,
             snapshot_every, snapshots, orthonormalise_start)
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(op, X, K, batch), V.device)
    code = getattr(lib(), fn_name)(ctypes.byref(m), k, l, ctypes.byref(p), _ptr(V), _ptr(ws),
                                   ws.numel(), _stream())
    _check(code, fn_name)
    return V


def prime_oja(X: Data, k: int, l: int, V: torch.Tensor, **kw) -> torch.Tensor:
    """Minibatch Sanger/Oja priming; V updated in place."""
    return _prime_sgd("ppca_prime_oja", OP_OJA, X, k, l, V, **kw)


def prime_eigengame(X: Data, k: int, l: int, V: torch.Tensor, **kw) -> torch.Tensor:
    """Minibatch EigenGame priming; V updated in place."""
    return _prime_sgd("ppca_prime_eigengame", OP_EIGENGAME, X, k, l, V, **kw)


def stream_pass(X: Data, K: int, V: torch.Tensor, r0: int = 0, nrows: int | None = None,
                ws=None, want_g: bool = True):
    """(Z d x K float32, G K x K float64) of one pass over rows r0.. (mod n);
    G is None when want_g is False (Z alone, as in a block power step)."""
    _check_v(V, X.d, K)
    nrows = X.n if nrows is None else nrows
    Z = torch.empty((X.d, K), dtype=torch.float32, device=V.device)
    G = torch.empty((K, K), dtype=torch.float64, device=V.device) if want_g else None
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_STREAM, X, K, nrows), V.device)
    code = lib().ppca_stream_pass(ctypes.byref(m), K, _ptr(V), r0, nrows, _ptr(Z),
                                  _ptr(G), _ptr(ws), ws.numel(), _stream())
    _check(code, "ppca_stream_pass")
    return Z, G


def project_gram(X: Data, K: int, V: torch.Tensor, ws=None):
    """(G, B): K x K float64 Gram of the projected data and of the operand."""
    _check_v(V, X.d, K)
    G = torch.empty((K, K), dtype=torch.float64, device=V.device)
    B = torch.empty((K, K), dtype=torch.float64, device=V.device)
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_PROJECT, X, K), V.device)
    code = lib().ppca_project_gram(ctypes.byref(m), K, _ptr(V), _ptr(G), _ptr(B), _ptr(ws),
                                   ws.numel(), _stream())
    _check(code, "ppca_project_gram")
    return G, B


def rayleigh_ritz(X: Data, K: int, k: int, G: torch.Tensor, B: torch.Tensor, V: torch.Tensor,
                  vectors: bool = True, ws=None):
    """(evals[k] float64 descending, E d x k float32 or None)."""
    _check_v(V, X.d, K)
    for t in (G, B):
        if t.dtype != torch.float64 or t.shape != (K, K) or not t.is_contiguous():
            raise TypeError("G and B must be contiguous K x K float64")
    ev = torch.empty(k, dtype=torch.float64, device=V.device)
    E = torch.empty((X.d, k), dtype=torch.float32, device=V.device) if vectors else None
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_RR, X, K), V.device)
    code = lib().ppca_rayleigh_ritz(ctypes.byref(m), K, k, _ptr(G), _ptr(B), _ptr(V), _ptr(E),
                                    _ptr(ev), _ptr(ws), ws.numel(), _stream())
    _check(code, "ppca_rayleigh_ritz")
    return ev, E


def rayleigh_ritz_noalloc(X: Data, K: int, k: int, G: torch.Tensor, B: torch.Tensor,
                          V: torch.Tensor, ev: torch.Tensor, E: torch.Tensor | None = None):
    """Rayleigh-Ritz into caller-allocated ev (k float64) and E (d x k float32,
    or None) with no workspace: the library's fixed device scratch is used."""
    _check_v(V, X.d, K)
    for t in (G, B):
        if t.dtype != torch.float64 or t.shape != (K, K) or not t.is_contiguous():
            raise TypeError("G and B must be contiguous K x K float64")
    if ev.dtype != torch.float64 or ev.numel() < k or not ev.is_contiguous():
        raise TypeError("ev must be a contiguous float64 tensor of at least k entries")
    if E is not None and (E.dtype != torch.float32 or E.shape != (X.d, k) or not E.is_contiguous()):
        raise TypeError(f"E must be a contiguous ({X.d}, {k}) float32 tensor")
    m = X.as_c()
    code = lib().ppca_rayleigh_ritz_noalloc(ctypes.byref(m), K, k, _ptr(G), _ptr(B), _ptr(V),
                                            _ptr(E), _ptr(ev), _stream())
    _check(code, "ppca_rayleigh_ritz_noalloc")
    return ev, E


def project_gram_rows(X: Data, K: int, V: torch.Tensor, r0: int, nrows: int, ws=None):
    """(G, B) of the projection over rows r0 .. r0 + nrows - 1 (mod n)."""
    _check_v(V, X.d, K)
    G = torch.empty((K, K), dtype=torch.float64, device=V.device)
    B = torch.empty((K, K), dtype=torch.float64, device=V.device)
    m = X.as_c()
    if ws is None:
        ws = _workspace(workspace_bytes(OP_PROJECT, X, K, nrows), V.device)
    code = lib().ppca_project_gram_rows(ctypes.byref(m), K, _ptr(V), r0, nrows, _ptr(G), _ptr(B),
                                        _ptr(ws), ws.numel(), _stream())
    _check(code, "ppca_project_gram_rows")
    return G, B


def read_probe(X: Data, mode: int, seg_bytes: int = 128, sink=None) -> torch.Tensor:
    """Streaming-read probe over the stored X (mode 0: vector loads; mode 1:
    the power pass's LDS-DMA pattern with seg_bytes of a row per step).
    Returns the per-workgroup XOR sink (uint32 viewed as int32)."""
    if sink is None:
        sink = torch.zeros(1024, dtype=torch.int32, device=X.x.device)
    m = X.as_c()
    code = lib().ppca_read_probe(ctypes.byref(m), mode, seg_bytes, _ptr(sink), sink.numel(),
                                 _stream())
    _check(code, "ppca_read_probe")
    return sink


def ppca(X: Data, V: torch.Tensor, k: int, rows: tuple[int, int] | None = None):
    """Alg. 1 steps 2-4 on primed directions V: (evals[k], E d x k).  rows =
    (r0, nrows) projects only that row window (Sec. 5.2 projects a tenth)."""
    K = V.shape[1]
    if rows is None:
        G, B = project_gram(X, K, V)
        return rayleigh_ritz(X, K, k, G, B, V)
    r0, nrows = rows
    G, B = project_gram_rows(X, K, V, r0, nrows)
    Xs = Data(X.x[:nrows], X.dtype, X.col_scale)     # descriptor with n = nrows (data not read)
    return rayleigh_ritz(Xs, K, k, G, B, V)


def _check_v(V: torch.Tensor, d: int, K: int):
    if V.dtype != torch.float32 or V.shape != (d, K) or not V.is_contiguous() or not V.is_cuda:
        raise TypeError(f"V must be a contiguous ({d}, {K}) float32 device tensor")


def set_kernel_timing(enable: bool):
    lib().ppca_set_kernel_timing(1 if enable else 0)


def kernel_stats(kernel: int):
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(lib().ppca_kernel_stats(kernel, ctypes.byref(n), ctypes.byref(ms)), "kernel_stats")
    return n.value, ms.value


def set_chunk_rows(rows: int):
    lib().ppca_set_chunk_rows(int(rows))


def set_fused_pass(enable: bool):
    """Single-read power pass on (True) or off (False, the default: two kernels)."""
    lib().ppca_set_fused_pass(1 if enable else 0)


# --------------------------------------------------------------- grouped
@dataclass
class Problem:
    """One problem of a grouped call: bf16 data X, k + l directions V (d x K
    float32, updated in place) and the outputs G, B (K x K float64), evals (k
    float64) and E (d x k float32, optional)."""
    X: Data
    k: int
    l: int
    V: torch.Tensor
    G: torch.Tensor | None = None
    B: torch.Tensor | None = None
    evals: torch.Tensor | None = None
    E: torch.Tensor | None = None

    def alloc(self, vectors: bool = True):
        K, dev = self.k + self.l, self.V.device
        if self.G is None:
            self.G = torch.empty((K, K), dtype=torch.float64, device=dev)
        if self.B is None:
            self.B = torch.empty((K, K), dtype=torch.float64, device=dev)
        if self.evals is None:
            self.evals = torch.empty(self.k, dtype=torch.float64, device=dev)
        if vectors and self.E is None:
            self.E = torch.empty((self.X.d, self.k), dtype=torch.float32, device=dev)
        return self

    def as_c(self) -> _Problem:
        _check_v(self.V, self.X.d, self.k + self.l)
        return _Problem(self.X.as_c(), self.k, self.l, self.V.data_ptr(), _ptr(self.G).value,
                        _ptr(self.B).value, _ptr(self.E).value, _ptr(self.evals).value)


def _problem_array(problems):
    arr = (_Problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = p.alloc(vectors=p.E is not None).as_c()
    return arr


class Group:
    """A fixed list of problems with its C descriptor array built once (the
    tensors behind it must stay alive and in place)."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.arr = _problem_array(self.problems)
        # 0 for invalid problems: the calls then report the precise status
        self.ws_bytes = int(lib().ppca_grouped_workspace_bytes(self.arr, len(self.problems)))

    def workspace(self):
        return _workspace(self.ws_bytes, self.problems[0].V.device)


def _group(problems) -> Group:
    return problems if isinstance(problems, Group) else Group(problems)


def grouped_workspace_bytes(problems) -> int:
    arr = _problem_array(problems)
    return int(lib().ppca_grouped_workspace_bytes(arr, len(problems)))


GROUP_ITEM_CANDIDATES = (1 << 20, 2 << 20, 3 << 20, 4 << 20, 6 << 20, 8 << 20)


def set_group_item_bytes(nbytes: int):
    """Work-item size (bytes of X) of later grouped calls; 0 = default."""
    _check(lib().ppca_set_group_item_bytes(int(nbytes)), "ppca_set_group_item_bytes")


def tune_group_items(problems, candidates=GROUP_ITEM_CANDIDATES, ws=None):
    """Time one fused power pass of these problems per candidate work-item
    size; returns (fastest size, [ms per candidate]).  The setting is not
    changed (see set_group_item_bytes)."""
    g = _group(problems)
    cand = (ctypes.c_int64 * len(candidates))(*[int(c) for c in candidates])
    if ws is None:
        need = max(int(lib().ppca_grouped_workspace_bytes_for(g.arr, len(g.problems), int(c)))
                   for c in candidates)
        ws = _workspace(need, g.problems[0].V.device)
    best = ctypes.c_int64(0)
    times = (ctypes.c_double * len(candidates))()
    code = lib().ppca_tune_group_items(g.arr, len(g.problems), cand, len(candidates), _ptr(ws),
                                       ws.numel(), _stream(), ctypes.byref(best), times)
    _check(code, "ppca_tune_group_items")
    return int(best.value), [float(t) for t in times]


def prime_power_grouped(problems, iters: int, graph: bool = False, ws=None):
    """Block power priming of every problem, then the projection Gram G and
    B of the primed V (one fused pass over X per iteration for all problems).
    problems: a list of Problem or a Group."""
    g = _group(problems)
    if ws is None:
        ws = g.workspace()
    code = lib().ppca_prime_power_grouped(g.arr, len(g.problems), iters,
                                          GROUP_GRAPH if graph else 0, _ptr(ws), ws.numel(),
                                          _stream())
    _check(code, "ppca_prime_power_grouped")
    return g.problems


def rayleigh_ritz_grouped(problems, ws=None):
    """Rayleigh-Ritz of every problem from its G, B and V: evals and E."""
    g = _group(problems)
    if ws is None:
        ws = g.workspace()
    code = lib().ppca_rayleigh_ritz_grouped(g.arr, len(g.problems), _ptr(ws), ws.numel(),
                                            _stream())
    _check(code, "ppca_rayleigh_ritz_grouped")
    return g.problems
