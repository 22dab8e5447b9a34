"""The C-ABI library loads and exports every symbol declared in include/ppca.h
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppca.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ppca_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ppca_prime_power", "ppca_prime_oja", "ppca_prime_eigengame",
                 "ppca_project_gram", "ppca_rayleigh_ritz", "ppca_center_quantize",
                 "ppca_workspace_bytes", "ppca_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2109_03709_amd import _lib
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(_declared()) == sorted(_lib.EXPORTS)


def test_host_only_calls():
    """Calls that touch no device memory: status strings, workspace sizes and
    argument validation (which returns before anything is enqueued)."""
    from paper_2109_03709_amd import _lib
    L = _lib.lib()
    assert _lib.strerror(0) == "success"
    assert "rank deficient" in _lib.strerror(-3)
    m = _lib._Matrix(16, 10000, 256, 256, _lib.F32, 0)
    ws_power = L.ppca_workspace_bytes(_lib.OP_POWER, ctypes.byref(m), 32, 0)
    assert ws_power > 10000 * 32 * 4          # at least the Y staging buffer
    assert L.ppca_workspace_bytes(_lib.OP_POWER, ctypes.byref(m), 0, 0) == 0
    assert L.ppca_workspace_bytes(_lib.OP_POWER, ctypes.byref(m), 129, 0) == 0
    assert L.ppca_workspace_bytes(_lib.OP_OJA, ctypes.byref(m), 32, 0) == 0
    assert L.ppca_workspace_bytes(_lib.OP_OJA, ctypes.byref(m), 32, 1000) > 0
    # invalid arguments are rejected on the host
    bad = _lib._Matrix(16, 100, 64, 32, _lib.F32, 0)          # ld < d
    assert L.ppca_prime_power(ctypes.byref(bad), 4, 4, 1, ctypes.c_void_p(16), None, None,
                              ctypes.c_void_p(256), 1 << 20, None) == -1
    fp8_no_scale = _lib._Matrix(16, 100, 64, 64, _lib.FP8_E4M3, 0)
    assert L.ppca_prime_power(ctypes.byref(fp8_no_scale), 4, 4, 1, ctypes.c_void_p(16), None,
                              None, ctypes.c_void_p(256), 1 << 20, None) == -2
    misaligned = _lib._Matrix(8, 100, 64, 64, _lib.F32, 0)
    assert L.ppca_prime_power(ctypes.byref(misaligned), 4, 4, 1, ctypes.c_void_p(16), None,
                              None, ctypes.c_void_p(256), 1 << 20, None) == -8
    odd_ld = _lib._Matrix(16, 100, 63, 63, _lib.F32, 0)
    assert L.ppca_prime_power(ctypes.byref(odd_ld), 4, 4, 1, ctypes.c_void_p(16), None,
                              None, ctypes.c_void_p(256), 1 << 20, None) == -8
    ok = _lib._Matrix(16, 100, 64, 64, _lib.F32, 0)
    assert L.ppca_prime_power(ctypes.byref(ok), 4, 4, 1, ctypes.c_void_p(16), None, None,
                              ctypes.c_void_p(256), 16, None) == -6    # workspace too small
    assert L.ppca_prime_power(ctypes.byref(ok), 0, 4, 1, ctypes.c_void_p(16), None, None,
                              ctypes.c_void_p(256), 1 << 30, None) == -1   # k = 0
    assert L.ppca_prime_power(ctypes.byref(ok), 64, 1, 1, ctypes.c_void_p(16), None, None,
                              ctypes.c_void_p(256), 1 << 30, None) == -1   # K > d


def test_grouped_work_split_host_calls():
    """Work-item size of the grouped calls: range check of the setter, and the
    workspace of a plan grows as the items shrink (more partial sums); a
    too-small workspace is rejected by the tuner before anything runs."""
    from paper_2109_03709_amd import _lib
    L = _lib.lib()
    probs = (_lib._Problem * 2)()
    for p, (n, d, k) in enumerate([(50_000, 256, 8), (20_000, 768, 16)]):
        probs[p].X = _lib._Matrix(16, n, d, d, _lib.BF16, 0)
        probs[p].k, probs[p].l = k, k
        probs[p].V = probs[p].G = probs[p].B = 16
    assert L.ppca_set_group_item_bytes(1024) == -1
    assert L.ppca_set_group_item_bytes(1 << 31) == -1
    small = L.ppca_grouped_workspace_bytes_for(probs, 2, 1 << 20)
    large = L.ppca_grouped_workspace_bytes_for(probs, 2, 8 << 20)
    assert small > large > 0
    assert L.ppca_grouped_workspace_bytes_for(probs, 2, 1024) == 0    # out of range
    try:
        assert L.ppca_set_group_item_bytes(1 << 20) == 0
        assert L.ppca_grouped_workspace_bytes(probs, 2) == small
    finally:
        assert L.ppca_set_group_item_bytes(0) == 0
    assert L.ppca_grouped_workspace_bytes(probs, 2) == L.ppca_grouped_workspace_bytes_for(
        probs, 2, 3 << 20)
    cand = (ctypes.c_int64 * 2)(1 << 20, 4 << 20)
    best = ctypes.c_int64(0)
    assert L.ppca_tune_group_items(probs, 2, cand, 2, ctypes.c_void_p(256), 4096, None,
                                   ctypes.byref(best), None) == -6
    bad = (ctypes.c_int64 * 1)(100)
    assert L.ppca_tune_group_items(probs, 2, bad, 1, ctypes.c_void_p(256), 1 << 40, None,
                                   ctypes.byref(best), None) == -1


def test_noalloc_rayleigh_ritz_host_checks():
    """The allocation-free Rayleigh-Ritz validates on the host before touching
    the device (bad arguments are rejected with no GPU call), and its
    workspace is bounded whatever n and d: the widest problems fit the fixed
    scratch at the largest K."""
    from paper_2109_03709_amd import _lib
    L = _lib.lib()
    assert _lib.NOALLOC_SCRATCH_BYTES == 4 << 20
    p = ctypes.c_void_p(256)
    for n, d in ((16, 64), (6654, 15_116_544), (1 << 40, 1 << 34)):
        for dt in (_lib.F32, _lib.BF16):
            m = _lib._Matrix(16, n, d, d, dt, 0)
            need = L.ppca_workspace_bytes(_lib.OP_RR, ctypes.byref(m), 128, 0)
            assert 0 < need <= 3 << 20, (n, d, dt, need)
    ok = _lib._Matrix(16, 1000, 64, 64, _lib.F32, 0)
    assert L.ppca_workspace_bytes(_lib.OP_RR, ctypes.byref(ok), 16, 0) < _lib.NOALLOC_SCRATCH_BYTES
    assert L.ppca_rayleigh_ritz_noalloc(ctypes.byref(ok), 0, 1, p, p, p, p, p, None) == -1
    assert L.ppca_rayleigh_ritz_noalloc(ctypes.byref(ok), 16, 17, p, p, p, p, p, None) == -1
    assert L.ppca_rayleigh_ritz_noalloc(ctypes.byref(ok), 16, 4, None, p, p, p, p, None) == -1
    fp8_no_scale = _lib._Matrix(16, 1000, 64, 64, _lib.FP8_E4M3, 0)
    assert L.ppca_rayleigh_ritz_noalloc(ctypes.byref(fp8_no_scale), 16, 4, p, p, p, p, p,
                                        None) == -2
