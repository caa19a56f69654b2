"""CPU oracle for the snapshot / validation hot path (ctypes over ``kco.c``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark import this package; the product library and
its Python binding never do, and this package imports nothing from them.

Every function here is a thin marshalling layer over the plain C in
``kco.c``; the arithmetic lives there, each part citing the paper passage it
serves (see the header of ``kco.h``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkco.so")
SOURCES = [os.path.join(HERE, "kco.c")]

OK, EINVAL, EALIGN, EORDER, ENOMEM, EDTYPE = 0, -1, -2, -3, -4, -6
F32, BF16, F16, FP8_E4M3FN, U8 = 0, 1, 2, 3, 4
F64, FP8_E4M3FNUZ, FP8_E5M2, FP8_E5M2FNUZ, I8, I16, I32, I64 = 5, 6, 7, 8, 9, 10, 11, 12
ELEM_SIZE = {F32: 4, BF16: 2, F16: 2, FP8_E4M3FN: 1, U8: 1, F64: 8, FP8_E4M3FNUZ: 1, FP8_E5M2: 1,
             FP8_E5M2FNUZ: 1, I8: 1, I16: 2, I32: 4, I64: 8}
PAGE = 4096


def build(force: bool = True) -> str:
    """Compile ``kco.c`` into ``libkco.so`` with plain ``gcc -O2``."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp",
           *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Range(ctypes.Structure):
    _fields_ = [("base", ctypes.c_uint64), ("size", ctypes.c_uint64)]


class ScanResult(ctypes.Structure):
    _fields_ = [("n_words", ctypes.c_uint64), ("n_ptr_like", ctypes.c_uint64),
                ("n_in_range", ctypes.c_uint64), ("n_oob", ctypes.c_uint64),
                ("n_written", ctypes.c_uint32), ("truncated", ctypes.c_uint32)]


class Oob(ctypes.Structure):
    _fields_ = [("word_va", ctypes.c_uint64), ("value", ctypes.c_uint64)]


class CmpResult(ctypes.Structure):
    _fields_ = [("n_elems", ctypes.c_uint64), ("n_mismatch_elems", ctypes.c_uint64),
                ("n_mismatch_bytes", ctypes.c_uint64), ("first_mismatch", ctypes.c_uint64),
                ("n_nan_both", ctypes.c_uint64), ("n_nan_cand_only", ctypes.c_uint64),
                ("n_nan_gold_only", ctypes.c_uint64), ("n_over_tol", ctypes.c_uint64),
                ("max_abs", ctypes.c_double), ("max_rel", ctypes.c_double),
                ("ulp_hist", ctypes.c_uint64 * 48),
                ("pass_", ctypes.c_uint32), ("status", ctypes.c_uint32),
                ("n_not_close", ctypes.c_uint64), ("pass_close", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = os.environ.get("KCO_LIB") or LIB_PATH  # KCO_LIB: load another build (mutation tests)
        if path == LIB_PATH and (not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
                os.path.getmtime(f) for f in SOURCES + [os.path.join(HERE, "kco.h")])):
            build()  # missing or older than its sources
        L = ctypes.CDLL(path)
        u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
        P = ctypes.POINTER
        L.kco_xxh64.argtypes = [vp, u64, u64]
        L.kco_xxh64.restype = u64
        L.kco_range_check.argtypes = [P(Range), u32, P(u64), P(u64)]
        L.kco_default_window.argtypes = [P(Range), u32, P(u64), P(u64)]
        L.kco_page_hash.argtypes = [P(Range), P(vp), u32, u64, vp, vp, vp, vp]
        L.kco_range_check_unit.argtypes = [P(Range), u32, u64, P(u64), P(u64)]
        L.kco_page_hash_unit.argtypes = [P(Range), P(vp), u32, u64, u64, vp, vp, vp, vp]
        L.kco_compact_unit.argtypes = [P(Range), P(vp), u32, u64, vp, vp, vp, vp, u64, P(u64)]
        L.kco_restore_unit.argtypes = [P(Range), P(vp), u32, u64, vp, vp, vp, vp, u64, u64, P(u64)]
        L.kco_region_diff_unit.argtypes = [P(Range), P(vp), u32, u64, vp, vp, vp, u64, u64, vp]
        L.kco_compact.argtypes = [P(Range), P(vp), u32, vp, vp, vp, vp, u64, P(u64)]
        L.kco_restore.argtypes = [P(Range), P(vp), u32, vp, vp, vp, vp, u64, u64, P(u64)]
        L.kco_closure_scan.argtypes = [P(Range), P(vp), u32, u64, u64, P(ScanResult), P(Oob), u64]
        L.kco_closure_scan_range.argtypes = [P(Range), u32, u32, vp, u64, u64, P(ScanResult), P(Oob), u64]
        L.kco_compare.argtypes = [vp, vp, u64, u32, u32, ctypes.c_double, ctypes.c_double, P(CmpResult)]
        L.kco_ulp.argtypes = [u32, u64, u64, P(u64)]
        L.kco_pointer_graph.argtypes = [P(Range), P(vp), u32, u64, u64, vp]
        L.kco_graph_reach.argtypes = [P(Range), u32, vp, vp, u64, vp]
        L.kco_region_diff.argtypes = [P(Range), P(vp), u32, vp, vp, vp, u64, u64, vp]
        L.kco_ulp_bin.argtypes = [u64]
        L.kco_ulp_bin.restype = u32
        for name in ("kco_range_check_unit", "kco_page_hash_unit", "kco_compact_unit", "kco_restore_unit",
                     "kco_region_diff_unit"):
            getattr(L, name).restype = i32
        for name in ("kco_range_check", "kco_default_window", "kco_page_hash", "kco_compact",
                     "kco_restore", "kco_closure_scan", "kco_closure_scan_range", "kco_compare", "kco_ulp", "kco_pointer_graph",
                     "kco_graph_reach", "kco_region_diff"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _check(code: int, what: str) -> None:
    if code != OK:
        raise OracleError(code, what)


def _ptr(a) -> int | None:
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _ranges(ranges):
    arr = (Range * max(1, len(ranges)))()
    for i, (b, s) in enumerate(ranges):
        arr[i].base, arr[i].size = int(b), int(s)
    return arr


def _hosts(views):
    arr = (ctypes.c_void_p * max(1, len(views)))()
    for i, v in enumerate(views):
        assert v.dtype == np.uint8 and v.flags["C_CONTIGUOUS"]
        arr[i] = v.ctypes.data
    return arr


def xxh64(data, seed: int = 0) -> int:
    buf = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data
    buf = np.ascontiguousarray(buf)
    return int(lib().kco_xxh64(buf.ctypes.data if buf.size else None, buf.nbytes, seed & (2**64 - 1)))


def range_check(ranges, unit: int = PAGE):
    """Returns (status, n_pages, first_page[n+1]); pages are hash units of
    ``unit`` bytes."""
    fp = np.zeros(len(ranges) + 1, dtype=np.uint64)
    n_pages = ctypes.c_uint64(0)
    st = lib().kco_range_check_unit(_ranges(ranges), len(ranges), unit,
                                    fp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    ctypes.byref(n_pages))
    return st, int(n_pages.value), fp


def default_window(ranges):
    lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().kco_default_window(_ranges(ranges), len(ranges), ctypes.byref(lo),
                                    ctypes.byref(hi)), "default_window")
    return int(lo.value), int(hi.value)


def _n_pages(ranges, unit: int = PAGE) -> int:
    st, n, _ = range_check(ranges, unit)
    _check(st, "range_check")
    return n


def page_hash(ranges, views, seed: int = 0, prior=None, unit: int = PAGE):
    """Returns (hash u64[N], zero_bm u64[W], changed_bm u64[W] or None) over
    hash units of ``unit`` bytes."""
    n = _n_pages(ranges, unit)
    w = (n + 63) // 64
    h = np.zeros(n, dtype=np.uint64)
    z = np.zeros(w, dtype=np.uint64)
    c = np.zeros(w, dtype=np.uint64) if prior is not None else None
    if prior is not None:
        prior = np.ascontiguousarray(prior, dtype=np.uint64)
        assert prior.size == n
    _check(lib().kco_page_hash_unit(_ranges(ranges), _hosts(views), len(ranges), unit, seed & (2**64 - 1),
                                    _ptr(prior), _ptr(h), _ptr(z), _ptr(c)), "page_hash")
    return h, z, c


def compact(ranges, views, zero_bm, changed_bm=None, cap_pages=None, unit: int = PAGE):
    """Returns (packed u8[min(n_kept,cap)*unit], page_va u64[min(n_kept,cap)], n_kept)."""
    n = _n_pages(ranges, unit)
    cap = n if cap_pages is None else int(cap_pages)
    packed = np.full(max(cap, 1) * unit, 0xEE, dtype=np.uint8)   # every byte of a slot must be written
    va = np.zeros(max(cap, 1), dtype=np.uint64)
    n_kept = ctypes.c_uint64(0)
    zero_bm = np.ascontiguousarray(zero_bm, dtype=np.uint64)
    if changed_bm is not None:
        changed_bm = np.ascontiguousarray(changed_bm, dtype=np.uint64)
    _check(lib().kco_compact_unit(_ranges(ranges), _hosts(views), len(ranges), unit, _ptr(zero_bm),
                                  _ptr(changed_bm), _ptr(packed), _ptr(va), cap,
                                  ctypes.byref(n_kept)), "compact")
    k = min(int(n_kept.value), cap)
    return packed[: k * unit], va[:k], int(n_kept.value)


def restore(ranges, views, zero_bm, changed_bm, packed, page_va, n_kept, cap_pages=None, unit: int = PAGE):
    """Writes into ``views`` in place; returns the number of rejected page VAs."""
    cap = len(page_va) if cap_pages is None else int(cap_pages)
    n_bad = ctypes.c_uint64(0)
    zero_bm = np.ascontiguousarray(zero_bm, dtype=np.uint64)
    if changed_bm is not None:
        changed_bm = np.ascontiguousarray(changed_bm, dtype=np.uint64)
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    page_va = np.ascontiguousarray(page_va, dtype=np.uint64)
    _check(lib().kco_restore_unit(_ranges(ranges), _hosts(views), len(ranges), unit, _ptr(zero_bm),
                                  _ptr(changed_bm), _ptr(packed) if packed.size else None,
                                  _ptr(page_va) if page_va.size else None, int(n_kept), cap,
                                  ctypes.byref(n_bad)), "restore")
    return int(n_bad.value)


def closure_scan(ranges, views, win_lo: int = 0, win_hi: int = 0, oob_cap: int = 64):
    """Returns (result dict, oob list of (word_va, value))."""
    res = ScanResult()
    oob = (Oob * max(1, oob_cap))()
    _check(lib().kco_closure_scan(_ranges(ranges), _hosts(views), len(ranges), win_lo, win_hi,
                                  ctypes.byref(res), oob, oob_cap), "closure_scan")
    d = {k: int(getattr(res, k)) for k, _ in ScanResult._fields_}
    return d, [(int(oob[i].word_va), int(oob[i].value)) for i in range(d["n_written"])]


def closure_scan_range(ranges, a: int, view, win_lo: int = 0, win_hi: int = 0, oob_cap: int = 64):
    """The closure scan of range ``a``'s words (host bytes ``view``) against
    every range: returns (result dict, oob list of (word_va, value))."""
    res = ScanResult()
    oob = (Oob * max(1, oob_cap))()
    v = np.ascontiguousarray(view).view(np.uint8)
    assert not 0 <= a < len(ranges) or v.nbytes >= ranges[a][1]
    _check(lib().kco_closure_scan_range(_ranges(ranges), len(ranges), a, _ptr(v), win_lo, win_hi,
                                        ctypes.byref(res), oob, oob_cap), "closure_scan_range")
    d = {k: int(getattr(res, k)) for k, _ in ScanResult._fields_}
    return d, [(int(oob[i].word_va), int(oob[i].value)) for i in range(d["n_written"])]


class RegionDiff(ctypes.Structure):
    _fields_ = [("n_diff_bytes", ctypes.c_uint64), ("n_diff_pages", ctypes.c_uint64),
                ("first_diff_va", ctypes.c_uint64), ("n_bad_pages", ctypes.c_uint64)]


def region_diff(ranges, views, gold_zero_bm, gold_packed, gold_page_va, gold_n_kept: int,
                cap_pages: int | None = None, unit: int = PAGE) -> list[dict]:
    """Per-range byte difference of the live bytes in ``views`` against a full snapshot."""
    n = len(ranges)
    zb = np.ascontiguousarray(gold_zero_bm, dtype=np.uint64)
    pk = np.ascontiguousarray(gold_packed, dtype=np.uint8)
    va = np.ascontiguousarray(gold_page_va, dtype=np.uint64)
    cap = len(va) if cap_pages is None else int(cap_pages)
    res = (RegionDiff * max(1, n))()
    _check(lib().kco_region_diff_unit(_ranges(ranges), _hosts(views), n, unit, _ptr(zb) if zb.size else None,
                                      _ptr(pk) if pk.size else None, _ptr(va) if va.size else None,
                                      int(gold_n_kept), cap, res), "region_diff")
    return [{k: int(getattr(res[i], k)) for k, _ in RegionDiff._fields_} for i in range(n)]


def pointer_graph(ranges, views, win_lo: int = 0, win_hi: int = 0) -> np.ndarray:
    """Edge bitmap: n rows of ceil(n / 64) uint64 words (row a, bit b = a -> b)."""
    n = len(ranges)
    rw = (n + 63) // 64
    edge = np.zeros(max(1, n * rw), dtype=np.uint64)
    _check(lib().kco_pointer_graph(_ranges(ranges), _hosts(views), n, win_lo, win_hi, _ptr(edge)),
           "pointer_graph")
    return edge[:n * rw].reshape(n, rw)


def edges_to_bool(edge_bm: np.ndarray, n: int) -> np.ndarray:
    """(n, ceil(n/64)) uint64 rows -> (n, n) boolean adjacency."""
    rows = np.ascontiguousarray(edge_bm, dtype=np.uint64).reshape(n, -1)
    bits = np.unpackbits(rows.view(np.uint8).reshape(n, -1), axis=1, bitorder="little")
    return bits[:, :n].astype(bool)


def graph_reach(ranges, edge_bm, root_words) -> np.ndarray:
    """Boolean mask of the ranges reachable from the root words."""
    n = len(ranges)
    rw = (n + 63) // 64
    edge = np.ascontiguousarray(edge_bm, dtype=np.uint64).reshape(-1)
    roots = np.ascontiguousarray(root_words, dtype=np.uint64).reshape(-1)
    reach = np.zeros(max(1, rw), dtype=np.uint64)
    _check(lib().kco_graph_reach(_ranges(ranges), n, _ptr(edge) if edge.size else None,
                                 _ptr(roots) if roots.size else None, roots.size, _ptr(reach)), "graph_reach")
    bits = np.unpackbits(reach.view(np.uint8), bitorder="little")
    return bits[:n].astype(bool)


def compare(cand, gold, dtype: int, ulp_tol: int = 0, atol: float = 0.0, rtol: float = 0.0):
    """cand / gold: numpy arrays (any dtype) holding n elements of ``dtype``."""
    es = ELEM_SIZE.get(dtype)
    if es is None:
        res = CmpResult()
        _check(lib().kco_compare(None, None, 0, dtype, ulp_tol, atol, rtol, ctypes.byref(res)), "compare")
    c = np.ascontiguousarray(cand).view(np.uint8)
    g = np.ascontiguousarray(gold).view(np.uint8)
    assert c.nbytes == g.nbytes and c.nbytes % es == 0
    res = CmpResult()
    _check(lib().kco_compare(_ptr(c) if c.size else None, _ptr(g) if g.size else None,
                             c.nbytes // es, dtype, ulp_tol, atol, rtol, ctypes.byref(res)), "compare")
    return cmp_to_dict(res)


def cmp_to_dict(res: CmpResult) -> dict:
    d = {}
    for k, _ in CmpResult._fields_:
        v = getattr(res, k)
        if k == "ulp_hist":
            d[k] = [int(x) for x in v]
        elif k == "pass_":
            d["pass"] = int(v)
        elif k == "reserved":
            continue
        else:
            d[k] = float(v) if k.startswith("max_") else int(v)
    return d


def ulp(dtype: int, cand_bits: int, gold_bits: int) -> int:
    d = ctypes.c_uint64(0)
    _check(lib().kco_ulp(dtype, cand_bits, gold_bits, ctypes.byref(d)), "ulp")
    return int(d.value)


def ulp_bin(d: int) -> int:
    return int(lib().kco_ulp_bin(d))
