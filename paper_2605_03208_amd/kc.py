"""ctypes binding of ``libkc.so`` (the C ABI declared in ``include/kc.h``).

Argument marshalling only: tensors become device pointers, the current torch
stream becomes the HIP stream, result structs are decoded.  Every step of the
path runs in the library's HIP kernels; if the library is missing this module
raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkc.so")
PAGE = 4096
ABI_VERSION = 7  # layout of the structs, the entry-point set and the range rules below

OK, EINVAL, EALIGN, EORDER, ENOMEM, EHIP, EDTYPE, ELIMIT, ERELOC = 0, -1, -2, -3, -4, -5, -6, -7, -8
F32, BF16, F16, FP8_E4M3FN, U8 = 0, 1, 2, 3, 4
F64, FP8_E4M3FNUZ, FP8_E5M2, FP8_E5M2FNUZ, I8, I16, I32, I64 = 5, 6, 7, 8, 9, 10, 11, 12
TORCH_TO_KC = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16, torch.float8_e4m3fn: FP8_E4M3FN,
               torch.uint8: U8, torch.float64: F64, torch.float8_e4m3fnuz: FP8_E4M3FNUZ,
               torch.float8_e5m2: FP8_E5M2, torch.float8_e5m2fnuz: FP8_E5M2FNUZ, torch.int8: I8,
               torch.int16: I16, torch.int32: I32, torch.int64: I64}
ELEM_SIZE = {k: torch.empty(0, dtype=t).element_size() for t, k in TORCH_TO_KC.items()}
OP_PAGE_HASH, OP_SNAPSHOT, OP_COMPACT, OP_RESTORE, OP_CLOSURE, OP_COMPARE, OP_GRAPH, OP_REGION_DIFF = range(8)
GRAPH_MAX_RANGES = 16384
NOALLOC_MAX_PAIRS = 4096

SYMBOLS = ["kc_strerror", "kc_last_error", "kc_abi_version", "kc_range_check", "kc_default_window",
           "kc_ctx_create", "kc_ctx_destroy", "kc_ctx_set_tuning", "kc_ctx_get_tuning",
           "kc_ctx_enable_timing", "kc_ctx_kernel_ms",
           "kc_rangeset_create", "kc_rangeset_destroy", "kc_page_hash", "kc_compact", "kc_snapshot",
           "kc_restore", "kc_closure_scan", "kc_compare", "kc_pairset_create", "kc_pairset_destroy",
           "kc_compare_pairset", "kc_snapshot_save", "kc_snapshot_load", "kc_pointer_graph", "kc_graph_reach",
           "kc_region_diff", "kc_vaspace_create", "kc_vaspace_destroy", "kc_vaspace_suggest", "kc_perturb",
           "kc_compare_noalloc", "kc_rangeset_create_unit", "kc_materialize"]


class KCError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        msg = f"{what}: {code} ({strerror(code)})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.code = code


class Range(ctypes.Structure):
    _fields_ = [("base", ctypes.c_uint64), ("size", ctypes.c_uint64)]


class ScanResult(ctypes.Structure):
    _fields_ = [("n_words", ctypes.c_uint64), ("n_ptr_like", ctypes.c_uint64),
                ("n_in_range", ctypes.c_uint64), ("n_oob", ctypes.c_uint64),
                ("n_written", ctypes.c_uint32), ("truncated", ctypes.c_uint32)]


class ScanArgs(ctypes.Structure):
    _fields_ = [("win_lo", ctypes.c_uint64), ("win_hi", ctypes.c_uint64),
                ("res_d", ctypes.c_void_p), ("oob_d", ctypes.c_void_p), ("oob_cap", ctypes.c_uint64)]


class Pair(ctypes.Structure):
    _fields_ = [("cand_d", ctypes.c_void_p), ("gold_d", ctypes.c_void_p), ("n_elems", ctypes.c_uint64),
                ("dtype", ctypes.c_uint32), ("ulp_tol", ctypes.c_uint32), ("atol", ctypes.c_double),
                ("rtol", ctypes.c_double)]


class PerturbBuf(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint64), ("length", ctypes.c_uint64), ("seed", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


_PERTURB_NP = np.dtype([("offset", "<u8"), ("length", "<u8"), ("seed", "<u4"), ("reserved", "<u4")])
assert _PERTURB_NP.itemsize == ctypes.sizeof(PerturbBuf)


class MaterializeBuf(ctypes.Structure):
    _fields_ = [("src_d", ctypes.c_uint64), ("offset", ctypes.c_uint64), ("length", ctypes.c_uint64),
                ("seed", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_MATERIALIZE_NP = np.dtype([("src_d", "<u8"), ("offset", "<u8"), ("length", "<u8"), ("seed", "<u4"),
                            ("reserved", "<u4")])
assert _MATERIALIZE_NP.itemsize == ctypes.sizeof(MaterializeBuf)


class CmpResult(ctypes.Structure):
    _fields_ = [("n_elems", ctypes.c_uint64), ("n_mismatch_elems", ctypes.c_uint64),
                ("n_mismatch_bytes", ctypes.c_uint64), ("first_mismatch", ctypes.c_uint64),
                ("n_nan_both", ctypes.c_uint64), ("n_nan_cand_only", ctypes.c_uint64),
                ("n_nan_gold_only", ctypes.c_uint64), ("n_over_tol", ctypes.c_uint64),
                ("max_abs", ctypes.c_double), ("max_rel", ctypes.c_double),
                ("ulp_hist", ctypes.c_uint64 * 48), ("pass_", ctypes.c_uint32), ("status", ctypes.c_uint32),
                ("n_not_close", ctypes.c_uint64), ("pass_close", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class IoStats(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_uint64), ("seconds", ctypes.c_double), ("copy_wait_s", ctypes.c_double),
                ("file_s", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("grid_per_cu", ctypes.c_uint32), ("tile_bytes", ctypes.c_uint32),
                ("per_item", ctypes.c_uint32), ("depth", ctypes.c_uint32)]


RESULT_BYTES = 488
assert ctypes.sizeof(CmpResult) == RESULT_BYTES and ctypes.sizeof(ScanResult) == 40 and ctypes.sizeof(Pair) == 48


_lib = None


def lib() -> ctypes.CDLL:
    """Load libkc.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_03208_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        P = ctypes.POINTER
        sig = {
            "kc_strerror": ([i32], ctypes.c_char_p),
            "kc_last_error": ([], ctypes.c_char_p),
            "kc_abi_version": ([], i32),
            "kc_range_check": ([P(Range), u32, P(u64)], i32),
            "kc_default_window": ([P(Range), u32, P(u64), P(u64)], i32),
            "kc_ctx_create": ([P(vp), i32], i32),
            "kc_ctx_destroy": ([vp], None),
            "kc_ctx_set_tuning": ([vp, u32, P(Tuning)], i32),
            "kc_ctx_get_tuning": ([vp, u32, P(Tuning)], i32),
            "kc_ctx_enable_timing": ([vp, i32], i32),
            "kc_ctx_kernel_ms": ([vp, u32, P(ctypes.c_float)], i32),
            "kc_rangeset_create": ([vp, P(Range), u32, P(vp), P(u64)], i32),
            "kc_rangeset_destroy": ([vp], None),
            "kc_page_hash": ([vp, vp, u64, vp, vp, vp, vp, P(ScanArgs), vp], i32),
            "kc_compact": ([vp, vp, vp, vp, vp, vp, u64, vp, vp], i32),
            "kc_snapshot": ([vp, vp, u64, vp, vp, vp, vp, vp, vp, u64, vp, P(ScanArgs), vp], i32),
            "kc_restore": ([vp, vp, vp, vp, vp, vp, vp, u64, vp, vp], i32),
            "kc_closure_scan": ([vp, vp, P(ScanArgs), vp], i32),
            "kc_compare": ([vp, P(Pair), u32, vp, vp], i32),
            "kc_pairset_create": ([vp, P(Pair), u32, P(vp)], i32),
            "kc_pairset_destroy": ([vp], None),
            "kc_compare_pairset": ([vp, vp, vp, vp], i32),
            "kc_compare_noalloc": ([vp, P(Pair), u32, vp, vp], i32),
            "kc_rangeset_create_unit": ([vp, P(Range), u32, u64, P(vp), P(u64)], i32),
            "kc_snapshot_save": ([vp, vp, ctypes.c_char_p, u64, vp, vp, vp, vp, vp, vp, u64, u64, vp, P(IoStats)],
                                 i32),
            "kc_snapshot_load": ([vp, vp, ctypes.c_char_p, vp, vp, vp, vp, vp, vp, u64, u64, vp, P(IoStats)], i32),
            "kc_pointer_graph": ([vp, vp, u64, u64, vp, vp], i32),
            "kc_graph_reach": ([P(Range), u32, vp, vp, u64, vp], i32),
            "kc_region_diff": ([vp, vp, u64, vp, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp], i32),
            "kc_vaspace_create": ([i32, P(Range), u32, P(vp), P(u32), P(u64)], i32),
            "kc_vaspace_destroy": ([vp], None),
            "kc_vaspace_suggest": ([i32, u64, P(u64)], i32),
            "kc_perturb": ([vp, vp, u64, u32, P(PerturbBuf), u32, u64, u32, vp], i32),
            "kc_materialize": ([vp, vp, u64, u32, P(MaterializeBuf), u32, u64, u32, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        if L.kc_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI {L.kc_abi_version()}, this binding expects {ABI_VERSION}: rebuild")
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().kc_strerror(code).decode()
    except Exception:  # library missing while formatting an error
        return "?"


def _check(code: int, what: str) -> None:
    if code != OK:
        detail = lib().kc_last_error().decode() if code in (EHIP, ERELOC) else ""
        raise KCError(code, what, detail)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ranges(ranges):
    arr = (Range * max(1, len(ranges)))()
    for i, (b, s) in enumerate(ranges):
        arr[i].base, arr[i].size = int(b), int(s)
    return arr


def range_check(ranges) -> tuple[int, int]:
    n = ctypes.c_uint64(0)
    st = lib().kc_range_check(_ranges(ranges), len(ranges), ctypes.byref(n))
    return st, int(n.value)


def default_window(ranges) -> tuple[int, int]:
    lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().kc_default_window(_ranges(ranges), len(ranges), ctypes.byref(lo), ctypes.byref(hi)),
           "kc_default_window")
    return int(lo.value), int(hi.value)


class Context:
    """A kc_ctx on one HIP device (the current torch device by default)."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        self.handle = ctypes.c_void_p()
        _check(lib().kc_ctx_create(ctypes.byref(self.handle), device), "kc_ctx_create")

    def set_tuning(self, op: int, grid_per_cu: int = 0, tile_bytes: int = 0, per_item: int = 0,
                   depth: int = 0) -> None:
        t = Tuning(grid_per_cu, tile_bytes, per_item, depth)
        _check(lib().kc_ctx_set_tuning(self.handle, op, ctypes.byref(t)), "kc_ctx_set_tuning")

    def get_tuning(self, op: int) -> dict:
        t = Tuning()
        _check(lib().kc_ctx_get_tuning(self.handle, op, ctypes.byref(t)), "kc_ctx_get_tuning")
        return dict(grid_per_cu=t.grid_per_cu, tile_bytes=t.tile_bytes, per_item=t.per_item, depth=t.depth)

    timing = False

    def enable_timing(self, on: bool = True) -> None:
        _check(lib().kc_ctx_enable_timing(self.handle, 1 if on else 0), "kc_ctx_enable_timing")
        self.timing = bool(on)

    def kernel_ms(self, op: int) -> float:
        """Duration of the main kernel(s) of the op's last call (waits for it)."""
        ms = ctypes.c_float(0)
        _check(lib().kc_ctx_kernel_ms(self.handle, op, ctypes.byref(ms)), "kc_ctx_kernel_ms")
        return float(ms.value)

    def close(self) -> None:
        if self.handle:
            lib().kc_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RangeSet:
    """Uploaded range table (tracked allocations) plus the scratch its calls use.
    ``unit``: the hash unit in bytes (4 KiB pages by default, a power of two up
    to 2 MiB); ``n_pages`` and ``n_words`` then count units."""

    def __init__(self, ctx: Context, ranges, unit: int = PAGE):
        self.ctx = ctx
        self.ranges = [(int(b), int(s)) for b, s in ranges]
        self.unit = int(unit)
        self.handle = ctypes.c_void_p()
        n = ctypes.c_uint64(0)
        _check(lib().kc_rangeset_create_unit(ctx.handle, _ranges(self.ranges), len(self.ranges), self.unit,
                                             ctypes.byref(self.handle), ctypes.byref(n)), "kc_rangeset_create_unit")
        self.n_pages = int(n.value)
        self.n_words = (self.n_pages + 63) // 64

    def close(self) -> None:
        if self.handle:
            lib().kc_rangeset_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VaSpace:
    """Device memory mapped at exactly the given ranges' VAs (create it before
    other device allocations of the process); raises KCError with code ERELOC
    when a range cannot be placed at its address."""

    def __init__(self, device: int, ranges):
        self.ranges = [(int(b), int(s)) for b, s in ranges]
        self.handle = ctypes.c_void_p()
        n_spans, mapped = ctypes.c_uint32(0), ctypes.c_uint64(0)
        _check(lib().kc_vaspace_create(device, _ranges(self.ranges), len(self.ranges), ctypes.byref(self.handle),
                                       ctypes.byref(n_spans), ctypes.byref(mapped)), "kc_vaspace_create")
        self.n_spans, self.mapped_bytes = int(n_spans.value), int(mapped.value)

    def close(self) -> None:
        if self.handle:
            lib().kc_vaspace_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vaspace_suggest(device: int, size: int) -> int:
    """An address where ``size`` bytes could be reserved a moment ago."""
    base = ctypes.c_uint64(0)
    _check(lib().kc_vaspace_suggest(device, size, ctypes.byref(base)), "kc_vaspace_suggest")
    return int(base.value)


class ScanOut:
    """Device buffers receiving a closure-scan result and its out-of-range list."""

    def __init__(self, device, oob_cap: int = 1024, win_lo: int = 0, win_hi: int = 0):
        self.res = torch.zeros(40, dtype=torch.uint8, device=device)
        self.oob = torch.zeros(max(1, oob_cap) * 16, dtype=torch.uint8, device=device)
        self.cap = oob_cap
        self.args = ScanArgs(win_lo, win_hi, self.res.data_ptr(), self.oob.data_ptr(), oob_cap)

    def result(self) -> tuple[dict, list]:
        r = ScanResult.from_buffer_copy(bytes(self.res.cpu().numpy()))
        d = {k: int(getattr(r, k)) for k, _ in ScanResult._fields_}
        raw = self.oob.cpu().numpy().view("<u8").reshape(-1, 2)
        return d, [(int(a), int(v)) for a, v in raw[: d["n_written"]]]


def _u64(n: int, device) -> torch.Tensor:
    return torch.empty(max(1, n), dtype=torch.int64, device=device)


def page_hash(ctx: Context, rs: RangeSet, seed: int = 0, prior: torch.Tensor | None = None,
              scan: ScanOut | None = None, out=None, stream=None):
    """Returns (hash[N], zero_bm[W], changed_bm[W] or None) as int64 device tensors."""
    dev = torch.device("cuda", ctx.device)
    h, z, c = out if out is not None else (_u64(rs.n_pages, dev), _u64(rs.n_words, dev),
                                           _u64(rs.n_words, dev) if prior is not None else None)
    _check(lib().kc_page_hash(ctx.handle, rs.handle, seed & (2**64 - 1), _ptr(prior), _ptr(h), _ptr(z),
                              _ptr(c), ctypes.byref(scan.args) if scan else None, _stream(stream)),
           "kc_page_hash")
    return h, z, c


def compact(ctx: Context, rs: RangeSet, zero_bm, changed_bm=None, cap_pages: int | None = None, out=None,
            stream=None):
    """Returns (packed u8[cap*unit], page_va int64[cap], n_kept int64[1]) device tensors."""
    dev = torch.device("cuda", ctx.device)
    cap = rs.n_pages if cap_pages is None else int(cap_pages)
    packed, va, nk = out if out is not None else (
        torch.empty(max(1, cap) * rs.unit, dtype=torch.uint8, device=dev), _u64(cap, dev), _u64(1, dev))
    _check(lib().kc_compact(ctx.handle, rs.handle, _ptr(zero_bm), _ptr(changed_bm), _ptr(packed), _ptr(va),
                            cap, _ptr(nk), _stream(stream)), "kc_compact")
    return packed, va, nk


def snapshot(ctx: Context, rs: RangeSet, seed: int = 0, prior=None, cap_pages: int | None = None,
             scan: ScanOut | None = None, out=None, stream=None):
    """Returns dict(hash, zero_bm, changed_bm, packed, page_va, n_kept) device tensors."""
    dev = torch.device("cuda", ctx.device)
    cap = rs.n_pages if cap_pages is None else int(cap_pages)
    if out is None:
        out = dict(hash=_u64(rs.n_pages, dev), zero_bm=_u64(rs.n_words, dev),
                   changed_bm=_u64(rs.n_words, dev) if prior is not None else None,
                   packed=torch.empty(max(1, cap) * rs.unit, dtype=torch.uint8, device=dev),
                   page_va=_u64(cap, dev), n_kept=_u64(1, dev))
    _check(lib().kc_snapshot(ctx.handle, rs.handle, seed & (2**64 - 1), _ptr(prior), _ptr(out["hash"]),
                             _ptr(out["zero_bm"]), _ptr(out.get("changed_bm")), _ptr(out["packed"]),
                             _ptr(out["page_va"]), cap, _ptr(out["n_kept"]),
                             ctypes.byref(scan.args) if scan else None, _stream(stream)), "kc_snapshot")
    return out


def restore(ctx: Context, rs: RangeSet, zero_bm, changed_bm, packed, page_va, n_kept, cap_pages: int | None = None,
            n_bad=None, stream=None):
    cap = page_va.numel() if cap_pages is None else int(cap_pages)
    _check(lib().kc_restore(ctx.handle, rs.handle, _ptr(zero_bm), _ptr(changed_bm), _ptr(packed), _ptr(page_va),
                            _ptr(n_kept), cap, _ptr(n_bad), _stream(stream)), "kc_restore")


def closure_scan(ctx: Context, rs: RangeSet, scan: ScanOut, stream=None) -> None:
    _check(lib().kc_closure_scan(ctx.handle, rs.handle, ctypes.byref(scan.args), _stream(stream)),
           "kc_closure_scan")


REGION_DIFF_FIELDS = ("n_diff_bytes", "n_diff_pages", "first_diff_va", "n_bad_pages")


def region_diff(ctx: Context, rs: RangeSet, gold: dict, seed: int = 0, cap_pages: int | None = None,
                out: dict | None = None, stream=None) -> dict:
    """Per-range byte difference of the live ranges against the full snapshot
    ``gold`` (as returned by ``snapshot``).  Returns device tensors: res
    (n_ranges x 4 int64), hash, zero_bm, changed_bm of the live pages."""
    dev = torch.device("cuda", ctx.device)
    cap = gold["page_va"].numel() if cap_pages is None else int(cap_pages)
    n = len(rs.ranges)
    if out is None:
        out = dict(res=torch.empty(max(1, n) * 4, dtype=torch.int64, device=dev), hash=_u64(rs.n_pages, dev),
                   zero_bm=_u64(rs.n_words, dev), changed_bm=_u64(rs.n_words, dev))
    _check(lib().kc_region_diff(ctx.handle, rs.handle, seed & (2**64 - 1), _ptr(gold["hash"]), _ptr(gold["zero_bm"]),
                                _ptr(gold["packed"]), _ptr(gold["page_va"]), _ptr(gold["n_kept"]), cap,
                                _ptr(out["hash"]), _ptr(out["zero_bm"]), _ptr(out["changed_bm"]), _ptr(out["res"]),
                                _stream(stream)), "kc_region_diff")
    return out


def decode_region_diff(res: torch.Tensor, n: int) -> list[dict]:
    """Per-range dicts of the kc_region_diff_result fields, as the library
    wrote them (a host copy; no field is derived here)."""
    raw = res[:n * 4].cpu().numpy().view(np.uint64).reshape(n, 4)
    return [{k: int(v) for k, v in zip(REGION_DIFF_FIELDS, row)} for row in raw]


def pointer_graph(ctx: Context, rs: RangeSet, win_lo: int = 0, win_hi: int = 0,
                  out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Edge bitmap on the device: (n_ranges, ceil(n_ranges / 64)) int64 words,
    row a bit b set iff range a holds a pointer-like word inside range b."""
    n = len(rs.ranges)
    rw = (n + 63) // 64
    if out is None:
        out = torch.empty(max(1, n * rw), dtype=torch.int64, device=torch.device("cuda", ctx.device))
    assert out.numel() * out.element_size() >= n * rw * 8
    _check(lib().kc_pointer_graph(ctx.handle, rs.handle, win_lo, win_hi, _ptr(out), _stream(stream)),
           "kc_pointer_graph")
    return out[:n * rw].view(n, rw) if n else out[:0].view(0, 0)


def graph_reach(ranges, edge_bm, root_words) -> np.ndarray:
    """Host: boolean mask of the ranges reachable from ``root_words`` over the
    edges of ``edge_bm`` (a host copy of ``pointer_graph``'s output)."""
    n = len(ranges)
    rw = (n + 63) // 64
    edge = np.ascontiguousarray(np.asarray(edge_bm).view(np.uint64).reshape(-1))
    assert edge.size >= n * rw
    roots = np.ascontiguousarray(np.asarray(root_words, dtype=np.uint64).reshape(-1))
    reach = np.zeros(max(1, rw), dtype=np.uint64)
    _check(lib().kc_graph_reach(_ranges(ranges), n, edge.ctypes.data if edge.size else None,
                                roots.ctypes.data if roots.size else None, roots.size, reach.ctypes.data),
           "kc_graph_reach")
    return np.unpackbits(reach.view(np.uint8), bitorder="little")[:n].astype(bool)


def make_pairs(pairs) -> tuple[ctypes.Array, int]:
    """pairs: iterable of (cand, gold, dtype, ulp_tol[, atol, rtol]) with device tensors."""
    pairs = list(pairs)
    arr = (Pair * max(1, len(pairs)))()
    for i, p in enumerate(pairs):
        c, g, dt, tol = p[:4]
        atol, rtol = (p[4], p[5]) if len(p) > 4 else (0.0, 0.0)
        n = c.numel() * c.element_size() // ELEM_SIZE[dt]
        assert g.numel() * g.element_size() == c.numel() * c.element_size()
        arr[i] = Pair(_ptr(c), _ptr(g), n, dt, tol, float(atol), float(rtol))
    return arr, len(pairs)


_PAIR_NP = np.dtype([("cand_d", "<u8"), ("gold_d", "<u8"), ("n_elems", "<u8"), ("dtype", "<u4"),
                     ("ulp_tol", "<u4"), ("atol", "<f8"), ("rtol", "<f8")])
assert _PAIR_NP.itemsize == ctypes.sizeof(Pair)


def pairs_from_arrays(cand_ptr, gold_ptr, n_elems, dtype, ulp_tol, atol=0.0, rtol=0.0) -> tuple[ctypes.Array, int]:
    """A kc_pair list from per-pair arrays of device addresses, element
    counts, element types and tolerances (no tensor per pair); the result
    goes to ``compare`` in place of a pair list."""
    n = len(cand_ptr)
    a = np.zeros(max(1, n), dtype=_PAIR_NP)
    a["cand_d"][:n], a["gold_d"][:n], a["n_elems"][:n] = cand_ptr, gold_ptr, n_elems
    a["dtype"][:n], a["ulp_tol"][:n], a["atol"][:n], a["rtol"][:n] = dtype, ulp_tol, atol, rtol
    return (Pair * max(1, n)).from_buffer(a), n


def compare(ctx: Context, pairs, res: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Returns the device buffer of kc_cmp_result structs (decode with ``decode_cmp``)."""
    arr, n = pairs if isinstance(pairs, tuple) else make_pairs(pairs)
    if res is None:
        res = torch.empty(max(1, n) * RESULT_BYTES, dtype=torch.uint8, device=torch.device("cuda", ctx.device))
    _check(lib().kc_compare(ctx.handle, arr, n, _ptr(res), _stream(stream)), "kc_compare")
    return res


def compare_noalloc(ctx: Context, pairs, res: torch.Tensor, stream=None) -> torch.Tensor:
    """kc_compare_noalloc: the compare with nothing allocated by the library;
    ``res`` (at least n * RESULT_BYTES bytes of device memory) is the caller's."""
    arr, n = pairs if isinstance(pairs, tuple) else make_pairs(pairs)
    _check(lib().kc_compare_noalloc(ctx.handle, arr, n, _ptr(res), _stream(stream)), "kc_compare_noalloc")
    return res


def perturb(ctx: Context, arena: torch.Tensor, offsets, lengths, seeds, block: int, kmax: int,
            stream=None) -> None:
    """kc_perturb: in place on the 1-D typed ``arena``, buffer b at element
    ``offsets[b]`` of ``lengths[b]`` elements moved by the perturbation of
    ``seeds[b]`` (one moved element per ``block``, 1..``kmax`` steps)."""
    dt = TORCH_TO_KC.get(arena.dtype)
    if dt is None:
        raise KCError(EDTYPE, "kc_perturb")
    n = len(offsets)
    a = np.zeros(max(1, n), dtype=_PERTURB_NP)
    a["offset"][:n], a["length"][:n] = np.asarray(offsets, dtype=np.int64), np.asarray(lengths, dtype=np.int64)
    a["seed"][:n] = np.asarray(seeds, dtype=np.int64) & 0xFFFFFFFF
    arr = (PerturbBuf * max(1, n)).from_buffer(a)
    _check(lib().kc_perturb(ctx.handle, _ptr(arena), arena.numel(), dt, arr, n, int(block), int(kmax),
                            _stream(stream)), "kc_perturb")


def materialize(ctx: Context, arena: torch.Tensor, src_ptrs, offsets, lengths, seeds, block: int, kmax: int,
                stream=None) -> None:
    """kc_materialize: buffer b of the 1-D typed ``arena`` (element ``offsets[b]``,
    ``lengths[b]`` elements) becomes the golden at device address ``src_ptrs[b]``
    moved by the perturbation of ``seeds[b]``: a copy and kc_perturb in one pass."""
    dt = TORCH_TO_KC.get(arena.dtype)
    if dt is None:
        raise KCError(EDTYPE, "kc_materialize")
    n = len(offsets)
    a = np.zeros(max(1, n), dtype=_MATERIALIZE_NP)
    a["src_d"][:n] = np.asarray(src_ptrs, dtype=np.uint64)
    a["offset"][:n], a["length"][:n] = np.asarray(offsets, dtype=np.int64), np.asarray(lengths, dtype=np.int64)
    a["seed"][:n] = np.asarray(seeds, dtype=np.int64) & 0xFFFFFFFF
    arr = (MaterializeBuf * max(1, n)).from_buffer(a)
    _check(lib().kc_materialize(ctx.handle, _ptr(arena), arena.numel(), dt, arr, n, int(block), int(kmax),
                                _stream(stream)), "kc_materialize")


def snapshot_save(ctx: Context, rs: RangeSet, directory: str, out: dict, seed: int = 0, cap_pages=None,
                  chunk_bytes: int = 0, stream=None) -> dict:
    """Write the snapshot in ``out`` (as returned by ``snapshot``) to files."""
    cap = out["page_va"].numel() if cap_pages is None else int(cap_pages)
    st = IoStats()
    _check(lib().kc_snapshot_save(ctx.handle, rs.handle, directory.encode(), seed & (2**64 - 1), _ptr(out["hash"]),
                                  _ptr(out["zero_bm"]), _ptr(out.get("changed_bm")), _ptr(out["packed"]),
                                  _ptr(out["page_va"]), _ptr(out["n_kept"]), cap, chunk_bytes, _stream(stream),
                                  ctypes.byref(st)), "kc_snapshot_save")
    return dict(bytes=int(st.bytes), seconds=float(st.seconds), copy_wait_s=float(st.copy_wait_s),
                file_s=float(st.file_s))


def snapshot_load(ctx: Context, rs: RangeSet, directory: str, cap_pages: int | None = None, delta: bool = False,
                  chunk_bytes: int = 0, stream=None):
    """Load a saved snapshot into fresh device buffers; returns (out dict, stats)."""
    dev = torch.device("cuda", ctx.device)
    cap = rs.n_pages if cap_pages is None else int(cap_pages)
    out = dict(hash=_u64(rs.n_pages, dev), zero_bm=_u64(rs.n_words, dev),
               changed_bm=_u64(rs.n_words, dev) if delta else None,
               packed=torch.empty(max(1, cap) * rs.unit, dtype=torch.uint8, device=dev),
               page_va=_u64(cap, dev), n_kept=_u64(1, dev))
    st = IoStats()
    _check(lib().kc_snapshot_load(ctx.handle, rs.handle, directory.encode(), _ptr(out["hash"]), _ptr(out["zero_bm"]),
                                  _ptr(out["changed_bm"]), _ptr(out["packed"]), _ptr(out["page_va"]),
                                  _ptr(out["n_kept"]), cap, chunk_bytes, _stream(stream), ctypes.byref(st)),
           "kc_snapshot_load")
    return out, dict(bytes=int(st.bytes), seconds=float(st.seconds), copy_wait_s=float(st.copy_wait_s),
                     file_s=float(st.file_s))


class PairSet:
    """A resident pair list (kc_pairset): compares through it allocate nothing
    and never synchronise, so they can be recorded into a graph."""

    def __init__(self, ctx: Context, pairs):
        self.ctx = ctx
        self.arr, self.n = pairs if isinstance(pairs, tuple) else make_pairs(pairs)
        self.handle = ctypes.c_void_p()
        _check(lib().kc_pairset_create(ctx.handle, self.arr, self.n, ctypes.byref(self.handle)),
               "kc_pairset_create")

    def close(self) -> None:
        if self.handle:
            lib().kc_pairset_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compare_pairset(ctx: Context, ps: PairSet, res: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if res is None:
        res = torch.empty(max(1, ps.n) * RESULT_BYTES, dtype=torch.uint8, device=torch.device("cuda", ctx.device))
    _check(lib().kc_compare_pairset(ctx.handle, ps.handle, _ptr(res), _stream(stream)), "kc_compare_pairset")
    return res


def decode_cmp(res: torch.Tensor, n: int) -> list[dict]:
    raw = bytes(res.cpu().numpy()[: n * RESULT_BYTES])
    out = []
    for i in range(n):
        r = CmpResult.from_buffer_copy(raw[i * RESULT_BYTES:(i + 1) * RESULT_BYTES])
        d = {}
        for k, _ in CmpResult._fields_:
            v = getattr(r, k)
            if k == "ulp_hist":
                d[k] = [int(x) for x in v]
            elif k == "pass_":
                d["pass"] = int(v)
            elif k == "reserved":
                continue
            else:
                d[k] = float(v) if k.startswith("max_") else int(v)
        out.append(d)
    return out
