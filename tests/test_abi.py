"""The C-ABI library loads and exports every function ``include/kc.h``
declares; its host-only checks agree with the oracle (no device needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def kc():
    from paper_2605_03208_amd import kc as K
    if not os.path.exists(K.LIB_PATH):
        from paper_2605_03208_amd import build
        build.build()
    K.lib()
    return K


def test_every_declared_symbol_is_exported(kc):
    names = declared_functions()
    assert len(names) >= 17
    L = kc.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(kc.SYMBOLS)


def test_abi_version_and_strerror(kc):
    assert kc.lib().kc_abi_version() == kc.ABI_VERSION == 7
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert kc.strerror(code) not in ("", "unknown status")


def test_range_check_agrees_with_oracle(kc, oracle_lib):
    rng = np.random.default_rng(7)
    cases = [[], [(0x10000, 0x1000)], [(0x10001, 0x1000)], [(0x10000, 0x1001)], [(0, 0x1000)],
             [(0x10000, 0)], [(2**64 - 0x1000, 0x2000)], [(0x20000, 0x1000), (0x10000, 0x1000)],
             [(0x10000, 0x2000), (0x11000, 0x1000)], [(0x10000, 0x2000), (0x12000, 0x1000)]]
    for _ in range(300):  # random mixes of good and bad ranges
        n = int(rng.integers(1, 6))
        base = 0x100000
        rs = []
        for _ in range(n):
            base += int(rng.integers(-3, 8)) * 0x1000 + int(rng.integers(0, 2)) * int(rng.integers(0, 4096)) * (rng.random() < 0.1)
            size = int(rng.integers(0, 5)) * 0x1000 + (1 if rng.random() < 0.05 else 0)
            rs.append((max(0, base), size))
            base += size
        cases.append(rs)
    for rs in cases:
        st_o, n_o, _ = oracle_lib.range_check(rs)
        st_k, n_k = kc.range_check(rs)
        assert st_o == st_k, rs
        if st_o == 0:
            assert n_o == n_k


def test_default_window_agrees_with_oracle(kc, oracle_lib):
    for rs in ([(0x7F8A00000000, 0x4000), (0x7F8A00100000, 0x1000)], [(0x2000, 0x1000)],
               [(2**64 - 2**33, 0x1000)]):
        assert kc.default_window(rs) == oracle_lib.default_window(rs)


def test_missing_library_fails_loudly(kc, monkeypatch, tmp_path):
    import importlib
    K = importlib.import_module("paper_2605_03208_amd.kc")
    monkeypatch.setattr(K, "_lib", None)
    monkeypatch.setattr(K, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        K.lib()


def test_binding_constants_match_header(kc):
    """Element-type, status and op codes in the binding are the header's."""
    text = open(os.path.join(ROOT, "include", "kc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    enum = {k: int(v) for k, v in re.findall(r"\b(KC_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    dts = [k for k in enum if k[3:] in ("F32", "BF16", "F16", "U8", "F64", "I8", "I16", "I32", "I64")
           or k.startswith("KC_FP8")]
    assert len(dts) == 13
    for k in dts:
        assert getattr(kc, k[3:]) == enum[k], k
        assert k[3:] in {name for name in dir(kc)}
    assert sorted(kc.TORCH_TO_KC.values()) == sorted(enum[k] for k in dts)
    for k in ("OK", "EINVAL", "EALIGN", "EORDER", "ENOMEM", "EHIP", "EDTYPE", "ELIMIT", "ERELOC"):
        assert getattr(kc, k) == enum["KC_" + k]
    for k in ("PAGE_HASH", "SNAPSHOT", "COMPACT", "RESTORE", "CLOSURE", "COMPARE", "GRAPH", "REGION_DIFF"):
        assert getattr(kc, "OP_" + k) == enum["KC_OP_" + k]


def test_graph_reach_agrees_with_oracle(kc, oracle_lib):
    """kc_graph_reach is host code: compare it with the oracle on random graphs."""
    rng = np.random.default_rng(5)
    for n in (0, 1, 2, 63, 64, 65, 200):
        ranges = [(0x400000 + i * 0x5000, 0x1000 * (1 + i % 3)) for i in range(n)]
        rw = (n + 63) // 64
        bits = np.zeros((n, rw * 64), np.uint8)
        bits[:, :n] = rng.random((n, n)) < 1.5 / max(n, 1)
        bits[:, n:] = 1 if n % 64 else 0        # garbage past the last range must be ignored
        edge = np.packbits(bits, axis=1, bitorder="little").view(np.uint64).reshape(n, rw)
        for roots in ([], [ranges[0][0]] if n else [], [r[0] + r[1] - 1 for r in ranges[::7]],
                      [0, 1, 2**64 - 1] + ([ranges[-1][0] + ranges[-1][1]] if n else [])):
            got = kc.graph_reach(ranges, edge, roots)
            clean = edge.copy()
            if n % 64:
                clean[:, -1] &= np.uint64((1 << (n % 64)) - 1)
            want = oracle_lib.graph_reach(ranges, clean, roots)
            assert (got == want).all(), (n, roots)
    with pytest.raises(kc.KCError):
        kc.graph_reach([(0x1010, 0x1000)], np.zeros(1, np.uint64), [])


def test_vaspace_rejects_bad_ranges_before_any_device_call(kc):
    """Range validation happens on the host, before the device is touched."""
    for ranges, code in (([(0x10001010, 0x1000)], kc.EALIGN), ([(0x20000000, 0x1000), (0x10000000, 0x1000)], kc.EORDER),
                         ([(0, 0x1000)], kc.EINVAL)):
        with pytest.raises(kc.KCError) as ei:
            kc.VaSpace(0, ranges)
        assert ei.value.code == code


def test_perturb_rejects_bad_arguments_before_any_device_call(kc):
    """kc_perturb validates its arguments on the host: no context, an unknown
    element type, a buffer past the arena, block or kmax 0."""
    L = kc.lib()
    bufs = (kc.PerturbBuf * 1)()
    bufs[0].offset, bufs[0].length, bufs[0].seed = 0, 10, 1
    assert L.kc_perturb(None, 0x1000, 10, kc.F32, bufs, 1, 1, 16, None) == kc.EINVAL
    # a context pointer is only dereferenced after validation; a dummy non-null one exercises the host checks
    dummy = ctypes.c_void_p(0x1000)
    assert L.kc_perturb(dummy, 0x1000, 10, kc.U8, bufs, 1, 1, 16, None) == kc.EDTYPE
    assert L.kc_perturb(dummy, 0x1000, 9, kc.F32, bufs, 1, 1, 16, None) == kc.EINVAL
    assert L.kc_perturb(dummy, 0x1000, 10, kc.F32, bufs, 1, 0, 16, None) == kc.EINVAL
    assert L.kc_perturb(dummy, 0x1000, 10, kc.F32, bufs, 1, 1, 0, None) == kc.EINVAL
    assert L.kc_perturb(dummy, 0x1002, 10, kc.F32, bufs, 1, 1, 16, None) == kc.EALIGN


def test_materialize_rejects_bad_arguments_before_any_device_call(kc):
    """kc_materialize validates its arguments on the host: no context, an
    unknown element type, a buffer past the arena, a null golden, block or
    kmax 0, a golden or a destination off 16 bytes."""
    L = kc.lib()
    bufs = (kc.MaterializeBuf * 1)()
    bufs[0].src_d, bufs[0].offset, bufs[0].length, bufs[0].seed = 0x2000, 4, 10, 1
    assert L.kc_materialize(None, 0x1000, 14, kc.F32, bufs, 1, 1, 16, None) == kc.EINVAL
    dummy = ctypes.c_void_p(0x1000)
    assert L.kc_materialize(dummy, 0x1000, 14, kc.U8, bufs, 1, 1, 16, None) == kc.EDTYPE
    assert L.kc_materialize(dummy, 0x1000, 13, kc.F32, bufs, 1, 1, 16, None) == kc.EINVAL
    assert L.kc_materialize(dummy, 0x1000, 14, kc.F32, bufs, 1, 0, 16, None) == kc.EINVAL
    assert L.kc_materialize(dummy, 0x1000, 14, kc.F32, bufs, 1, 1, 0, None) == kc.EINVAL
    assert L.kc_materialize(dummy, 0x1008, 14, kc.F32, bufs, 1, 1, 16, None) == kc.EALIGN
    bufs[0].offset = 3
    assert L.kc_materialize(dummy, 0x1000, 14, kc.F32, bufs, 1, 1, 16, None) == kc.EALIGN
    bufs[0].offset, bufs[0].src_d = 4, 0x2004
    assert L.kc_materialize(dummy, 0x1000, 14, kc.F32, bufs, 1, 1, 16, None) == kc.EALIGN
    bufs[0].src_d = 0
    assert L.kc_materialize(dummy, 0x1000, 14, kc.F32, bufs, 1, 1, 16, None) == kc.EINVAL


def test_pair_arrays_marshal_like_pair_structs(kc):
    """The array form of a pair list (used by the server) lays out kc_pair
    exactly as the per-pair constructor does."""
    arr, n = kc.pairs_from_arrays(np.array([0x1000, 0x2000], dtype=np.uint64),
                                  np.array([0x3000, 2**63 + 0x4000], dtype=np.uint64), np.array([5, 2**40]),
                                  np.array([0, 12]), np.array([2, 9]), 1e-8, 1e-5)
    want = [kc.Pair(0x1000, 0x3000, 5, 0, 2, 1e-8, 1e-5), kc.Pair(0x2000, 2**63 + 0x4000, 2**40, 12, 9, 1e-8, 1e-5)]
    assert n == 2
    assert [bytes(p) for p in arr] == [bytes(p) for p in want]
    arr, n = kc.pairs_from_arrays([], [], [], [], [])
    assert n == 0 and len(arr) == 1
