"""Pins the oracle's typed compare.

Independent pins: closed-form ULP distances fixed by the encodings (IEEE-754
binary32/binary16/binary64, bfloat16 = upper half of binary32, OCP fp8 E4M3FN
and E5M2, the FNUZ fp8 variants), the rank of every fp8 code among the
torch-decoded values of its format, exact Python-integer differences for the
integer types,
perturbations by k steps of the library ``nextafter`` (or the torch-decoded
fp8 code table) whose k the generator records, numpy float64 formulas for
the max abs / rel error, and numpy byte counts for the paper's
differing-byte metric (Sec. 4.5.2, byte-exact comparison).
"""
import struct

import numpy as np
import pytest
import torch

from paper_2605_03208_amd import workloads as W


def f32_bits(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


def test_ulp_closed_forms(oracle_lib):
    o = oracle_lib
    one = f32_bits(1.0)
    nxt = int(np.nextafter(np.float32(1.0), np.float32(2.0)).view(np.uint32))
    assert o.ulp(o.F32, nxt, one) == 1
    assert o.ulp(o.F32, f32_bits(0.0), f32_bits(-0.0)) == 0
    dmin = int(np.float32(1e-45).view(np.uint32))            # +denorm_min
    assert o.ulp(o.F32, dmin, dmin | 0x80000000) == 2
    fmax = int(np.finfo(np.float32).max.view(np.uint32))
    assert o.ulp(o.F32, fmax, f32_bits(float("inf"))) == 1
    assert o.ulp(o.F32, f32_bits(2.0), f32_bits(1.0)) == 1 << 23   # one binade of fp32
    assert o.ulp(o.BF16, 0x3F81, 0x3F80) == 1
    assert o.ulp(o.BF16, f32_bits(2.0) >> 16, f32_bits(1.0) >> 16) == 1 << 7
    assert o.ulp(o.F16, int(np.float16(2.0).view(np.uint16)), int(np.float16(1.0).view(np.uint16))) == 1 << 10
    assert o.ulp(o.FP8_E4M3FN, 0x7E, 0x7D) == 1
    assert o.ulp(o.FP8_E4M3FN, 0x01, 0x81) == 2
    inf, ninf = f32_bits(float("inf")), f32_bits(float("-inf"))
    d = o.ulp(o.F32, inf, ninf)
    assert d == 0xFF000000 and o.ulp_bin(d) == 44


def test_ulp_bins(oracle_lib):
    o = oracle_lib
    assert [o.ulp_bin(d) for d in range(17)] == list(range(17))
    # octaves above 16: (16, 32] -> 17, (32, 64] -> 18, ...
    assert o.ulp_bin(17) == 17 and o.ulp_bin(32) == 17 and o.ulp_bin(33) == 18
    assert o.ulp_bin(1 << 23) == 35 and o.ulp_bin((1 << 23) + 1) == 36
    assert o.ulp_bin((1 << 32) - 1) == 44
    # the last bin takes every distance above 2^34 (binary64, 64-bit integers)
    assert o.ulp_bin(1 << 34) == 46 and o.ulp_bin((1 << 34) + 1) == 47
    assert o.ulp_bin(1 << 52) == 47 and o.ulp_bin(2**64 - 1) == 47


def _check_pair(o, pair, dt, atol=0.0, rtol=0.0):
    gold = pair.gold.cpu()
    cand = pair.cand.cpu()
    gv = gold.view(torch.uint8).numpy()
    cv = cand.view(torch.uint8).numpy()
    r = o.compare(cv, gv, dt, pair.ulp_tol, atol, rtol)
    n = gold.numel()
    assert r["n_elems"] == n
    mism = np.sort(np.concatenate([pair.pos, pair.nan_pos]))
    assert r["n_mismatch_elems"] == len(mism)
    assert r["first_mismatch"] == (int(mism[0]) if len(mism) else 2**64 - 1)
    assert r["n_mismatch_bytes"] == int((cv != gv).sum())
    assert r["n_nan_cand_only"] == len(pair.nan_pos) and r["n_nan_gold_only"] == 0 and r["n_nan_both"] == 0
    hist = np.zeros(48, dtype=np.int64)
    np.add.at(hist, np.abs(pair.k), 1)          # all |k| <= 16 here: bin == distance
    hist[0] = n - len(pair.pos) - len(pair.nan_pos)
    assert r["ulp_hist"] == hist.tolist()
    assert r["n_over_tol"] == int((np.abs(pair.k) > pair.ulp_tol).sum())
    assert r["pass"] == int(r["n_over_tol"] == 0 and len(pair.nan_pos) == 0)
    g64 = gold.to(torch.float64).numpy()
    c64 = cand.to(torch.float64).numpy()
    ok = ~np.isnan(c64) & ~np.isnan(g64)
    diff = np.abs(c64[ok] - g64[ok])
    assert r["max_abs"] == (diff.max() if diff.size else 0.0)
    nz = ok & (g64 != 0)
    rel = np.abs(c64[nz] - g64[nz]) / np.abs(g64[nz])
    assert r["max_rel"] == (rel.max() if rel.size else 0.0)
    close = np.isclose(c64[ok], g64[ok], rtol=rtol, atol=atol)    # library routine, float64
    assert r["n_not_close"] == int((~close).sum())
    assert r["pass_close"] == int(r["n_not_close"] == 0 and len(pair.nan_pos) == 0)
    return r


FLOAT_DTS = [W.DT_F32, W.DT_BF16, W.DT_F16, W.DT_FP8, W.DT_F64, W.DT_FP8_E4M3FNUZ, W.DT_FP8_E5M2,
             W.DT_FP8_E5M2FNUZ]
INT_DTS = [W.DT_I8, W.DT_I16, W.DT_I32, W.DT_I64]


def _gold(dt, n, gen):
    t = W.TORCH_DTYPE[dt]
    if t in W.INT_TYPES:   # away from the range ends so k steps stay inside
        hi = min(torch.iinfo(t).max, 1 << 40) - 64
        return torch.randint(-hi, hi, (n,), generator=gen, dtype=torch.int64).to(t)
    if t in W.FP8_TYPES:   # keep away from the fp8 range ends so k steps stay inside
        return (torch.randn(n, generator=gen) * 0.5).to(t)
    return torch.randn(n, generator=gen, dtype=torch.float64).to(t)


@pytest.mark.parametrize("dt", FLOAT_DTS + INT_DTS)
def test_known_perturbations(oracle_lib, dt):
    rng = np.random.default_rng(100 + dt)
    gen = torch.Generator().manual_seed(dt)
    t = W.TORCH_DTYPE[dt]
    for n, tol in [(4099, 0), (20000, 3), (1, 0), (64, 16)]:
        gold = _gold(dt, n, gen)
        pair = W.perturb_pair(gold, dt, rng, max(1, n // 50), 4 if t in W.FP8_TYPES else 16,
                              n_nan=2 if n > 10 and t not in W.INT_TYPES else 0, ulp_tol=tol)
        for atol, rtol in ((0.0, 0.0), (1e-8, 1e-5), (1e-3, 0.0), (0.0, 1e-2)):
            _check_pair(oracle_lib, pair, dt, atol, rtol)


def test_c1_compare_pairs_scaled(oracle_lib):
    for pair in W.c1_compare(scale=1 / 16, n_pairs=3):
        r = _check_pair(oracle_lib, pair, W.DT_F32)
        assert r["pass"] == 0 and r["n_nan_cand_only"] == 2


def test_special_values(oracle_lib):
    o = oracle_lib
    nan_a, nan_b = 0x7FC00000, 0x7FC00001
    inf = f32_bits(float("inf"))
    fmax = int(np.finfo(np.float32).max.view(np.uint32))
    gold = np.array([f32_bits(1.0), nan_a, nan_a, f32_bits(2.0), f32_bits(-0.0), inf, f32_bits(3.0), 0, inf],
                    dtype=np.uint32)
    cand = np.array([f32_bits(1.0), nan_a, nan_b, nan_a, f32_bits(0.0), fmax, f32_bits(3.0), f32_bits(1.0), inf],
                    dtype=np.uint32)
    r = o.compare(cand, gold, o.F32, 0)
    assert r["n_nan_both"] == 2 and r["n_nan_cand_only"] == 1 and r["n_nan_gold_only"] == 0
    assert r["n_mismatch_elems"] == 5 and r["first_mismatch"] == 2
    assert r["max_abs"] == float("inf")       # fmax vs +inf
    # rel: gold +inf and gold 0 are excluded; only finite non-zero golds count
    assert r["max_rel"] == 0.0
    assert r["ulp_hist"][0] == 4 and r["ulp_hist"][1] == 1   # equal x3 (incl. inf) + (+0,-0); fmax/inf
    assert r["ulp_hist"][12 + 30] == 1                       # 1.0 vs +0: 0x3F800000 ULPs
    assert r["n_over_tol"] == 2 and r["pass"] == 0
    # bit-identical NaNs count as both-NaN, not in the histogram
    r = o.compare(np.array([nan_a], np.uint32), np.array([nan_a], np.uint32), o.F32, 0)
    assert r["n_nan_both"] == 1 and sum(r["ulp_hist"]) == 0 and r["pass"] == 1
    # gold-only NaN fails
    r = o.compare(np.array([f32_bits(1.0)], np.uint32), np.array([nan_a], np.uint32), o.F32, 8)
    assert r["n_nan_gold_only"] == 1 and r["pass"] == 0
    # fp8: 0x7F is NaN, 0xFF too
    r = o.compare(np.array([0x7F, 0xFF, 0x7E], np.uint8), np.array([0x7F, 0x7F, 0x7F], np.uint8), o.FP8_E4M3FN, 0)
    assert r["n_nan_both"] == 2 and r["n_nan_gold_only"] == 1


def test_u8_bytes(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(1)
    g = rng.integers(0, 256, 10007, dtype=np.uint8)
    c = g.copy()
    idx = rng.choice(len(g), 37, replace=False)
    c[idx] ^= 0x10
    r = o.compare(c, g, o.U8, 0)
    assert r["n_mismatch_elems"] == r["n_mismatch_bytes"] == 37
    assert r["first_mismatch"] == int(idx.min()) and r["pass"] == 0
    assert sum(r["ulp_hist"]) == 0 and r["max_abs"] == 0.0
    r = o.compare(g, g, o.U8, 0)
    assert r["pass"] == 1 and r["first_mismatch"] == 2**64 - 1


def test_empty_and_bad_dtype(oracle_lib):
    o = oracle_lib
    r = o.compare(np.zeros(0, np.float32), np.zeros(0, np.float32), o.F32, 0)
    assert r["n_elems"] == 0 and r["pass"] == 1 and r["first_mismatch"] == 2**64 - 1
    with pytest.raises(o.OracleError):
        o.compare(np.zeros(4, np.uint8), np.zeros(4, np.uint8), 13, 0)


def test_tolerance_comparison_specials(oracle_lib):
    """Infinities are close only to themselves; NaNs never enter the count;
    the bound is atol + rtol * |golden| (checked against numpy.isclose)."""
    o = oracle_lib
    inf, ninf = float("inf"), float("-inf")
    g = np.array([1.0, 1.0, 1.0, inf, inf, 0.0, -2.0, 1e-30, 3.0, np.nan], dtype=np.float32)
    c = np.array([1.0, 1.00001, 1.1, inf, ninf, 1e-9, -2.00002, 0.0, np.float32(np.finfo(np.float32).max), 1.0],
                 dtype=np.float32)
    for atol, rtol in ((0.0, 0.0), (1e-8, 1e-5), (1e-6, 1e-4), (0.2, 0.0)):
        r = o.compare(c, g, o.F32, 0, atol, rtol)
        ok = ~np.isnan(c) & ~np.isnan(g)
        want = int((~np.isclose(c[ok].astype(np.float64), g[ok].astype(np.float64), rtol=rtol, atol=atol)).sum())
        assert r["n_not_close"] == want, (atol, rtol)
        assert r["n_nan_gold_only"] == 1 and r["pass_close"] == 0
    with pytest.raises(o.OracleError):
        o.compare(c, g, o.F32, 0, -1.0, 0.0)


def test_mismatch_bytes_count_per_byte(oracle_lib):
    o = oracle_lib
    g = np.array([0x3F800000, 0x40000000], np.uint32)
    c = np.array([0x3F800001, 0x40010100], np.uint32)
    r = o.compare(c, g, o.F32, 1 << 30)
    assert r["n_mismatch_elems"] == 2 and r["n_mismatch_bytes"] == 3 and r["pass"] == 1


FP8_FORMATS = [(W.DT_FP8, torch.float8_e4m3fn), (W.DT_FP8_E4M3FNUZ, torch.float8_e4m3fnuz),
               (W.DT_FP8_E5M2, torch.float8_e5m2), (W.DT_FP8_E5M2FNUZ, torch.float8_e5m2fnuz)]


@pytest.mark.parametrize("dt,tdt", FP8_FORMATS)
def test_fp8_codes_against_torch(oracle_lib, dt, tdt):
    """Every code of each fp8 format: its NaN class, its value (as the max abs
    error against the zero code) and, for every pair of non-NaN codes, its ULP
    distance = the difference of their ranks among the distinct values."""
    o = oracle_lib
    vals = torch.arange(256, dtype=torch.uint8).view(tdt).to(torch.float64).numpy()
    codes = np.arange(256, dtype=np.uint8)
    r = o.compare(codes, codes, dt, 0)
    assert r["n_nan_both"] == int(np.isnan(vals).sum())
    for c in range(256):
        r = o.compare(np.array([c], np.uint8), np.array([0], np.uint8), dt, 0)
        if np.isnan(vals[c]):
            assert r["n_nan_cand_only"] == 1
        else:
            assert r["max_abs"] == abs(vals[c]), hex(c)
    distinct = np.unique(vals[~np.isnan(vals)])          # -0 and +0 are one value
    rank = {c: int(np.searchsorted(distinct, vals[c])) for c in range(256) if not np.isnan(vals[c])}
    for a in rank:
        for b in rank:
            assert o.ulp(dt, a, b) == abs(rank[a] - rank[b]), (hex(a), hex(b))


def f64_bits(x):
    return int(np.float64(x).view(np.uint64))


def test_f64_closed_forms(oracle_lib):
    o = oracle_lib
    assert o.ulp(o.F64, f64_bits(np.nextafter(1.0, 2.0)), f64_bits(1.0)) == 1
    assert o.ulp(o.F64, f64_bits(0.0), f64_bits(-0.0)) == 0
    dmin = f64_bits(5e-324)
    assert o.ulp(o.F64, dmin, dmin | (1 << 63)) == 2
    assert o.ulp(o.F64, f64_bits(np.finfo(np.float64).max), f64_bits(np.inf)) == 1
    assert o.ulp(o.F64, f64_bits(2.0), f64_bits(1.0)) == 1 << 52
    d = o.ulp(o.F64, f64_bits(np.inf), f64_bits(-np.inf))
    assert d == 2 * 0x7FF0000000000000 and o.ulp_bin(d) == 47
    g = np.array([1.0, np.inf, 3.0, 0.0, 2.0, np.nan], np.float64)
    c = np.array([np.nextafter(1.0, 0.0), np.inf, 3.5, -0.0, np.nan, np.nan], np.float64)
    r = o.compare(c, g, o.F64, 0)
    assert r["n_nan_both"] == 1 and r["n_nan_cand_only"] == 1
    assert r["max_abs"] == 0.5 and r["max_rel"] == 0.5 / 3.0
    assert r["ulp_hist"][0] == 2 and r["ulp_hist"][1] == 1 and r["ulp_hist"][47] == 1
    # signalling-NaN encodings and the all-ones payload are NaN; the inf is not
    s = np.array([0x7FF0000000000001, 0xFFFFFFFFFFFFFFFF, 0x7FF0000000000000], np.uint64)
    r = o.compare(s, s, o.F64, 0)
    assert r["n_nan_both"] == 2 and r["ulp_hist"][0] == 1


@pytest.mark.parametrize("dt", INT_DTS)
def test_integers_exact(oracle_lib, dt):
    """Integer pairs against exact Python-integer differences, including the
    range ends (a difference of up to 2^64 - 1)."""
    o = oracle_lib
    t = W.TORCH_DTYPE[dt]
    info = np.iinfo(torch.empty(0, dtype=t).numpy().dtype)
    rng = np.random.default_rng(dt)
    n = 3001
    g = rng.integers(info.min, info.max, n, dtype=np.int64, endpoint=True).astype(info.dtype)
    c = g.copy()
    idx = rng.choice(n, 400, replace=False)
    c[idx] = rng.integers(info.min, info.max, len(idx), dtype=np.int64, endpoint=True).astype(info.dtype)
    c[idx[:3]] = [info.max, info.min, info.max]
    g[idx[:3]] = [info.min, info.max, info.max - 1]
    for atol, rtol, tol in ((0.0, 0.0, 0), (1e3, 1e-3, 7), (5.0, 0.5, 1 << 20)):
        r = o.compare(c, g, dt, tol, atol, rtol)
        gi, ci = [int(x) for x in g], [int(x) for x in c]
        dist = [abs(a - b) for a, b in zip(ci, gi)]
        hist = [0] * 48
        for d in dist:
            hist[d if d <= 16 else min(12 + (d - 1).bit_length(), 47)] += 1
        assert r["ulp_hist"] == hist
        assert r["n_mismatch_elems"] == sum(d != 0 for d in dist)
        assert r["n_over_tol"] == sum(d > tol for d in dist)
        assert r["max_abs"] == float(max(dist))
        assert r["max_rel"] == max(float(d) / abs(float(b)) for d, b in zip(dist, gi) if b != 0)
        assert r["n_not_close"] == sum(float(d) > atol + rtol * abs(float(b)) for d, b in zip(dist, gi))
        assert r["n_nan_both"] == r["n_nan_cand_only"] == r["n_nan_gold_only"] == 0
        assert r["pass"] == int(r["n_over_tol"] == 0) and r["pass_close"] == int(r["n_not_close"] == 0)
        assert r["first_mismatch"] == min(i for i, d in enumerate(dist) if d)
