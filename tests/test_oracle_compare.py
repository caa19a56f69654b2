"""Pins the oracle's typed compare.

Independent pins: closed-form ULP distances fixed by the encodings (IEEE-754
binary32/binary16, bfloat16 = upper half of binary32, OCP fp8 E4M3FN),
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


@pytest.mark.parametrize("dt", [W.DT_F32, W.DT_BF16, W.DT_F16, W.DT_FP8])
def test_known_perturbations(oracle_lib, dt):
    rng = np.random.default_rng(100 + dt)
    gen = torch.Generator().manual_seed(dt)
    for n, tol in [(4099, 0), (20000, 3), (1, 0), (64, 16)]:
        gold = torch.randn(n, generator=gen).to(W.TORCH_DTYPE[dt])
        if dt == W.DT_FP8:  # keep away from the fp8 range ends so k steps stay inside
            gold = (torch.randn(n, generator=gen) * 0.5).to(W.TORCH_DTYPE[dt])
        pair = W.perturb_pair(gold, dt, rng, max(1, n // 50), 16 if dt != W.DT_FP8 else 4,
                              n_nan=2 if n > 10 else 0, ulp_tol=tol)
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
        o.compare(np.zeros(4, np.uint8), np.zeros(4, np.uint8), 9, 0)


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
