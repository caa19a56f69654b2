"""HIP path vs the CPU oracle, element by element, through the C ABI.

Every case prints its name before touching the GPU.  Inputs come from the
seeded generators; expected values come from the oracle run on a host copy
of the same device bytes.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_03208_amd import workloads as W

pytestmark = pytest.mark.gpu

PAGE = 4096


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kc():
    from paper_2605_03208_amd import kc as K
    K.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return K


@pytest.fixture(scope="module")
def ctx(kc):
    c = kc.Context(0)
    yield c
    c.close()


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def host_of(case):
    host = case.arena.host_copy()
    return host, W.host_views(case.layout, host)


def check_scan(kc, scan, ranges, views, win=(0, 0)):
    res, oob = scan.result()
    o_res, o_oob = oracle.closure_scan(ranges, views, win[0], win[1], oob_cap=scan.cap)
    assert res == o_res
    assert oob == o_oob
    return res, oob


def snapshot_vs_oracle(kc, ctx, case, fused=True, seed=0, cap=None, oob_cap=64, win=(0, 0)):
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    host, views = host_of(case)
    scan = kc.ScanOut("cuda", oob_cap=oob_cap, win_lo=win[0], win_hi=win[1])
    if fused:
        out = kc.snapshot(ctx, rs, seed=seed, cap_pages=cap, scan=scan)
        h, z, packed, va, nk = out["hash"], out["zero_bm"], out["packed"], out["page_va"], out["n_kept"]
    else:
        h, z, _ = kc.page_hash(ctx, rs, seed=seed, scan=scan)
        packed, va, nk = kc.compact(ctx, rs, z, None, cap_pages=cap)
    torch.cuda.synchronize()
    oh, oz, _ = oracle.page_hash(ranges, views, seed=seed)
    assert np.array_equal(u64(h)[: rs.n_pages], oh)
    assert np.array_equal(u64(z)[: rs.n_words], oz)
    op, ova, onk = oracle.compact(ranges, views, oz, cap_pages=cap)
    n_kept = int(u64(nk)[0])
    assert n_kept == onk
    k = len(ova)
    assert np.array_equal(u64(va)[:k], ova)
    assert np.array_equal(packed[: k * PAGE].cpu().numpy(), op)
    check_scan(kc, scan, ranges, views, win)
    return rs, dict(hash=h, zero_bm=z, packed=packed, page_va=va, n_kept=nk), host, views


def test_page_hash_small_c1(kc, ctx):
    say("page_hash c1 scale 1/16 (seed 0 and seed 7), fused closure scan")
    case = W.c1_snapshot("cuda", scale=1 / 16)
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    host, views = host_of(case)
    for seed in (0, 7, 2**64 - 1):
        scan = kc.ScanOut("cuda", oob_cap=16)
        h, z, c = kc.page_hash(ctx, rs, seed=seed, scan=scan)
        torch.cuda.synchronize()
        oh, oz, _ = oracle.page_hash(ranges, views, seed=seed)
        assert np.array_equal(u64(h)[: rs.n_pages], oh)
        assert np.array_equal(u64(z)[: rs.n_words], oz)
        check_scan(kc, scan, ranges, views)


def test_snapshot_fused_c1_full(kc, ctx):
    say("snapshot fused c1 full (64 MiB, 48 ranges)")
    case = W.c1_snapshot("cuda")
    rs, out, host, views = snapshot_vs_oracle(kc, ctx, case, fused=True)
    assert int(u64(out["n_kept"])[0]) == 16384 - 4915
    say("snapshot two-pass c1 full")
    snapshot_vs_oracle(kc, ctx, case, fused=False)


def test_restore_roundtrip_c1(kc, ctx):
    say("restore round trip c1 full: clobber 0xA5, restore, re-hash")
    case = W.c1_snapshot("cuda")
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    original = case.arena.buf.clone()
    out = kc.snapshot(ctx, rs)
    for i in range(case.layout.n):
        case.arena.view(i).fill_(0xA5)
    n_bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 0
    for i in range(case.layout.n):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        assert torch.equal(case.arena.buf[o:o + s], original[o:o + s]), i
    h2, _, _ = kc.page_hash(ctx, rs)
    assert torch.equal(h2[: rs.n_pages], out["hash"][: rs.n_pages])
    say("restore with corrupted page-VA entries")
    va = out["page_va"].clone()
    va[0] = ranges[-1][0] + ranges[-1][1]   # one past the end
    va[5] = va[5] + 8                        # misaligned
    host, views = host_of(case)
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], va, out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 2
    o_views = [v.copy() for v in views]
    packed = out["packed"].cpu().numpy()
    nk = int(u64(out["n_kept"])[0])
    assert oracle.restore(ranges, o_views, u64(out["zero_bm"])[: rs.n_words], None, packed[: nk * PAGE],
                          u64(va)[:nk], nk) == 2
    host2, views2 = host_of(case)
    assert all(np.array_equal(a, b) for a, b in zip(views2, o_views))
    say("delta restore (every page marked changed) with the same corrupted entries")
    for i in range(case.layout.n):
        case.arena.view(i).fill_(0xA5)
    every = torch.full((rs.n_words,), -1, dtype=torch.int64, device="cuda")
    n_bad.zero_()
    kc.restore(ctx, rs, out["zero_bm"], every, out["packed"], va, out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 2
    o_views = [np.full_like(v, 0xA5) for v in views]
    assert oracle.restore(ranges, o_views, u64(out["zero_bm"])[: rs.n_words], u64(every), packed[: nk * PAGE],
                          u64(va)[:nk], nk) == 2
    host3, views3 = host_of(case)
    assert all(np.array_equal(a, b) for a, b in zip(views3, o_views))


def _tuned_context(kc, signature, ops):
    """A context in the launch shapes the benchmark tunes for ``signature``
    (built-in shapes where the shipped table has none)."""
    from paper_2605_03208_amd import autotune
    c = kc.Context(0)
    shapes = {}
    for op in ops:
        hit = autotune.lookup(autotune.cache_key(op, signature))
        if hit:
            c.set_tuning(op, **hit["best"])
            shapes[autotune.OP_NAMES[op]] = hit["best"]
    return c, shapes


def test_delta_c2_scaled(kc, ctx):
    _delta_c2(kc, ctx, 1 / 32)


def test_delta_c2_full_in_bench_shapes(kc):
    """The 4096-range, 2 GiB set at full size, in the shapes the benchmark's
    batched delta snapshot runs."""
    c, shapes = _tuned_context(kc, "c2-delta-4096-ranges", (kc.OP_PAGE_HASH, kc.OP_COMPACT))
    say(f"delta snapshot c2 full size, shapes {shapes or 'built-in'}")
    _delta_c2(kc, c, 1.0)
    c.close()


def _delta_c2(kc, ctx, scale):
    say(f"delta snapshot c2 scale {scale}: full, rewrite 5 %, delta, restore chain")
    case = W.c2_snapshot("cuda", scale=scale)
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    s1 = kc.snapshot(ctx, rs, seed=3)
    base_img = case.arena.buf.clone()
    W.c2_rewrite(case)
    mutated = case.arena.buf.clone()
    host, views = host_of(case)
    s2 = kc.snapshot(ctx, rs, seed=3, prior=s1["hash"])
    torch.cuda.synchronize()
    oh, oz, oc = oracle.page_hash(ranges, views, seed=3, prior=u64(s1["hash"])[: rs.n_pages])
    assert np.array_equal(u64(s2["hash"])[: rs.n_pages], oh)
    assert np.array_equal(u64(s2["zero_bm"])[: rs.n_words], oz)
    assert np.array_equal(u64(s2["changed_bm"])[: rs.n_words], oc)
    changed = np.unpackbits(oc.view(np.uint8), bitorder="little")[: rs.n_pages].astype(bool)
    assert np.array_equal(np.nonzero(changed)[0], case.truth["rewritten"])
    op, ova, onk = oracle.compact(ranges, views, oz, oc)
    assert int(u64(s2["n_kept"])[0]) == onk == len(case.truth["rewritten"])
    assert np.array_equal(u64(s2["page_va"])[:onk], ova)
    assert np.array_equal(s2["packed"][: onk * PAGE].cpu().numpy(), op)
    say("delta restore chain: clobber, restore base, restore delta")
    case.arena.buf.fill_(0x5A)
    kc.restore(ctx, rs, s1["zero_bm"], None, s1["packed"], s1["page_va"], s1["n_kept"])
    torch.cuda.synchronize()
    for i in range(case.layout.n):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        assert torch.equal(case.arena.buf[o:o + s], base_img[o:o + s])
    kc.restore(ctx, rs, s2["zero_bm"], s2["changed_bm"], s2["packed"], s2["page_va"], s2["n_kept"])
    torch.cuda.synchronize()
    for i in range(case.layout.n):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        assert torch.equal(case.arena.buf[o:o + s], mutated[o:o + s])


def _ragged_case(seed, n_ranges, max_pages, zero_frac=0.3, ptr_frac=0.002):
    """Ranges of 1..max_pages pages with random gaps, random bytes, zero pages,
    in-range and out-of-range pointer words."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, max_pages + 1, size=n_ranges) * PAGE
    lay = W.make_layout(rng, sizes, gap_pages=(1, 3))
    arena = W.Arena(lay, "cuda")
    content = rng.integers(0, 256, size=lay.total, dtype=np.uint8)
    pages = content.reshape(-1, PAGE)
    pages[rng.random(len(pages)) < zero_frac] = 0
    words = content.view(np.uint64)
    ranges = lay.ranges(arena.va_base)
    k = max(1, int(ptr_frac * len(words)))
    pos = rng.choice(len(words), size=k, replace=False)
    tgt = rng.integers(0, n_ranges, size=k)
    vals = np.array([ranges[t][0] for t in tgt], dtype=np.uint64) + rng.integers(0, PAGE, size=k).astype(np.uint64)
    bad = rng.random(k) < 0.3
    vals[bad] = np.uint64(ranges[-1][0] + ranges[-1][1]) + rng.integers(0, 1 << 20, size=int(bad.sum())).astype(np.uint64)
    words[pos] = vals
    arena.load_concat(content)
    return W.SnapshotCase(f"ragged{seed}", arena, {})


@pytest.mark.parametrize("seed,n_ranges,max_pages", [(11, 1, 1), (12, 3, 17), (13, 37, 40), (14, 300, 9),
                                                     (15, 700, 3)])
def test_ragged_tiles_and_capacities(kc, ctx, seed, n_ranges, max_pages):
    say(f"ragged snapshot seed={seed} ranges={n_ranges} max_pages={max_pages}")
    case = _ragged_case(seed, n_ranges, max_pages)
    rs, out, host, views = snapshot_vs_oracle(kc, ctx, case, fused=True, seed=seed, oob_cap=8)
    n_kept = int(u64(out["n_kept"])[0])
    say(f"ragged seed={seed}: capacity {n_kept // 2} truncation, fused and two-pass")
    snapshot_vs_oracle(kc, ctx, case, fused=True, seed=seed, cap=n_kept // 2, oob_cap=3)
    snapshot_vs_oracle(kc, ctx, case, fused=False, seed=seed, cap=max(0, n_kept // 3), oob_cap=0)
    say(f"ragged seed={seed}: explicit windows")
    lo = case.ranges()[0][0]
    snapshot_vs_oracle(kc, ctx, case, fused=True, seed=seed, win=(lo, lo + 3 * PAGE))
    snapshot_vs_oracle(kc, ctx, case, fused=True, seed=seed, win=(1, 2**64 - 1), oob_cap=5000)


def test_standalone_closure_scan(kc, ctx):
    say("standalone closure scan c1 scale 1/4 and a ragged case")
    for case in (W.c1_snapshot("cuda", scale=1 / 4), _ragged_case(21, 500, 6, ptr_frac=0.01)):
        ranges = case.ranges()
        rs = kc.RangeSet(ctx, ranges)
        host, views = host_of(case)
        for cap in (0, 2, 100000):
            scan = kc.ScanOut("cuda", oob_cap=cap)
            kc.closure_scan(ctx, rs, scan)
            torch.cuda.synchronize()
            check_scan(kc, scan, ranges, views)


def test_per_item_launches_equal_batched(kc, ctx):
    say("per-range launches vs one persistent launch (hash, compact, closure)")
    case = _ragged_case(31, 200, 20)
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    outs = []
    for per_item, grid in ((0, 0), (1, 0), (0, 1), (0, 32)):
        c2 = kc.Context(0)
        for op in (kc.OP_PAGE_HASH, kc.OP_SNAPSHOT, kc.OP_COMPACT, kc.OP_CLOSURE):
            c2.set_tuning(op, grid_per_cu=grid, per_item=per_item)
        rs2 = kc.RangeSet(c2, ranges)
        scan = kc.ScanOut("cuda", oob_cap=50)
        o = kc.snapshot(c2, rs2, seed=5, scan=scan)
        h, z, _ = kc.page_hash(c2, rs2, seed=5)
        p2, va2, nk2 = kc.compact(c2, rs2, z)
        scan2 = kc.ScanOut("cuda", oob_cap=50)
        kc.closure_scan(c2, rs2, scan2)
        torch.cuda.synchronize()
        nk = int(u64(o["n_kept"])[0])
        outs.append((u64(o["hash"])[: rs2.n_pages].copy(), u64(o["zero_bm"])[: rs2.n_words].copy(),
                     o["packed"][: nk * PAGE].cpu().numpy(), u64(o["page_va"])[:nk].copy(), nk, scan.result(),
                     u64(h)[: rs2.n_pages].copy(), p2[: nk * PAGE].cpu().numpy(), scan2.result()))
        rs2.close()
        c2.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            if isinstance(a, np.ndarray):
                assert np.array_equal(a, b)
            else:
                assert a == b


def test_empty_rangeset(kc, ctx):
    say("empty range set")
    rs = kc.RangeSet(ctx, [])
    scan = kc.ScanOut("cuda", oob_cap=4)
    out = kc.snapshot(ctx, rs, scan=scan, cap_pages=0)
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], cap_pages=0)
    torch.cuda.synchronize()
    assert int(u64(out["n_kept"])[0]) == 0
    res, oob = scan.result()
    assert res["n_words"] == 0 and res["n_oob"] == 0 and oob == []


def test_rangeset_errors(kc, ctx):
    say("range-set argument errors")
    for bad, code in (([(0x10001010, 0x1000)], kc.EALIGN), ([(0x20000, 0x1000), (0x10000, 0x1000)], kc.EORDER),
                      ([(0x10000, 0)], kc.EINVAL)):
        with pytest.raises(kc.KCError) as ei:
            kc.RangeSet(ctx, bad)
        assert ei.value.code == code


# ------------------------------------------------------------------ compare --

def cmp_vs_oracle(kc, ctx, pairs, tile_bytes=None, per_item=0, grid=0):
    """pairs: list of (cand, gold, dtype, tol) device tensors."""
    c2 = kc.Context(0)
    c2.set_tuning(kc.OP_COMPARE, grid_per_cu=grid, tile_bytes=tile_bytes or 0, per_item=per_item)
    res = kc.compare(c2, pairs)
    torch.cuda.synchronize()
    got = kc.decode_cmp(res, len(pairs))
    c2.close()
    for p, r in zip(pairs, got):
        c, g, dt, tol = p[:4]
        atol, rtol = (p[4], p[5]) if len(p) > 4 else (0.0, 0.0)
        o = oracle.compare(c.cpu().view(torch.uint8).numpy(), g.cpu().view(torch.uint8).numpy(), dt, tol, atol, rtol)
        assert r == o, (dt, tol, c.numel())
    return got


def test_compare_c1_pairs(kc, ctx):
    say("compare c1: 16 fp32 pairs x 2^20, tol 0")
    pairs = W.c1_compare("cuda")
    got = cmp_vs_oracle(kc, ctx, [(p.cand, p.gold, W.DT_F32, p.ulp_tol) for p in pairs])
    for p, r in zip(pairs, got):
        assert r["n_mismatch_elems"] == 1049 + 2 and r["n_nan_cand_only"] == 2 and r["pass"] == 0


SPECIALS = {  # NaN, inf / max, -inf / -max, smallest subnormal, -0 / 0, largest finite ...
    W.DT_F32: [0x7FC00000, 0x7F800000, 0xFF800000, 0x00000001, 0x80000000, 0x7F7FFFFF],
    W.DT_BF16: [0x7FC0, 0x7F80, 0xFF80, 0x0001, 0x8000, 0x7F7F],
    W.DT_F16: [0x7E00, 0x7C00, 0xFC00, 0x0001, 0x8000, 0x7BFF],
    W.DT_FP8: [0x7F, 0xFF, 0x7E, 0x01, 0x80, 0x00],
    W.DT_F64: [0x7FF8000000000000, 0x7FF0000000000000, 0xFFF0000000000000, 0x1, 0x8000000000000000,
               0x7FEFFFFFFFFFFFFF, 0x7FF0000000000001],
    W.DT_FP8_E4M3FNUZ: [0x80, 0x7F, 0xFF, 0x01, 0x00, 0x08],
    W.DT_FP8_E5M2: [0x7E, 0x7C, 0xFC, 0x01, 0x80, 0x7B, 0xFF],
    W.DT_FP8_E5M2FNUZ: [0x80, 0x7F, 0xFF, 0x01, 0x00, 0x04],
}
for _dt, _t in ((W.DT_I8, torch.int8), (W.DT_I16, torch.int16), (W.DT_I32, torch.int32), (W.DT_I64, torch.int64)):
    _i = torch.iinfo(_t)
    _m = (1 << (8 * W.ELEM_SIZE[_dt])) - 1
    SPECIALS[_dt] = [_i.min & _m, _i.max, _m, 0, 1, (_i.min + 1) & _m]
ALL_DTS = [W.DT_F32, W.DT_BF16, W.DT_F16, W.DT_FP8, W.DT_U8, W.DT_F64, W.DT_FP8_E4M3FNUZ, W.DT_FP8_E5M2,
           W.DT_FP8_E5M2FNUZ, W.DT_I8, W.DT_I16, W.DT_I32, W.DT_I64]
BITS_VIEW = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}


def _special_pair(dt, n, seed):
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    t = W.TORCH_DTYPE[dt]
    es = W.ELEM_SIZE[dt]
    if dt == W.DT_U8:
        gold = torch.randint(0, 256, (n,), device="cuda", dtype=torch.uint8, generator=gen)
    elif t in W.INT_TYPES:
        hi = 100 if es == 1 else 1 << 20
        gold = torch.randint(-hi, hi, (n,), device="cuda", dtype=torch.int64, generator=gen).to(t)
    else:
        gold = torch.randn(n, device="cuda", generator=gen, dtype=torch.float64).to(t)
    cand = gold.clone()
    gb = gold.view(BITS_VIEW[es])
    cb = cand.view(gb.dtype)
    m = max(1, n // 20)
    idx = torch.from_numpy(rng.choice(n, size=min(n, m), replace=False)).cuda()
    flips = torch.from_numpy(rng.integers(1, 1 << (8 * es - 1), size=len(idx))).cuda().to(cb.dtype)
    cb[idx] ^= flips          # arbitrary bit flips: NaNs, infs, sign changes, huge ULP distances
    if n > 8 and dt != W.DT_U8:
        special = SPECIALS[dt]
        for j, v in enumerate(special):
            val = v if es == 1 or v < (1 << (8 * es - 1)) else v - (1 << (8 * es))
            gb[j] = val
            cb[(j + 1) % len(special)] = val
    return cand, gold


@pytest.mark.parametrize("dt", ALL_DTS)
def test_compare_dtypes_specials_and_tails(kc, ctx, dt):
    say(f"compare dtype={dt}: bit flips, specials, ragged tails, empty")
    pairs = []
    for i, n in enumerate([0, 1, 3, 7, 8, 15, 16, 17, 255, 4096 + 5, 70001, 300007]):
        c, g = _special_pair(dt, max(n, 1), 100 * dt + i)
        c, g = c[:n], g[:n]
        pairs.append((c, g, dt, int(i % 9), (0.0, 1e-8, 1e-3)[i % 3], (0.0, 1e-5, 0.0, 1e-2)[i % 4]))
    for tb, per_item in ((None, 0), (4096, 0), (4096, 1), (1 << 20, 0)):
        cmp_vs_oracle(kc, ctx, pairs, tile_bytes=tb, per_item=per_item)


def test_compare_mixed_dtypes_one_launch(kc, ctx):
    say("compare: every dtype in one batched launch, 1-ULP perturbations")
    rng = np.random.default_rng(77)
    gen = torch.Generator().manual_seed(77)
    pairs = []
    for dt in ALL_DTS:
        if dt == W.DT_U8:
            continue
        t = W.TORCH_DTYPE[dt]
        for n in (1000, 65536 + 3):
            if t in W.INT_TYPES:
                gold = torch.randint(-100, 100, (n,), generator=gen, dtype=torch.int64).to(t)
            else:
                gold = (torch.randn(n, generator=gen, dtype=torch.float64) * 0.5).to(t)
            pr = W.perturb_pair(gold.cuda(), dt, rng, n // 100, 3, n_nan=0 if t in W.INT_TYPES else 2, ulp_tol=1)
            pairs.append((pr.cand, pr.gold, dt, 1, 1e-8, 1e-5))
    got = cmp_vs_oracle(kc, ctx, pairs)
    assert all(r["n_mismatch_elems"] > 0 for r in got)


def test_compare_c3_scaled(kc, ctx):
    say("compare c3 scale 1/256: 1000 mixed pairs, batched vs per-buffer vs tile sizes")
    ps = W.c3_pairs("cuda", scale=1 / 256, n_pairs=1000)
    pairs = [(ps.cand(i), ps.gold(i), int(ps.dtypes[i]), int(ps.tols[i]), 1e-8, 1e-5) for i in range(len(ps))]
    got = cmp_vs_oracle(kc, ctx, pairs)
    for i, r in enumerate(got):
        assert r["n_mismatch_elems"] == len(ps.pos[i])
        assert r["n_over_tol"] == int((np.abs(ps.k[i]) > ps.tols[i]).sum())
    for kw in (dict(per_item=1), dict(tile_bytes=16384), dict(tile_bytes=1 << 20, grid=1)):
        c2 = kc.Context(0)
        c2.set_tuning(kc.OP_COMPARE, grid_per_cu=kw.get("grid", 0), tile_bytes=kw.get("tile_bytes", 0),
                      per_item=kw.get("per_item", 0))
        res = kc.compare(c2, pairs)
        torch.cuda.synchronize()
        assert kc.decode_cmp(res, len(pairs)) == got
        c2.close()


def test_compare_unaligned_views(kc, ctx):
    """Views at odd element offsets (both sides, one side, different offsets)
    on every element type: each report equal to the oracle's, and to the
    aligned copies' report."""
    say("compare views at odd element offsets vs oracle")
    rng = np.random.default_rng(91)
    gen = torch.Generator().manual_seed(91)
    pairs, aligned = [], []
    for dt in ALL_DTS:
        t = W.TORCH_DTYPE[dt]
        for n, (oc, og) in ((1000, (1, 1)), (4099, (3, 0)), (70001, (0, 5)), (65536, (2, 7)), (5, (1, 2))):
            if t in W.INT_TYPES:
                gold = torch.randint(-100, 100, (n,), generator=gen, dtype=torch.int64).to(t)
            elif dt == W.DT_U8:
                gold = torch.randint(0, 256, (n,), generator=gen, dtype=torch.int64).to(torch.uint8)
            else:
                gold = (torch.randn(n, generator=gen, dtype=torch.float64)).to(t)
            gold = gold.cuda()
            if dt == W.DT_U8:
                cand = gold.clone()
                idx = torch.from_numpy(rng.choice(n, size=min(n, 9), replace=False)).cuda()
                cand[idx] ^= 0x11
            else:
                nan = 0 if t in W.INT_TYPES or n < 10 else 2
                cand = W.perturb_pair(gold, dt, rng, max(1, n // 300), 4, n_nan=nan, ulp_tol=2).cand
            cbuf = torch.empty(n + 8, dtype=t, device="cuda")
            gbuf = torch.empty(n + 8, dtype=t, device="cuda")
            cbuf[oc:oc + n] = cand
            gbuf[og:og + n] = gold
            pairs.append((cbuf[oc:oc + n], gbuf[og:og + n], dt, 2, 1e-7, 1e-4))
            aligned.append((cand, gold, dt, 2, 1e-7, 1e-4))
    got = cmp_vs_oracle(kc, ctx, pairs)
    assert got == kc.decode_cmp(kc.compare(ctx, aligned), len(aligned))
    assert sum(r["n_mismatch_elems"] for r in got) > 0
    for tb in (16384, 65536):   # several tiles per pair, tiles ending mid-pair
        assert cmp_vs_oracle(kc, ctx, pairs, tile_bytes=tb) == got


def test_compare_errors(kc, ctx):
    say("compare argument errors")
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(kc.KCError) as ei:                # fp32 elements at an odd byte address
        kc.compare(ctx, [(a[1:33], a[1:33], W.DT_F32, 0)])
    assert ei.value.code == kc.EALIGN
    arr, n = kc.make_pairs([(a, a, W.DT_U8, 0)])
    arr[0].dtype = 13
    with pytest.raises(kc.KCError) as ei:
        kc.compare(ctx, (arr, n))
    assert ei.value.code == kc.EDTYPE
