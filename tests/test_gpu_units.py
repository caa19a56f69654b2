"""Hash units larger than the 4 KiB page (8 KiB to 2 MiB), on the GPU vs the
CPU oracle through the C ABI: snapshot (fused and two-pass), delta snapshot,
restore (full and delta, corrupted page-VA entries), region diff, closure scan
and snapshot files, on ranges with partial last units and zero units, then the
2 GiB 4096-range set and the 30 GiB MoE pool at 64 KiB and 2 MiB.  No byte
outside a range may ever be written (the arena around the ranges holds a
sentinel that must survive).

Every case prints its name before touching the GPU."""
import concurrent.futures as cf
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_03208_amd import workloads as W
from tests.helpers import words_to_bits

pytestmark = pytest.mark.gpu

PAGE = 4096
WORKERS = min(16, os.cpu_count() or 1)


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


def _outside_unchanged(case, before):
    """Every arena byte outside the ranges equals ``before``."""
    buf = case.arena.buf.cpu().numpy()
    mask = np.ones(len(buf), dtype=bool)
    for o, s in zip(case.layout.offsets, case.layout.sizes):
        mask[int(o):int(o) + int(s)] = False
    return np.array_equal(buf[mask], before[mask])


def test_unit_argument_checks(kc, ctx):
    say("units: unit sizes that are not a power of two from 4 KiB to 2 MiB are refused")
    case = W.units_case("cuda", unit=8192, n_ranges=3, seed=1)
    for bad in (0, 2048, 12288, 4 << 20):
        with pytest.raises(kc.KCError) as ei:
            kc.RangeSet(ctx, case.ranges(), unit=bad)
        assert ei.value.code == kc.EINVAL


@pytest.mark.parametrize("unit,n_ranges,seed", [(8192, 30, 21), (65536, 24, 22), (1 << 21, 12, 23),
                                                (1 << 21, 40, 24)])
def test_units_snapshot_restore_scan_diff_files(kc, ctx, tmp_path, unit, n_ranges, seed):
    say(f"units {unit}: {n_ranges} ranges seed {seed}: snapshot, compact, restore, scan, region diff, files")
    case = W.units_case("cuda", unit=unit, n_ranges=n_ranges, seed=seed)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    views = W.host_views(case.layout, host)
    rs = kc.RangeSet(ctx, ranges, unit=unit)
    st, n_units, _ = oracle.range_check(ranges, unit)
    assert st == 0 and rs.n_pages == n_units
    # fused entry point: probe, scan, hashing pass with the packed writes, closure scan as its own pass
    scan = kc.ScanOut("cuda", oob_cap=64)
    out = kc.snapshot(ctx, rs, seed=7, scan=scan)
    torch.cuda.synchronize()
    oh, oz, _ = oracle.page_hash(ranges, views, seed=7, unit=unit)
    assert np.array_equal(u64(out["hash"])[:rs.n_pages], oh)
    assert np.array_equal(u64(out["zero_bm"])[:rs.n_words], oz)
    zbits = words_to_bits(oz, n_units)
    assert 0 < zbits.sum() < n_units
    op, ova, onk = oracle.compact(ranges, views, oz, unit=unit)
    assert int(u64(out["n_kept"])[0]) == onk
    assert np.array_equal(u64(out["page_va"])[:onk], ova)
    assert np.array_equal(out["packed"][:onk * unit].cpu().numpy(), op)
    res, oob = scan.result()
    o_res, o_oob = oracle.closure_scan(ranges, views, oob_cap=64)
    assert res == o_res and oob == o_oob and res["n_in_range"] > 0
    # two passes: hash (with the closure scan) then compaction, and a capacity below the kept count
    scan2 = kc.ScanOut("cuda", oob_cap=3)
    h, z, _ = kc.page_hash(ctx, rs, seed=7, scan=scan2)
    cap = max(1, onk // 2)
    packed, va, nk = kc.compact(ctx, rs, z, None, cap_pages=cap)
    torch.cuda.synchronize()
    assert torch.equal(h, out["hash"]) and torch.equal(z, out["zero_bm"])
    assert int(u64(nk)[0]) == onk
    op2, ova2, _ = oracle.compact(ranges, views, oz, cap_pages=cap, unit=unit)
    assert np.array_equal(u64(va)[:cap], ova2) and np.array_equal(packed[:cap * unit].cpu().numpy(), op2)
    r2, l2 = scan2.result()
    o2, ol2 = oracle.closure_scan(ranges, views, oob_cap=3)
    assert r2 == o2 and l2 == ol2
    # the fused entry point under the same capacity: slots past it are not written (guard bytes after them)
    guard = dict(hash=torch.empty_like(out["hash"]), zero_bm=torch.empty_like(out["zero_bm"]), changed_bm=None,
                 packed=torch.full(((cap + 2) * unit,), 0xA5, dtype=torch.uint8, device="cuda"),
                 page_va=torch.full((cap + 2,), -1, dtype=torch.int64, device="cuda"),
                 n_kept=torch.empty(1, dtype=torch.int64, device="cuda"))
    kc.snapshot(ctx, rs, seed=7, cap_pages=cap, out=guard)
    torch.cuda.synchronize()
    assert int(u64(guard["n_kept"])[0]) == onk and torch.equal(guard["hash"], out["hash"])
    assert np.array_equal(u64(guard["page_va"])[:cap], ova2)
    assert np.array_equal(guard["packed"][:cap * unit].cpu().numpy(), op2)
    assert bool((guard["packed"][cap * unit:] == 0xA5).all()) and bool((guard["page_va"][cap:] == -1).all())

    say(f"units {unit}: clobber the ranges, restore, outside bytes untouched")
    before = case.arena.buf.cpu().numpy().copy()
    for i in range(case.layout.n):
        case.arena.view(i).fill_(0x3C)
    n_bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 0
    assert np.array_equal(case.arena.buf.cpu().numpy(), before)

    say(f"units {unit}: restore with page-VA entries inside a unit, past the end and misaligned")
    bad_va = out["page_va"].clone()
    k = int(onk)
    picks = [0, k // 3, k - 1]
    bad_va[picks[0]] += PAGE          # inside a unit: not the start of one
    bad_va[picks[1]] = ranges[-1][0] + ranges[-1][1] + unit
    bad_va[picks[2]] += 8
    for i in range(case.layout.n):
        case.arena.view(i).fill_(0x3C)
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], bad_va, out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    o_views = [np.full(v.shape, 0x3C, dtype=np.uint8) for v in views]
    o_bad = oracle.restore(ranges, o_views, oz, None, op, u64(bad_va)[:k], k, unit=unit)
    assert int(n_bad.item()) == o_bad >= 1
    got_views = W.host_views(case.layout, case.arena.host_copy())
    assert all(np.array_equal(a, b) for a, b in zip(got_views, o_views))
    assert _outside_unchanged(case, before)
    case.arena.load_concat(np.concatenate(views))

    say(f"units {unit}: region diff against the snapshot after planted changes")
    gen = np.random.default_rng(seed + 100)
    live = [v.copy() for v in views]
    for a in gen.choice(n_ranges, size=min(5, n_ranges), replace=False):
        a = int(a)
        pos = gen.choice(len(live[a]), size=min(7, len(live[a])), replace=False)
        live[a][pos] ^= 0x81
    case.arena.load_concat(np.concatenate(live))
    rd = kc.region_diff(ctx, rs, out, seed=7)
    torch.cuda.synchronize()
    got = kc.decode_region_diff(rd["res"], n_ranges)
    want = oracle.region_diff(ranges, live, oz, op, ova, onk, unit=unit)
    assert got == want and sum(r["n_diff_bytes"] for r in got) > 0

    say(f"units {unit}: delta snapshot against the first, then the restore chain")
    s2 = kc.snapshot(ctx, rs, seed=7, prior=out["hash"])
    torch.cuda.synchronize()
    dh, dz, dc = oracle.page_hash(ranges, live, seed=7, prior=oh, unit=unit)
    assert np.array_equal(u64(s2["hash"])[:rs.n_pages], dh)
    assert np.array_equal(u64(s2["changed_bm"])[:rs.n_words], dc)
    dp, dva, dnk = oracle.compact(ranges, live, dz, dc, unit=unit)
    assert int(u64(s2["n_kept"])[0]) == dnk > 0
    assert np.array_equal(u64(s2["page_va"])[:dnk], dva)
    assert np.array_equal(s2["packed"][:dnk * unit].cpu().numpy(), dp)
    case.arena.load_concat(np.concatenate(views))          # back to the base image, then the delta on top
    kc.restore(ctx, rs, s2["zero_bm"], s2["changed_bm"], s2["packed"], s2["page_va"], s2["n_kept"])
    torch.cuda.synchronize()
    after = W.host_views(case.layout, case.arena.host_copy())
    assert all(np.array_equal(a, b) for a, b in zip(after, live))

    say(f"units {unit}: snapshot files: save, load, restore; a set of another unit is refused")
    d = str(tmp_path / "snap")
    kc.snapshot_save(ctx, rs, d, out, seed=7)
    man = json.load(open(os.path.join(d, "manifest.json")))
    assert man["page_size"] == unit and man["n_pages"] == n_units and man["n_kept"] == onk
    assert np.array_equal(np.fromfile(os.path.join(d, "packed.bin"), dtype=np.uint8), op)
    back, _ = kc.snapshot_load(ctx, rs, d)
    for i in range(case.layout.n):
        case.arena.view(i).fill_(0x3C)
    kc.restore(ctx, rs, back["zero_bm"], None, back["packed"], back["page_va"], back["n_kept"])
    torch.cuda.synchronize()
    assert np.array_equal(case.arena.buf.cpu().numpy(), before)
    other = kc.RangeSet(ctx, ranges, unit=PAGE if unit != PAGE else 8192)
    with pytest.raises(kc.KCError) as ei:
        kc.snapshot_load(ctx, other, d)
    assert ei.value.code == kc.EINVAL
    other.close()
    rs.close()


@pytest.mark.parametrize("unit", [4096, 65536, 1 << 21])
def test_hashing_depths_agree(kc, unit):
    """The hashing pass with one chunk in flight per wave and with two to four
    (the pipeline of large units, forced here at every unit) gives the same
    snapshot and delta, equal to the oracle."""
    say(f"units {unit}: hashing pass at depth 1 to 4")
    case = W.units_case("cuda", unit=max(unit, 8192), n_ranges=20, seed=31)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    views = W.host_views(case.layout, host)
    outs = []
    for depth in (1, 2, 3, 4):
        c = kc.Context(0)
        for op in (kc.OP_SNAPSHOT, kc.OP_PAGE_HASH):
            c.set_tuning(op, depth=depth)
            with pytest.raises(kc.KCError) as ei:
                c.set_tuning(op, depth=5)
            assert ei.value.code == kc.EINVAL and c.get_tuning(op)["depth"] == depth
        rs = kc.RangeSet(c, ranges, unit=unit)
        s1 = kc.snapshot(c, rs, seed=4)
        h2, z2, c2 = kc.page_hash(c, rs, seed=5, prior=s1["hash"])
        torch.cuda.synchronize()
        outs.append([u64(s1["hash"])[:rs.n_pages].copy(), u64(s1["zero_bm"])[:rs.n_words].copy(),
                     s1["packed"][:int(u64(s1["n_kept"])[0]) * unit].cpu().numpy(), u64(h2)[:rs.n_pages].copy(),
                     u64(c2)[:rs.n_words].copy()])
        rs.close()
        c.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)
    oh, oz, _ = oracle.page_hash(ranges, views, seed=4, unit=unit)
    assert np.array_equal(outs[0][0], oh) and np.array_equal(outs[0][1], oz)
    op, _, _ = oracle.compact(ranges, views, oz, unit=unit)
    assert np.array_equal(outs[1][2], op)
    h5, _, ch = oracle.page_hash(ranges, views, seed=5, prior=oh, unit=unit)
    assert np.array_equal(outs[1][3], h5) and np.array_equal(outs[1][4], ch)


def test_unit_runs_per_quad(kc):
    """2400 ranges of up to 40 units of 8 KiB: enough tiles that the
    pipelined pass gives each lane quad a run of two units (32-unit tiles) on a
    256-CU device, with zero units, partial last units and ranges under one
    unit among them.  At two to four chunks in flight, and with one launch per
    range: the snapshot (and under a capacity below the kept count), the
    read-only hash with its zero bits, and the delta against the set after a
    rewrite, all against the oracle."""
    unit = 8192
    say("units 8192: 2400 ranges, runs of units per quad, depths 2-4")
    case = W.units_case("cuda", unit=unit, n_ranges=2400, seed=41, max_units=40)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    views = W.host_views(case.layout, host)
    oh, oz, _ = oracle.page_hash(ranges, views, seed=9, unit=unit)
    op, ova, onk = oracle.compact(ranges, views, oz, unit=unit)
    cap = onk - onk // 3
    op2, ova2, _ = oracle.compact(ranges, views, oz, cap_pages=cap, unit=unit)
    rng = np.random.default_rng(41)
    picks = rng.choice(len(ranges), size=300, replace=False)
    outs = []
    for depth, per_item in ((2, 0), (3, 0), (4, 0), (2, 1)):
        c = kc.Context(0)
        for op_ in (kc.OP_SNAPSHOT, kc.OP_PAGE_HASH):
            c.set_tuning(op_, depth=depth, per_item=per_item)
        rs = kc.RangeSet(c, ranges, unit=unit)
        say(f"units 8192: depth {depth}, one launch per range {per_item}: snapshot, capacity {cap} of {onk}, "
            "read-only hash")
        out = kc.snapshot(c, rs, seed=9)
        torch.cuda.synchronize()
        assert np.array_equal(u64(out["hash"])[:rs.n_pages], oh)
        assert np.array_equal(u64(out["zero_bm"])[:rs.n_words], oz)
        assert int(u64(out["n_kept"])[0]) == onk
        assert np.array_equal(u64(out["page_va"])[:onk], ova)
        assert np.array_equal(out["packed"][:onk * unit].cpu().numpy(), op)
        guard = dict(hash=torch.empty_like(out["hash"]), zero_bm=torch.empty_like(out["zero_bm"]), changed_bm=None,
                     packed=torch.full(((cap + 2) * unit,), 0xA5, dtype=torch.uint8, device="cuda"),
                     page_va=torch.full((cap + 2,), -1, dtype=torch.int64, device="cuda"),
                     n_kept=torch.empty(1, dtype=torch.int64, device="cuda"))
        kc.snapshot(c, rs, seed=9, cap_pages=cap, out=guard)
        h, z, _ = kc.page_hash(c, rs, seed=9)
        torch.cuda.synchronize()
        assert int(u64(guard["n_kept"])[0]) == onk
        assert np.array_equal(u64(guard["page_va"])[:cap], ova2)
        assert np.array_equal(guard["packed"][:cap * unit].cpu().numpy(), op2)
        assert bool((guard["packed"][cap * unit:] == 0xA5).all()) and bool((guard["page_va"][cap:] == -1).all())
        assert np.array_equal(u64(h)[:rs.n_pages], oh) and np.array_equal(u64(z)[:rs.n_words], oz)
        outs.append((c, rs, out))
    say("units 8192: rewrite a byte in 300 ranges (zero units among them), delta in each context")
    for a in picks:
        o, sz = int(case.layout.offsets[a]), int(case.layout.sizes[a])
        pos = o + int(rng.integers(0, sz))
        case.arena.buf[pos] = (int(host[pos]) + 1) % 256
    v2 = W.host_views(case.layout, case.arena.host_copy())
    dh, dz, dc = oracle.page_hash(ranges, v2, seed=9, prior=oh, unit=unit)
    assert words_to_bits(dc, len(oh)).sum() == 300
    for c, rs, out in outs:
        h2, z2, c2 = kc.page_hash(c, rs, seed=9, prior=out["hash"])
        torch.cuda.synchronize()
        assert np.array_equal(u64(h2)[:rs.n_pages], dh)
        assert np.array_equal(u64(z2)[:rs.n_words], dz)
        assert np.array_equal(u64(c2)[:rs.n_words], dc)
        rs.close()
        c.close()


@pytest.mark.parametrize("unit", [65536, 1 << 21])
def test_units_c2_full(kc, ctx, unit):
    """The 2 GiB set of 4096 ranges (sizes 4 KiB to 64 MiB): most ranges end in
    a partial unit at 64 KiB, nearly all are one partial unit at 2 MiB."""
    say(f"units {unit}: c2 full (4096 ranges, 2 GiB): full snapshot, 5 % rewrite, delta, restore chain")
    case = W.c2_snapshot("cuda")
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges, unit=unit)
    s1 = kc.snapshot(ctx, rs, seed=2)
    host1 = case.arena.host_copy().copy()
    v1 = W.host_views(case.layout, host1)
    torch.cuda.synchronize()
    oh, oz, _ = oracle.page_hash(ranges, v1, seed=2, unit=unit)
    assert np.array_equal(u64(s1["hash"])[:rs.n_pages], oh)
    assert np.array_equal(u64(s1["zero_bm"])[:rs.n_words], oz)
    op, ova, onk = oracle.compact(ranges, v1, oz, unit=unit)
    assert int(u64(s1["n_kept"])[0]) == onk
    assert np.array_equal(u64(s1["page_va"])[:onk], ova)
    assert np.array_equal(s1["packed"][:onk * unit].cpu().numpy(), op)
    del op
    W.c2_rewrite(case)
    host2 = case.arena.host_copy().copy()
    v2 = W.host_views(case.layout, host2)
    s2 = kc.snapshot(ctx, rs, seed=2, prior=s1["hash"])
    torch.cuda.synchronize()
    dh, dz, dc = oracle.page_hash(ranges, v2, seed=2, prior=oh, unit=unit)
    assert np.array_equal(u64(s2["hash"])[:rs.n_pages], dh)
    assert np.array_equal(u64(s2["changed_bm"])[:rs.n_words], dc)
    dp, dva, dnk = oracle.compact(ranges, v2, dz, dc, unit=unit)
    assert int(u64(s2["n_kept"])[0]) == dnk
    assert np.array_equal(u64(s2["page_va"])[:dnk], dva)
    assert np.array_equal(s2["packed"][:dnk * unit].cpu().numpy(), dp)
    case.arena.buf.fill_(0x5A)
    kc.restore(ctx, rs, s1["zero_bm"], None, s1["packed"], s1["page_va"], s1["n_kept"])
    kc.restore(ctx, rs, s2["zero_bm"], s2["changed_bm"], s2["packed"], s2["page_va"], s2["n_kept"])
    torch.cuda.synchronize()
    got = W.host_views(case.layout, case.arena.host_copy())
    assert all(np.array_equal(a, b) for a, b in zip(got, v2))
    rs.close()


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("unit", [65536, 1 << 21])
def test_units_c4_full(kc, unit):
    """The 30 GiB MoE pool: every unit hash, zero bit, page VA and packed unit
    against the oracle run one range at a time, the closure scan (its own pass
    at these units) against the per-range oracle scans, and a restore of every
    byte."""
    from tests.test_gpu_fullsize import _bounded, _scan_totals
    from tests.test_gpu_parity import _tuned_context
    ctx, shapes = _tuned_context(kc, "c4-moe-pool-scale1.0", (kc.OP_SNAPSHOT, kc.OP_RESTORE))
    say(f"units {unit}: c4 full (30 GiB, 200 ranges), shapes {shapes or 'built-in'}")
    case = W.c4_snapshot("cuda")
    ranges = case.ranges()
    n = len(ranges)
    rs = kc.RangeSet(ctx, ranges, unit=unit)
    st, N, fp = oracle.range_check(ranges, unit)
    assert st == 0 and N == rs.n_pages
    fp = [int(x) for x in fp]
    scan = kc.ScanOut("cuda", oob_cap=16)
    out = kc.snapshot(ctx, rs, seed=0, scan=scan)
    torch.cuda.synchronize()
    g_hash = u64(out["hash"])[:N].copy()
    g_zero = words_to_bits(u64(out["zero_bm"])[:rs.n_words], N)
    g_kept = int(u64(out["n_kept"])[0])
    g_res, g_oob = scan.result()
    hosts = [None] * n

    def phase1(a, host):
        oh, oz, _ = oracle.page_hash([ranges[a]], [host], unit=unit)
        zb = words_to_bits(oz, fp[a + 1] - fp[a])
        assert np.array_equal(g_hash[fp[a]:fp[a + 1]], oh), f"unit hashes differ in range {a}"
        assert np.array_equal(g_zero[fp[a]:fp[a + 1]], zb), f"zero bits differ in range {a}"
        return a, int(len(zb) - zb.sum()), oz, oracle.closure_scan_range(ranges, a, host, oob_cap=16)

    def jobs1():
        for a in range(n):
            hosts[a] = case.arena.view(a).cpu().numpy()
            yield phase1, (a, hosts[a])

    kept, zw, scans = [0] * n, [None] * n, [None] * n
    with cf.ThreadPoolExecutor(WORKERS) as pool:
        for a, k, oz, sc in _bounded(pool, jobs1(), 2 * WORKERS):
            kept[a], zw[a], scans[a] = k, oz, sc
    assert g_kept == sum(kept)
    o_res, o_oob = _scan_totals(scans, 16)
    assert g_res == o_res and g_oob == o_oob
    say(f"units {unit}: c4 full: every packed unit and page VA vs the oracle")
    slot0 = np.concatenate([[0], np.cumsum(kept)]).astype(np.int64)
    g_va = u64(out["page_va"])[:g_kept].copy()

    def phase2(a, host, dev_packed):
        op, ova, onk = oracle.compact([ranges[a]], [host], zw[a], unit=unit)
        assert onk == kept[a]
        assert np.array_equal(g_va[slot0[a]:slot0[a + 1]], ova), f"page VAs differ in range {a}"
        assert np.array_equal(dev_packed, op), f"packed units differ in range {a}"
        return a

    def jobs2():
        for a in range(n):
            yield phase2, (a, hosts[a], out["packed"][int(slot0[a]) * unit:int(slot0[a + 1]) * unit].cpu().numpy())

    with cf.ThreadPoolExecutor(WORKERS) as pool:
        list(_bounded(pool, jobs2(), WORKERS))
    say(f"units {unit}: c4 full: clobber, restore, every byte")
    golden = case.arena.buf.clone()
    case.arena.buf.fill_(0xA5)
    n_bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 0
    for a in range(n):
        o, sz = int(case.layout.offsets[a]), int(case.layout.sizes[a])
        assert torch.equal(case.arena.buf[o:o + sz], golden[o:o + sz]), a
    rs.close()
    ctx.close()
