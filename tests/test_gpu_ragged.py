"""Ranges whose sizes are not multiples of the page, on the GPU vs the CPU
oracle through the C ABI: every step over the partial last pages, and no
byte outside a range ever written (the arena around the ranges holds a
sentinel pattern that must survive).

Every case prints its name before touching the GPU."""
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


@pytest.mark.parametrize("n_ranges,seed", [(40, 9), (300, 10), (3, 11)])
def test_ragged_snapshot_restore_scan_graph(kc, ctx, n_ranges, seed):
    say(f"ragged ranges: n={n_ranges} seed={seed}: snapshot, compact, restore, scan, graph, region diff")
    case = W.ragged_case("cuda", n_ranges=n_ranges, seed=seed)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    views = W.host_views(case.layout, host)
    rs = kc.RangeSet(ctx, ranges)
    assert rs.n_pages == case.layout.n_pages
    # fused snapshot with the closure scan
    scan = kc.ScanOut("cuda", oob_cap=64)
    out = kc.snapshot(ctx, rs, seed=5, scan=scan)
    torch.cuda.synchronize()
    oh, oz, _ = oracle.page_hash(ranges, views, seed=5)
    assert np.array_equal(u64(out["hash"])[:rs.n_pages], oh)
    assert np.array_equal(u64(out["zero_bm"])[:rs.n_words], oz)
    op, ova, onk = oracle.compact(ranges, views, oz)
    assert int(u64(out["n_kept"])[0]) == onk
    assert np.array_equal(u64(out["page_va"])[:onk], ova)
    assert np.array_equal(out["packed"][:onk * PAGE].cpu().numpy(), op)
    res, oob = scan.result()
    assert (res, oob) == oracle.closure_scan(ranges, views, oob_cap=64)
    # hash-only pass, standalone scan, pointer graph
    h, z, _ = kc.page_hash(ctx, rs, seed=5)
    scan2 = kc.ScanOut("cuda", oob_cap=64)
    kc.closure_scan(ctx, rs, scan2)
    edge = kc.pointer_graph(ctx, rs)
    torch.cuda.synchronize()
    assert np.array_equal(u64(h)[:rs.n_pages], oh) and np.array_equal(u64(z)[:rs.n_words], oz)
    assert scan2.result() == (res, oob)
    assert np.array_equal(edge.cpu().numpy().view(np.uint64), oracle.pointer_graph(ranges, views))
    # restore over clobbered ranges: range bytes come back, nothing outside is touched
    for (o, s) in zip(case.layout.offsets, case.layout.sizes):
        case.arena.buf[int(o): int(o) + int(s)] = 0x3C
    n_bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 0
    assert np.array_equal(case.arena.host_copy(), host)
    # region diff: the last byte of a partial page counts, a byte past the range's end does not
    a = next(i for i, (_, s) in enumerate(ranges) if s % PAGE != 0 and s > 64)
    end = int(case.layout.offsets[a]) + int(case.layout.sizes[a])
    case.arena.buf[end - 1] ^= 0xFF
    case.arena.buf[end] ^= 0xFF
    torch.cuda.synchronize()
    got = kc.decode_region_diff(kc.region_diff(ctx, rs, out, seed=5)["res"], len(ranges))
    live = case.arena.host_copy()
    want = oracle.region_diff(ranges, W.host_views(case.layout, live), oz, op, ova, onk)
    assert got == want
    assert got[a]["n_diff_bytes"] == 1 and got[a]["first_diff_va"] == ranges[a][0] + ranges[a][1] - 1
    rs.close()


def test_ragged_delta_compact_and_per_range_launches(kc, ctx):
    say("ragged ranges: delta compact against a prior table, per-range launches equal batched")
    case = W.ragged_case("cuda", n_ranges=60, seed=12)
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    h0, _, _ = kc.page_hash(ctx, rs)
    torch.cuda.synchronize()
    prior = h0.clone()
    rng = np.random.default_rng(4)
    for a in rng.choice(len(ranges), size=20, replace=False):   # rewrite one byte in 20 ranges
        o = int(case.layout.offsets[a]) + int(rng.integers(0, int(case.layout.sizes[a])))
        case.arena.buf[o] ^= 0x5A
    torch.cuda.synchronize()
    host = case.arena.host_copy()
    views = W.host_views(case.layout, host)
    h, z, c = kc.page_hash(ctx, rs, prior=prior)
    packed, va, nk = kc.compact(ctx, rs, z, c)
    torch.cuda.synchronize()
    oh, oz, oc = oracle.page_hash(ranges, views, prior=u64(prior)[:rs.n_pages])
    assert np.array_equal(u64(c)[:rs.n_words], oc)
    op, ova, onk = oracle.compact(ranges, views, oz, oc)
    assert int(u64(nk)[0]) == onk
    assert np.array_equal(u64(va)[:onk], ova) and np.array_equal(packed[:onk * PAGE].cpu().numpy(), op)
    ctx2 = kc.Context(0)
    for op_ in (kc.OP_PAGE_HASH, kc.OP_SNAPSHOT, kc.OP_CLOSURE, kc.OP_RESTORE):
        ctx2.set_tuning(op_, per_item=1)
    rs2 = kc.RangeSet(ctx2, ranges)
    out2 = kc.snapshot(ctx2, rs2)
    out1 = kc.snapshot(ctx, rs)
    torch.cuda.synchronize()
    n = int(u64(out1["n_kept"])[0])
    assert torch.equal(out1["hash"], out2["hash"]) and torch.equal(out1["zero_bm"], out2["zero_bm"])
    assert torch.equal(out1["packed"][:n * PAGE], out2["packed"][:n * PAGE])
    rs2.close()
    ctx2.close()
    rs.close()


def test_ragged_snapshot_files_roundtrip(kc, ctx, tmp_path):
    say("ragged ranges: snapshot saved to files, loaded, restored over clobbered ranges")
    case = W.ragged_case("cuda", n_ranges=25, seed=13)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    rs = kc.RangeSet(ctx, ranges)
    out = kc.snapshot(ctx, rs)
    torch.cuda.synchronize()
    d = str(tmp_path / "snap")
    kc.snapshot_save(ctx, rs, d, out)
    for (o, s) in zip(case.layout.offsets, case.layout.sizes):
        case.arena.buf[int(o): int(o) + int(s)] = 0x3C
    back, _ = kc.snapshot_load(ctx, rs, d)
    kc.restore(ctx, rs, back["zero_bm"], None, back["packed"], back["page_va"], back["n_kept"])
    torch.cuda.synchronize()
    assert np.array_equal(case.arena.host_copy(), host)
    rs.close()
