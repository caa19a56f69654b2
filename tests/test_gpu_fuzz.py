"""Seeded sweep over random range sets on the GPU vs the CPU oracle: range
counts from 1 to 600 (one to three LDS fence strides), sizes from a few bytes
to 80 KiB (partial and whole last pages, ragged tiles), gaps of zero to three
pages, zero pages, pointer words.  Each case checks the fused snapshot with the
closure scan, the restore (nothing outside the ranges written), the pointer
graph and the region diff.

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


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("seed", range(64))
def test_random_range_sets(kc, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.choice([1, 2, 7, 63, 64, 65, 255, 256, 257, 600]))
    max_bytes = int(rng.choice([40, 5000, 20 * PAGE]))
    say(f"fuzz seed={seed}: {n} ranges, sizes up to {max_bytes} bytes")
    case = W.ragged_case("cuda", n_ranges=n, seed=2000 + seed, max_bytes=max_bytes)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    views = W.host_views(case.layout, host)
    ctx = kc.Context(0)
    if seed % 3 == 1:   # other launch shapes give the same results
        for op in (kc.OP_SNAPSHOT, kc.OP_RESTORE, kc.OP_GRAPH, kc.OP_REGION_DIFF, kc.OP_PAGE_HASH):
            ctx.set_tuning(op, grid_per_cu=int(rng.integers(1, 9)))
    rs = kc.RangeSet(ctx, ranges)
    scan = kc.ScanOut("cuda", oob_cap=int(rng.integers(0, 8)))
    seed_h = int(rng.integers(0, 2**63))
    out = kc.snapshot(ctx, rs, seed=seed_h, scan=scan)
    edge = kc.pointer_graph(ctx, rs)
    torch.cuda.synchronize()
    oh, oz, _ = oracle.page_hash(ranges, views, seed=seed_h)
    assert np.array_equal(u64(out["hash"])[:rs.n_pages], oh)
    assert np.array_equal(u64(out["zero_bm"])[:rs.n_words], oz)
    op, ova, onk = oracle.compact(ranges, views, oz)
    assert int(u64(out["n_kept"])[0]) == onk
    assert np.array_equal(u64(out["page_va"])[:onk], ova)
    assert np.array_equal(out["packed"][:onk * PAGE].cpu().numpy(), op)
    assert scan.result() == oracle.closure_scan(ranges, views, oob_cap=scan.cap)
    assert np.array_equal(edge.cpu().numpy().view(np.uint64), oracle.pointer_graph(ranges, views))
    for (o, s) in zip(case.layout.offsets, case.layout.sizes):
        case.arena.buf[int(o): int(o) + int(s)] = int(rng.integers(1, 256))
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"])
    torch.cuda.synchronize()
    assert np.array_equal(case.arena.host_copy(), host)
    flips = rng.integers(0, case.arena.buf.numel(), size=20)
    case.arena.buf[torch.from_numpy(flips).cuda()] ^= 0x11
    torch.cuda.synchronize()
    got = kc.decode_region_diff(kc.region_diff(ctx, rs, out, seed=seed_h)["res"], len(ranges))
    live = case.arena.host_copy()
    assert got == oracle.region_diff(ranges, W.host_views(case.layout, live), oz, op, ova, onk)
    rs.close()
    ctx.close()
