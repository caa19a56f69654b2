"""Pointer graph on the GPU vs the CPU oracle, bit for bit, through the C ABI,
and the reachable-only snapshot built on it.

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


def graph_vs_oracle(kc, ctx, case, win=(0, 0), per_cu=None):
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    host = case.arena.host_copy()
    views = W.host_views(case.layout, host)
    if per_cu is not None:
        ctx.set_tuning(kc.OP_GRAPH, grid_per_cu=per_cu)
    edge = kc.pointer_graph(ctx, rs, win[0], win[1])
    torch.cuda.synchronize()
    got = edge.cpu().numpy().view(np.uint64)
    want = oracle.pointer_graph(ranges, views, win[0], win[1])
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    if per_cu is not None:
        ctx.set_tuning(kc.OP_GRAPH, grid_per_cu=0)
    return rs, got


@pytest.mark.parametrize("n,seed", [(1, 1), (7, 2), (64, 3), (130, 4), (700, 5)])
def test_planted_graph(kc, ctx, n, seed):
    say(f"pointer graph: planted digraph n_ranges={n} seed={seed}")
    case = W.graph_case("cuda", n_ranges=n, seed=seed)
    rs, got = graph_vs_oracle(kc, ctx, case)
    adj = oracle.edges_to_bool(got, n)
    want = np.zeros((n, n), bool)
    for a, b in case.truth["edges"]:
        want[a, b] = True
    assert (adj == want).all()
    for per_cu in (1, 32):   # launch shape must not change the result
        graph_vs_oracle(kc, ctx, case, per_cu=per_cu)
    rs.close()


@pytest.mark.parametrize("n,seed", [(4096, 6), (5000, 7)])
def test_many_ranges_graph_and_scans(kc, ctx, n, seed):
    """The graph and the standalone scan keep up to 4096 ranges in one LDS
    table per workgroup; past that the table strides and the search finishes
    in global memory.  The fused scan keeps 256."""
    say(f"pointer graph and closure scans over {n} ranges")
    case = W.graph_case("cuda", n_ranges=n, seed=seed, max_pages=3)
    rs, got = graph_vs_oracle(kc, ctx, case)
    want = np.zeros((n, n), bool)
    for a, b in case.truth["edges"]:
        want[a, b] = True
    assert (oracle.edges_to_bool(got, n) == want).all()
    ranges = case.ranges()
    host = case.arena.host_copy()
    views = W.host_views(case.layout, host)
    o_res, o_oob = oracle.closure_scan(ranges, views, oob_cap=64)
    assert o_res["n_oob"] > 0 and o_res["n_in_range"] > 0
    say(f"closure scans over {n} ranges: standalone and fused vs oracle")
    scan = kc.ScanOut("cuda", oob_cap=64)
    kc.closure_scan(ctx, rs, scan)
    scan2 = kc.ScanOut("cuda", oob_cap=64)
    kc.snapshot(ctx, rs, scan=scan2)
    torch.cuda.synchronize()
    assert scan.result() == (o_res, o_oob)
    assert scan2.result() == (o_res, o_oob)
    rs.close()


def test_windows_and_dense_pointers(kc, ctx):
    say("pointer graph: custom windows; c1 scaled (1 % of words are pointers)")
    case = W.graph_case("cuda", n_ranges=40, seed=21)
    vals = sorted(v for _, _, v in case.truth["plants"])
    for win in ((vals[len(vals) // 3], vals[2 * len(vals) // 3]), (vals[0], vals[0] + 1), (1, 2**64 - 1)):
        graph_vs_oracle(kc, ctx, case, win=win)[0].close()
    c1 = W.c1_snapshot("cuda", scale=1 / 16, seed=3)
    graph_vs_oracle(kc, ctx, c1)[0].close()


def test_reachable_only_snapshot(kc, ctx):
    say("pointer graph: reach from kernel-argument words, snapshot of the reachable ranges only")
    case = W.graph_case("cuda", n_ranges=200, seed=31, mean_out=0.8)
    ranges = case.ranges()
    rs, got = graph_vs_oracle(kc, ctx, case)
    reach = kc.graph_reach(ranges, got, case.truth["root_words"])
    assert (reach == oracle.graph_reach(ranges, got, case.truth["root_words"])).all()
    sub = [r for r, keep in zip(ranges, reach) if keep]
    assert 0 < len(sub) <= len(ranges)
    rs_sub = kc.RangeSet(ctx, sub)
    out = kc.snapshot(ctx, rs_sub)
    torch.cuda.synchronize()
    host = case.arena.host_copy()
    views = [v for v, keep in zip(W.host_views(case.layout, host), reach) if keep]
    oh, oz, _ = oracle.page_hash(sub, views)
    assert np.array_equal(out["hash"].cpu().numpy().view(np.uint64)[:rs_sub.n_pages], oh)
    op, ova, onk = oracle.compact(sub, views, oz)
    assert int(out["n_kept"].cpu().numpy().view(np.uint64)[0]) == onk
    assert np.array_equal(out["page_va"].cpu().numpy().view(np.uint64)[:onk], ova)
    assert np.array_equal(out["packed"][:onk * PAGE].cpu().numpy(), op)
    rs_sub.close()
    rs.close()


def test_graph_limits_and_empty(kc, ctx):
    say("pointer graph: empty range set, too many ranges, bad window")
    rs = kc.RangeSet(ctx, [])
    e = kc.pointer_graph(ctx, rs)
    assert e.numel() == 0
    rs.close()
    many = [(0x7F0000000000 + i * 2 * PAGE, PAGE) for i in range(kc.GRAPH_MAX_RANGES + 1)]
    rs = kc.RangeSet(ctx, many)   # the table only: nothing is read before the limit check
    with pytest.raises(kc.KCError) as ei:
        kc.pointer_graph(ctx, rs)
    assert ei.value.code == kc.ELIMIT
    rs.close()
    case = W.graph_case("cuda", n_ranges=3, seed=2)
    rs = kc.RangeSet(ctx, case.ranges())
    with pytest.raises(kc.KCError) as ei:
        kc.pointer_graph(ctx, rs, 0, 100)
    assert ei.value.code == kc.EINVAL
    rs.close()


def test_ranges_from_far_apart_allocations(kc, ctx):
    say("range lookups: 520 small ranges plus two at the ends of a 3 GiB allocation, cross pointers, "
        "scan + graph + hash vs oracle")
    a = W.graph_case("cuda", n_ranges=260, seed=41, max_pages=3)
    b = W.graph_case("cuda", n_ranges=260, seed=42, max_pages=3)
    spacer = torch.zeros(3 << 30, dtype=torch.uint8, device="cuda")
    s0 = (spacer.data_ptr() + PAGE - 1) // PAGE * PAGE
    s1 = (spacer.data_ptr() + spacer.numel()) // PAGE * PAGE - 2 * PAGE
    far = [(s0, 2 * PAGE), (s1, 2 * PAGE)]           # the span of the set now covers gigabytes
    # pointers between the arenas and into the far ranges, at known words
    rng = np.random.default_rng(3)
    targets = a.ranges() + b.ranges() + far
    for src in (a, b):
        words = src.arena.buf.view(torch.int64)
        for _ in range(60):
            base, size = targets[int(rng.integers(0, len(targets)))]
            r0, sz0 = src.ranges()[int(rng.integers(0, 260))]
            words[(r0 - src.arena.va_base) // 8 + int(rng.integers(0, sz0 // 8))] = base + int(rng.integers(0, size))
    spacer[s0 - spacer.data_ptr():s0 - spacer.data_ptr() + 8] = torch.tensor(
        [a.ranges()[5][0] + 16], dtype=torch.int64).view(torch.uint8).cuda()
    torch.cuda.synchronize()
    views_by_base = {}
    for c in (a, b):
        for (base, _), v in zip(c.ranges(), W.host_views(c.layout, c.arena.host_copy())):
            views_by_base[base] = v
    for base, size in far:
        off = base - spacer.data_ptr()
        views_by_base[base] = spacer[off:off + size].cpu().numpy()
    ranges = sorted(targets)
    views = [views_by_base[base] for base, _ in ranges]
    say(f"span of the set: {(ranges[-1][0] + ranges[-1][1] - ranges[0][0]) / 2**30:.2f} GiB, {len(ranges)} ranges")
    rs = kc.RangeSet(ctx, ranges)
    edge = kc.pointer_graph(ctx, rs)
    scan = kc.ScanOut("cuda", oob_cap=256)
    h, z, _ = kc.page_hash(ctx, rs, scan=scan)
    torch.cuda.synchronize()
    assert np.array_equal(edge.cpu().numpy().view(np.uint64), oracle.pointer_graph(ranges, views))
    res, oob = scan.result()
    o_res, o_oob = oracle.closure_scan(ranges, views, oob_cap=256)
    assert res == o_res and oob == o_oob
    assert res["n_in_range"] >= 120
    oh, oz, _ = oracle.page_hash(ranges, views)
    assert np.array_equal(h.cpu().numpy().view(np.uint64)[:rs.n_pages], oh)
    rs.close()
    del spacer
