"""Pins the oracle on ranges whose sizes are not multiples of the page (the
pointer-to-size map holds exact allocation sizes, paper Sec. 4.1.1): the
partial last page of a range is hashed, zero-tested, packed, restored and
scanned over its own bytes only.

Independent pins: python-xxhash of each page's exact bytes (library), numpy
per-page zero tests, numpy construction of the packed slots (bytes, then
zeros), a sentinel byte pattern outside every range that no step may change,
and the generator's record of its planted pointer words."""
import numpy as np
import pytest

from paper_2605_03208_amd import workloads as W

xxhash = pytest.importorskip("xxhash")
PAGE = 4096


@pytest.fixture(scope="module")
def rcase():
    case = W.ragged_case(seed=9)
    host = case.arena.host_copy().copy()
    return case, host


def _pages(case, host):
    out = []
    for (o, s) in zip(case.layout.offsets, case.layout.sizes):
        for p in range((int(s) + PAGE - 1) // PAGE):
            lo = int(o) + p * PAGE
            out.append(host[lo: lo + min(PAGE, int(s) - p * PAGE)])
    return out


def test_range_check_accepts_any_size_on_page_bases(oracle_lib):
    o = oracle_lib
    assert o.range_check([(0x10000, 0x1001)])[:2] == (0, 2)
    assert o.range_check([(0x10000, 1), (0x11000, 4096), (0x12000, 4097)])[:2] == (0, 1 + 1 + 2)
    assert o.range_check([(0x10010, 0x1000)])[0] == o.EALIGN
    assert o.range_check([(0x10000, 0x1001), (0x11000, 8)])[0] == o.EORDER   # the partial page is the range's


def test_hash_and_zero_over_the_page_bytes_only(oracle_lib, rcase):
    case, host = rcase
    ranges = case.ranges()
    views = W.host_views(case.layout, host)
    h, z, _ = oracle_lib.page_hash(ranges, views, seed=3)
    pages = _pages(case, host)
    assert len(h) == len(pages) == case.layout.n_pages
    assert [int(x) for x in h] == [xxhash.xxh64_intdigest(p.tobytes(), 3) for p in pages]
    zb = np.unpackbits(z.view(np.uint8), bitorder="little")[: len(pages)]
    assert zb.tolist() == [int(not p.any()) for p in pages]
    assert any(len(p) < PAGE for p in pages) and any(len(p) < 16 for p in pages)


def test_packed_slots_hold_the_bytes_then_zeros(oracle_lib, rcase):
    case, host = rcase
    ranges = case.ranges()
    views = W.host_views(case.layout, host)
    _, z, _ = oracle_lib.page_hash(ranges, views)
    packed, va, n_kept = oracle_lib.compact(ranges, views, z)
    pages = _pages(case, host)
    page_va = [b + p * PAGE for (b, s) in ranges for p in range((s + PAGE - 1) // PAGE)]
    kept = [i for i, p in enumerate(pages) if p.any()]
    assert n_kept == len(kept) and [int(x) for x in va] == [page_va[i] for i in kept]
    want = np.zeros((len(kept), PAGE), np.uint8)
    for k, i in enumerate(kept):
        want[k, : len(pages[i])] = pages[i]
    assert np.array_equal(packed.reshape(-1, PAGE), want)


def test_restore_writes_only_range_bytes(oracle_lib, rcase):
    case, host = rcase
    ranges = case.ranges()
    views = W.host_views(case.layout, host)
    _, z, _ = oracle_lib.page_hash(ranges, views)
    packed, va, n_kept = oracle_lib.compact(ranges, views, z)
    clob = host.copy()
    cviews = W.host_views(case.layout, clob)
    for v in cviews:
        v[:] = 0x3C
    assert oracle_lib.restore(ranges, cviews, z, None, packed, va, n_kept) == 0
    assert np.array_equal(clob, host)       # ranges restored, sentinel bytes outside untouched
    inside = np.zeros(len(host), bool)
    for o, s in zip(case.layout.offsets, case.layout.sizes):
        inside[int(o): int(o) + int(s)] = True
    assert (host[~inside] == W.SENTINEL).all()


def test_closure_scan_reads_whole_words_inside(oracle_lib, rcase):
    case, host = rcase
    ranges = case.ranges()
    views = W.host_views(case.layout, host)
    res, oob = oracle_lib.closure_scan(ranges, views, oob_cap=64)
    assert res["n_words"] == sum(s // 8 for _, s in ranges)
    lo = ranges[0][0] - (1 << 32)
    hi = ranges[-1][0] + ranges[-1][1] + (1 << 32)
    n_ptr = n_in = 0
    for (b, s), v in zip(ranges, views):
        w = v[: s // 8 * 8].view(np.uint64)
        like = (w >= lo) & (w < hi)
        n_ptr += int(like.sum())
        for x in w[like]:
            n_in += any(rb <= int(x) < rb + rs for rb, rs in ranges)
    assert res["n_ptr_like"] == n_ptr and res["n_in_range"] == n_in
    assert n_in >= len(case.truth["ptr"])
    edge = oracle_lib.pointer_graph(ranges, views)
    adj = oracle_lib.edges_to_bool(edge, len(ranges))
    for a, off, v in case.truth["ptr"]:
        b = next(i for i, (rb, rs) in enumerate(ranges) if rb <= v < rb + rs)
        assert adj[a, b]


def test_region_diff_counts_range_bytes_only(oracle_lib, rcase):
    case, host = rcase
    ranges = case.ranges()
    views = W.host_views(case.layout, host)
    _, z, _ = oracle_lib.page_hash(ranges, views)
    packed, va, n_kept = oracle_lib.compact(ranges, views, z)
    live = host.copy()
    lviews = W.host_views(case.layout, live)
    a = next(i for i, (_, s) in enumerate(ranges) if s % PAGE > 100)
    lviews[a][-1] ^= 0xFF                                         # the last byte of a partial page
    o = int(case.layout.offsets[a]) + int(case.layout.sizes[a])
    live[o: o + 7] ^= 0xFF                                        # past the range's end: not part of it
    got = oracle_lib.region_diff(ranges, lviews, z, packed, va, n_kept)
    assert [r["n_diff_bytes"] for r in got] == [int(i == a) for i in range(len(ranges))]
    assert got[a]["first_diff_va"] == ranges[a][0] + ranges[a][1] - 1
