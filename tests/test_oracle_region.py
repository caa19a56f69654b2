"""Pins the oracle's per-range byte difference against a full snapshot.

Independent pins: the generator's own record of which bytes it changed (as
Python sets: counts, pages and the lowest changed address per range), numpy
counts of non-zero bytes for pages that are wiped, and planted corruptions of
the snapshot's page-VA table or capacity whose effect is known in advance."""
import numpy as np
import pytest

from paper_2605_03208_amd import workloads as W

PAGE = 4096


@pytest.fixture(scope="module")
def base(oracle_lib):
    case = W.c1_snapshot(scale=1 / 64, seed=7)
    ranges = case.ranges()
    host = case.arena.host_copy().copy()
    views = W.host_views(case.layout, host)
    _, zb, _ = oracle_lib.page_hash(ranges, views)
    packed, va, n_kept = oracle_lib.compact(ranges, views, zb)
    return case, ranges, host, zb, packed, va, n_kept


def _fresh(base):
    case, ranges, host, zb, packed, va, n_kept = base
    h = host.copy()
    return case, ranges, h, W.host_views(case.layout, h), zb, packed, va, n_kept


def test_identical_memory_has_no_difference(oracle_lib, base):
    case, ranges, h, views, zb, packed, va, n_kept = _fresh(base)
    for r in oracle_lib.region_diff(ranges, views, zb, packed, va, n_kept):
        assert r == dict(n_diff_bytes=0, n_diff_pages=0, first_diff_va=2**64 - 1, n_bad_pages=0)


def test_planted_byte_changes(oracle_lib, base):
    case, ranges, h, views, zb, packed, va, n_kept = _fresh(base)
    rng = np.random.default_rng(11)
    changed = {}                                   # range -> set of byte offsets
    for a in rng.choice(len(ranges), size=len(ranges) // 2, replace=False):
        offs = set(int(x) for x in rng.integers(0, ranges[a][1], size=int(rng.integers(1, 40))))
        for o in offs:
            views[a][o] ^= np.uint8(rng.integers(1, 256))   # always a different byte
        changed[int(a)] = offs
    got = oracle_lib.region_diff(ranges, views, zb, packed, va, n_kept)
    for a, r in enumerate(got):
        offs = changed.get(a, set())
        assert r["n_diff_bytes"] == len(offs)
        assert r["n_diff_pages"] == len({o // PAGE for o in offs})
        assert r["first_diff_va"] == (ranges[a][0] + min(offs) if offs else 2**64 - 1)
        assert r["n_bad_pages"] == 0


def test_zero_pages_filled_and_pages_wiped(oracle_lib, base):
    case, ranges, h, views, zb, packed, va, n_kept = _fresh(base)
    # a zero page of the snapshot gets three bytes; a non-zero page is wiped
    bits = np.unpackbits(zb.view(np.uint8), bitorder="little")
    cum = np.concatenate([[0], np.cumsum([s // PAGE for _, s in ranges])])
    g_zero = int(np.flatnonzero(bits[:cum[-1]])[3])
    g_full = int(np.flatnonzero(bits[:cum[-1]] == 0)[5])
    a0 = int(np.searchsorted(cum, g_zero, side="right") - 1)
    a1 = int(np.searchsorted(cum, g_full, side="right") - 1)
    p0, p1 = g_zero - cum[a0], g_full - cum[a1]
    views[a0][p0 * PAGE + 5] = 1
    views[a0][p0 * PAGE + 100] = 2
    views[a0][p0 * PAGE + 4095] = 3
    nz = int(np.count_nonzero(views[a1][p1 * PAGE:(p1 + 1) * PAGE]))
    first = int(np.flatnonzero(views[a1][p1 * PAGE:(p1 + 1) * PAGE])[0])
    views[a1][p1 * PAGE:(p1 + 1) * PAGE] = 0
    got = oracle_lib.region_diff(ranges, views, zb, packed, va, n_kept)
    want = {a0: [3, 1, ranges[a0][0] + p0 * PAGE + 5]}
    if a1 == a0:
        want[a0] = [3 + nz, 2, ranges[a0][0] + min(p0 * PAGE + 5, p1 * PAGE + first)]
    else:
        want[a1] = [nz, 1, ranges[a1][0] + p1 * PAGE + first]
    for a, r in enumerate(got):
        w = want.get(a, [0, 0, 2**64 - 1])
        assert [r["n_diff_bytes"], r["n_diff_pages"], r["first_diff_va"]] == w, a


def test_bad_page_table_entries_and_capacity(oracle_lib, base):
    case, ranges, h, views, zb, packed, va, n_kept = _fresh(base)
    va2 = va.copy()
    va2[10] += PAGE                  # entry 10 names the wrong page
    got = oracle_lib.region_diff(ranges, views, zb, packed, va2, n_kept)
    cum = np.concatenate([[0], np.cumsum([s // PAGE for _, s in ranges])])
    bad_range = next(a for a, (b, s) in enumerate(ranges) if b <= int(va[10]) < b + s)
    assert [r["n_bad_pages"] for r in got] == [int(a == bad_range) for a in range(len(ranges))]
    assert all(r["n_diff_bytes"] == 0 for r in got)
    # a capacity of k pages: every non-zero page at slot >= k is bad
    k = n_kept // 3
    got = oracle_lib.region_diff(ranges, views, zb, packed[:k * PAGE], va[:k], n_kept, cap_pages=k)
    assert sum(r["n_bad_pages"] for r in got) == n_kept - k
    per_range = np.zeros(len(ranges), np.int64)
    for s in range(k, n_kept):
        per_range[next(a for a, (b, sz) in enumerate(ranges) if b <= int(va[s]) < b + sz)] += 1
    assert [r["n_bad_pages"] for r in got] == per_range.tolist()
