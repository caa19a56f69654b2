"""Pins the oracle's snapshot, restore and closure-scan definitions.

Independent pins: python-xxhash per page (library), numpy boolean page
masks and fancy indexing (zero bitmap, compaction), numpy searchsorted
(closure scan), the generator's record of what it injected (zero pages,
rewritten pages, pointers), closed-form counts, and the restore invariant.
"""
import numpy as np
import pytest

from paper_2605_03208_amd import workloads as W
from tests.helpers import PAGE, bits_to_words, concat_pages, numpy_closure, page_vas, words_to_bits

xxhash = pytest.importorskip("xxhash")


def _case(scale=1 / 32):
    case = W.c1_snapshot(scale=scale)
    host = case.arena.host_copy()
    return case, host, W.host_views(case.layout, host)


def test_range_check_errors(oracle_lib):
    o = oracle_lib
    good = [(0x10000, 0x2000), (0x20000, 0x1000)]
    assert o.range_check(good)[:2] == (o.OK, 3)
    assert o.range_check([])[:2] == (o.OK, 0)
    assert o.range_check([(0x10001, 0x1000)])[0] == o.EALIGN
    assert o.range_check([(0x10000, 0x1001)])[0] == o.OK          # a partial last page
    assert o.range_check([(0x10000, 0)])[0] == o.EINVAL
    assert o.range_check([(0, 0x1000)])[0] == o.EINVAL
    assert o.range_check([(2**64 - 0x1000, 0x2000)])[0] == o.EINVAL
    assert o.range_check([(0x20000, 0x1000), (0x10000, 0x1000)])[0] == o.EORDER
    assert o.range_check([(0x10000, 0x2000), (0x11000, 0x1000)])[0] == o.EORDER
    st, n, fp = o.range_check([(0x10000, 0x2000), (0x12000, 0x3000), (0x40000, 0x1000)])
    assert (st, n) == (o.OK, 6) and list(fp) == [0, 2, 5, 6]


def test_page_hash_matches_library_and_numpy(oracle_lib):
    case, host, views = _case()
    h, z, c = oracle_lib.page_hash(case.ranges(), views, seed=7)
    pages = concat_pages(views)
    assert c is None
    assert [int(x) for x in h] == [xxhash.xxh64_intdigest(p.tobytes(), 7) for p in pages]
    zero = ~pages.any(axis=1)
    assert np.array_equal(z, bits_to_words(zero))
    assert np.array_equal(np.nonzero(zero)[0], case.truth["zero_pages"])


def test_full_c1_zero_count_closed_form(oracle_lib):
    case, host, views = _case(scale=1.0)
    h, z, _ = oracle_lib.page_hash(case.ranges(), views)
    zero = words_to_bits(z, case.layout.n_pages)
    assert case.layout.n_pages == 16384 and int(zero.sum()) == 4915
    _, va, n_kept = oracle_lib.compact(case.ranges(), views, z)
    assert n_kept == 16384 - 4915 == 11469
    assert np.all(np.diff(va.astype(np.int64)) > 0)


def test_changed_bitmap_is_exactly_the_rewritten_set(oracle_lib):
    case = W.c2_snapshot(scale=1 / 512)
    v1 = W.host_views(case.layout, case.arena.host_copy())
    h1, _, _ = oracle_lib.page_hash(case.ranges(), v1, seed=3)
    W.c2_rewrite(case)
    v2 = W.host_views(case.layout, case.arena.host_copy())
    h2, z2, c2 = oracle_lib.page_hash(case.ranges(), v2, seed=3, prior=h1)
    changed = words_to_bits(c2, case.layout.n_pages)
    assert np.array_equal(np.nonzero(changed)[0], case.truth["rewritten"])
    assert np.array_equal(changed, h1 != h2)


def test_changed_flags_follow_prior_table(oracle_lib):
    case, host, views = _case()
    h, _, _ = oracle_lib.page_hash(case.ranges(), views)
    prior = h.copy()
    rng = np.random.default_rng(5)
    flip = rng.choice(len(h), size=len(h) // 7, replace=False)
    prior[flip] ^= np.uint64(1) << np.uint64(17)
    _, _, c = oracle_lib.page_hash(case.ranges(), views, prior=prior)
    want = np.zeros(len(h), dtype=bool)
    want[flip] = True
    assert np.array_equal(c, bits_to_words(want))


def test_compact_full_and_delta(oracle_lib):
    case, host, views = _case()
    rngs = case.ranges()
    h, z, _ = oracle_lib.page_hash(rngs, views)
    pages = concat_pages(views)
    vas = page_vas(rngs)
    zero = words_to_bits(z, len(pages))
    packed, va, n_kept = oracle_lib.compact(rngs, views, z)
    assert n_kept == int((~zero).sum())
    assert np.array_equal(packed.reshape(-1, PAGE), pages[~zero])
    assert np.array_equal(va, vas[~zero])
    assert packed.reshape(-1, PAGE).any(axis=1).all()  # no packed page is all-zero
    rng = np.random.default_rng(9)
    changed = rng.random(len(pages)) < 0.2
    packed, va, n_kept = oracle_lib.compact(rngs, views, z, bits_to_words(changed))
    keep = changed & ~zero
    assert n_kept == int(keep.sum())
    assert np.array_equal(packed.reshape(-1, PAGE), pages[keep])
    assert np.array_equal(va, vas[keep])


def test_compact_capacity_truncates_but_counts(oracle_lib):
    case, host, views = _case()
    _, z, _ = oracle_lib.page_hash(case.ranges(), views)
    full_packed, full_va, n_kept = oracle_lib.compact(case.ranges(), views, z)
    cap = n_kept // 3
    packed, va, n2 = oracle_lib.compact(case.ranges(), views, z, cap_pages=cap)
    assert n2 == n_kept
    assert np.array_equal(packed, full_packed[: cap * PAGE]) and np.array_equal(va, full_va[:cap])


def test_restore_roundtrip_full_and_delta(oracle_lib):
    case, host, views = _case()
    rngs = case.ranges()
    original = host.copy()
    h1, z1, _ = oracle_lib.page_hash(rngs, views)
    packed, va, n_kept = oracle_lib.compact(rngs, views, z1)
    # delta on top: mutate some pages (including zero <-> non-zero moves)
    rng = np.random.default_rng(3)
    mutated = host.copy()
    mviews = W.host_views(case.layout, mutated)
    mp = concat_pages(mviews)  # copy
    sel = rng.choice(len(mp), size=len(mp) // 10, replace=False)
    for j, g in enumerate(sel):
        a, p = W.page_views(case, np.array([g]))
        page = mviews[int(a[0])][int(p[0]) * PAGE:(int(p[0]) + 1) * PAGE]
        page[:] = 0 if j % 3 == 0 else rng.integers(0, 256, PAGE, dtype=np.uint8)
    h2, z2, c2 = oracle_lib.page_hash(rngs, mviews, prior=h1)
    dpacked, dva, dn = oracle_lib.compact(rngs, mviews, z2, c2)
    # clobber and restore base, then delta
    work = np.full_like(host, 0xA5)
    wviews = W.host_views(case.layout, work)
    assert oracle_lib.restore(rngs, wviews, z1, None, packed, va, n_kept) == 0
    assert all(np.array_equal(a, b) for a, b in zip(wviews, W.host_views(case.layout, original)))
    assert oracle_lib.restore(rngs, wviews, z2, c2, dpacked, dva, dn) == 0
    assert all(np.array_equal(a, b) for a, b in zip(wviews, mviews))
    hh, _, _ = oracle_lib.page_hash(rngs, wviews)
    assert np.array_equal(hh, h2)


def test_restore_rejects_bad_page_va(oracle_lib):
    case, host, views = _case()
    rngs = case.ranges()
    _, z, _ = oracle_lib.page_hash(rngs, views)
    packed, va, n_kept = oracle_lib.compact(rngs, views, z)
    bad = va.copy()
    bad[0] = rngs[-1][0] + rngs[-1][1]          # one past the end
    bad[1] = va[1] + 8                           # not page aligned
    work = host.copy()
    wviews = W.host_views(case.layout, work)
    assert oracle_lib.restore(rngs, wviews, z, None, packed, bad, n_kept) == 2


def test_closure_scan_matches_numpy_and_truth(oracle_lib):
    case, host, views = _case(scale=1 / 8)
    rngs = case.ranges()
    lo, hi = oracle_lib.default_window(rngs)
    assert lo == rngs[0][0] - 2**32 and hi == rngs[-1][0] + rngs[-1][1] + 2**32
    res, oob = oracle_lib.closure_scan(rngs, views, oob_cap=1000)
    want, want_oob = numpy_closure(rngs, views, lo, hi)
    for k, v in want.items():
        assert res[k] == v, k
    assert oob == want_oob and res["truncated"] == 0
    assert res["n_words"] == case.layout.n_pages * 512
    assert res["n_in_range"] >= len(case.truth["ptr_pos"])
    got_vals = sorted(v for _, v in oob)
    assert all(int(v) in got_vals for v in case.truth["oob_val"])  # every injected OOB reported


def test_closure_scan_truncation_and_window(oracle_lib):
    case, host, views = _case()
    rngs = case.ranges()
    full, oob_full = oracle_lib.closure_scan(rngs, views, oob_cap=100)
    res, oob = oracle_lib.closure_scan(rngs, views, oob_cap=2)
    assert res["n_oob"] == full["n_oob"] >= 3 and res["truncated"] == 1 and res["n_written"] == 2
    assert oob == oob_full[:2]
    res0, oob0 = oracle_lib.closure_scan(rngs, views, oob_cap=0)
    assert res0["n_oob"] == full["n_oob"] and res0["n_written"] == 0 and oob0 == []
    # a window that excludes everything
    res, _ = oracle_lib.closure_scan(rngs, views, win_lo=1, win_hi=2)
    assert res["n_ptr_like"] == 0
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.closure_scan(rngs, views, win_lo=0, win_hi=10)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.closure_scan(rngs, views, win_lo=10, win_hi=10)


def test_closure_scan_brute_force_tiny(oracle_lib):
    """Hand-built words at the edges of three ranges, checked by a linear scan."""
    rngs = [(0x100000, 0x1000), (0x103000, 0x2000), (0x200000, 0x1000)]
    host = np.zeros(4 * PAGE, dtype=np.uint8)
    words = host.view("<u8")
    probes = [0x100000, 0x100FFF, 0x101000, 0x102FF8, 0x103000, 0x104FFF, 0x105000,
              0x1FFFFF, 0x200000, 0x200FFF, 0x201000, 0x50, 0xFFFFFFFF00000000, 0x103001,
              0x1000, 0xFFF, 0x300000, 0x2FFFFF]   # window edges: lo, lo - 1, hi, hi - 1
    for i, v in enumerate(probes):
        words[i * 37 % len(words)] = v
    views = [host[:PAGE], host[PAGE:3 * PAGE], host[3 * PAGE:]]
    lo, hi = 0x1000, 0x300000
    res, oob = oracle_lib.closure_scan(rngs, views, lo, hi, oob_cap=64)
    exp_oob = []
    n_ptr = n_in = 0
    for (b, s), v in zip(rngs, views):
        for i, w in enumerate(v.view("<u8")):
            w = int(w)
            if not (lo <= w < hi):
                continue
            n_ptr += 1
            if any(rb <= w < rb + rs for rb, rs in rngs):
                n_in += 1
            else:
                exp_oob.append((b + 8 * i, w))
    assert (res["n_ptr_like"], res["n_in_range"], res["n_oob"]) == (n_ptr, n_in, len(exp_oob))
    assert oob == exp_oob
    assert res["n_words"] == 4 * 512
    # the per-range scan over the same edge words: the pieces add up to the linear scan
    parts = [oracle_lib.closure_scan_range(rngs, a, views[a], lo, hi, oob_cap=64) for a in range(len(rngs))]
    assert sum(r["n_ptr_like"] for r, _ in parts) == n_ptr and sum(r["n_in_range"] for r, _ in parts) == n_in
    assert [e for _, o in parts for e in o] == exp_oob


def test_closure_scan_range_pieces_make_the_whole(oracle_lib):
    """The per-range scan: each range's words against the numpy searchsorted
    formulation over the whole table (the range alone as the word source), and
    over all ranges the counts sum to, and the lists concatenate into, the
    whole-set scan, with and without truncation and under explicit windows."""
    for scale, win in ((1 / 8, (0, 0)), (1 / 32, (0, 0)), (1 / 32, None)):
        case, host, views = _case(scale=scale)
        rngs = case.ranges()
        if win is None:  # a window that cuts through the ranges
            win = (rngs[3][0] + 4096, rngs[-5][0] + 12345)
        lo, hi = win if win != (0, 0) else oracle_lib.default_window(rngs)
        whole, whole_oob = oracle_lib.closure_scan(rngs, views, win[0], win[1], oob_cap=10**6)
        tot = dict(n_words=0, n_ptr_like=0, n_in_range=0, n_oob=0)
        cat = []
        for a in range(len(rngs)):
            res, oob = oracle_lib.closure_scan_range(rngs, a, views[a], win[0], win[1], oob_cap=10**6)
            want, want_oob = _numpy_closure_of_range(rngs, a, views[a], lo, hi)
            assert {k: res[k] for k in want} == want and oob == want_oob, a
            for k in tot:
                tot[k] += res[k]
            cat += oob
            short, short_oob = oracle_lib.closure_scan_range(rngs, a, views[a], win[0], win[1], oob_cap=1)
            assert short["n_oob"] == res["n_oob"] and short_oob == oob[:1]
            assert short["truncated"] == (1 if res["n_oob"] > 1 else 0)
        assert all(whole[k] == v for k, v in tot.items()) and cat == whole_oob
        assert whole["n_oob"] >= (3 if win == (0, 0) else 1)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.closure_scan_range(rngs, len(rngs), views[0])


def _numpy_closure_of_range(ranges, a, view, lo, hi):
    bases = np.array([b for b, _ in ranges], dtype=np.uint64)
    ends = np.array([b + s for b, s in ranges], dtype=np.uint64)
    w = np.ascontiguousarray(view[: ranges[a][1] // 8 * 8]).view("<u8")
    ptr = (w >= np.uint64(lo)) & (w < np.uint64(hi))
    idx = np.searchsorted(bases, w, side="right").astype(np.int64) - 1
    inr = np.zeros(len(w), dtype=bool)
    ok = idx >= 0
    inr[ok] = w[ok] < ends[idx[ok]]
    bad = np.nonzero(ptr & ~inr)[0]
    counts = dict(n_words=len(w), n_ptr_like=int(ptr.sum()), n_in_range=int((ptr & inr).sum()), n_oob=len(bad))
    return counts, [(ranges[a][0] + 8 * int(i), int(w[i])) for i in bad]


def test_empty_rangeset(oracle_lib):
    h, z, _ = oracle_lib.page_hash([], [])
    assert len(h) == 0 and len(z) == 0
    packed, va, n = oracle_lib.compact([], [], z)
    assert n == 0
    res, oob = oracle_lib.closure_scan([], [])
    assert res["n_words"] == 0 and oob == []


def test_zero_flag_single_nonzero_byte_anywhere(oracle_lib):
    """A page is zero only if every one of its 4096 bytes is zero: one set
    byte at the first, last or any interior offset clears the flag."""
    offsets = [0, 1, 7, 8, 63, 64, 2047, 2048, 4088, 4095]
    host = np.zeros((len(offsets) + 2) * PAGE, dtype=np.uint8)
    for i, off in enumerate(offsets):
        host[(i + 1) * PAGE + off] = 0x80 if i % 2 else 1
    rngs = [(0x200000, len(host))]
    h, z, _ = oracle_lib.page_hash(rngs, [host])
    pages = host.reshape(-1, PAGE)
    assert np.array_equal(z, bits_to_words(~pages.any(axis=1)))
    assert [int(x) for x in h] == [xxhash.xxh64_intdigest(p.tobytes(), 0) for p in pages]
