"""Pins the oracle's hash units above 4 KiB (64 KiB and 2 MiB pages for
whole-allocation capture of large tensors, paper Sec. 4.2.1).

Independent pins: python-xxhash over exactly each unit's bytes (library),
numpy boolean masks per unit (zero bits, changed bits, compaction), the
ceil-division unit count, the restore invariant, planted page-table
corruptions whose count is known in advance, and Python sets of the bytes a
test flips (region diff).  With a 4096-byte unit every function equals the
page form the other pins cover."""
import numpy as np
import pytest

from tests.helpers import bits_to_words, words_to_bits

xxhash = pytest.importorskip("xxhash")
PAGE = 4096
BASE = 0x7F8A00000000


def _case(unit, seed=0):
    """Ranges of uneven sizes (partial last units, ranges shorter than a unit)
    with all-zero units, units zero but for one byte, and random bytes."""
    rng = np.random.default_rng(seed + unit)
    sizes = [unit * 3, unit * 2 + 4096 * 3, unit + 1, 4096, 777, unit * 4 - 8, unit // 2 + 16, 5 * 4096]
    ranges, views, va = [], [], BASE
    for sz in sizes:
        v = rng.integers(0, 256, size=sz, dtype=np.uint8)
        n_units = -(-sz // unit)
        for p in range(n_units):
            lo, hi = p * unit, min(sz, (p + 1) * unit)
            r = rng.random()
            if r < 0.3:
                v[lo:hi] = 0                                   # an all-zero unit
            elif r < 0.45:
                v[lo:hi] = 0
                v[int(rng.integers(lo, hi))] = int(rng.integers(1, 256))  # zero but for one byte
        ranges.append((va, sz))
        views.append(v)
        va += -(-sz // PAGE) * PAGE + PAGE * int(rng.integers(1, 5))
    return ranges, views


def _units(ranges, views, unit):
    """(range, unit index, bytes) of every unit, in global order."""
    out = []
    for a, ((b, sz), v) in enumerate(zip(ranges, views)):
        for p in range(-(-sz // unit)):
            out.append((a, p, v[p * unit: min(sz, (p + 1) * unit)]))
    return out


@pytest.mark.parametrize("unit", [PAGE, 16 << 10, 64 << 10, 2 << 20])
def test_unit_hash_zero_changed_compact(oracle_lib, unit):
    o = oracle_lib
    ranges, views = _case(unit)
    units = _units(ranges, views, unit)
    st, n, fp = o.range_check(ranges, unit)
    assert st == o.OK and n == len(units) == sum(-(-sz // unit) for _, sz in ranges)
    h, z, _ = o.page_hash(ranges, views, seed=5, unit=unit)
    assert [int(x) for x in h] == [xxhash.xxh64_intdigest(u.tobytes(), seed=5) for _, _, u in units]
    zero = np.array([not u.any() for _, _, u in units])
    assert np.array_equal(z, bits_to_words(zero))
    assert 0 < zero.sum() < len(units)
    prior = h.copy()
    flip = np.random.default_rng(1).choice(len(units), size=max(1, len(units) // 3), replace=False)
    prior[flip] ^= np.uint64(1)
    _, _, c = o.page_hash(ranges, views, seed=5, prior=prior, unit=unit)
    want_c = np.zeros(len(units), dtype=bool)
    want_c[flip] = True
    assert np.array_equal(words_to_bits(c, len(units)), want_c)
    for changed in (None, c):
        keep = ~zero & (want_c if changed is not None else True)
        packed, va, nk = o.compact(ranges, views, z, changed, unit=unit)
        sel = [i for i in range(len(units)) if keep[i]]
        assert nk == len(sel)
        want_va = [ranges[units[i][0]][0] + units[i][1] * unit for i in sel]
        assert [int(x) for x in va] == want_va
        want = np.zeros(len(sel) * unit, dtype=np.uint8)
        for k, i in enumerate(sel):
            u = units[i][2]
            want[k * unit: k * unit + len(u)] = u                  # a partial unit padded with zeros
        assert np.array_equal(packed, want)
        cap = max(1, nk // 2)
        p2, va2, nk2 = o.compact(ranges, views, z, changed, cap_pages=cap, unit=unit)
        assert nk2 == nk and np.array_equal(p2, want[: cap * unit]) and list(va2) == want_va[:cap]


@pytest.mark.parametrize("unit", [16 << 10, 64 << 10, 2 << 20])
def test_unit_restore_roundtrip_and_bad_addresses(oracle_lib, unit):
    o = oracle_lib
    ranges, views = _case(unit, seed=3)
    h, z, _ = o.page_hash(ranges, views, unit=unit)
    packed, va, nk = o.compact(ranges, views, z, unit=unit)
    target = [np.full_like(v, 0xA5) for v in views]
    assert o.restore(ranges, target, z, None, packed, va, nk, unit=unit) == 0
    assert all(np.array_equal(t, v) for t, v in zip(target, views))
    # one VA 4 KiB into a unit, one past every range, one unaligned: each is skipped and counted
    bad = va.copy()
    inside = [i for i in range(nk) if int(va[i]) + PAGE < ranges[-1][0] + ranges[-1][1]]
    bad[inside[0]] = va[inside[0]] + np.uint64(PAGE)
    bad[1] = np.uint64(ranges[-1][0] + ranges[-1][1] + 10 * unit)
    bad[2] = va[2] + np.uint64(8)
    target = [np.full_like(v, 0xA5) for v in views]
    assert o.restore(ranges, target, z, None, packed, bad, nk, unit=unit) == 3
    # delta: change some units, restore the delta over the old image
    new_views = [v.copy() for v in views]
    new_views[0][5] ^= 0xFF
    new_views[1][:] = 0
    h2, z2, c2 = o.page_hash(ranges, new_views, prior=h, unit=unit)
    dp, dva, dnk = o.compact(ranges, new_views, z2, c2, unit=unit)
    img = [v.copy() for v in views]
    assert o.restore(ranges, img, z2, c2, dp, dva, dnk, unit=unit) == 0
    assert all(np.array_equal(a, b) for a, b in zip(img, new_views))


@pytest.mark.parametrize("unit", [64 << 10, 2 << 20])
def test_unit_region_diff(oracle_lib, unit):
    o = oracle_lib
    ranges, views = _case(unit, seed=7)
    _, z, _ = o.page_hash(ranges, views, unit=unit)
    packed, va, nk = o.compact(ranges, views, z, unit=unit)
    live = [v.copy() for v in views]
    rng = np.random.default_rng(9)
    flipped = {}
    for a in (0, 2, 5):
        pos = sorted(set(int(x) for x in rng.integers(0, len(live[a]), size=20)))
        for p in pos:
            live[a][p] ^= 0x3C
        flipped[a] = pos
    res = o.region_diff(ranges, live, z, packed, va, nk, unit=unit)
    for a, r in enumerate(res):
        pos = flipped.get(a, [])
        assert r["n_diff_bytes"] == len(pos) and r["n_bad_pages"] == 0
        assert r["n_diff_pages"] == len({p // unit for p in pos})
        assert r["first_diff_va"] == (ranges[a][0] + pos[0] if pos else 2**64 - 1)
    bad = va.copy()
    bad[0] = bad[0] + np.uint64(PAGE)                              # the first non-zero unit loses its copy
    res = o.region_diff(ranges, live, z, packed, bad, nk, unit=unit)
    assert sum(r["n_bad_pages"] for r in res) == 1


def test_unit_limits_and_page_form(oracle_lib):
    o = oracle_lib
    ranges, views = _case(PAGE)
    for bad_unit in (2048, 3 * PAGE, 4 << 20, 0):
        assert o.range_check(ranges, bad_unit)[0] == o.EINVAL
    assert o.range_check([(BASE + PAGE, 10)], 64 << 10)[:2] == (o.OK, 1)   # base only 4 KiB aligned
    assert o.range_check([(BASE + 8, 10)], 64 << 10)[0] == o.EALIGN
    h1, z1, _ = o.page_hash(ranges, views)
    h2, z2, _ = o.page_hash(ranges, views, unit=PAGE)
    assert np.array_equal(h1, h2) and np.array_equal(z1, z2)
