"""The seeded generators produce the shapes and tallies their workloads declare."""
import pytest
import numpy as np
import torch

from paper_2605_03208_amd import workloads as W


def test_fit_sizes_exact_total():
    rng = np.random.default_rng(0)
    for n, lo, hi, total, align in [(48, 4096, 8 << 20, 64 << 20, 4096), (10000, 256, 64 << 20, 8 << 30, 256),
                                    (7, 4096, 1 << 20, 7 * 4096, 4096)]:
        s = W.fit_sizes(W.loguniform(rng, n, lo, hi), lo, hi, total, align)
        assert s.sum() == total and (s % align == 0).all() and s.min() >= lo


def test_c1_tallies():
    case = W.c1_snapshot()
    lay, t = case.layout, case.truth
    assert lay.n == 48 and lay.n_pages == 16384 and lay.total == 64 << 20
    assert len(t["zero_pages"]) == 4915 and len(t["ptr_pos"]) == 83886 and len(t["oob_val"]) == 3
    assert (lay.sizes >= 4096).all() and (lay.sizes <= 8 << 20).all()
    host = case.arena.host_copy()
    views = W.host_views(lay, host)
    pages = np.concatenate([v.reshape(-1, 4096) for v in views])
    assert not pages[t["zero_pages"]].any()
    words = np.concatenate([v.view("<u8") for v in views])
    assert np.array_equal(words[t["ptr_pos"]], t["ptr_val"])
    rngs = case.ranges()
    # VA gaps: ranges sorted, disjoint, page aligned
    for (b0, s0), (b1, _) in zip(rngs, rngs[1:]):
        assert b0 % 4096 == 0 and b0 + s0 < b1


def test_c1_compare_tallies():
    pairs = W.c1_compare(scale=1 / 64, n_pairs=2)
    for p in pairs:
        n = p.gold.numel()
        assert len(p.pos) == round(0.001 * n) and len(p.nan_pos) == 2
        assert set(np.abs(p.k)) <= {1, 2, 3, 4}
        assert not set(p.pos) & set(p.nan_pos)
        assert torch.isnan(p.cand[torch.from_numpy(p.nan_pos)]).all()


def test_c2_layout_and_rewrite():
    _, lay = W.c2_layout()
    assert lay.n == 4096 and lay.n_pages == 524288
    case = W.c2_snapshot(scale=1 / 1024)
    before = case.arena.host_copy().copy()
    W.c2_rewrite(case)
    after = case.arena.host_copy()
    bp = np.concatenate([v.reshape(-1, 4096) for v in W.host_views(case.layout, before)])
    ap = np.concatenate([v.reshape(-1, 4096) for v in W.host_views(case.layout, after)])
    diff = np.nonzero((bp != ap).any(axis=1))[0]
    assert np.array_equal(diff, case.truth["rewritten"])
    assert len(case.truth["rewritten"]) == int(case.layout.n_pages * 0.05)


def test_c3_layout():
    ps = W.c3_pairs(scale=1 / 4096, n_pairs=64)
    assert len(ps) == 64 and ps.nbytes.sum() == (8 << 30) // 4096
    assert (ps.nbytes % 256 == 0).all() and (ps.offsets % 256 == 0).all()
    assert list(ps.dtypes[:4]) == [W.DT_F32, W.DT_F32, W.DT_BF16, W.DT_F16]
    assert ps.tols.min() >= 0 and ps.tols.max() <= 8


def test_c4_layout():
    _, lay = W.c4_layout()
    assert lay.n == 200 and lay.n_pages == 7864320 and lay.total == 30 << 30
    assert lay.sizes[0] == 4096 * 14336 * 2 and lay.sizes[192] == 512 << 10 and lay.sizes[193] == 1 << 30
    case = W.c4_snapshot(scale=1 / 2048, oob_entries=1)
    t = case.truth
    tab = case.arena.view(192).view(torch.int64).numpy().view(np.uint64)
    rngs = case.ranges()
    assert tab[0] == rngs[0][0] and tab[193 % len(tab)] in (rngs[1][0], rngs[-1][0] + rngs[-1][1])
    assert tab[t["oob_slots"][0]] == rngs[-1][0] + rngs[-1][1]


def test_c5_schedule():
    reqs = W.c5_requests(rate_hz=200, duration_s=2.0)
    assert 300 < len(reqs) < 500
    assert all(1 <= len(r.golden_ids) <= 64 and 0 <= r.ulp_tol <= 8 for r in reqs)
    assert all(a.arrival_s < b.arrival_s for a, b in zip(reqs, reqs[1:]))


@pytest.mark.parametrize("t,dt", [(torch.float32, W.DT_F32), (torch.float64, W.DT_F64), (torch.bfloat16, W.DT_BF16),
                                  (torch.float16, W.DT_F16)])
def test_perturbation_steps_equal_nextafter(t, dt):
    """perturb_many moves a float k ULP in one integer step; it must equal k
    nextafter steps towards +-inf, including at zero, subnormals, the largest
    finite value, infinities and NaNs."""
    fi = torch.finfo(t)
    iv = {2: torch.int16, 4: torch.int32, 8: torch.int64}[torch.tensor(0, dtype=t).element_size()]
    base = [0.0, -0.0, float("inf"), float("-inf"), float("nan"), fi.max, -fi.max, fi.tiny, -fi.tiny, fi.eps,
            -fi.eps, 1.0, -1.0]
    sub = torch.tensor([1, 2, 3], dtype=iv).view(t)
    vals = torch.cat([torch.tensor(base * 300, dtype=torch.float64).to(t), sub, -sub,
                      torch.randn(2000, generator=torch.Generator().manual_seed(3), dtype=torch.float64).to(t)])
    n = vals.numel()
    got = vals.clone()
    W.perturb_many(got, dt, [0], [n], [777], p_pert=1.0, kmax=16)  # every element moves
    j, sd = torch.arange(n), torch.full((n,), 777)
    h1 = W._hash32(sd * 0x9E37 + j * 0x85EB + 1)
    h2 = W._hash32(h1 + sd + 0x27D4EB2F)
    k = 1 + (h2 % 16)
    k = torch.where(((h2 >> 20) & 1) == 1, -k, k)
    want = vals.clone()
    target = torch.where(k > 0, torch.full_like(want, float("inf")), torch.full_like(want, float("-inf")))
    for i in range(16):
        want = torch.where(k.abs() > i, torch.nextafter(want, target), want)
    same = (got.view(iv) == want.view(iv)) | (torch.isnan(got) & torch.isnan(want))
    assert bool(same.all())


def test_batched_perturbation_equals_each_buffer_alone():
    a = torch.randn(300000, generator=torch.Generator().manual_seed(4), dtype=torch.float32)
    b = a.clone()
    spans = ((0, 100000, 11), (100000, 150000, 22), (250000, 50000, 33))
    W.perturb_many(a, W.DT_F32, [o for o, _, _ in spans], [n for _, n, _ in spans], [s for _, _, s in spans], 1e-3)
    for o, n, s in spans:
        W.perturb_device(b[o:o + n], W.DT_F32, s, 1e-3)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32)) and not torch.equal(a, a.clone().fill_(0))


def test_perturbation_keeps_fp8_nans_and_saturates_int64():
    for t in (torch.float8_e4m3fn, torch.float8_e4m3fnuz, torch.float8_e5m2, torch.float8_e5m2fnuz):
        dt = {v: k for k, v in W.TORCH_DTYPE.items()}[t]
        codes = torch.arange(256, dtype=torch.int64).to(torch.uint8)
        got = codes.clone().view(t)
        W.perturb_many(got, dt, [0], [256], [9], p_pert=1.0, kmax=16)
        nan = torch.isnan(codes.view(t).to(torch.float32))
        assert bool(nan.any()) and torch.equal(got.view(torch.uint8)[nan], codes[nan])
        assert not torch.equal(got.view(torch.uint8)[~nan], codes[~nan])
    ii = torch.iinfo(torch.int64)
    v = torch.tensor([ii.max, ii.min] * 200, dtype=torch.int64)
    got = v.clone()
    W.perturb_many(got, W.DT_I64, [0], [400], [5], p_pert=1.0, kmax=16)
    assert bool(((got == ii.max) | (got == ii.min) | ((got - v).abs() <= 16)).all())
    assert bool(((v == ii.max) & (got < 0)).logical_not().all()) and bool(((v == ii.min) & (got > 0)).logical_not().all())
