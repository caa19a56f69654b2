"""Systems layers on the GPU: resident pair sets, graph replay, autotuner
candidates, and the serving loop (alone vs in the mix, and vs the oracle)."""
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
    assert torch.cuda.is_available()
    return K


def test_pairset_equals_compare(kc):
    say("pair set vs one-shot compare, c3 scale 1/512")
    ctx = kc.Context(0)
    ps = W.c3_pairs("cuda", scale=1 / 512, n_pairs=300)
    plist = [(ps.cand(i), ps.gold(i), int(ps.dtypes[i]), int(ps.tols[i])) for i in range(len(ps))]
    a = kc.compare(ctx, plist)
    pset = kc.PairSet(ctx, plist)
    b = kc.compare_pairset(ctx, pset)
    b2 = kc.compare_pairset(ctx, pset)
    torch.cuda.synchronize()
    assert torch.equal(a[: 300 * kc.RESULT_BYTES], b[: 300 * kc.RESULT_BYTES]) and torch.equal(b, b2)
    pset.close()
    ctx.close()


def test_graph_replay_matches_eager(kc):
    say("graph: snapshot + restore + compare recorded once, replayed with eager work between")
    ctx = kc.Context(0)
    case = W.c1_snapshot("cuda", scale=1 / 4)
    rs = kc.RangeSet(ctx, case.ranges())
    N = rs.n_pages
    dev = torch.device("cuda", 0)
    out = dict(hash=torch.empty(N, dtype=torch.int64, device=dev),
               zero_bm=torch.empty(rs.n_words, dtype=torch.int64, device=dev), changed_bm=None,
               packed=torch.empty(N * PAGE, dtype=torch.uint8, device=dev),
               page_va=torch.empty(N, dtype=torch.int64, device=dev),
               n_kept=torch.empty(1, dtype=torch.int64, device=dev))
    scan = kc.ScanOut(dev, oob_cap=16)
    pairs = W.c1_compare("cuda", scale=1 / 16, n_pairs=4)
    pset = kc.PairSet(ctx, [(p.cand, p.gold, W.DT_F32, 0) for p in pairs])
    res = torch.empty(4 * kc.RESULT_BYTES, dtype=torch.uint8, device=dev)

    def step():
        kc.snapshot(ctx, rs, scan=scan, out=out)
        kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"])
        kc.compare_pairset(ctx, pset, res=res)

    step()
    torch.cuda.synchronize()
    nk = int(out["n_kept"].item())
    nw = int(scan.result()[0]["n_written"])

    def outputs():   # everything the step defines (slots past n_kept are not written)
        return (out["hash"], out["zero_bm"], out["packed"][: nk * PAGE], out["page_va"][:nk], out["n_kept"],
                scan.res, scan.oob[: nw * 16], res)

    ref = tuple(t.clone() for t in outputs())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        for t in (out["hash"], out["zero_bm"], out["page_va"], out["n_kept"], scan.res, res):
            t.fill_(-1 if t.dtype == torch.int64 else 0xEE)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outputs(), ref):
            assert torch.equal(a, b), rep
    pset.close()
    rs.close()
    ctx.close()


def test_graph_replay_region_diff_and_pointer_graph(kc):
    say("graph: region diff + pointer graph recorded once, replayed over clobbered outputs and changed memory")
    ctx = kc.Context(0)
    case = W.graph_case("cuda", n_ranges=300, seed=17, max_pages=8)
    rs = kc.RangeSet(ctx, case.ranges())
    n = len(case.ranges())
    dev = torch.device("cuda", 0)
    gold = kc.snapshot(ctx, rs)
    torch.cuda.synchronize()

    def buffers():
        return dict(res=torch.empty(n * 4, dtype=torch.int64, device=dev),
                    hash=torch.empty(rs.n_pages, dtype=torch.int64, device=dev),
                    zero_bm=torch.empty(rs.n_words, dtype=torch.int64, device=dev),
                    changed_bm=torch.empty(rs.n_words, dtype=torch.int64, device=dev),
                    edge=torch.empty(n * ((n + 63) // 64), dtype=torch.int64, device=dev))

    def step(b):
        kc.region_diff(ctx, rs, gold, out=b)
        kc.pointer_graph(ctx, rs, out=b["edge"])

    live = buffers()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(live)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(live)
    rng = np.random.default_rng(3)
    for rep in range(4):
        if rep >= 2:   # change the live memory between replays
            idx = torch.from_numpy(rng.integers(0, case.arena.buf.numel(), size=50)).cuda()
            case.arena.buf[idx] ^= 0x5A
        eager = buffers()
        step(eager)
        torch.cuda.synchronize()
        for t in live.values():
            t.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in live:
            assert torch.equal(live[k], eager[k]), (rep, k)
    rs.close()
    ctx.close()


def test_autotuner_candidates_are_bit_identical(kc, tmp_path, monkeypatch):
    say("autotuner: every candidate of snapshot / compare gives the same outputs")
    from paper_2605_03208_amd import autotune
    monkeypatch.setenv("KC_TUNE_CACHE", str(tmp_path / "tune.json"))
    ctx = kc.Context(0)
    case = W.c1_snapshot("cuda", scale=1 / 4)
    rs = kc.RangeSet(ctx, case.ranges())
    scan = kc.ScanOut("cuda", oob_cap=16)
    out = kc.snapshot(ctx, rs, scan=scan)
    run = lambda: kc.snapshot(ctx, rs, scan=scan, out=out)
    dig = lambda: autotune.digest_tensors(out["hash"][: rs.n_pages], out["zero_bm"][: rs.n_words], out["n_kept"],
                                          out["packed"][: int(out["n_kept"].item()) * PAGE], scan.res, scan.oob)
    r = autotune.tune(ctx, kc.OP_SNAPSHOT, run, dig, signature="test-c1")
    assert not r["cached"] and len(r["table"]) == len(autotune.CANDIDATES[kc.OP_SNAPSHOT])
    r2 = autotune.tune(ctx, kc.OP_SNAPSHOT, run, dig, signature="test-c1")
    assert r2["cached"] and r2["best"] == r["best"]
    ps = W.c3_pairs("cuda", scale=1 / 1024, n_pairs=200)
    plist = [(ps.cand(i), ps.gold(i), int(ps.dtypes[i]), int(ps.tols[i])) for i in range(len(ps))]
    res = torch.empty(200 * kc.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    state = {}

    def prep(c):
        state["ps"] = kc.PairSet(ctx, plist)

    r = autotune.tune(ctx, kc.OP_COMPARE, lambda: kc.compare_pairset(ctx, state["ps"], res=res),
                      lambda: autotune.digest_tensors(res), signature="test-c3", prepare=prep)
    assert len(r["table"]) == len(autotune.CANDIDATES[kc.OP_COMPARE])
    rs.close()
    ctx.close()


def test_serving_alone_equals_mix_and_oracle(kc):
    say("serving: 40 requests in the mix vs each alone, and vs the oracle")
    from paper_2605_03208_amd import serve
    golds, dtypes = W.c5_pool("cuda", scale=1 / 64, n_buffers=24)
    raw = W.c5_requests(rate_hz=2000.0, duration_s=0.02, n_buffers=24, max_k=6)
    # the first twelve arrive together, so that the first loop pass launches a batch on every stream before
    # any can complete; the rest keep their Poisson arrival times and join while others are in flight
    reqs = [serve.Request(r.rid, 0.0 if i < 12 else r.arrival_s, r.golden_ids, r.ulp_tol, r.seed)
            for i, r in enumerate(raw[:40])]
    ex = serve.DeviceExecutor(golds, dtypes, n_streams=3)
    budget = int(np.sort([ex.request_bytes(r) for r in reqs])[-1] * 8)
    srv = serve.Server(ex, budget, max_batch=2)
    mix = {d.rid: d for d in srv.run(reqs)}
    assert len(mix) == len(reqs) and srv.budget.peak <= budget
    # the mix really mixed: some batch held several requests, and some batch
    # was launched while an earlier one was still in flight
    batches = {}
    for d in mix.values():
        batches.setdefault(d.launch_s, []).append(d)
    assert max(len(v) for v in batches.values()) >= 2
    spans = sorted((k, max(x.done_s for x in v)) for k, v in batches.items())
    assert any(spans[i + 1][0] < max(e for _, e in spans[: i + 1]) for i in range(len(spans) - 1))
    for r in reqs:
        alone = serve.Server(ex, budget).run([serve.Request(r.rid, 0.0, r.golden_ids, r.ulp_tol, r.seed)])
        assert alone[0].results == mix[r.rid].results, r.rid
    for r in reqs[:6]:
        for gid, got in zip(r.golden_ids, mix[r.rid].results):
            gold = golds[int(gid)]
            cand = gold.clone()
            W.perturb_device(cand, int(dtypes[int(gid)]), ex.candidate_seed(r, int(gid)))
            want = oracle.compare(cand.cpu().view(torch.uint8).numpy(), gold.cpu().view(torch.uint8).numpy(),
                                  int(dtypes[int(gid)]), r.ulp_tol, *serve.DEFAULT_CLOSE)
            assert got == want


def test_serving_batch_past_2g_elements_equals_alone(kc):
    """A batch whose fp8 candidate arena holds more than 2^31 elements (the
    overload regime) gives every request the results it gets alone."""
    say("serving: one batch with an fp8 arena past 2^31 elements vs each request alone")
    from paper_2605_03208_amd import serve
    golds, dtypes = W.c5_pool("cuda")
    fp8 = np.nonzero(np.asarray(dtypes) == W.DT_FP8)[0]
    assert sum(golds[int(g)].numel() for g in fp8) * 2 > 2**31
    reqs = [serve.Request(i, 0.0, fp8[i::2] if i < 2 else fp8, tol, 100 + i) for i, tol in enumerate((0, 3, 8))]
    ex = serve.DeviceExecutor(golds, dtypes, n_streams=1)
    srv = serve.Server(ex, 64 << 30, max_batch=3)
    mix = {d.rid: d for d in srv.run(reqs)}
    assert len({d.launch_s for d in mix.values()}) == 1           # one batch
    for r in reqs:
        alone = serve.Server(ex, 64 << 30).run([serve.Request(r.rid, 0.0, r.golden_ids, r.ulp_tol, r.seed)])
        assert alone[0].results == mix[r.rid].results, r.rid
        assert sum(x["n_mismatch_elems"] for x in mix[r.rid].results) > 0


def _perturb_inputs(dt, n, seed):
    """Every code of an 8-bit type, or a type's specials (zeros, infinities,
    NaNs, extremes, subnormals, integer bounds) repeated, then random values."""
    t = W.TORCH_DTYPE[dt]
    width = W.ELEM_SIZE[dt]
    iv = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}[width]
    g = torch.Generator().manual_seed(seed)
    if width == 1:
        bits = torch.arange(256, dtype=torch.int64).repeat(n // 256 + 1)[:n].to(torch.uint8)
        return bits.view(t)
    if t.is_floating_point:
        fi = torch.finfo(t)
        sub = torch.tensor([1, 2, 3], dtype=iv).view(t)
        base = torch.cat([torch.tensor([0.0, -0.0, float("inf"), float("-inf"), float("nan"), fi.max, -fi.max,
                                        fi.tiny, -fi.tiny, 1.0, -1.0], dtype=torch.float64).to(t), sub, -sub])
        rnd = torch.randn(n, generator=g, dtype=torch.float64).to(t)
    else:
        ii = torch.iinfo(t)
        base = torch.tensor([ii.min, ii.min + 1, ii.max, ii.max - 1, -1, 0, 1], dtype=torch.int64).to(t)
        rnd = torch.randint(ii.min, ii.max, (n,), generator=g, dtype=torch.int64).to(t)
    head = base.repeat(40)
    return torch.cat([head, rnd])[:n]


@pytest.mark.parametrize("dt", [W.DT_F32, W.DT_BF16, W.DT_F16, W.DT_F64, W.DT_FP8, W.DT_FP8_E4M3FNUZ,
                                W.DT_FP8_E5M2, W.DT_FP8_E5M2FNUZ, W.DT_I8, W.DT_I16, W.DT_I32, W.DT_I64])
def test_kc_perturb_equals_generator(kc, dt):
    """The server's candidate kernel moves exactly the elements, by exactly
    the steps, that the seeded generator moves on the CPU: specials, every
    code of the 8-bit types, ragged buffers, and more buffers than one launch
    carries."""
    say(f"kc_perturb vs the generator, dtype {dt}")
    ctx = kc.Context(0)
    n = 70000
    host = _perturb_inputs(dt, n, 7 + dt)
    rng = np.random.default_rng(dt)
    cuts = np.sort(rng.choice(np.arange(1, n), size=130, replace=False))
    offs = np.concatenate([[0], cuts])
    lens = np.diff(np.concatenate([offs, [n]]))
    lens[5] = 0                                     # an empty buffer
    seeds = rng.integers(0, 2**31, size=len(offs))
    for p_pert, kmax in ((1.0, 16), (1 / 3, 5), (1e-2, 16)):
        want = host.clone()
        W.perturb_many(want, dt, offs, lens, seeds, p_pert, kmax)
        got = host.to("cuda")
        kc.perturb(ctx, got, offs, lens, seeds, max(1, int(round(1.0 / p_pert))), kmax)
        torch.cuda.synchronize()
        iv = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}[W.ELEM_SIZE[dt]]
        assert torch.equal(got.cpu().view(iv), want.view(iv)), p_pert
        assert not torch.equal(want.view(iv), host.view(iv))
    ctx.close()


@pytest.mark.parametrize("dt", [W.DT_F32, W.DT_BF16, W.DT_F64, W.DT_FP8_E4M3FNUZ, W.DT_I8, W.DT_I16, W.DT_I64])
def test_kc_materialize_equals_copy_then_generator(kc, dt):
    """One-pass candidates: each golden copied into its place in the arena and
    moved exactly as the seeded generator moves it on the CPU; ragged lengths
    (short last vectors, empty buffers), more buffers than one launch carries,
    and the arena outside the buffers left as it was."""
    say(f"kc_materialize vs copy + the generator, dtype {dt}")
    ctx = kc.Context(0)
    esz = W.ELEM_SIZE[dt]
    rng = np.random.default_rng(100 + dt)
    lens = rng.integers(0, 900, size=150)
    lens[:6] = [0, 1, 16 // esz - 1, 16 // esz, 16 // esz + 1, 3]
    host = _perturb_inputs(dt, int(lens.sum()), 11 + dt)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    golds = [host[a: a + n].to("cuda") for a, n in zip(starts.tolist(), lens.tolist())]
    align = 16 // esz
    room = -(-lens // align) * align + align      # a gap of at least one vector after every buffer
    offs = np.concatenate([[0], np.cumsum(room)[:-1]]).astype(np.int64)
    seeds = rng.integers(0, 2**31, size=len(lens))
    iv = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}[esz]
    for p_pert, kmax in ((1.0, 16), (1 / 3, 5), (1e-2, 16)):
        block = max(1, int(round(1.0 / p_pert)))
        arena = torch.full((int(room.sum()) * esz,), 0x5A, dtype=torch.uint8, device="cuda").view(host.dtype)
        want = arena.cpu().clone()
        for g, o, n in zip(golds, offs.tolist(), lens.tolist()):
            want[o: o + n] = g.cpu()
        W.perturb_many(want, dt, offs, lens, seeds, p_pert, kmax)
        kc.materialize(ctx, arena, [g.data_ptr() for g in golds], offs, lens, seeds, block, kmax)
        torch.cuda.synchronize()
        assert torch.equal(arena.cpu().view(iv), want.view(iv)), p_pert
    for g, a, n in zip(golds, starts.tolist(), lens.tolist()):   # goldens untouched
        assert torch.equal(g.cpu().view(iv), host[a: a + n].view(iv))
    ctx.close()


def test_kc_perturb_offsets_past_4g_elements(kc):
    """Element offsets and moved-element indices past 2^32: a 4.5 GiB int8
    arena whose second buffer starts below 2^32 and ends above it."""
    say("kc_perturb: 4.5 GiB int8 arena, a buffer across element 2^32")
    ctx = kc.Context(0)
    n = (9 << 29)
    offs, lens, seeds = [0, (1 << 32) - 12345], [1 << 30, n - ((1 << 32) - 12345)], [3, 4]
    got = torch.zeros(n, dtype=torch.int8, device="cuda")
    kc.perturb(ctx, got, offs, lens, seeds, 1000, 16)
    torch.cuda.synchronize()
    want = torch.zeros(n, dtype=torch.int8)
    W.perturb_many(want, W.DT_I8, offs, lens, seeds, p_pert=1e-3, kmax=16)
    assert torch.equal(got.cpu(), want)
    assert int((want[(1 << 32):] != 0).sum()) > 0
    del got
    ctx.close()


def test_kc_materialize_past_4g_elements(kc):
    """Vector and element indices past 2^32: a 4.5 GiB int8 golden copied and
    moved into an arena at an offset, its buffer crossing element 2^32 of the
    arena, next to a small buffer with a short last vector."""
    say("kc_materialize: 4.5 GiB int8 golden, its place crossing arena element 2^32")
    ctx = kc.Context(0)
    n = (9 << 29)
    g = torch.randint(-128, 128, (1 << 26,), dtype=torch.int8, generator=torch.Generator().manual_seed(9)).repeat(72)
    small = torch.arange(37, dtype=torch.int64).to(torch.int8)
    gold, gold_small = g.to("cuda"), small.to("cuda")
    offs, lens, seeds = [1 << 20, (1 << 20) + n + 16], [n, 37], [5, 6]
    arena = torch.zeros(offs[1] + 48, dtype=torch.int8, device="cuda")
    kc.materialize(ctx, arena, [gold.data_ptr(), gold_small.data_ptr()], offs, lens, seeds, 1000, 16)
    torch.cuda.synchronize()
    want = torch.zeros(offs[1] + 48, dtype=torch.int8)
    want[offs[0]: offs[0] + n] = g
    want[offs[1]: offs[1] + 37] = small
    W.perturb_many(want, W.DT_I8, offs, lens, seeds, p_pert=1e-3, kmax=16)
    assert torch.equal(arena.cpu(), want)
    assert not torch.equal(want[(1 << 32): offs[0] + n], g[(1 << 32) - offs[0]:])
    del arena, gold
    ctx.close()


def test_kc_perturb_errors(kc):
    say("kc_perturb argument errors")
    ctx = kc.Context(0)
    a = torch.zeros(100, dtype=torch.float32, device="cuda")
    for args, code in (((a, [0], [101], [1], 1, 16), kc.EINVAL), ((a, [90], [11], [1], 1, 16), kc.EINVAL),
                       ((a, [0], [10], [1], 0, 16), kc.EINVAL), ((a, [0], [10], [1], 1, 0), kc.EINVAL),
                       ((a.view(torch.uint8), [0], [10], [1], 1, 16), kc.EDTYPE)):
        with pytest.raises(kc.KCError) as ei:
            kc.perturb(ctx, *args)
        assert ei.value.code == code
    kc.perturb(ctx, a, [], [], [], 1, 16)                  # nothing to move
    kc.perturb(ctx, a, [0, 50], [7, 9], [1, 2], 10, 16)    # buffers shorter than a block
    torch.cuda.synchronize()
    assert bool((a == 0).all())                            # rejected and empty calls wrote nothing
    ctx.close()


def test_sets_may_outlive_their_context(kc):
    say("context destroyed before its range set and pair set; caller's HIP state stays clean")
    ctx = kc.Context(0)
    case = W.c1_snapshot("cuda", scale=1 / 64)
    rs = kc.RangeSet(ctx, case.ranges())
    a = torch.ones(4096, dtype=torch.float32, device="cuda")
    ps = kc.PairSet(ctx, [(a, a, W.DT_F32, 0)])
    ctx.close()
    with pytest.raises(kc.KCError):
        kc.compare_pairset(ctx, ps)      # a closed context is rejected, not dereferenced
    rs.close()
    ps.close()
    b = torch.zeros(1 << 20, device="cuda").add_(1.0)
    torch.cuda.synchronize()
    assert float(b.sum().item()) == float(1 << 20)
