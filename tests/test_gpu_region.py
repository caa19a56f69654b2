"""Per-range byte difference against a snapshot (hash first, then only the
changed pages byte by byte) on the GPU vs the CPU oracle, through the C ABI.

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


def diff_vs_oracle(kc, ctx, case, rs, gold, seed=0, cap=None, gold_host=None):
    ranges = case.ranges()
    out = kc.region_diff(ctx, rs, gold, seed=seed, cap_pages=cap)
    torch.cuda.synchronize()
    got = kc.decode_region_diff(out["res"], len(ranges))
    host = case.arena.host_copy()
    views = W.host_views(case.layout, host)
    zb, packed, va, n_kept = gold_host
    k = len(va) if cap is None else cap
    want = oracle.region_diff(ranges, views, zb, packed[:k * PAGE], va[:k], n_kept, cap_pages=k)
    assert got == want
    # the live hash table and the changed bitmap are the oracle's page hash against the snapshot's table
    oh, oz, oc = oracle.page_hash(ranges, views, seed=seed, prior=u64(gold["hash"])[:rs.n_pages])
    assert np.array_equal(u64(out["hash"])[:rs.n_pages], oh)
    assert np.array_equal(u64(out["zero_bm"])[:rs.n_words], oz)
    assert np.array_equal(u64(out["changed_bm"])[:rs.n_words], oc)
    return got


def take_snapshot(kc, ctx, rs, seed=0):
    gold = kc.snapshot(ctx, rs, seed=seed)
    torch.cuda.synchronize()
    n_kept = int(u64(gold["n_kept"])[0])
    host = (u64(gold["zero_bm"])[:rs.n_words].copy(), gold["packed"][:n_kept * PAGE].cpu().numpy(),
            u64(gold["page_va"])[:n_kept].copy(), n_kept)
    return gold, host


@pytest.mark.parametrize("name,seed", [("c1", 0), ("c1", 12345), ("graph", 0)])
def test_region_diff_planted_changes(kc, ctx, name, seed):
    say(f"region diff: {name} scaled, seed {seed}: unchanged, then planted byte changes")
    case = W.c1_snapshot("cuda", scale=1 / 16, seed=5) if name == "c1" else \
        W.graph_case("cuda", n_ranges=600, seed=9, max_pages=6)
    rs = kc.RangeSet(ctx, case.ranges())
    gold, gh = take_snapshot(kc, ctx, rs, seed)
    got = diff_vs_oracle(kc, ctx, case, rs, gold, seed, gold_host=gh)
    assert all(r["n_diff_bytes"] == 0 and r["n_bad_pages"] == 0 for r in got)
    rng = np.random.default_rng(seed + 1)
    buf = case.arena.buf
    for a in rng.choice(len(case.ranges()), size=min(50, len(case.ranges())), replace=False):
        o = int(case.layout.offsets[a])
        s = int(case.layout.sizes[a])
        offs = torch.from_numpy(np.unique(rng.integers(0, s, size=int(rng.integers(1, 30))))).cuda() + o
        buf[offs] ^= torch.from_numpy(rng.integers(1, 256, size=len(offs), dtype=np.uint8)).cuda()
    # wipe one page and fill one zero page
    zb = np.unpackbits(gh[0].view(np.uint8), bitorder="little")[:rs.n_pages]
    cum = case.layout.cum() // PAGE
    for g, val in ((int(np.flatnonzero(zb == 0)[7]), 0), (int(np.flatnonzero(zb)[2]) if zb.any() else None, 9)):
        if g is None:
            continue
        a = int(np.searchsorted(cum, g, side="right") - 1)
        o = int(case.layout.offsets[a]) + (g - int(cum[a])) * PAGE
        buf[o:o + PAGE] = val
    torch.cuda.synchronize()
    got = diff_vs_oracle(kc, ctx, case, rs, gold, seed, gold_host=gh)
    assert sum(r["n_diff_pages"] for r in got) > 0
    rs.close()


def test_region_diff_bad_table_and_capacity(kc, ctx):
    say("region diff: corrupted page-VA entries, reduced capacity")
    case = W.c1_snapshot("cuda", scale=1 / 32, seed=6)
    rs = kc.RangeSet(ctx, case.ranges())
    gold, gh = take_snapshot(kc, ctx, rs)
    case.arena.buf[::7777] ^= 1
    gold["page_va"][5] += PAGE
    gold["page_va"][gh[3] - 1] = 0
    gh = (gh[0], gh[1], u64(gold["page_va"])[:gh[3]].copy(), gh[3])
    diff_vs_oracle(kc, ctx, case, rs, gold, gold_host=gh)
    for cap in (0, 1, gh[3] // 2):
        diff_vs_oracle(kc, ctx, case, rs, gold, cap=cap, gold_host=gh)
    rs.close()
