"""Full-size configurations checked against the oracle with no sampling.

The 30 GiB MoE-shaped pool (192 bf16 expert matrices, a pointer table, an
80 %-zero workspace and six activation buffers; 200 ranges, 7,864,320 pages)
and the 10,000-pair uneven compare (8 GiB a side) run in the launch shapes the
benchmark times.  The oracle cannot hold the pool and its packed copy in one
call, so it runs one range at a time, on a thread pool (its C calls release the
interpreter lock), and the per-range results are assembled in range order:
every hash, every zero bit, every page VA and packed page, the kept count, the
exact closure-scan counts and ordered out-of-range list, the restored bytes and
all 200 compare reports.  Nothing here samples or uses a bound.
"""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_03208_amd import workloads as W
from tests.helpers import words_to_bits
from tests.test_gpu_parity import BITS_VIEW, SPECIALS, _tuned_context

pytestmark = pytest.mark.gpu

PAGE = 4096
WORKERS = min(16, os.cpu_count() or 1)


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


def _bounded(pool, jobs, limit):
    """Submits (fn, args) jobs keeping at most ``limit`` in flight; yields
    results in submission order.  Jobs are produced lazily, so the host copies
    a job carries are made only when a slot is free."""
    pending = []
    for fn, args in jobs:
        pending.append(pool.submit(fn, *args))
        if len(pending) >= limit:
            yield pending.pop(0).result()
    for f in pending:
        yield f.result()


def _scan_totals(parts, cap):
    """Sum of per-range closure-scan results and the first ``cap`` entries of
    their concatenated lists (the form the whole-table scan takes)."""
    tot = dict(n_words=0, n_ptr_like=0, n_in_range=0, n_oob=0)
    lst = []
    for res, oob in parts:
        for k in tot:
            tot[k] += res[k]
        lst.extend(oob)
    tot["n_written"] = min(tot["n_oob"], cap)
    tot["truncated"] = 1 if tot["n_oob"] > cap else 0
    return tot, lst[:cap]


@pytest.mark.timeout(1200)
def test_c4_full_exact(kc):
    ctx, shapes = _tuned_context(kc, "c4-moe-pool-scale1.0", (kc.OP_SNAPSHOT, kc.OP_RESTORE, kc.OP_COMPARE))
    say(f"c4 full exact: launch shapes {shapes or 'built-in'}; generate the 30 GiB MoE pool on device")
    case = W.c4_snapshot("cuda")
    ranges = case.ranges()
    n = len(ranges)
    rs = kc.RangeSet(ctx, ranges)
    N = rs.n_pages
    st, o_pages, fp = oracle.range_check(ranges)
    assert st == 0 and o_pages == N == 7864320
    fp = [int(x) for x in fp]
    cap = 16

    say("c4 full exact: fused snapshot + closure scan on the device")
    scan = kc.ScanOut("cuda", oob_cap=cap)
    out = kc.snapshot(ctx, rs, seed=0, scan=scan)
    torch.cuda.synchronize()
    g_hash = u64(out["hash"])[:N].copy()
    g_zero = words_to_bits(u64(out["zero_bm"])[: rs.n_words], N)
    g_kept = int(u64(out["n_kept"])[0])
    g_res, g_oob = scan.result()

    # phase 1: per range, hash / zero bits and the closure scan of its words
    say(f"c4 full exact: oracle page hash + closure scan, one range at a time on {WORKERS} threads")
    hosts = [None] * n

    def phase1(a, host):
        oh, oz, _ = oracle.page_hash([ranges[a]], [host])
        np_a = fp[a + 1] - fp[a]
        zbits = words_to_bits(oz, np_a)
        assert np.array_equal(g_hash[fp[a]:fp[a + 1]], oh), f"hash table differs in range {a}"
        assert np.array_equal(g_zero[fp[a]:fp[a + 1]], zbits), f"zero bitmap differs in range {a}"
        sres, soob = oracle.closure_scan_range(ranges, a, host, oob_cap=cap)
        return a, int(np_a - zbits.sum()), oz, (sres, soob)

    def jobs1():
        for a in range(n):
            hosts[a] = case.arena.view(a).cpu().numpy()
            yield phase1, (a, hosts[a])

    kept, zwords, scans = [0] * n, [None] * n, [None] * n
    with cf.ThreadPoolExecutor(WORKERS) as pool:
        for a, k, oz, sc in _bounded(pool, jobs1(), 2 * WORKERS):
            kept[a], zwords[a], scans[a] = k, oz, sc
            if a % 50 == 49:
                say(f"c4 full exact: phase 1 through range {a}")
    assert g_kept == sum(kept) == N - 209715
    o_res, o_oob = _scan_totals(scans, cap)
    assert g_res == o_res and g_oob == o_oob
    assert o_res["n_words"] == N * 512 and o_res["n_oob"] == 0

    # phase 2: per range, the oracle's packed pages and page VAs against the
    # device's slots, placed by the oracle's own kept counts
    say("c4 full exact: oracle compaction vs every packed page and page VA")
    slot0 = np.concatenate([[0], np.cumsum(kept)]).astype(np.int64)
    g_va = u64(out["page_va"])[:g_kept].copy()

    def phase2(a, host, dev_packed):
        op, ova, onk = oracle.compact([ranges[a]], [host], zwords[a])
        assert onk == kept[a]
        assert np.array_equal(g_va[slot0[a]:slot0[a + 1]], ova), f"page VAs differ in range {a}"
        assert np.array_equal(dev_packed, op), f"packed pages differ in range {a}"
        return a

    def jobs2():
        for a in range(n):
            s, e = int(slot0[a]) * PAGE, int(slot0[a + 1]) * PAGE
            yield phase2, (a, hosts[a], out["packed"][s:e].cpu().numpy())

    with cf.ThreadPoolExecutor(WORKERS) as pool:
        for a in _bounded(pool, jobs2(), WORKERS):
            if a % 50 == 49:
                say(f"c4 full exact: phase 2 through range {a}")

    say("c4 full exact: one injected out-of-range pointer in the table")
    tab = case.arena.view(192).view(torch.int64)
    tslot = 12345
    saved = int(tab[tslot].item())
    max_end = ranges[-1][0] + ranges[-1][1]
    tab[tslot] = max_end
    scan2 = kc.ScanOut("cuda", oob_cap=cap)
    kc.closure_scan(ctx, rs, scan2)
    torch.cuda.synchronize()
    parts = list(scans)
    parts[192] = oracle.closure_scan_range(ranges, 192, case.arena.view(192).cpu().numpy(), oob_cap=cap)
    o2_res, o2_oob = _scan_totals(parts, cap)
    r2, l2 = scan2.result()
    assert r2 == o2_res and l2 == o2_oob
    assert r2["n_oob"] == 1 and l2 == [(ranges[192][0] + 8 * tslot, max_end)]
    tab[tslot] = saved

    say("c4 full exact: clobber every range, restore, every byte and every hash")
    golden = case.arena.buf.clone()
    case.arena.buf.fill_(0xA5)
    n_bad = torch.zeros(1, dtype=torch.int64, device="cuda")
    kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], n_bad=n_bad)
    torch.cuda.synchronize()
    assert int(n_bad.item()) == 0
    for a in range(n):
        o, sz = int(case.layout.offsets[a]), int(case.layout.sizes[a])
        assert torch.equal(case.arena.buf[o:o + sz], golden[o:o + sz]), a
    h2, _, _ = kc.page_hash(ctx, rs)
    torch.cuda.synchronize()
    assert np.array_equal(u64(h2)[:N], g_hash)
    del out, h2

    say("c4 full exact: all 200 ranges compared with a golden copy, differences planted in four, vs oracle")
    kinds = [W.DT_BF16] * 192 + [W.DT_U8, W.DT_F32] + [W.DT_F16] * 6
    planted = {5: (W.DT_BF16, 2, 0.0, 0.0), 192: (W.DT_U8, 0, 0.0, 0.0), 193: (W.DT_F32, 1, 1e-6, 1e-3),
               197: (W.DT_F16, 4, 0.0, 1e-2)}
    gen = torch.Generator(device="cuda").manual_seed(45)
    for i, (dt, _, _, _) in planted.items():
        es = W.ELEM_SIZE[dt]
        bits = case.arena.view(i).view(BITS_VIEW[es])
        idx = torch.randint(0, bits.numel(), (4000,), device="cuda", generator=gen)
        step = torch.randint(1, 6, (4000,), device="cuda", generator=gen).to(bits.dtype)
        bits[idx[:3000]] += step[:3000]                               # a few ULPs (or byte values) away
        bits[idx[3000:]] ^= (step[3000:] << (8 * es - 4)).to(bits.dtype)  # high bits: signs, NaNs, infs
        if dt != W.DT_U8:
            bits[idx[:2]] = SPECIALS[dt][0]                           # NaN in the candidate only
    pairs = []
    for i in range(n):
        o, sz = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        dt, tol, atol, rtol = planted.get(i, (kinds[i], 0, 0.0, 0.0))
        pairs.append((case.arena.buf[o:o + sz], golden[o:o + sz], dt, tol, atol, rtol))
    ps = kc.PairSet(ctx, pairs)
    res = kc.compare_pairset(ctx, ps)
    torch.cuda.synchronize()
    got = kc.decode_cmp(res, n)

    def cmp_job(i, cand_host):
        _, _, dt, tol, atol, rtol = pairs[i]
        o = oracle.compare(cand_host, hosts[i], dt, tol, atol, rtol)   # hosts[i]: the bytes before planting
        assert got[i] == o, i
        return i

    def jobs3():
        for i in range(n):
            yield cmp_job, (i, case.arena.view(i).cpu().numpy() if i in planted else hosts[i])

    with cf.ThreadPoolExecutor(WORKERS) as pool:
        list(_bounded(pool, jobs3(), 2 * WORKERS))
    for i in planted:
        assert got[i]["n_mismatch_elems"] > 0 and got[i]["pass"] == 0
    assert all(got[i]["n_mismatch_bytes"] == 0 and got[i]["pass"] == 1 for i in range(n) if i not in planted)
    ps.close()
    rs.close()
    ctx.close()


@pytest.mark.timeout(1200)
def test_c3_full_exact(kc):
    """10,000 pairs, 8 GiB a side, in the shape the benchmark's batched compare
    runs: every pair's whole report against the oracle, and its mismatch and
    over-tolerance counts against the generator's record."""
    c, shapes = _tuned_context(kc, "c3-10000-pairs", (kc.OP_COMPARE,))
    say(f"compare c3 full exact (10,000 pairs, 8 GiB a side), shape {shapes or 'built-in'}")
    ps = W.c3_pairs("cuda")
    pairs = [(ps.cand(i), ps.gold(i), int(ps.dtypes[i]), int(ps.tols[i]), 1e-8, 1e-5) for i in range(len(ps))]
    res = kc.compare(c, pairs)
    torch.cuda.synchronize()
    got = kc.decode_cmp(res, len(pairs))
    for i, r in enumerate(got):
        assert r["n_elems"] == ps.n_elems(i)
        assert r["n_mismatch_elems"] == len(ps.pos[i])
        assert r["n_over_tol"] == int((np.abs(ps.k[i]) > ps.tols[i]).sum())
    say(f"compare c3 full exact: all 10,000 reports vs oracle on {WORKERS} threads")
    gold_h = ps.gold_arena.cpu().numpy()
    cand_h = ps.cand_arena.cpu().numpy()

    def job(i):
        o, s = int(ps.offsets[i]), int(ps.nbytes[i])
        _, _, dt, tol, atol, rtol = pairs[i]
        r = oracle.compare(cand_h[o:o + s], gold_h[o:o + s], dt, tol, atol, rtol)
        assert got[i] == r, i
        return i

    with cf.ThreadPoolExecutor(WORKERS) as pool:
        done = 0
        for _ in pool.map(job, range(len(ps))):
            done += 1
            if done % 2500 == 0:
                say(f"compare c3 full exact: {done} pairs checked")
    c.close()
