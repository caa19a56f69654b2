"""Benchmark of the snapshot / validation hot path on one MI355X.

One step = one pass of the whole path over the 30 GiB MoE-shaped pool
(200 ranges: 192 bf16 4096x14336 experts, a 512 KiB table of expert
pointers, a 1 GiB fp32 workspace with 80 % zero pages, 6 fp16 activation
buffers):

  1. kc_snapshot        -- zero probe, keep scan, then one pass that hashes
                           every page (XXH64), runs the closure scan over every
                           aligned word and writes the packed snapshot and its
                           page-VA table;
  2. kc_restore         -- zero-fill + scatter of the packed pages back to their
                           original VAs;
  3. kc_compare_pairset -- the 200 restored buffers against a resident golden
                           copy (typed: bf16 / u8 / fp32 / fp16), one launch.

Inputs are resident in HBM before timing.  ``value`` is algorithmic bytes per
step (``step_bytes``) over the timed GPU time of K steps on the stream the
library launches on.  Launch shapes come from the autotuner (every candidate
must give bit-identical outputs).  The roofline object reports the kernel with
the largest time share, timed by HIP events the library records around it.
Also reported: the same step replayed from a HIP graph, the c1 latency case
(stream vs graph), batched persistent launches vs one launch per buffer (c2
delta snapshot over 4096 ranges, c3 compare over 10,000 pairs), and the
validation serving loop (c5: p50 / p99 latency, aggregate GB/s).

    python bench.py [--steps K] [--warmup W] [--scale S] [--no-cpu] [--no-extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import shutil
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PAGE = 4096

# HBM traffic of the main kernels from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) of `bench.py --steps 2 --warmup 1 --no-cpu --no-extras`
# (the tuned launch shapes), per launch, scaled by the factors a plain 4 GiB
# device copy gives (fetch x2.0, write x1.0).  Valid only for the kernel
# sources they were taken from.
PMC_TRAFFIC = {
    "source_sha256": "e1c6a004cddd500c648e60c69194f8845c910135b386660677fe57bc9c581063",
    "snapshot": 62869523365,   # fetch 31385126181 + write 31484397184
    "restore": 63687466317,    # fetch 32333170304 + write 31354296013
    "compare": 64440925107,    # fetch 64440925107 + write 0
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Sources the step's kernels are compiled from (kernels, their device helpers
# and the shared definitions); the counter values below belong to one version.
STEP_KERNEL_SOURCES = ("kc_compare.hip", "kc_device.h", "kc_internal.h", "kc_snapshot.hip", "kc_xxh64.h")


def code_tokens(text: str) -> str:
    """The source with comments removed and whitespace runs collapsed: edits to
    comments or layout do not change what the counters describe."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest(read=None) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_03208_amd", "csrc")
    for name in STEP_KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(name)
        h.update(name.encode() + b"\0" + code_tokens(text).encode())
    return h.hexdigest()


def step_bytes(n_pages: int, n_kept: int, cmp_bytes: int) -> dict:
    """Algorithmic bytes of one step, per op."""
    snap = 4096 * n_pages + 8 * n_pages + (n_pages + 7) // 8 + n_kept * (4096 + 8)
    restore = 4096 * n_kept + 8 * n_kept + 4096 * n_pages
    compare = 2 * cmp_bytes
    return dict(snapshot=snap, restore=restore, compare=compare)


def kernel_bytes(n_pages: int, n_kept: int, cmp_bytes: int) -> dict:
    """Algorithmic bytes of each op's main kernel per launch."""
    return dict(
        snapshot=n_kept * (4096 + 4096 + 8) + 8 * n_pages,  # fused pass: kept pages read + packed + va, all hashes
        restore=n_kept * (4096 + 4096 + 8),                 # scatter: packed read + page write + va read
        compare=2 * cmp_bytes,
    )


def cpu_baseline(case, ranges, sample_idx) -> dict:
    """The oracle, single-threaded, on a bounded sample of the pool's ranges."""
    import numpy as np

    import oracle
    sub = [ranges[i] for i in sample_idx]
    views = [case.arena.view(i).cpu().numpy() for i in sample_idx]
    gold = [v.copy() for v in views]
    nb = sum(s for _, s in sub)
    n_pages = nb // PAGE
    dtypes = [oracle.BF16 if ri < 192 else (oracle.U8 if ri == 192 else (oracle.F32 if ri == 193 else oracle.F16))
              for ri in sample_idx]
    secs = {}
    t0 = time.perf_counter()
    h, z, _ = oracle.page_hash(sub, views)
    secs["page_hash"] = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.closure_scan(sub, views, oob_cap=16)
    secs["closure_scan"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    packed, va, n_kept = oracle.compact(sub, views, z)
    secs["compact"] = time.perf_counter() - t1
    work = [np.empty_like(v) for v in views]
    t1 = time.perf_counter()
    oracle.restore(sub, work, z, None, packed, va, n_kept)
    secs["restore"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    for w, g, dt in zip(work, gold, dtypes):
        oracle.compare(w, g, dt, 0)
    secs["compare"] = time.perf_counter() - t1
    t = time.perf_counter() - t0
    b = step_bytes(n_pages, n_kept, nb)
    total = sum(b.values())
    op_bytes = {"page_hash": nb + 8 * n_pages, "closure_scan": nb, "compact": 4104 * n_kept + 4096 * n_kept,
                "restore": b["restore"], "compare": b["compare"]}
    ops = {k: {"s": round(v, 3), "GBps": round(op_bytes[k] / v / 1e9, 3)} for k, v in secs.items()}
    return {"value": round(total / t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sample_idx)} of the 200 ranges ({nb / 2**30:.2f} GiB: 8 experts, the pointer table, "
                      f"the workspace, one activation buffer) through page hash + closure scan + compact + "
                      f"restore + compare, {t:.1f} s single-threaded",
            "seconds": round(t, 2), "ops": ops, "host": host_cpu(),
            "threads": cpu_threads(sub, gold, dtypes, total)}


def host_cpu() -> dict:
    """The host's CPU model and logical CPU count (what this process may use)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable": usable}


def cpu_threads(sub, views, dtypes, total_bytes: int, chunk: int = 64 << 20) -> dict:
    """The same oracle calls over the same sample, cut into independent 64 MiB chunks on a thread pool.

    ctypes drops the GIL inside each C call, so the chunks run in parallel.  Each chunk's closure scan uses
    the sample's pointer window but only its own chunk as the range table (a word pointing into another
    chunk counts as out of range there): the work per word is the same, the counts are not the sample's.
    """
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    lo, hi = oracle.default_window(sub)
    jobs = []
    for (base, size), v, dt in zip(sub, views, dtypes):
        for off in range(0, size, chunk):
            n = min(chunk, size - off)
            jobs.append(((base + off, n), v[off:off + n], dt))

    def run(job):
        r, v, dt = job
        _, z, _ = oracle.page_hash([r], [v])
        oracle.closure_scan([r], [v], lo, hi, oob_cap=16)
        packed, va, n_kept = oracle.compact([r], [v], z)
        w = np.empty_like(v)
        oracle.restore([r], [w], z, None, packed, va, n_kept)
        oracle.compare(w, v, dt, 0)

    n_threads = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(n_threads) as ex:
        list(ex.map(run, jobs))
    t = time.perf_counter() - t0
    return {"value": round(total_bytes / t / 1e9, 3), "unit": "GB/s", "cores": n_threads, "kind": "oracle",
            "sample": f"the same sample in {len(jobs)} chunks of at most {chunk >> 20} MiB on {n_threads} "
                      f"threads, {t:.1f} s",
            "seconds": round(t, 2)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 30 GiB pool (1.0 = full)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip graph / batching / serving measurements")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in launch shapes")
    ap.add_argument("--retune", action="store_true", help="sweep launch shapes even if a tuned table has them")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the c5 serving run at 200 req/s (after a 2 s warm-up run)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="GIB",
                    help="only run a plain device copy of GIB GiB three times (counter calibration) and exit")
    ap.add_argument("--c1-only", action="store_true",
                    help="only measure the small latency-bound case (64 MiB snapshot + restore + compare) and exit")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving measurement (c5 and the overload burst) and exit")
    ap.add_argument("--units-only", action="store_true",
                    help="only measure snapshot and restore of the pool at 4 KiB, 64 KiB and 2 MiB hash units")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path would shard "
              f"by allocation: each GPU snapshots its own ranges).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration << 30
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(7)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "reps": 3}), flush=True)
        return 0

    from paper_2605_03208_amd import autotune, kc
    from paper_2605_03208_amd import workloads as W

    kc.lib()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.c1_only:
        print(json.dumps({"c1_latency": c1_latency(torch, kc, W, dev)}), flush=True)
        return 0
    if args.serve_only:
        print(json.dumps({"serving": serving(torch, kc, W, dev, args.serve_seconds)}), flush=True)
        return 0
    log(f"generating the MoE pool at scale {args.scale}")
    case = W.c4_snapshot("cuda", scale=args.scale)
    ranges = case.ranges()
    if args.units_only:
        ctx = kc.Context(0)
        print(json.dumps({"hash_units": hash_units(torch, kc, ctx, case, ranges, args.steps)}), flush=True)
        return 0
    golden = case.arena.buf.clone()
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, ranges)
    N = rs.n_pages
    cap = N
    out = dict(hash=torch.empty(N, dtype=torch.int64, device=dev),
               zero_bm=torch.empty(rs.n_words, dtype=torch.int64, device=dev), changed_bm=None,
               packed=torch.empty(cap * PAGE, dtype=torch.uint8, device=dev),
               page_va=torch.empty(cap, dtype=torch.int64, device=dev),
               n_kept=torch.empty(1, dtype=torch.int64, device=dev))
    scan = kc.ScanOut(dev, oob_cap=64)
    n_bad = torch.zeros(1, dtype=torch.int64, device=dev)
    kinds = [W.DT_BF16] * 192 + [W.DT_U8, W.DT_F32] + [W.DT_F16] * 6
    pair_list = []
    for i in range(len(ranges)):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        pair_list.append((case.arena.buf[o:o + s], golden[o:o + s], kinds[i] if i < len(kinds) else W.DT_U8, 0))
    cmp_bytes = sum(int(s) for _, s in ranges)
    res = torch.empty(len(pair_list) * kc.RESULT_BYTES, dtype=torch.uint8, device=dev)
    state = {"ps": kc.PairSet(ctx, pair_list)}

    def snap():
        kc.snapshot(ctx, rs, seed=0, scan=scan, out=out)

    def restore():
        kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"], cap_pages=cap,
                   n_bad=n_bad)

    def compare():
        kc.compare_pairset(ctx, state["ps"], res=res)

    def step():
        snap()
        restore()
        compare()

    tuned = {}
    if not args.no_tune:
        log("autotuning launch shapes on this workload (tuned table reused unless --retune)")
        sig = f"c4-moe-pool-scale{args.scale}"
        use_cache = not args.retune
        snap_digest = lambda: autotune.digest_tensors(out["hash"], out["zero_bm"], out["n_kept"], scan.res)
        r = autotune.tune(ctx, kc.OP_SNAPSHOT, snap, snap_digest, sig, use_cache=use_cache)
        tuned["snapshot"] = dict(r["best"], cached=r["cached"])
        restore_digest = lambda: autotune.digest_tensors(n_bad)
        r = autotune.tune(ctx, kc.OP_RESTORE, restore, restore_digest, sig, use_cache=use_cache)
        tuned["restore"] = dict(r["best"], cached=r["cached"])

        def prep(cand):
            state["ps"].close()
            state["ps"] = kc.PairSet(ctx, pair_list)

        cmp_digest = lambda: autotune.digest_tensors(res)
        r = autotune.tune(ctx, kc.OP_COMPARE, compare, cmp_digest, sig, use_cache=use_cache, prepare=prep)
        tuned["compare"] = dict(r["best"], cached=r["cached"])
        log(f"tuned: {tuned}")

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_kept = int(out["n_kept"].item())
    sres, _ = scan.result()
    got = kc.decode_cmp(res, len(pair_list))
    assert all(r["pass"] == 1 and r["n_mismatch_bytes"] == 0 for r in got), "restored pool differs from golden"
    assert int(n_bad.item()) == 0 and sres["n_oob"] == 0

    log(f"timing {args.steps} steps")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps

    log("per-kernel timing pass")
    ctx.enable_timing(True)
    kms = {"snapshot": [], "restore": [], "compare": []}
    for _ in range(args.steps):
        step()
        kms["snapshot"].append(ctx.kernel_ms(kc.OP_SNAPSHOT))
        kms["restore"].append(ctx.kernel_ms(kc.OP_RESTORE))
        kms["compare"].append(ctx.kernel_ms(kc.OP_COMPARE))
    ctx.enable_timing(False)
    avg = {k: float(np.mean(v)) for k, v in kms.items()}
    sb = step_bytes(N, n_kept, cmp_bytes)
    kb = kernel_bytes(N, n_kept, cmp_bytes)
    total_bytes = sum(sb.values())
    value = total_bytes / (ms_per_step / 1e3) / 1e9
    dom = max(avg, key=avg.get)
    achieved = kb[dom] / (avg[dom] / 1e3) / 1e9
    kernel_names = {"snapshot": "k_page_hash<gather,scan>", "restore": "k_restore_scatter", "compare": "k_compare"}
    traffic_ok = PMC_TRAFFIC["source_sha256"] == source_digest() and args.scale == 1.0
    ops = {k: {"kernel": kernel_names[k], "kernel_ms": round(avg[k], 4),
               "kernel_GBps": round(kb[k] / (avg[k] / 1e3) / 1e9, 1),
               "kernel_frac_of_peak": round(kb[k] / (avg[k] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
               "kernel_alg_bytes": kb[k], "op_alg_bytes_per_step": sb[k],
               "pmc_traffic_bytes": PMC_TRAFFIC[k] if traffic_ok else None} for k in avg}

    line = {
        "metric": "hash+compact/compare GB/s (% HBM peak), batched vs per-buffer; p99 latency",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8/u64 (XXH64, scans); fp64 (compare errors)", "data": "synthetic",
        "frac_of_hbm_peak": round(value / HBM_PEAK_GBS, 4),
        "config": {"workload": "MoE-shaped pool snapshot -> restore -> validate: 200 ranges, "
                               f"{N * PAGE / 2**30:.2f} GiB ({N} pages, {n_kept} kept), 192 bf16 4096x14336 "
                               "experts + 512 KiB pointer table + 1 GiB fp32 workspace (80% zero pages) + "
                               "6 fp16 activations; fused closure scan vs the 200 sorted ranges; "
                               "200-pair typed compare against a resident golden copy",
                   "scale": args.scale, "pages": N, "kept_pages": n_kept, "alg_bytes_per_step": total_bytes,
                   "launch_shapes": tuned or "built-in"},
        "roofline": {"bound": "hbm", "kernel": kernel_names[dom], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": ops[dom]["pmc_traffic_bytes"]},
        "ops": ops,
        "wall_s_timed": round(wall, 3),
    }

    # the snapshot op alone (probe + scans + fused pass + out-of-range emission)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        snap()
    e1.record(stream)
    torch.cuda.synchronize()
    snap_op_ms = e0.elapsed_time(e1) / args.steps
    line["snapshot_op"] = {"ms": round(snap_op_ms, 4),
                           "GBps": round(sb["snapshot"] / (snap_op_ms / 1e3) / 1e9, 1),
                           "frac_of_peak": round(sb["snapshot"] / (snap_op_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    sample_idx = list(range(0, 8)) + [192, 193, 194] if args.scale == 1.0 else list(range(min(11, len(ranges))))
    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline on a bounded sample")
        cpu = cpu_baseline(case, ranges, sample_idx)
    if not args.no_extras:
        log("copy ceiling: plain 4 GiB device-to-device copy")
        line["copy_ceiling"] = copy_ceiling(torch, dev)
        log("pointer graph over the same ranges")
        line["pointer_graph"] = pointer_graph_pass(torch, kc, ctx, rs, N, args.steps, tune=not args.no_tune)
        log("region diff of the live pool against the step's snapshot, 1 % of pages touched")
        line["region_diff"] = region_diff_pass(torch, kc, ctx, rs, out, case, N, args.steps, tune=not args.no_tune)
        log("graph replay of the step")
        line["graph"] = graph_step(torch, step, res, pair_list, kc, args.steps)
        log("hash units of 4 KiB, 64 KiB and 2 MiB: snapshot and restore of the same pool")
        line["hash_units"] = hash_units(torch, kc, ctx, case, ranges, args.steps)
        log("plain copies between the restore's own buffers, both directions (the pool is clobbered after this)")
        line["copy_same_buffers"] = same_buffer_copies(torch, case, out, n_kept, avg["restore"], avg["snapshot"])
        state["ps"].close()
        rs.close()
        del case, golden, out, state, pair_list, rs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        line["graph"]["c1_latency"] = c1_latency(torch, kc, W, dev)
        line["batching"] = batching(torch, kc, W, dev, tune=not args.no_tune)
        line["snapshot_files"] = snapshot_files(torch, kc, W, dev)
        line["partial_pages"] = partial_pages(torch, kc, W, dev)
        line["scan_many_ranges"] = scan_many_ranges(torch, kc, W, dev)
        line["serving"] = serving(torch, kc, W, dev, args.serve_seconds)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    return 0


def same_buffer_copies(torch, case, out, n_kept: int, restore_ms: float, snapshot_ms: float, reps: int = 3) -> dict:
    """A plain elementwise copy kernel (torch, 16-byte vectors) moving the
    restore's bytes (n_kept pages) between the restore's own two buffers:
    packed snapshot -> pool (the restore's direction) and pool -> packed (the
    fused snapshot pass's direction).  The copy's GB/s count read + write;
    *_speed_vs_copy is the copy's time over the kernel's (1.0 = as fast as
    the copy in its direction).  Leaves the pool holding packed bytes."""
    nbytes = n_kept * PAGE
    packed = out["packed"][:nbytes].view(torch.int32)
    pool = case.arena.buf[:nbytes].view(torch.int32)
    res = {"bytes_copied": nbytes}
    for name, src, dst in (("packed_to_pool", packed, pool), ("pool_to_packed", pool, packed)):
        torch.mul(src, 1, out=dst)  # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch.mul(src, 1, out=dst)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": round(ms, 4), "GBps": round(2 * nbytes / (ms / 1e3) / 1e9, 1)}
    res["restore_scatter_speed_vs_copy"] = round(res["packed_to_pool"]["ms"] / restore_ms, 4)
    res["snapshot_pass_speed_vs_copy"] = round(res["pool_to_packed"]["ms"] / snapshot_ms, 4)
    return res


def hash_units(torch, kc, ctx, case, ranges, reps: int) -> dict:
    """The snapshot (probe, keep scan, hashing pass with the packed writes; no
    closure scan) and the restore of the same pool at hash units of 4 KiB,
    64 KiB and 2 MiB, each in its own range set.  Algorithmic bytes: the
    ranges' bytes read, 8 B of hash and a zero bit per unit, a packed slot of
    `unit` bytes and an 8 B page VA per kept unit (restore: the packed slots
    read, the ranges' bytes written, the page VAs read)."""
    import numpy as np
    dev = case.arena.buf.device
    pool = sum(int(s) for _, s in ranges)
    res = {}
    for unit, depth in ((4096, 0), (64 << 10, 0), (64 << 10, 1), (2 << 20, 0), (2 << 20, 4)):
        ctx.set_tuning(kc.OP_SNAPSHOT, depth=depth)
        rs = kc.RangeSet(ctx, ranges, unit=unit)
        n = rs.n_pages
        out = dict(hash=torch.empty(n, dtype=torch.int64, device=dev),
                   zero_bm=torch.empty(rs.n_words, dtype=torch.int64, device=dev), changed_bm=None,
                   packed=torch.empty(n * unit, dtype=torch.uint8, device=dev),
                   page_va=torch.empty(n, dtype=torch.int64, device=dev),
                   n_kept=torch.empty(1, dtype=torch.int64, device=dev))
        kc.snapshot(ctx, rs, out=out)
        torch.cuda.synchronize()
        kept = int(out["n_kept"].item())
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.enable_timing(True)
        kms = []
        ev0.record()
        for _ in range(reps):
            kc.snapshot(ctx, rs, out=out)
            kms.append(ctx.kernel_ms(kc.OP_SNAPSHOT))
        ev1.record()
        torch.cuda.synchronize()
        snap_ms = ev0.elapsed_time(ev1) / reps
        rms = []
        ev0.record()
        for _ in range(reps):
            kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"])
            rms.append(ctx.kernel_ms(kc.OP_RESTORE))
        ev1.record()
        torch.cuda.synchronize()
        ctx.enable_timing(False)
        restore_ms = ev0.elapsed_time(ev1) / reps
        snap_bytes = pool + 8 * n + n // 8 + kept * (unit + 8)
        restore_bytes = kept * (unit + 8) + pool
        res[f"{unit // 1024}KiB" + (f"_depth{depth}" if depth else "")] = {
            "units": n, "kept_units": kept,
            "snapshot_ms": round(snap_ms, 4), "snapshot_GBps": round(snap_bytes / snap_ms / 1e6, 1),
            "hash_pass_ms": round(float(np.mean(kms)), 4),
            "restore_ms": round(restore_ms, 4), "restore_GBps": round(restore_bytes / restore_ms / 1e6, 1),
            "restore_scatter_ms": round(float(np.mean(rms)), 4)}
        del out
        rs.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    ctx.set_tuning(kc.OP_SNAPSHOT)
    return res


def copy_ceiling(torch, dev, gib: int = 4, reps: int = 5) -> dict:
    """A plain device copy (torch's copy kernel): what a read+write stream reaches on this part."""
    src = torch.empty(gib << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * (gib << 30) / (ms / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * (gib << 30), "ms": round(ms, 4), "GBps": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def region_diff_pass(torch, kc, ctx, rs, gold, case, n_pages: int, reps: int, tune: bool = True) -> dict:
    """kc_region_diff over the step's ranges against the step's snapshot, after
    one byte of every 100th page was flipped (flipped back afterwards)."""
    import numpy as np
    shape = None
    cum = case.layout.cum()
    pages = np.arange(0, n_pages, 100)
    a = np.searchsorted(cum // PAGE, pages, side="right") - 1
    offs = case.layout.offsets[a] + (pages - cum[a] // PAGE) * PAGE + 123
    idx = torch.from_numpy(offs.astype(np.int64)).cuda()
    buf = case.arena.buf
    buf[idx] ^= 0x5A
    out = kc.region_diff(ctx, rs, gold)
    if tune:
        from paper_2605_03208_amd import autotune
        run = lambda: kc.region_diff(ctx, rs, gold, out=out)
        dig = lambda: autotune.digest_tensors(out["res"], out["changed_bm"], out["hash"])
        shape = {name: autotune.tune(ctx, op, run, dig, f"c4-moe-pool-pages{n_pages}")["best"]
                 for op, name in ((kc.OP_PAGE_HASH, "hash"), (kc.OP_REGION_DIFF, "diff"))}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        kc.region_diff(ctx, rs, gold, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ctx.enable_timing(True)
    kc.region_diff(ctx, rs, gold, out=out)
    kms = ctx.kernel_ms(kc.OP_REGION_DIFF)
    hms = ctx.kernel_ms(kc.OP_PAGE_HASH)
    ctx.enable_timing(False)
    diff = kc.decode_region_diff(out["res"], len(rs.ranges))
    buf[idx] ^= 0x5A
    torch.cuda.synchronize()
    changed = len(pages)
    alg = n_pages * PAGE + 2 * changed * PAGE
    return {"op_ms": round(ms, 4), "GBps": round(alg / (ms / 1e3) / 1e9, 1),
            "frac_of_peak": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "hash_kernel_ms": round(hms, 4), "diff_kernel_ms": round(kms, 4), "pages_changed": changed,
            "diff_bytes": sum(r["n_diff_bytes"] for r in diff), "diff_pages": sum(r["n_diff_pages"] for r in diff),
            "diff_shape": shape}


def pointer_graph_pass(torch, kc, ctx, rs, n_pages: int, reps: int, tune: bool = True) -> dict:
    """kc_pointer_graph over the step's ranges: one read of every page."""
    import numpy as np
    out = kc.pointer_graph(ctx, rs)
    shape = None
    if tune:
        from paper_2605_03208_amd import autotune
        r = autotune.tune(ctx, kc.OP_GRAPH, lambda: kc.pointer_graph(ctx, rs, out=out),
                          lambda: autotune.digest_tensors(out), f"c4-moe-pool-pages{n_pages}")
        shape = r["best"]
    ctx.enable_timing(True)
    ms = []
    for _ in range(reps):
        kc.pointer_graph(ctx, rs, out=out)
        ms.append(ctx.kernel_ms(kc.OP_GRAPH))
    ctx.enable_timing(False)
    edges = int(np.unpackbits(out.cpu().numpy().view(np.uint8)).sum())
    k = float(np.mean(ms))
    gbs = n_pages * PAGE / (k / 1e3) / 1e9
    return {"kernel": "k_pointer_graph", "kernel_ms": round(k, 4), "GBps": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "n_ranges": len(rs.ranges), "n_edges": edges,
            "shape": shape}


def graph_step(torch, step, res, pair_list, kc, reps: int) -> dict:
    """Record one step into a HIP graph, replay it, check the replays."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    got = kc.decode_cmp(res, len(pair_list))
    ok = all(r["pass"] == 1 and r["n_mismatch_bytes"] == 0 for r in got)
    return {"ms_per_step": round(e0.elapsed_time(e1) / reps, 4), "replays_checked": ok}


def c1_latency(torch, kc, W, dev) -> dict:
    """Latency-bound small case: 64 MiB snapshot + restore + 16-pair compare."""
    log("c1 latency: stream vs graph")
    case = W.c1_snapshot("cuda")
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, case.ranges())
    N = rs.n_pages
    out = dict(hash=torch.empty(N, dtype=torch.int64, device=dev),
               zero_bm=torch.empty(rs.n_words, dtype=torch.int64, device=dev), changed_bm=None,
               packed=torch.empty(N * PAGE, dtype=torch.uint8, device=dev),
               page_va=torch.empty(N, dtype=torch.int64, device=dev),
               n_kept=torch.empty(1, dtype=torch.int64, device=dev))
    scan = kc.ScanOut(dev, oob_cap=16)
    pairs = W.c1_compare("cuda")
    ps = kc.PairSet(ctx, [(p.cand, p.gold, W.DT_F32, 0) for p in pairs])
    res = torch.empty(len(pairs) * kc.RESULT_BYTES, dtype=torch.uint8, device=dev)

    def step():
        kc.snapshot(ctx, rs, scan=scan, out=out)
        kc.restore(ctx, rs, out["zero_bm"], None, out["packed"], out["page_va"], out["n_kept"])
        kc.compare_pairset(ctx, ps, res=res)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    ref = res.clone()
    reps = 50
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    stream_host_us = (time.perf_counter() - t0) / reps * 1e6  # host time to issue one step
    e1.record(stream)
    torch.cuda.synchronize()
    stream_us = e0.elapsed_time(e1) / reps * 1e3
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    with torch.cuda.stream(s):
        step()
    stream.wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    ok = True
    for _ in range(3):  # replays with eager work in between, each checked
        g.replay()
        torch.cuda.synchronize()
        ok = ok and torch.equal(res, ref)
        res.zero_()
        torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    graph_host_us = (time.perf_counter() - t0) / reps * 1e6
    e1.record(stream)
    torch.cuda.synchronize()
    graph_us = e0.elapsed_time(e1) / reps * 1e3
    ok = ok and torch.equal(res, ref)
    ps.close()
    rs.close()
    ctx.close()
    return {"workload": "c1: 64 MiB / 48 ranges snapshot + restore + 16 x 2^20 fp32 compare",
            "stream_us": round(stream_us, 1), "graph_us": round(graph_us, 1),
            "graph_speedup": round(stream_us / graph_us, 3),
            "stream_host_issue_us": round(stream_host_us, 1), "graph_host_issue_us": round(graph_host_us, 1),
            "replays_match_eager": ok}


def partial_pages(torch, kc, W, dev) -> dict:
    """Full snapshot of the c2 pool (4096 ranges, 2 GiB) with its page-multiple
    sizes, then with every range 1-4095 bytes shorter (every range ends in a
    partial page): what the partial-page path costs."""
    import numpy as np
    log("partial pages: c2 full snapshot, whole vs every range ending in a partial page")
    case = W.c2_snapshot("cuda")
    rng = np.random.default_rng(7)
    whole = case.ranges()
    ragged = [(b, s - int(rng.integers(1, 4096))) for b, s in whole]
    out = {"ranges": len(whole)}
    for name, ranges in (("whole", whole), ("ragged", ragged)):
        ctx = kc.Context(0)
        rs = kc.RangeSet(ctx, ranges)
        snap = kc.snapshot(ctx, rs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            kc.snapshot(ctx, rs, out=snap)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        nbytes = sum(s for _, s in ranges)
        out[f"{name}_ms"] = round(ms, 4)
        out[f"{name}_GBps_read"] = round(nbytes / (ms / 1e3) / 1e9, 1)
        rs.close()
        ctx.close()
    out["ragged_over_whole"] = round(out["ragged_ms"] / out["whole_ms"], 3)
    del case
    torch.cuda.empty_cache()
    return out


def scan_many_ranges(torch, kc, W, dev, reps: int = 5) -> dict:
    """Closure scan over the 4096-range, 2 GiB set with 1 % of every range's
    words set to addresses inside random ranges: the fused snapshot and the
    standalone scan, against the same set without planted pointers."""
    log("closure scan over 4096 ranges, with and without 1 % pointer words")
    case = W.c2_snapshot("cuda")
    ranges = case.ranges()
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, ranges)
    out = kc.snapshot(ctx, rs, seed=0)
    scan = kc.ScanOut(dev, oob_cap=16)
    nbytes = sum(s for _, s in ranges)

    def timed():
        ctx.enable_timing(True)
        snap, cl = [], []
        for _ in range(reps):
            kc.snapshot(ctx, rs, scan=scan, out=out)
            snap.append(ctx.kernel_ms(kc.OP_SNAPSHOT))
            kc.closure_scan(ctx, rs, scan)
            cl.append(ctx.kernel_ms(kc.OP_CLOSURE))
        ctx.enable_timing(False)
        return min(snap), min(cl)

    res = {"ranges": len(ranges), "bytes": nbytes}
    res["fused_ms_no_pointers"], res["standalone_ms_no_pointers"] = (round(x, 4) for x in timed())
    gen = torch.Generator(device=dev).manual_seed(7)
    bases = torch.tensor([b for b, _ in ranges], dtype=torch.int64, device=dev)
    sizes = torch.tensor([s for _, s in ranges], dtype=torch.int64, device=dev)
    for i in range(len(ranges)):
        w = case.arena.view(i).view(torch.int64)
        k = max(1, w.numel() // 100)
        pos = torch.randint(0, w.numel(), (k,), device=dev, generator=gen)
        tgt = torch.randint(0, len(ranges), (k,), device=dev, generator=gen)
        off = (torch.rand(k, device=dev, generator=gen, dtype=torch.float64) * sizes[tgt].double()).long()
        w[pos] = bases[tgt] + off
    res["fused_ms"], res["standalone_ms"] = (round(x, 4) for x in timed())
    r, _ = scan.result()
    res["n_ptr_like"], res["n_in_range"] = r["n_ptr_like"], r["n_in_range"]
    res["standalone_GBps"] = round(nbytes / (res["standalone_ms"] / 1e3) / 1e9, 1)
    rs.close()
    ctx.close()
    del case, out
    torch.cuda.empty_cache()
    return res


def batching(torch, kc, W, dev, tune: bool = True) -> dict:
    """Batched persistent launches (autotuned shapes unless ``tune`` is off) vs one launch per buffer on uneven
    sizes."""
    from paper_2605_03208_amd import autotune
    out = {}
    log("batching: c3 compare, 10,000 pairs / 8 GiB per side")
    ps = W.c3_pairs("cuda", n_pairs=10000)
    plist = [(ps.cand(i), ps.gold(i), int(ps.dtypes[i]), int(ps.tols[i]), 1e-8, 1e-5) for i in range(len(ps))]
    arr = kc.make_pairs(plist)
    nbytes = 2 * int(ps.nbytes.sum())
    res = torch.empty(len(ps) * kc.RESULT_BYTES, dtype=torch.uint8, device=dev)
    results = {}
    for mode in ("batched", "per_buffer"):
        c2 = kc.Context(0)
        c2.set_tuning(kc.OP_COMPARE, per_item=1 if mode == "per_buffer" else 0)
        if mode == "batched" and tune:
            r = autotune.tune(c2, kc.OP_COMPARE, lambda: kc.compare(c2, arr, res=res),
                              lambda: autotune.digest_tensors(res), "c3-10000-pairs")
            out["c3_batched_shape"] = r["best"]
        kc.compare(c2, arr, res=res)
        torch.cuda.synchronize()
        results[mode] = res.clone()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            kc.compare(c2, arr, res=res)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[f"c3_compare_{mode}_ms"] = round(dt * 1e3, 3)
        out[f"c3_compare_{mode}_GBps"] = round(nbytes / dt / 1e9, 1)
        c2.close()
    out["c3_results_identical"] = bool(torch.equal(results["batched"], results["per_buffer"]))
    out["c3_batched_speedup"] = round(out["c3_compare_per_buffer_ms"] / out["c3_compare_batched_ms"], 2)
    del ps, plist, arr, results
    torch.cuda.empty_cache()
    log("batching: c2 delta snapshot, 4096 ranges / 2 GiB")
    case = W.c2_snapshot("cuda")
    rngs = case.ranges()
    c0 = kc.Context(0)
    rs0 = kc.RangeSet(c0, rngs)
    s1 = kc.snapshot(c0, rs0, seed=2)  # the base image P1 (full snapshot)
    prior = s1["hash"].clone()
    W.c2_rewrite(case)
    torch.cuda.synchronize()
    rs0.close()
    c0.close()
    digests = {}
    for mode in ("batched", "per_buffer"):
        c2 = kc.Context(0)
        for op in (kc.OP_PAGE_HASH, kc.OP_COMPACT):
            c2.set_tuning(op, per_item=1 if mode == "per_buffer" else 0)
        rs = kc.RangeSet(c2, rngs)
        s2 = kc.snapshot(c2, rs, seed=2, prior=prior)
        if mode == "batched" and tune:
            run = lambda: kc.snapshot(c2, rs, seed=2, prior=prior, out=s2)
            dig = lambda: autotune.digest_tensors(s2["hash"], s2["changed_bm"], s2["n_kept"], s2["page_va"])
            out["c2_batched_shape"] = {kc_name: autotune.tune(c2, op, run, dig, "c2-delta-4096-ranges")["best"]
                                       for op, kc_name in ((kc.OP_PAGE_HASH, "page_hash"),
                                                           (kc.OP_COMPACT, "compact"))}
            run()
        torch.cuda.synchronize()
        nk = int(s2["n_kept"].item())
        digests[mode] = (s2["hash"].cpu(), s2["changed_bm"].cpu(), s2["packed"][: nk * PAGE].cpu())
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            kc.snapshot(c2, rs, seed=2, prior=prior, out=s2)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        n = rs.n_pages
        b = 4096 * n + 8 * n + 8 * n + n // 4 + nk * 4104
        out[f"c2_delta_{mode}_ms"] = round(dt * 1e3, 3)
        out[f"c2_delta_{mode}_GBps"] = round(b / dt / 1e9, 1)
        out["c2_delta_kept_pages"] = nk
        if mode == "batched":  # restore chain: the base image P1, then the delta D on top of it
            nk1 = int(s1["n_kept"].item())
            full = lambda: kc.restore(c2, rs, s1["zero_bm"], None, s1["packed"], s1["page_va"], s1["n_kept"])
            delta = lambda: kc.restore(c2, rs, s2["zero_bm"], s2["changed_bm"], s2["packed"], s2["page_va"],
                                       s2["n_kept"])
            full()
            delta()
            h, _, _ = kc.page_hash(c2, rs, seed=2)
            torch.cuda.synchronize()
            out["c2_restore_chain_matches_delta_hashes"] = bool(torch.equal(h[:n], s2["hash"][:n]))
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            tf = td = 0.0
            for _ in range(reps):
                ev[0].record()
                full()
                ev[1].record()
                delta()
                ev[2].record()
                torch.cuda.synchronize()
                tf += ev[0].elapsed_time(ev[1]) / reps
                td += ev[1].elapsed_time(ev[2]) / reps
            bf = 4104 * nk1 + 4096 * n          # packed read + page writes (kept and zero) + VA reads
            bd = 8200 * nk                       # changed non-zero pages: packed read + page write + VA
            out["c2_restore_full_ms"] = round(tf, 3)
            out["c2_restore_full_GBps"] = round(bf / (tf / 1e3) / 1e9, 1)
            out["c2_restore_delta_ms"] = round(td, 3)
            out["c2_restore_delta_GBps"] = round(bd / (td / 1e3) / 1e9, 1)
        rs.close()
        c2.close()
    out["c2_results_identical"] = all(torch.equal(a, b) for a, b in zip(digests["batched"], digests["per_buffer"]))
    out["c2_batched_speedup"] = round(out["c2_delta_per_buffer_ms"] / out["c2_delta_batched_ms"], 2)
    del case, s1
    torch.cuda.empty_cache()
    return out


def _mount_of(path: str) -> dict:
    """The mount holding ``path`` (longest matching mount point in
    /proc/mounts): device, file system type, and whether it is held in memory."""
    path = os.path.realpath(path)
    best = ("", "", "")
    try:
        with open("/proc/mounts") as f:
            for line in f:
                dev, mnt, fs = line.split()[:3]
                mnt = mnt.replace("\\040", " ")
                if (path == mnt or path.startswith(mnt.rstrip("/") + "/")) and len(mnt) >= len(best[1]):
                    best = (dev, mnt, fs)
    except OSError:
        pass
    dev, mnt, fs = best
    info = {"device": dev, "mount": mnt, "fstype": fs, "in_memory": fs in ("tmpfs", "ramfs")}
    name = os.path.basename(dev)
    for blk in (name, name.rstrip("0123456789").rstrip("p") if name.startswith("nvme") else name.rstrip("0123456789")):
        model = f"/sys/block/{blk}/device/model"
        if blk and os.path.exists(model):
            info["model"] = open(model).read().strip()
            info["rotational"] = open(f"/sys/block/{blk}/queue/rotational").read().strip() == "1"
            break
    return info


def _disk_dir(min_free: int):
    """A directory on a block device (not a memory file system) with room to spare, else None."""
    cands = [os.environ.get("GRAFT_REPO_ROOT", ""), os.path.dirname(os.path.abspath(__file__)), "/var/tmp",
             os.path.expanduser("~"), "/tmp"]
    for c in cands:
        if c and os.path.isdir(c) and os.access(c, os.W_OK):
            m = _mount_of(c)
            if not m["in_memory"] and m["fstype"] not in ("", "proc", "sysfs") and \
                    shutil.disk_usage(c).free > min_free:
                return c, m
    return None, None


def snapshot_files(torch, kc, W, dev) -> dict:
    """The packed snapshot of the 2 GiB / 4096-range pool streamed to host
    files and loaded back (the paper's capture writes regions to files at
    ~1.7 GB/s, Sec. 5.3), through four 64 MiB pinned buffers, to a memory file
    system and to a directory on a block device.  Each side reports the wall
    time split into waiting for device copies and file I/O.  On the block
    device the save is also made durable (fsync of every file, timed apart),
    the files' cached pages are then dropped (fadvise), and the load reads
    them back from the device."""
    import tempfile
    log("snapshot files: c2 full snapshot saved and loaded back, RAM and block-device targets")
    case = W.c2_snapshot("cuda")
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, case.ranges())
    out = kc.snapshot(ctx, rs, seed=2)
    torch.cuda.synchronize()
    n_kept = int(out["n_kept"].item())
    shm = "/dev/shm" if os.path.isdir("/dev/shm") and shutil.disk_usage("/dev/shm").free > (8 << 30) else None
    disk, disk_mount = _disk_dir(8 << 30)
    res = {"workload": "c2 full snapshot (4096 ranges, 2 GiB)"}
    for label, base, mount in (("ram", shm, _mount_of(shm) if shm else None), ("disk", disk, disk_mount)):
        if base is None:
            res[label] = None
            continue
        d = tempfile.mkdtemp(prefix="kc_snap_", dir=base)
        try:
            sd = os.path.join(d, "s")
            save = kc.snapshot_save(ctx, rs, sd, out, seed=2)
            r = {"dir": base, "mount": mount, "bytes": save["bytes"],
                 "save_GBps": round(save["bytes"] / save["seconds"] / 1e9, 2), "save_s": round(save["seconds"], 4),
                 "save_copy_wait_s": round(save["copy_wait_s"], 4), "save_file_s": round(save["file_s"], 4)}
            if label == "disk":
                t0 = time.perf_counter()
                for name in os.listdir(sd):
                    fd = os.open(os.path.join(sd, name), os.O_RDONLY)
                    os.fsync(fd)
                    os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)   # the load must come from the device
                    os.close(fd)
                fs = time.perf_counter() - t0
                r["fsync_s"] = round(fs, 4)
                r["save_durable_GBps"] = round(save["bytes"] / (save["seconds"] + fs) / 1e9, 2)
            back, load = kc.snapshot_load(ctx, rs, sd)
            r.update(load_GBps=round(load["bytes"] / load["seconds"] / 1e9, 2), load_s=round(load["seconds"], 4),
                     load_copy_wait_s=round(load["copy_wait_s"], 4), load_file_s=round(load["file_s"], 4),
                     reload_identical=bool(torch.equal(back["packed"][: n_kept * PAGE], out["packed"][: n_kept * PAGE])))
            del back
        finally:
            shutil.rmtree(d, ignore_errors=True)
        res[label] = r
    rs.close()
    ctx.close()
    del case, out
    torch.cuda.empty_cache()
    return res


def serving(torch, kc, W, dev, seconds: float) -> dict:
    """c5: Poisson 200 req/s, 1-64 candidate buffers per request, 32 GiB budget."""
    from paper_2605_03208_amd import serve
    log(f"serving: c5 for {seconds:.1f} s at 200 req/s")
    torch.cuda.empty_cache()  # arenas come from the server's streams, which cannot reuse earlier cached blocks
    free, total = torch.cuda.mem_get_info()
    log(f"serving: device memory free {free / 2**30:.1f} of {total / 2**30:.1f} GiB, torch holds "
        f"{torch.cuda.memory_allocated() / 2**30:.1f} GiB allocated, {torch.cuda.memory_reserved() / 2**30:.1f} GiB reserved")
    golds, dtypes = W.c5_pool("cuda")
    reqs = W.c5_requests(rate_hz=200.0, duration_s=seconds)
    reqs = [serve.Request(r.rid, r.arrival_s, r.golden_ids, r.ulp_tol, r.seed) for r in reqs]
    ex = serve.DeviceExecutor(golds, dtypes, n_streams=4, arena_bytes=32 << 30)
    log("serving: 2 s warm-up run of the same schedule law (another seed)")
    warm_reqs = W.c5_requests(rate_hz=200.0, duration_s=2.0, seed=55)
    warm = serve.Server(ex, 32 << 30)
    warm.run([serve.Request(r.rid, r.arrival_s, r.golden_ids, r.ulp_tol, r.seed) for r in warm_reqs])
    torch.cuda.synchronize()
    srv = serve.Server(ex, 32 << 30)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    summ = serve.summarize(done, wall)
    summ.update(offered_req_per_s=200.0, budget_GiB=32, budget_peak_GiB=round(srv.budget.peak / 2**30, 2),
                streams=4, pool_buffers=len(golds),
                pool_GiB=round(sum(g.numel() * g.element_size() for g in golds) / 2**30, 2))
    burst_s = min(2.0, seconds / 3)   # long enough to fill the budget; longer only lengthens the queue
    log(f"serving: overload burst (2,000 req/s for {burst_s:.1f} s)")
    burst = W.c5_requests(rate_hz=2000.0, duration_s=burst_s)
    burst = [serve.Request(r.rid, r.arrival_s, r.golden_ids, r.ulp_tol, r.seed) for r in burst]
    # warm-up burst (another seed): the first budget-sized arenas are fresh device allocations
    warm_burst = W.c5_requests(rate_hz=2000.0, duration_s=min(0.5, burst_s), seed=56)
    serve.Server(ex, 32 << 30).run([serve.Request(r.rid, r.arrival_s, r.golden_ids, r.ulp_tol, r.seed)
                                    for r in warm_burst])
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    log(f"serving: after the warm-up burst, device memory free {free / 2**30:.1f} GiB, torch reserved "
        f"{torch.cuda.memory_reserved() / 2**30:.1f} GiB")
    srv2 = serve.Server(ex, 32 << 30)
    t0 = time.perf_counter()
    done2 = srv2.run(burst)
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    b = serve.summarize(done2, wall2)
    b.update(offered_req_per_s=2000.0, budget_peak_GiB=round(srv2.budget.peak / 2**30, 2))
    summ["overload"] = b
    return summ


if __name__ == "__main__":
    sys.exit(main())
