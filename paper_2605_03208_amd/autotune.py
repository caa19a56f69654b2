"""Launch-shape autotuner for the kc operations.

For one operation on the caller's real inputs, every candidate launch shape
(persistent waves per CU, and for compare workgroups per CU and the bytes per tile) is run,
timed with the library's kernel events, and its outputs are digested; a
candidate whose outputs differ from the first one's raises, so tuning can
never change a result.  The fastest candidate is applied to the context and
stored in a JSON cache keyed by (arch, HIP version, op, workload signature).

    from paper_2605_03208_amd import autotune
    best = autotune.tune(ctx, kc.OP_SNAPSHOT, run=lambda: ..., digest=lambda: ..., signature="c4")
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import torch

from . import kc

ARCH = "gfx950"

CANDIDATES = {
    kc.OP_PAGE_HASH: [dict(grid_per_cu=g) for g in (2, 3, 4, 6, 8, 12, 16, 24)],
    kc.OP_SNAPSHOT: [dict(grid_per_cu=g) for g in (2, 3, 4, 6, 8, 12)],
    kc.OP_COMPACT: [dict(grid_per_cu=g) for g in (4, 8, 16, 32, 48, 64, 96, 128, 192, 256)],
    kc.OP_RESTORE: [dict(grid_per_cu=g) for g in (8, 12, 16, 24, 32, 48, 64, 96, 128)],
    kc.OP_CLOSURE: [dict(grid_per_cu=g) for g in (4, 8, 16)],
    kc.OP_COMPARE: [dict(grid_per_cu=g, tile_bytes=t) for g in (1, 2, 3, 4, 16, 64, 128, 256, 512, 1024)
                    for t in (16 << 10, 32 << 10, 64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20)],
    kc.OP_GRAPH: [dict(grid_per_cu=g) for g in (4, 8, 12, 16, 24, 32)],
    kc.OP_REGION_DIFF: [dict(grid_per_cu=g) for g in (8, 12, 16, 20, 32, 48, 64)],
}

OP_NAMES = {kc.OP_PAGE_HASH: "page_hash", kc.OP_SNAPSHOT: "snapshot", kc.OP_COMPACT: "compact",
            kc.OP_RESTORE: "restore", kc.OP_CLOSURE: "closure_scan", kc.OP_COMPARE: "compare",
            kc.OP_GRAPH: "pointer_graph", kc.OP_REGION_DIFF: "region_diff"}


class TuningChangedResult(RuntimeError):
    """A candidate launch shape produced different outputs."""


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def cache_path() -> str:
    """The writable cache (tuning results of this machine)."""
    return os.environ.get("KC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "kc", "tune.json"))


def lookup(key: str):
    """A cached winner: this machine's cache first, then the table shipped
    with the package (winners of this autotuner on an MI355X)."""
    hit = _load_cache(cache_path()).get(key)
    if hit is None and os.environ.get("KC_TUNE_SHIPPED", "1") != "0":
        hit = _load_cache(SHIPPED).get(key)
    return hit


def size_class(nbytes: int) -> int:
    return int(math.log2(max(1, nbytes)))


def cache_key(op: int, signature: str) -> str:
    hip = getattr(torch.version, "hip", None) or "unknown"
    return f"{ARCH}|{hip}|{OP_NAMES[op]}|{signature}"


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, key: str, entry: dict) -> None:
    data = _load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def digest_tensors(*tensors) -> str:
    """SHA-256 of the bytes of device tensors (copied to the host)."""
    h = hashlib.sha256()
    for t in tensors:
        if t is None:
            h.update(b"none")
            continue
        h.update(t.detach().contiguous().view(torch.uint8).cpu().numpy().tobytes())
    return h.hexdigest()


def tune(ctx: kc.Context, op: int, run, digest=None, signature: str = "", candidates=None, reps: int = 3,
         use_cache: bool = True, prepare=None) -> dict:
    """Pick the fastest launch shape of ``op`` for ``run`` (a callable that
    issues the op once on the current stream).  ``digest`` (optional) returns
    a comparable summary of the outputs; ``prepare(cand)`` (optional) rebuilds
    state that depends on the shape (e.g. a pair set's tile table) and may
    return a replacement ``run``."""
    key = cache_key(op, signature)
    path = cache_path()
    if use_cache and signature:
        hit = lookup(key)
        if hit:
            best = hit["best"]
            ctx.set_tuning(op, **best)
            if prepare is not None:
                prepare(best)
            return dict(best=best, cached=True, table=hit.get("table", []))
    cands = candidates if candidates is not None else CANDIDATES[op]
    was_timing = getattr(ctx, "timing", False)
    ctx.enable_timing(True)
    table = []
    ref = None
    try:
        for cand in cands:
            ctx.set_tuning(op, **cand)
            fn = run
            if prepare is not None:
                r = prepare(cand)
                if r is not None:
                    fn = r
            fn()
            torch.cuda.synchronize()
            if digest is not None:
                d = digest()
                if ref is None:
                    ref = d
                elif d != ref:
                    raise TuningChangedResult(f"{OP_NAMES[op]}: candidate {cand} changed the outputs")
            times = []
            for _ in range(reps):
                fn()
                times.append(ctx.kernel_ms(op))
            table.append(dict(cand=cand, ms=min(times)))
    finally:
        ctx.enable_timing(was_timing)
    best = min(table, key=lambda e: e["ms"])["cand"]
    ctx.set_tuning(op, **best)
    if prepare is not None:
        prepare(best)
    entry = dict(best=best, table=table, when=time.strftime("%Y-%m-%dT%H:%M:%S"))
    if signature:
        _store_cache(path, key, entry)
    return dict(best=best, cached=False, table=table)
