"""Writes ``oracle_c1_small.json``: the oracle's outputs on the small c1
snapshot (1/64 scale) and two c1 compare pairs (1/64 scale).

Calls only the oracle and the seeded generators; nothing here touches the
HIP library.  Re-run it (and say why in the commit message) only when the
oracle's arithmetic changes for a reason the paper or a documented reading
justifies.

    python -m tests.golden.make_golden
"""
import hashlib
import json
import os

import numpy as np
import torch

import oracle
from paper_2605_03208_amd import workloads as W

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c1_small.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def compute() -> dict:
    case = W.c1_snapshot(scale=1 / 64)
    views = W.host_views(case.layout, case.arena.host_copy())
    rngs = [(b - W.SYNTH_BASE, s) for b, s in case.ranges()]  # VA-relative, base-independent
    rngs_abs = case.ranges()
    h, z, _ = oracle.page_hash(rngs_abs, views, seed=0)
    packed, va, n_kept = oracle.compact(rngs_abs, views, z)
    res, oob = oracle.closure_scan(rngs_abs, views, oob_cap=16)
    cmp = []
    for p in W.c1_compare(scale=1 / 64, n_pairs=2):
        cmp.append(oracle.compare(p.cand.view(torch.uint8).numpy(), p.gold.view(torch.uint8).numpy(),
                                  oracle.F32, 0))
    return dict(
        ranges_rel=rngs, synth_base=W.SYNTH_BASE, n_pages=int(len(h)),
        hash_sha256=digest(h), zero_bm_sha256=digest(z), n_kept=n_kept,
        packed_sha256=digest(packed), page_va_rel_sha256=digest(va - np.uint64(W.SYNTH_BASE)),
        closure=res, oob=[(a - W.SYNTH_BASE, v) for a, v in oob],
        compare=[{k: (v if k != "ulp_hist" else v[:45]) for k, v in c.items()} for c in cmp],
    )


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(compute(), f, indent=1, sort_keys=True)
    print("wrote", OUT)
