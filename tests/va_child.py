"""Two processes of a VA-faithful capture and replay, run by
``tests/test_gpu_vaspace.py`` (not a test module itself).

``capture DIR``: build seeded ranges holding data and pointers into each
other at whatever VAs this process's allocator gives, snapshot them, save the
snapshot to DIR with the raw bytes, the closure-scan result and the pointer
graph.

``replay DIR``: in a fresh process, map device memory at exactly the saved
VAs before anything else allocates (exit 3 if a range cannot be placed there),
load the snapshot, restore it, and check the restored state byte for byte and
by its hashes, closure scan and pointer graph.  Prints one JSON line."""
import json
import os
import sys

import numpy as np


def raw_view(torch, base, size):
    class Mem:   # a device address range as a torch tensor, without copying
        __cuda_array_interface__ = {"shape": (size,), "typestr": "|u1", "data": (base, False), "version": 2}
    return torch.as_tensor(Mem(), device="cuda")


def capture(d):
    import torch
    from paper_2605_03208_amd import kc, workloads as W
    case = W.graph_case("cuda", n_ranges=40, seed=77, max_pages=32)
    ranges = case.ranges()
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, ranges)
    scan = kc.ScanOut("cuda", oob_cap=64)
    out = kc.snapshot(ctx, rs, scan=scan)
    torch.cuda.synchronize()
    kc.snapshot_save(ctx, rs, d, out)
    edge = kc.pointer_graph(ctx, rs).cpu().numpy().view(np.uint64)
    host = case.arena.host_copy()
    np.concatenate(W.host_views(case.layout, host)).tofile(os.path.join(d, "raw.bin"))
    res, oob = scan.result()
    info = dict(ranges=ranges, scan=res, oob=oob, n_kept=int(out["n_kept"].item()),
                edges=[int(x) for x in edge.reshape(-1)])
    with open(os.path.join(d, "capture.json"), "w") as f:
        json.dump(info, f)
    probe = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")   # where this allocator goes next
    print(json.dumps({"captured": len(ranges), "n_kept": info["n_kept"], "n_in_range": res["n_in_range"],
                      "lowest": hex(ranges[0][0]), "highest_end": hex(ranges[-1][0] + ranges[-1][1]),
                      "next_allocation": hex(probe.data_ptr())}))
    return 0


def replay(d):
    with open(os.path.join(d, "capture.json")) as f:
        info = json.load(f)
    ranges = [tuple(r) for r in info["ranges"]]
    import torch
    from paper_2605_03208_amd import kc
    try:
        vs = kc.VaSpace(0, ranges)          # the first device allocation of this process
    except kc.KCError as e:
        if e.code == kc.ERELOC:
            probe = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
            print(json.dumps({"relocated": str(e), "first_allocation_here": hex(probe.data_ptr())}), flush=True)
            return 3
        raise
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, ranges)
    gold, _ = kc.snapshot_load(ctx, rs, d)
    kc.restore(ctx, rs, gold["zero_bm"], None, gold["packed"], gold["page_va"], gold["n_kept"])
    diff = kc.decode_region_diff(kc.region_diff(ctx, rs, gold)["res"], len(ranges))
    scan = kc.ScanOut("cuda", oob_cap=64)
    again = kc.snapshot(ctx, rs, scan=scan)
    edge = kc.pointer_graph(ctx, rs).cpu().numpy().view(np.uint64)
    torch.cuda.synchronize()
    res, oob = scan.result()
    raw = np.fromfile(os.path.join(d, "raw.bin"), dtype=np.uint8)
    try:
        live = np.concatenate([raw_view(torch, b, s).cpu().numpy() for b, s in ranges])
        bytes_equal = bool(np.array_equal(live, raw))
    except (TypeError, RuntimeError, ValueError) as e:   # no foreign-pointer import in this torch
        print(json.dumps({"bytes_check_unavailable": str(e)}), flush=True)
        bytes_equal = None
    checks = {
        "bytes_equal": bytes_equal,
        "no_region_diff": all(r["n_diff_bytes"] == 0 and r["n_bad_pages"] == 0 for r in diff),
        "hash_equal": bool(torch.equal(again["hash"], gold["hash"])),
        "scan_equal": res == info["scan"] and [list(x) for x in oob] == info["oob"],
        "graph_equal": [int(x) for x in edge.reshape(-1)] == info["edges"],
    }
    rs.close()
    ctx.close()
    vs.close()
    print(json.dumps({"spans": vs.n_spans, "mapped_bytes": vs.mapped_bytes, **checks}), flush=True)
    return 0 if all(v is not False for v in checks.values()) else 1


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    mode, directory = sys.argv[1], sys.argv[2]
    sys.exit(capture(directory) if mode == "capture" else replay(directory))
