"""Two processes of a VA-faithful capture and replay, run by
``tests/test_gpu_vaspace.py`` (not a test module itself).

``capture DIR``: map the tracked memory at an address the runtime offers,
fill seeded ranges with data and pointers into each other, snapshot them, and
save the snapshot to DIR with the raw bytes, the closure-scan result and the
pointer graph.

``replay DIR``: in a fresh process, map device memory at exactly the saved
VAs before anything else allocates (exit 3 if a range cannot be placed there),
load the snapshot, restore it, read the restored bytes back, and snapshot,
scan and graph the restored state again.  Everything the replay computed is
written to DIR (``replay.npz``, ``replay.json``), so the test can hold it
against the oracle run on the generator's raw bytes.  Prints one JSON line."""
import json
import os
import sys

import numpy as np


def raw_view(torch, base, size):
    class Mem:   # a device address range as a torch tensor, without copying
        __cuda_array_interface__ = {"shape": (size,), "typestr": "|u1", "data": (base, False), "version": 2}
    return torch.as_tensor(Mem(), device="cuda")


def read_device(base, size):
    """Host copy of ``size`` bytes at device address ``base`` through the HIP
    runtime's own synchronous copy (no torch wrapping of a foreign pointer)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(size, dtype=np.uint8)
    rc = hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(base), size, 2)   # 2 = device to host
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")
    return out


def capture(d):
    """The tracked memory is mapped at an address the runtime offers for it
    (kc_vaspace_suggest), filled with seeded bytes and pointers between the
    ranges, snapshotted and saved."""
    import torch
    from paper_2605_03208_amd import kc, workloads as W
    page = 4096
    rng = np.random.default_rng(77)
    sizes = rng.integers(1, 33, size=40) * page
    sizes[::9] -= rng.integers(1, page, size=len(sizes[::9]))      # a few partial last pages
    lay = W.make_layout(rng, sizes, gap_pages=(1, 8))
    total = (lay.arena_bytes + page - 1) // page * page
    base = kc.vaspace_suggest(0, total)
    vs = kc.VaSpace(0, [(base, total)])                            # the capture's tracked memory
    ranges = lay.ranges(base)
    host = np.zeros(total, dtype=np.uint8)
    n_ptr = 0
    for (o, s) in zip(lay.offsets, lay.sizes):
        o, s = int(o), int(s)
        host[o:o + s] = rng.integers(0, 256, size=s, dtype=np.uint8)
        for p in range((s + page - 1) // page):
            if rng.random() < 0.15:
                host[o + p * page: min(o + (p + 1) * page, o + s)] = 0
        for w in np.flatnonzero(rng.random(s // 8) < 0.005):
            b, bs = ranges[int(rng.integers(0, len(ranges)))]
            host[o + 8 * int(w): o + 8 * int(w) + 8] = np.frombuffer(
                np.uint64(b + int(rng.integers(0, bs))).tobytes(), dtype=np.uint8)
            n_ptr += 1
    raw_view(torch, base, total).copy_(torch.from_numpy(host).cuda())
    ctx = kc.Context(0)
    rs = kc.RangeSet(ctx, ranges)
    scan = kc.ScanOut("cuda", oob_cap=64)
    out = kc.snapshot(ctx, rs, scan=scan)
    torch.cuda.synchronize()
    kc.snapshot_save(ctx, rs, d, out)
    edge = kc.pointer_graph(ctx, rs).cpu().numpy().view(np.uint64)
    np.concatenate([host[int(o): int(o) + int(s)] for o, s in zip(lay.offsets, lay.sizes)]).tofile(
        os.path.join(d, "raw.bin"))
    res, oob = scan.result()
    info = dict(ranges=ranges, scan=res, oob=oob, n_kept=int(out["n_kept"].item()),
                edges=[int(x) for x in edge.reshape(-1)])
    with open(os.path.join(d, "capture.json"), "w") as f:
        json.dump(info, f)
    print(json.dumps({"captured": len(ranges), "at": hex(base), "bytes": total, "n_kept": info["n_kept"],
                      "pointers_planted": n_ptr, "n_in_range": res["n_in_range"]}))
    rs.close()
    ctx.close()
    vs.close()
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
    live = np.concatenate([read_device(b, s) for b, s in ranges])
    n_kept = int(again["n_kept"].item())
    u64 = lambda t: t.detach().cpu().numpy().view(np.uint64)
    np.savez(os.path.join(d, "replay.npz"), live=live, hash=u64(again["hash"])[: rs.n_pages],
             zero_bm=u64(again["zero_bm"])[: rs.n_words], page_va=u64(again["page_va"])[:n_kept],
             packed=again["packed"][: n_kept * 4096].cpu().numpy(), n_kept=np.array([n_kept], dtype=np.uint64),
             edges=edge.reshape(-1))
    with open(os.path.join(d, "replay.json"), "w") as f:
        json.dump({"scan": res, "oob": [list(x) for x in oob]}, f)
    checks = {
        "bytes_equal": bool(np.array_equal(live, raw)),
        "no_region_diff": all(r["n_diff_bytes"] == 0 and r["n_bad_pages"] == 0 for r in diff),
    }
    rs.close()
    ctx.close()
    vs.close()
    print(json.dumps({"spans": vs.n_spans, "mapped_bytes": vs.mapped_bytes, **checks}), flush=True)
    return 0 if all(checks.values()) else 1


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    mode, directory = sys.argv[1], sys.argv[2]
    sys.exit(capture(directory) if mode == "capture" else replay(directory))
