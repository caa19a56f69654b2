"""Snapshot files: what kc_snapshot_save writes equals the oracle's snapshot
byte for byte; kc_snapshot_load + kc_restore brings the original bytes back
at the same VAs (full and delta snapshots)."""
import json
import struct
import os
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


def _file(d, name, dtype=np.uint8):
    return np.fromfile(os.path.join(d, name), dtype=dtype)


@pytest.mark.parametrize("chunk", [0, 1 << 20, 4096 * 3])
def test_save_matches_oracle_and_reload_restores(kc, tmp_path, chunk):
    say(f"snapshot files c1 full, chunk={chunk}")
    ctx = kc.Context(0)
    case = W.c1_snapshot("cuda")
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    out = kc.snapshot(ctx, rs, seed=11)
    original = case.arena.buf.clone()
    d = str(tmp_path / "snap")
    st = kc.snapshot_save(ctx, rs, d, out, seed=11, chunk_bytes=chunk)
    host = case.arena.host_copy()
    views = W.host_views(case.layout, host)
    oh, oz, _ = oracle.page_hash(ranges, views, seed=11)
    op, ova, onk = oracle.compact(ranges, views, oz)
    assert np.array_equal(_file(d, "hash.bin", "<u8"), oh)
    assert np.array_equal(_file(d, "zero_bm.bin", "<u8"), oz)
    assert np.array_equal(_file(d, "page_va.bin", "<u8"), ova)
    assert np.array_equal(_file(d, "packed.bin"), op)
    assert not os.path.exists(os.path.join(d, "changed_bm.bin"))
    man = json.load(open(os.path.join(d, "manifest.json")))
    assert man["n_kept"] == onk == man["n_packed"] and man["n_pages"] == rs.n_pages and man["seed"] == 11
    assert [(int(r["base"], 16), r["size"]) for r in man["regions"]] == ranges
    assert st["bytes"] == 8 * rs.n_pages + 8 * rs.n_words + 8 * onk + PAGE * onk
    say("reload into fresh buffers, clobber, restore")
    back, _ = kc.snapshot_load(ctx, rs, d, chunk_bytes=chunk)
    case.arena.buf.fill_(0xA5)
    kc.restore(ctx, rs, back["zero_bm"], None, back["packed"], back["page_va"], back["n_kept"])
    torch.cuda.synchronize()
    for i in range(case.layout.n):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        assert torch.equal(case.arena.buf[o:o + s], original[o:o + s])
    assert torch.equal(back["hash"][: rs.n_pages], out["hash"][: rs.n_pages])
    rs.close()
    ctx.close()


def test_delta_files_and_errors(kc, tmp_path):
    say("snapshot files: delta chain on c2 scale 1/64, mismatched range set, small capacity")
    ctx = kc.Context(0)
    case = W.c2_snapshot("cuda", scale=1 / 64)
    ranges = case.ranges()
    rs = kc.RangeSet(ctx, ranges)
    s1 = kc.snapshot(ctx, rs, seed=2)
    base_img = case.arena.buf.clone()
    W.c2_rewrite(case)
    mutated = case.arena.buf.clone()
    s2 = kc.snapshot(ctx, rs, seed=2, prior=s1["hash"])
    d1, d2 = str(tmp_path / "base"), str(tmp_path / "delta")
    kc.snapshot_save(ctx, rs, d1, s1, seed=2, chunk_bytes=1 << 16)
    kc.snapshot_save(ctx, rs, d2, s2, seed=2, chunk_bytes=1 << 16)
    host = case.arena.host_copy()
    views = W.host_views(case.layout, host)
    _, oz, oc = oracle.page_hash(ranges, views, seed=2, prior=s1["hash"].cpu().numpy().view(np.uint64)[: rs.n_pages])
    op, ova, onk = oracle.compact(ranges, views, oz, oc)
    assert np.array_equal(_file(d2, "changed_bm.bin", "<u8"), oc)
    assert np.array_equal(_file(d2, "packed.bin"), op) and np.array_equal(_file(d2, "page_va.bin", "<u8"), ova)
    b1, _ = kc.snapshot_load(ctx, rs, d1)
    b2, _ = kc.snapshot_load(ctx, rs, d2, delta=True)
    case.arena.buf.fill_(0x5A)
    kc.restore(ctx, rs, b1["zero_bm"], None, b1["packed"], b1["page_va"], b1["n_kept"])
    torch.cuda.synchronize()
    for i in range(case.layout.n):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        assert torch.equal(case.arena.buf[o:o + s], base_img[o:o + s])
    kc.restore(ctx, rs, b2["zero_bm"], b2["changed_bm"], b2["packed"], b2["page_va"], b2["n_kept"])
    torch.cuda.synchronize()
    for i in range(case.layout.n):
        o, s = int(case.layout.offsets[i]), int(case.layout.sizes[i])
        assert torch.equal(case.arena.buf[o:o + s], mutated[o:o + s])
    other = kc.RangeSet(ctx, ranges[:-1])
    with pytest.raises(kc.KCError) as ei:
        kc.snapshot_load(ctx, other, d1)
    assert ei.value.code == kc.EINVAL
    with pytest.raises(kc.KCError) as ei:
        kc.snapshot_load(ctx, rs, d1, cap_pages=3)
    assert ei.value.code == kc.ELIMIT
    with pytest.raises(kc.KCError) as ei:
        kc.snapshot_load(ctx, rs, d2)          # delta needs a changed bitmap buffer
    assert ei.value.code == kc.EINVAL
    say("snapshot files: a snapshot saved below its kept count is refused on load")
    d3 = str(tmp_path / "truncated")
    nk1 = int(s1["n_kept"].item())
    kc.snapshot_save(ctx, rs, d3, s1, seed=2, cap_pages=nk1 // 2)
    man = json.load(open(os.path.join(d3, "manifest.json")))
    assert man["n_kept"] == nk1 and man["n_packed"] == nk1 // 2
    assert np.array_equal(_file(d3, "page_va.bin", "<u8"), _file(d1, "page_va.bin", "<u8")[: nk1 // 2])
    with pytest.raises(kc.KCError) as ei:
        kc.snapshot_load(ctx, rs, d3)
    assert ei.value.code == kc.ELIMIT
    say("snapshot files: a header whose packed count exceeds its kept count is refused")
    hdr = bytearray(open(os.path.join(d1, "header.bin"), "rb").read())
    d4 = str(tmp_path / "bad_header")
    os.makedirs(d4)
    for name in os.listdir(d1):
        with open(os.path.join(d1, name), "rb") as fi, open(os.path.join(d4, name), "wb") as fo:
            fo.write(fi.read())
    fields = list(struct.unpack("<8s2I5Q2I", bytes(hdr[:64])))   # magic, version, page size, seed, ranges,
    fields[7] = fields[6] + 1                                    # pages, kept, packed, delta: packed = kept + 1
    open(os.path.join(d4, "header.bin"), "wb").write(struct.pack("<8s2I5Q2I", *fields))
    with pytest.raises(kc.KCError) as ei:
        kc.snapshot_load(ctx, rs, d4)
    assert ei.value.code == kc.EINVAL
    other.close()
    rs.close()
    ctx.close()
