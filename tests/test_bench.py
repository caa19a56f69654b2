"""The benchmark's host-side contract: one-GPU refusal, the byte formulas the
GB/s figures divide by, and the kernel-source digest that ties stored counter
values to the code they were taken from."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_step_bytes_of_the_moe_pool():
    # 7,864,320 pages of which 209,715 are zero; both compare sides are the whole 30 GiB
    n_pages, n_kept, cmp_bytes = 7864320, 7864320 - 209715, 30 << 30
    b = bench.step_bytes(n_pages, n_kept, cmp_bytes)
    assert b["snapshot"] == 4096 * n_pages + 8 * n_pages + n_pages // 8 + 4104 * n_kept
    assert round(b["snapshot"] / 1e9, 2) == 63.69
    assert round(b["restore"] / 1e9, 2) == 63.63
    assert round(b["compare"] / 1e9, 2) == 64.42
    assert round(sum(b.values()) / 1e9, 2) == 191.74
    k = bench.kernel_bytes(n_pages, n_kept, cmp_bytes)
    assert k["restore"] == 8200 * n_kept and k["compare"] == b["compare"]


def test_source_digest_ignores_comments_not_code():
    csrc = os.path.join(ROOT, "paper_2605_03208_amd", "csrc")
    texts = {n: open(os.path.join(csrc, n), encoding="utf-8").read() for n in bench.STEP_KERNEL_SOURCES}
    base = bench.source_digest(lambda n: texts[n])
    assert base == bench.source_digest()
    name = "kc_snapshot.hip"
    commented = dict(texts)
    commented[name] = "// a new comment\n/* and a block\n   comment */\n" + texts[name].replace("\n", "\n  \n", 3)
    assert bench.source_digest(lambda n: commented[n]) == base
    changed = dict(texts)
    changed[name] = texts[name] + "\nstatic int kc_digest_probe = 1;\n"
    assert bench.source_digest(lambda n: changed[n]) != base
    for n in bench.STEP_KERNEL_SOURCES:  # every listed source takes part
        other = dict(texts)
        other[n] = texts[n] + "\n;\n"
        assert bench.source_digest(lambda m: other[m]) != base, n
