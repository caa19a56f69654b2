"""kc_compare_noalloc (the compare that allocates nothing) against kc_compare,
through the C ABI: two calls in a row, the second with fewer pairs, each
report bit-identical to kc_compare's on the same pairs; device memory free
before and after the second call is unchanged; more pairs than the static
scratch holds is refused before anything runs."""
import sys

import numpy as np
import pytest
import torch

from paper_2605_03208_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kc():
    from paper_2605_03208_amd import kc as K
    K.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return K


DTS = [W.DT_F32, W.DT_BF16, W.DT_F16, W.DT_FP8, W.DT_U8, W.DT_F64, W.DT_FP8_E5M2, W.DT_FP8_E4M3FNUZ,
       W.DT_I8, W.DT_I32, W.DT_I64]


def _pairs(n_pairs, seed):
    """Mixed element types and ragged sizes (empty pairs included), a few
    elements moved by 1-6 ULPs and candidate NaNs in the float types."""
    rng = np.random.default_rng(seed)
    gen = torch.Generator().manual_seed(seed)
    out = []
    for i in range(n_pairs):
        dt = DTS[i % len(DTS)]
        t = W.TORCH_DTYPE[dt]
        es = W.ELEM_SIZE[dt]
        n = 0 if i % 29 == 7 else int(rng.integers(1, 50_000))
        n = n - n % (16 // es) if n > 16 and i % 3 else n      # some tails, some whole 16-byte runs
        if t in W.INT_TYPES:
            gold = torch.randint(-1000, 1000, (n,), generator=gen, dtype=torch.int64).to(t)
        elif dt == W.DT_U8:
            gold = torch.randint(0, 256, (n,), generator=gen, dtype=torch.int64).to(torch.uint8)
        else:
            gold = torch.randn(n, generator=gen, dtype=torch.float64).to(t)
        gold = gold.cuda()
        n_nan = 0 if (t in W.INT_TYPES or dt == W.DT_U8 or n < 10) else int(rng.integers(0, 3))
        if dt == W.DT_U8:
            cand = gold.clone()
            if n:
                idx = torch.from_numpy(rng.choice(n, size=min(n, 5), replace=False)).cuda()
                cand[idx] ^= 0x5A
            out.append((cand, gold, dt, 0, 0.0, 0.0))
            continue
        pr = W.perturb_pair(gold, dt, rng, n // 500, 6, n_nan=n_nan, ulp_tol=int(rng.integers(0, 5)))
        out.append((pr.cand, pr.gold, dt, pr.ulp_tol, 1e-6 * (i % 2), 1e-3 * (i % 3)))
    return out


def test_noalloc_equals_compare_on_two_calls(kc):
    ctx = kc.Context(0)
    for call, (n_pairs, seed) in enumerate(((300, 11), (37, 12))):
        say(f"kc_compare_noalloc call {call + 1}: {n_pairs} mixed pairs vs kc_compare")
        pairs = _pairs(n_pairs, seed)
        want = kc.decode_cmp(kc.compare(ctx, pairs), n_pairs)
        res = torch.full((n_pairs * kc.RESULT_BYTES,), 0xEE, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        free_before, _ = torch.cuda.mem_get_info()
        kc.compare_noalloc(ctx, pairs, res)
        torch.cuda.synchronize()
        free_after, _ = torch.cuda.mem_get_info()
        got = kc.decode_cmp(res, n_pairs)
        assert got == want
        assert sum(r["n_mismatch_elems"] for r in got) > 0
        if call == 1:
            assert free_after == free_before
    say("kc_compare_noalloc: more pairs than the static scratch holds")
    z = torch.zeros(16, dtype=torch.uint8, device="cuda")
    too_many = [(z[:0], z[:0], W.DT_U8, 0)] * (kc.NOALLOC_MAX_PAIRS + 1)
    res = torch.empty(len(too_many) * kc.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(kc.KCError) as ei:
        kc.compare_noalloc(ctx, too_many, res)
    assert ei.value.code == kc.ELIMIT
    ctx.close()
