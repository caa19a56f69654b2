"""Seeded synthetic inputs for the snapshot / validation hot path.

This module holds none of the method's arithmetic (no hashing, zero tests,
prefix scans, pointer-range tests or ULP distances).  It draws layouts (range
sizes, gaps), contents (random bytes, normal floats, int8-quantised blocks),
injects pointer words and perturbations, and records what it injected.  Both
the HIP path and the CPU oracle consume these inputs; neither is imported
here.

The workloads stand in for the paper's captures (Table 2: 10-186 regions,
152 MB - 30 GB; the vLLM MoE capture of Sec. 5.2 with 24 x 702 MB +
24 x 330 MB expert tensors plus activations) and for the outputs a tuning
agent would validate; no dataset or model is involved.

Layout rule shared by all size laws: draw the law, rescale the unclamped
items until the sizes sum to the requested total, clamp to [lo, hi], round
to the alignment, and put the rounding residual on the largest item.
Perturbations by k ULP are k applications of the library ``nextafter``
(fp32 / bf16 / fp16) or k steps through the value-sorted table of the 254
non-NaN fp8-e4m3fn codes (decoded by torch).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

PAGE = 4096
KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30
SYNTH_BASE = 0x7F8A00000000  # synthetic arena VA for CPU-only runs

DT_F32, DT_BF16, DT_F16, DT_FP8, DT_U8 = 0, 1, 2, 3, 4
DT_F64, DT_FP8_E4M3FNUZ, DT_FP8_E5M2, DT_FP8_E5M2FNUZ = 5, 6, 7, 8
DT_I8, DT_I16, DT_I32, DT_I64 = 9, 10, 11, 12
TORCH_DTYPE = {DT_F32: torch.float32, DT_BF16: torch.bfloat16, DT_F16: torch.float16,
               DT_FP8: torch.float8_e4m3fn, DT_U8: torch.uint8, DT_F64: torch.float64,
               DT_FP8_E4M3FNUZ: torch.float8_e4m3fnuz, DT_FP8_E5M2: torch.float8_e5m2,
               DT_FP8_E5M2FNUZ: torch.float8_e5m2fnuz, DT_I8: torch.int8, DT_I16: torch.int16,
               DT_I32: torch.int32, DT_I64: torch.int64}
ELEM_SIZE = {dt: torch.empty(0, dtype=t).element_size() for dt, t in TORCH_DTYPE.items()}
FP8_TYPES = (torch.float8_e4m3fn, torch.float8_e4m3fnuz, torch.float8_e5m2, torch.float8_e5m2fnuz)
INT_TYPES = (torch.int8, torch.int16, torch.int32, torch.int64)
# one NaN encoding per fp8 format (E4M3FN: S.1111.111; E5M2: exponent 31 with a
# non-zero mantissa; the FNUZ formats: 0x80, their only NaN)
FP8_NAN = {torch.float8_e4m3fn: 0x7F, torch.float8_e4m3fnuz: 0x80, torch.float8_e5m2: 0x7E,
           torch.float8_e5m2fnuz: 0x80}


# --------------------------------------------------------------------------
# size laws
# --------------------------------------------------------------------------

def fit_sizes(raw: np.ndarray, lo: int, hi: int, total: int, align: int) -> np.ndarray:
    """Scale ``raw`` so it sums to ``total`` with every item in [lo, hi],
    multiples of ``align``; the residual goes on the largest item."""
    n = len(raw)
    if n * lo > total or n * hi < total:
        raise ValueError("total not reachable with n items in [lo, hi]")
    x = raw.astype(np.float64).copy()
    clamped = np.zeros(n, dtype=bool)
    for _ in range(64):
        free = ~clamped
        fixed = np.clip(x[clamped], lo, hi).sum()
        s = x[free].sum()
        if s <= 0:
            break
        x[free] *= (total - fixed) / s
        newly = free & ((x < lo) | (x > hi))
        x = np.clip(x, lo, hi)
        if not newly.any():
            break
        clamped |= newly
    sizes = np.maximum(lo, np.minimum(hi, (np.round(x / align) * align))).astype(np.int64)
    resid = total - int(sizes.sum())
    order = np.argsort(-sizes, kind="stable")
    for i in order:  # push the residual into the largest items that can take it
        if resid == 0:
            break
        if resid > 0:
            step = min(resid, hi - int(sizes[i]))
        else:
            step = max(resid, lo - int(sizes[i]))
        sizes[i] += step
        resid -= step
    if resid != 0:
        sizes[order[0]] += resid
    assert int(sizes.sum()) == total and (sizes % align == 0).all()
    return sizes


def loguniform(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))


def pareto(rng: np.random.Generator, n: int, alpha: float, lo: float) -> np.ndarray:
    return lo * (1.0 + rng.pareto(alpha, size=n))


# --------------------------------------------------------------------------
# layouts and arenas
# --------------------------------------------------------------------------

@dataclass
class Layout:
    sizes: np.ndarray          # bytes per range (int64)
    offsets: np.ndarray        # byte offset of each range inside the arena
    arena_bytes: int

    @property
    def n(self) -> int:
        return len(self.sizes)

    @property
    def total(self) -> int:
        return int(self.sizes.sum())

    @property
    def n_pages(self) -> int:
        return int(((self.sizes + PAGE - 1) // PAGE).sum())   # a partial last page counts

    def cum(self) -> np.ndarray:
        """Start of each range in range-concatenated byte space."""
        return np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)

    def ranges(self, va_base: int):
        return [(va_base + int(o), int(s)) for o, s in zip(self.offsets, self.sizes)]


def make_layout(rng: np.random.Generator, sizes: np.ndarray, gap_pages=(1, 16)) -> Layout:
    gaps = rng.integers(gap_pages[0], gap_pages[1] + 1, size=len(sizes) + 1) * PAGE
    offsets = np.zeros(len(sizes), dtype=np.int64)
    pos = int(gaps[0])
    for i, s in enumerate(sizes):
        offsets[i] = pos
        pos += (int(s) + PAGE - 1) // PAGE * PAGE + int(gaps[i + 1])   # every range starts on a page
    return Layout(np.asarray(sizes, dtype=np.int64), offsets, pos)


class Arena:
    """One byte buffer holding every range at its layout offset.

    ``va_base`` is the address the ranges are reported at: the real device
    address of the (4 KiB aligned) buffer on a GPU, or ``SYNTH_BASE`` on the
    CPU, where ``buf`` is only a host stand-in for device memory."""

    def __init__(self, layout: Layout, device="cpu", fill_zero: bool = True):
        self.layout = layout
        self.device = torch.device(device)
        alloc = torch.zeros if fill_zero else torch.empty
        raw = alloc(layout.arena_bytes + PAGE, dtype=torch.uint8, device=self.device)
        shift = (-raw.data_ptr()) % PAGE
        self._raw = raw
        self.buf = raw[shift: shift + layout.arena_bytes]
        self.va_base = self.buf.data_ptr() if self.device.type == "cuda" else SYNTH_BASE

    def view(self, i: int) -> torch.Tensor:
        o, s = int(self.layout.offsets[i]), int(self.layout.sizes[i])
        return self.buf[o: o + s]

    def ranges(self):
        return self.layout.ranges(self.va_base)

    def load_concat(self, content: np.ndarray) -> None:
        """Copy range-concatenated host bytes into the ranges."""
        cum = self.layout.cum()
        src = torch.from_numpy(content)
        for i in range(self.layout.n):
            self.view(i).copy_(src[cum[i]: cum[i + 1]], non_blocking=False)

    def host_copy(self) -> np.ndarray:
        """Whole arena as a host numpy array (a D2H copy on a GPU)."""
        return self.buf.cpu().numpy() if self.device.type == "cuda" else self.buf.numpy()


def host_views(layout: Layout, host: np.ndarray):
    """Per-range contiguous uint8 views into a host copy of an arena."""
    return [host[int(o): int(o) + int(s)] for o, s in zip(layout.offsets, layout.sizes)]


# --------------------------------------------------------------------------
# c1: small plain snapshot (64 MiB, 48 allocations) + 16 fp32 compare pairs
# --------------------------------------------------------------------------

@dataclass
class SnapshotCase:
    name: str
    arena: Arena
    truth: dict = field(default_factory=dict)

    @property
    def layout(self) -> Layout:
        return self.arena.layout

    def ranges(self):
        return self.arena.ranges()


def c1_layout(scale: float = 1.0, seed: int = 1):
    rng = np.random.default_rng(seed)
    n = 48
    total_pages = max(n, int(round(16384 * scale)))
    hi = min(8 * MiB, max(PAGE, (total_pages * PAGE) // 4) // PAGE * PAGE)
    hi = max(hi, -(-total_pages // n) * PAGE)
    raw = loguniform(rng, n, 4 * KiB, 8 * MiB)
    sizes = fit_sizes(raw, PAGE, hi, total_pages * PAGE, PAGE)
    return rng, make_layout(rng, sizes)


def c1_snapshot(device="cpu", scale: float = 1.0, seed: int = 1) -> SnapshotCase:
    """48 ranges, uniform random bytes, 30 % of pages zero, 1 % of aligned
    words overwritten with pointers into the ranges, plus 3 out-of-range
    pointers (max_end, min_base - 8, middle of the largest gap)."""
    rng, lay = c1_layout(scale, seed)
    arena = Arena(lay, device)
    ranges = arena.ranges()
    N = lay.n_pages
    content = rng.integers(0, 256, size=lay.total, dtype=np.uint8)
    zero_pages = np.sort(rng.choice(N, size=int(round(0.3 * N)), replace=False))
    pages = content.reshape(N, PAGE)
    pages[zero_pages] = 0
    nonzero = np.setdiff1d(np.arange(N), zero_pages)
    n_ptr = int(round(0.01 * N * (PAGE // 8)))
    # candidate words: word w of non-zero page p  ->  global word p*512 + w
    picks = rng.choice(len(nonzero) * (PAGE // 8), size=n_ptr + 3, replace=False)
    words_pos = nonzero[picks // (PAGE // 8)] * (PAGE // 8) + picks % (PAGE // 8)
    ptr_pos, oob_pos = words_pos[:n_ptr], words_pos[n_ptr:]
    tgt = rng.integers(0, lay.n, size=n_ptr)
    off = (rng.random(n_ptr) * lay.sizes[tgt]).astype(np.int64)
    bases = np.array([b for b, _ in ranges], dtype=np.uint64)
    ptr_val = bases[tgt] + off.astype(np.uint64)
    min_base = ranges[0][0]
    max_end = ranges[-1][0] + ranges[-1][1]
    gap_lo = np.array([ranges[i][0] + ranges[i][1] for i in range(lay.n - 1)], dtype=np.int64)
    gap_len = np.array([ranges[i + 1][0] for i in range(lay.n - 1)], dtype=np.int64) - gap_lo
    if lay.n > 1:
        j = int(np.argmax(gap_len))
        in_gap = int(gap_lo[j] + (gap_len[j] // 2) // 8 * 8)
    else:
        in_gap = max_end + 2 * MiB
    oob_val = np.array([max_end, min_base - 8, in_gap], dtype=np.uint64)
    w = content.view(np.uint64)
    w[ptr_pos] = ptr_val
    w[oob_pos] = oob_val
    arena.load_concat(content)
    truth = dict(zero_pages=zero_pages, ptr_pos=ptr_pos, ptr_val=ptr_val, oob_pos=oob_pos,
                 oob_val=oob_val, n_pages=N)
    return SnapshotCase("c1", arena, truth)


# --------------------------------------------------------------------------
# ragged ranges: sizes that are not multiples of the page
# --------------------------------------------------------------------------

SENTINEL = 0xA5


def ragged_case(device="cpu", n_ranges: int = 40, seed: int = 9, max_bytes: int = 9 * PAGE + 123) -> SnapshotCase:
    """Ranges of arbitrary byte sizes (a few whole-page sizes, a few under
    16 bytes) on page-aligned bases, 0-3 pages apart.  Every byte of the arena
    outside the ranges (the rest of each partial last page, the gaps) holds
    ``SENTINEL``; range bytes are random, with about a fifth of the pages (or
    partial pages) zeroed and about 0.2 % of the words wholly inside a range
    set to addresses inside some range.  ``truth['ptr']`` lists those planted
    (range, byte offset, value) words."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, max_bytes + 1, size=n_ranges)
    sizes[::7] = (sizes[::7] + PAGE - 1) // PAGE * PAGE
    sizes[1::11] = rng.integers(1, 16, size=len(sizes[1::11]))
    lay = make_layout(rng, sizes, gap_pages=(0, 3))
    arena = Arena(lay, device)
    arena.buf.fill_(SENTINEL)
    ranges = arena.ranges()
    content = rng.integers(0, 256, size=lay.total, dtype=np.uint8)
    cum = lay.cum()
    for a in range(n_ranges):   # zero about a fifth of each range's pages (partial ones included)
        for p in range((int(sizes[a]) + PAGE - 1) // PAGE):
            if rng.random() < 0.2:
                lo = int(cum[a]) + p * PAGE
                content[lo:min(lo + PAGE, int(cum[a + 1]))] = 0
    ptr = []
    for a in range(n_ranges):
        n_words = int(sizes[a]) // 8
        for w in np.flatnonzero(rng.random(n_words) < 0.002):
            b = int(rng.integers(0, n_ranges))
            v = ranges[b][0] + int(rng.integers(0, int(sizes[b])))
            content[int(cum[a]) + 8 * int(w): int(cum[a]) + 8 * int(w) + 8] = np.frombuffer(
                np.uint64(v).tobytes(), dtype=np.uint8)
            ptr.append((a, 8 * int(w), v))
    arena.load_concat(content)
    return SnapshotCase("ragged", arena, dict(ptr=ptr, sentinel=SENTINEL))


def units_case(device="cpu", unit: int = 64 * KiB, n_ranges: int = 24, seed: int = 21,
               max_units: int = 5) -> SnapshotCase:
    """Ranges for hash units larger than the page: byte sizes up to
    ``max_units`` units (a few whole multiples of the unit, a few under one
    unit), on page-aligned bases 0-3 pages apart, gaps filled with
    ``SENTINEL``.  About a quarter of the units (partial ones included) are
    all zero, a few more have only their first 4 KiB page zero (so a probe of
    the first bytes alone would misjudge them), and about 0.2 % of the words
    wholly inside a range hold addresses inside some range."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, max_units * unit + 1, size=n_ranges)
    sizes[::5] = (sizes[::5] + unit - 1) // unit * unit
    sizes[2::7] = rng.integers(1, PAGE, size=len(sizes[2::7]))
    lay = make_layout(rng, sizes, gap_pages=(0, 3))
    arena = Arena(lay, device)
    arena.buf.fill_(SENTINEL)
    ranges = arena.ranges()
    content = rng.integers(0, 256, size=lay.total, dtype=np.uint8)
    cum = lay.cum()
    for a in range(n_ranges):   # pointers first: the zeroing below clears those in zeroed units
        for w in np.flatnonzero(rng.random(int(sizes[a]) // 8) < 0.002):
            b = int(rng.integers(0, n_ranges))
            v = ranges[b][0] + int(rng.integers(0, int(sizes[b])))
            content[int(cum[a]) + 8 * int(w): int(cum[a]) + 8 * int(w) + 8] = np.frombuffer(
                np.uint64(v).tobytes(), dtype=np.uint8)
    for a in range(n_ranges):
        for u in range((int(sizes[a]) + unit - 1) // unit):
            lo = int(cum[a]) + u * unit
            hi = min(lo + unit, int(cum[a + 1]))
            r = rng.random()
            if r < 0.25:
                content[lo:hi] = 0
            elif r < 0.35:
                content[lo:min(lo + PAGE, hi)] = 0
    arena.load_concat(content)
    return SnapshotCase("units", arena, dict(unit=unit, sentinel=SENTINEL))


# --------------------------------------------------------------------------
# pointer graphs: a planted sparse digraph between ranges
# --------------------------------------------------------------------------

def graph_case(device="cpu", n_ranges: int = 64, seed: int = 5, mean_out: float = 1.5,
               max_pages: int = 24) -> SnapshotCase:
    """Ranges of 1..max_pages pages holding N(0,1) fp32 data (never
    pointer-like), a few zero pages, and a random digraph planted as pointer
    words: for each edge a -> b, 1..3 aligned words of range a hold addresses
    anywhere inside range b (first and last byte included).  One range also
    holds a whole page of pointers into three targets.  Out-of-range
    pointer-like values (range ends, gap middles) are planted too and make no
    edge.  ``truth['edges']`` is the planted edge set, ``truth['plants']`` the
    planted (source, target, value) words; ``truth['root_words']``
    imitates a kernel-argument block: addresses into two root ranges mixed with
    scalars and one out-of-range pointer."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, max_pages + 1, size=n_ranges) * PAGE
    lay = make_layout(rng, sizes, gap_pages=(1, 8))
    arena = Arena(lay, device)
    ranges = arena.ranges()
    bases = np.array([b for b, _ in ranges], dtype=np.uint64)
    ends = bases + lay.sizes.astype(np.uint64)
    gen = torch.Generator().manual_seed(seed)
    content = torch.randn(lay.total // 4, generator=gen).numpy().view(np.uint8).copy()
    w = content.view(np.uint64)
    cum_w = lay.cum() // 8
    N = lay.n_pages
    zero_pages = rng.choice(N, size=N // 10, replace=False)
    content.reshape(N, PAGE)[zero_pages] = 0
    taken = set()

    def free_word(a):  # an unused aligned word of range a
        while True:
            x = int(cum_w[a] + rng.integers(0, lay.sizes[a] // 8))
            if x not in taken:
                taken.add(x)
                return x

    def addr_in(b):
        off = int(rng.integers(0, lay.sizes[b]))
        off = (0, int(lay.sizes[b]) - 1, off)[int(rng.integers(0, 3))]
        return int(bases[b]) + off

    edges, plants = set(), []
    for a in range(n_ranges):
        for b in rng.choice(n_ranges, size=min(n_ranges, rng.poisson(mean_out)), replace=False):
            edges.add((a, int(b)))
            for _ in range(int(rng.integers(1, 4))):
                v = addr_in(int(b))
                w[free_word(a)] = v
                plants.append((a, int(b), v))
    # a page-sized pointer array in one range, three targets
    a = int(np.argmax(lay.sizes))
    tg = rng.choice(n_ranges, size=min(3, n_ranges), replace=False)
    p0 = int(cum_w[a])
    for j in range(PAGE // 8):
        if p0 + j not in taken:
            taken.add(p0 + j)
            b = int(tg[j % len(tg)])
            v = addr_in(b)
            w[p0 + j] = v
            plants.append((a, b, v))
            edges.add((a, b))
    # pointer-like values outside every range: no edge
    gaps = [int(ends[i]) + (int(bases[i + 1]) - int(ends[i])) // 2 for i in range(n_ranges - 1)]
    oob_vals = [int(ends[-1]), int(bases[0]) - 8] + gaps[:8] + [int(ends[i]) for i in range(min(8, n_ranges))]
    for v in oob_vals:
        w[free_word(int(rng.integers(0, n_ranges)))] = v
    arena.load_concat(content)
    roots = rng.choice(n_ranges, size=min(2, n_ranges), replace=False)
    root_words = np.array([addr_in(int(roots[0])), 42, 0x3FF0000000000000, addr_in(int(roots[-1])),
                           int(ends[-1]) + PAGE, 0], dtype=np.uint64)
    truth = dict(edges=edges, plants=plants, oob_vals=oob_vals, roots=[int(r) for r in roots],
                 root_words=root_words)
    return SnapshotCase("graph", arena, truth)


# --------------------------------------------------------------------------
# perturbation by k ULP (library nextafter / sorted fp8 code table)
# --------------------------------------------------------------------------

_FP8_TABLES = {}


def _fp8_tables(tdtype=torch.float8_e4m3fn):
    """Codes of an fp8 format sorted by their torch-decoded value (NaNs left
    out, -0 sharing the rank of +0), and the rank of every code (-1: NaN)."""
    if tdtype not in _FP8_TABLES:
        codes = torch.arange(256, dtype=torch.uint8)
        vals = codes.view(tdtype).to(torch.float32)
        keep = [c for c in range(256) if not math.isnan(vals[c].item())
                and not (vals[c].item() == 0.0 and c != 0)]
        order = sorted(keep, key=lambda c: vals[c].item())
        code_of_rank = torch.tensor(order, dtype=torch.uint8)
        rank_of_code = torch.full((256,), -1, dtype=torch.int64)
        for r, c in enumerate(order):
            rank_of_code[c] = r
        for c in range(256):  # -0 sits where +0 does
            if vals[c].item() == 0.0:
                rank_of_code[c] = rank_of_code[0]
        _FP8_TABLES[tdtype] = (code_of_rank, rank_of_code)
    return _FP8_TABLES[tdtype]


def step_ulps(vals: torch.Tensor, k: torch.Tensor) -> torch.Tensor:
    """Move each element |k| representable values toward sign(k) * inf
    (CPU tensors).  fp32/bf16/fp16 use ``torch.nextafter``."""
    k = k.to(torch.int64)
    if vals.dtype in FP8_TYPES:
        code_of_rank, rank_of_code = _fp8_tables(vals.dtype)
        r = rank_of_code[vals.view(torch.uint8).to(torch.int64)] + k
        r = r.clamp(0, len(code_of_rank) - 1)
        return code_of_rank[r].view(vals.dtype)
    if vals.dtype in INT_TYPES:  # integers: one step is one unit
        info = torch.iinfo(vals.dtype)
        return (vals.to(torch.int64) + k).clamp(info.min, info.max).to(vals.dtype)
    out = vals.clone()
    up = torch.full_like(out, float("inf"))
    down = torch.full_like(out, float("-inf"))
    target = torch.where(k > 0, up, down)
    for i in range(int(k.abs().max().item()) if k.numel() else 0):
        step = k.abs() > i
        out = torch.where(step, torch.nextafter(out, target), out)
    return out


@dataclass
class ComparePair:
    gold: torch.Tensor          # typed tensor (device)
    cand: torch.Tensor
    dtype: int
    ulp_tol: int
    pos: np.ndarray             # perturbed element positions (sorted)
    k: np.ndarray               # signed ULP steps at those positions
    nan_pos: np.ndarray         # candidate-only NaN positions


def perturb_pair(gold: torch.Tensor, dtype: int, rng: np.random.Generator, n_pert: int,
                 kmax: int, n_nan: int = 0, ulp_tol: int = 0) -> ComparePair:
    n = gold.numel()
    n_pert = min(n_pert, n)
    n_nan = min(n_nan, n - n_pert)
    pick = rng.choice(n, size=n_pert + n_nan, replace=False) if n_pert + n_nan else np.zeros(0, np.int64)
    pos = np.sort(pick[:n_pert])
    nan_pos = np.sort(pick[n_pert:])
    k = rng.integers(1, kmax + 1, size=n_pert) * np.where(rng.random(n_pert) < 0.5, -1, 1)
    cand = gold.clone()
    if n_pert:
        idx = torch.from_numpy(pos).to(gold.device)
        moved = step_ulps(gold[idx].cpu(), torch.from_numpy(k)).to(gold.device)
        cand[idx] = moved
    if n_nan:
        idx = torch.from_numpy(nan_pos).to(gold.device)
        if gold.dtype in FP8_TYPES:
            cand.view(torch.uint8)[idx] = FP8_NAN[gold.dtype]
        elif gold.dtype in INT_TYPES:
            raise ValueError("integers have no NaN")
        else:
            cand[idx] = float("nan")
    return ComparePair(gold, cand, dtype, ulp_tol, pos, k, nan_pos)


def c1_compare(device="cpu", scale: float = 1.0, seed: int = 1, n_pairs: int = 16):
    """16 fp32 pairs of 2^20 elements, gold N(0,1), 0.1 % of elements moved by
    1-4 ULP, two candidate-only quiet NaNs per buffer, tolerance 0."""
    rng = np.random.default_rng(seed + 1000)
    gen = torch.Generator(device=device).manual_seed(seed)
    n = max(64, int(round((1 << 20) * scale)))
    pairs = []
    for _ in range(n_pairs):
        gold = torch.randn(n, dtype=torch.float32, device=device, generator=gen)
        pairs.append(perturb_pair(gold, DT_F32, rng, int(round(0.001 * n)), 4, n_nan=2, ulp_tol=0))
    return pairs


# --------------------------------------------------------------------------
# c2: dirty-page diff at 2 GiB (4096 Pareto allocations, Q8 blocks + fp16)
# --------------------------------------------------------------------------

def q8_stream(n_blocks: int, gen: torch.Generator, device) -> torch.Tensor:
    """Blocks of [fp16 scale | 32 x int8], absmax-quantised N(0, 0.02)."""
    x = torch.randn(n_blocks, 32, device=device, generator=gen) * 0.02
    scale = x.abs().amax(dim=1, keepdim=True).clamp_min(1e-12) / 127.0
    q = torch.round(x / scale).clamp(-127, 127).to(torch.int8)
    out = torch.empty(n_blocks, 34, dtype=torch.uint8, device=device)
    out[:, :2] = scale.to(torch.float16).view(torch.uint8).view(n_blocks, 2)
    out[:, 2:] = q.view(torch.uint8)
    return out.reshape(-1)


def c2_layout(scale: float = 1.0, seed: int = 2):
    rng = np.random.default_rng(seed)
    n = max(4, int(round(4096 * min(1.0, scale * 16))))
    total_pages = max(n, int(round(524288 * scale)))
    hi = max(PAGE, min(64 * MiB, (total_pages * PAGE) // 4) // PAGE * PAGE)
    hi = max(hi, -(-total_pages // n) * PAGE)
    sizes = fit_sizes(pareto(rng, n, 1.2, 4 * KiB), PAGE, hi, total_pages * PAGE, PAGE)
    return rng, make_layout(rng, sizes)


def c2_snapshot(device="cpu", scale: float = 1.0, seed: int = 2) -> SnapshotCase:
    """Allocation i holds fp16 N(0,1) activations if i % 4 == 3, else Q8
    blocks cut at the allocation end.  ``rewrite()`` puts fresh uniform
    bytes into 5 % of the pages (seeded) for the second snapshot."""
    rng, lay = c2_layout(scale, seed)
    arena = Arena(lay, device, fill_zero=False)
    arena.buf.zero_()
    gen = torch.Generator(device=device).manual_seed(seed)
    total = lay.total
    act = torch.randn(total // 2 + 1, dtype=torch.float16, device=device, generator=gen).view(torch.uint8)
    q8 = q8_stream(total // 34 + lay.n + 2, gen, device)
    cum = lay.cum()
    for i in range(lay.n):
        s = int(lay.sizes[i])
        if i % 4 == 3:
            src = act[cum[i]: cum[i] + s]
        else:
            start = -(-int(cum[i]) // 34) * 34
            src = q8[start: start + s]
        arena.view(i).copy_(src)
    N = lay.n_pages
    rewritten = np.sort(rng.choice(N, size=int(N * 0.05), replace=False))
    case = SnapshotCase("c2", arena, dict(rewritten=rewritten, n_pages=N, seed=seed))
    return case


def page_views(case: SnapshotCase, pages: np.ndarray):
    """(range index, page-in-range) for global page indices."""
    fp = np.concatenate([[0], np.cumsum(case.layout.sizes // PAGE)])
    a = np.searchsorted(fp, pages, side="right") - 1
    return a, pages - fp[a]


def c2_rewrite(case: SnapshotCase) -> None:
    """Second-snapshot mutation: fresh uniform bytes in the recorded pages."""
    pages = case.truth["rewritten"]
    gen = torch.Generator(device=case.arena.device).manual_seed(case.truth["seed"] + 77)
    fresh = torch.randint(0, 256, (len(pages), PAGE), dtype=torch.uint8,
                          device=case.arena.device, generator=gen)
    a, p = page_views(case, pages)
    offs = case.layout.offsets[a] + p * PAGE
    idx = torch.from_numpy(offs).to(case.arena.device)
    case.arena.buf.view(-1, PAGE).index_copy_(0, idx // PAGE, fresh)


# --------------------------------------------------------------------------
# c3: batched uneven compare (10,000 pairs, 8 GiB per side)
# --------------------------------------------------------------------------

@dataclass
class PairSet:
    gold_arena: torch.Tensor
    cand_arena: torch.Tensor
    offsets: np.ndarray
    nbytes: np.ndarray
    dtypes: np.ndarray
    tols: np.ndarray
    pos: list
    k: list

    def n_elems(self, i: int) -> int:
        return int(self.nbytes[i]) // ELEM_SIZE[int(self.dtypes[i])]

    def gold(self, i: int) -> torch.Tensor:
        o, s = int(self.offsets[i]), int(self.nbytes[i])
        return self.gold_arena[o: o + s].view(TORCH_DTYPE[int(self.dtypes[i])])

    def cand(self, i: int) -> torch.Tensor:
        o, s = int(self.offsets[i]), int(self.nbytes[i])
        return self.cand_arena[o: o + s].view(TORCH_DTYPE[int(self.dtypes[i])])

    def __len__(self) -> int:
        return len(self.nbytes)


def c3_pairs(device="cpu", scale: float = 1.0, seed: int = 3, n_pairs: int = 10000,
             p_pert: float = 1e-4, kmax: int = 16) -> PairSet:
    rng = np.random.default_rng(seed)
    n_pairs = max(4, int(n_pairs))
    total = max(n_pairs * 256, int(round(8 * GiB * scale)) // 256 * 256)
    hi = max(256, min(64 * MiB, total // 4) // 256 * 256)
    hi = max(hi, -(-total // n_pairs + 255) // 256 * 256)
    sizes = fit_sizes(loguniform(rng, n_pairs, 256, 64 * MiB), 256, hi, total, 256)
    dtypes = np.array([(DT_F32, DT_F32, DT_BF16, DT_F16)[i % 4] for i in range(n_pairs)], dtype=np.int64)
    tols = rng.integers(0, 9, size=n_pairs)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    gold_arena = torch.empty(total, dtype=torch.uint8, device=device)
    gen = torch.Generator(device=device).manual_seed(seed)
    for dt in (DT_F32, DT_BF16, DT_F16):
        sel = np.nonzero(dtypes == dt)[0]
        n_el = int(sizes[sel].sum()) // ELEM_SIZE[dt]
        vals = torch.randn(n_el, dtype=torch.float32, device=device, generator=gen).to(TORCH_DTYPE[dt])
        vb = vals.view(torch.uint8)
        c = 0
        for i in sel:
            o, s = int(offsets[i]), int(sizes[i])
            gold_arena[o: o + s].copy_(vb[c: c + s])
            c += s
        del vals, vb
    cand_arena = gold_arena.clone()
    pos_l, k_l = [], []
    for dt in (DT_F32, DT_BF16, DT_F16):
        sel = np.nonzero(dtypes == dt)[0]
        gidx, ks = [], []
        for i in sel:
            n_el = int(sizes[i]) // ELEM_SIZE[dt]
            m = int(rng.binomial(n_el, p_pert))
            pos = np.sort(rng.choice(n_el, size=m, replace=False)) if m else np.zeros(0, np.int64)
            k = rng.integers(1, kmax + 1, size=m) * np.where(rng.random(m) < 0.5, -1, 1)
            pos_l.append((int(i), pos))
            k_l.append((int(i), k))
            gidx.append(int(offsets[i]) // ELEM_SIZE[dt] + pos)
            ks.append(k)
        if not gidx:
            continue
        gidx = np.concatenate(gidx)
        ks = np.concatenate(ks)
        if len(gidx) == 0:
            continue
        typed = cand_arena.view(TORCH_DTYPE[dt]) if total % ELEM_SIZE[dt] == 0 else None
        idx = torch.from_numpy(gidx).to(device)
        moved = step_ulps(typed[idx].cpu(), torch.from_numpy(ks)).to(device)
        typed[idx] = moved
    pos_d = dict(pos_l)
    k_d = dict(k_l)
    return PairSet(gold_arena, cand_arena, offsets, sizes, dtypes, tols,
                   [pos_d[i] for i in range(n_pairs)], [k_d[i] for i in range(n_pairs)])


# --------------------------------------------------------------------------
# c4: 30 GiB MoE-shaped weight pool
# --------------------------------------------------------------------------

def c4_layout(scale: float = 1.0, seed: int = 4):
    """192 bf16 4096x14336 expert matrices, a 512 KiB table of u64 pointers
    to the expert bases, a 1 GiB fp32 workspace (80 % of its pages zero) and
    6 fp16 activation buffers of 1365.25 MiB: 200 ranges, 30 GiB."""
    rng = np.random.default_rng(seed)

    def pages(b):
        return max(1, int(round(b * scale / PAGE)))

    sizes = ([pages(4096 * 14336 * 2)] * 192 + [pages(512 * KiB)] + [pages(1 * GiB)]
             + [pages(349504 * PAGE)] * 6)
    sizes = np.array(sizes, dtype=np.int64) * PAGE
    return rng, make_layout(rng, sizes)


def c4_snapshot(device="cpu", scale: float = 1.0, seed: int = 4, oob_entries: int = 0) -> SnapshotCase:
    rng, lay = c4_layout(scale, seed)
    arena = Arena(lay, device, fill_zero=False)
    arena.buf.zero_()
    gen = torch.Generator(device=device).manual_seed(seed)
    for i in range(192):
        arena.view(i).view(torch.bfloat16).normal_(0.0, 0.02, generator=gen)
    ranges = arena.ranges()
    table = arena.view(192).view(torch.int64)
    n_tab = table.numel()
    bases = np.array([ranges[i % 192][0] for i in range(n_tab)], dtype=np.uint64)
    max_end = ranges[-1][0] + ranges[-1][1]
    oob_slots = []
    if oob_entries:
        oob_slots = list(rng.choice(n_tab, size=oob_entries, replace=False))
        for s in oob_slots:
            bases[s] = max_end
    table.copy_(torch.from_numpy(bases.view(np.int64)).to(device))
    ws = arena.view(193).view(torch.float32)
    ws.normal_(0.0, 1.0, generator=gen)
    ws_pages = int(lay.sizes[193]) // PAGE
    zero = np.sort(rng.choice(ws_pages, size=int(ws_pages * 0.8), replace=False))
    ws.view(ws_pages, PAGE // 4).index_fill_(0, torch.from_numpy(zero).to(device), 0.0)
    for i in range(194, 200):
        arena.view(i).view(torch.float16).normal_(0.0, 1.0, generator=gen)
    fp = np.concatenate([[0], np.cumsum(lay.sizes // PAGE)])
    truth = dict(zero_pages=fp[193] + zero, n_table=n_tab, oob_slots=oob_slots, n_pages=lay.n_pages,
                 table_range=192)
    return SnapshotCase("c4", arena, truth)


# --------------------------------------------------------------------------
# c5: validation serving loop (request schedule; goldens resident on device)
# --------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival_s: float
    golden_ids: np.ndarray
    ulp_tol: int
    seed: int


def c5_pool(device="cpu", scale: float = 1.0, seed: int = 5, n_buffers: int = 256):
    """Resident golden pool: log-uniform 4 KiB - 256 MiB, fp32/bf16/fp8 1:1:1."""
    rng = np.random.default_rng(seed)
    hi = max(8 * KiB, int(256 * MiB * scale) // PAGE * PAGE)
    sizes = (np.round(loguniform(rng, n_buffers, 4 * KiB, max(hi, 8 * KiB)) / PAGE) * PAGE).astype(np.int64)
    sizes = np.clip(sizes, 4 * KiB, None)
    dtypes = np.array([(DT_F32, DT_BF16, DT_FP8)[i % 3] for i in range(n_buffers)])
    gen = torch.Generator(device=device).manual_seed(seed)
    golds = []
    for s, dt in zip(sizes, dtypes):
        n = int(s) // ELEM_SIZE[int(dt)]
        golds.append(torch.randn(n, device=device, generator=gen).to(TORCH_DTYPE[int(dt)]))
    return golds, dtypes


def c5_requests(rate_hz: float = 200.0, duration_s: float = 30.0, seed: int = 5,
                n_buffers: int = 256, max_k: int = 64):
    rng = np.random.default_rng(seed + 1)
    t, out, rid = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        k = int(rng.integers(1, max_k + 1))
        ids = rng.choice(n_buffers, size=k, replace=False)
        out.append(Request(rid, t, ids, int(rng.integers(0, 9)), int(rng.integers(0, 2**31))))
        rid += 1
    return out


_FP8_DEV = {}


def _fp8_tables_on(device, tdtype=torch.float8_e4m3fn):
    key = (str(device), tdtype)
    if key not in _FP8_DEV:
        c, r = _fp8_tables(tdtype)
        _FP8_DEV[key] = (c.to(device), r.to(device))
    return _FP8_DEV[key]


def _hash32(x: torch.Tensor) -> torch.Tensor:
    """A 32-bit integer mix on int64 tensors (values stay below 2^59, so no
    overflow on any device)."""
    m = 0xFFFFFFFF
    x = x & m
    for _ in range(2):
        x = ((x >> 16) ^ x) * 0x45D9F3B & m
    return ((x >> 16) ^ x) & m


def perturb_many(arena: torch.Tensor, dtype: int, offsets, lengths, seeds, p_pert: float = 1e-4,
                 kmax: int = 16) -> None:
    """In place, on the arena's device, without host synchronisation.

    ``arena`` is a 1-D typed tensor holding several candidate buffers at
    element ``offsets`` with element ``lengths``.  In buffer b, element
    j * B + (h mod B) of each block j of B = round(1/p_pert) elements moves by
    1..kmax ULP in a direction, where h and the step come from a hash of
    (seeds[b], j): a buffer's perturbation depends only on its own seed.  A
    float moves in sign-magnitude order of its bits (the order the compare's
    ULP distance counts), stopping at an infinity; NaNs stay; integers and fp8
    codes move by k and k ranks, clamped (fp8 NaN codes stay too)."""
    block = max(1, int(round(1.0 / p_pert)))
    lengths = np.asarray(lengths, dtype=np.int64)
    m = lengths // block
    total = int(m.sum())
    if total == 0:
        return
    dev = arena.device
    keep = m > 0
    per = torch.from_numpy(np.stack([np.asarray(offsets, dtype=np.int64)[keep], m[keep],
                                     np.asarray(seeds, dtype=np.int64)[keep] & 0x7FFFFFFF]))
    if dev.type == "cuda":  # a pageable upload would wait for the other streams' work
        per = per.pin_memory()
    off_t, m_t, seed_t = per.to(dev, non_blocking=True)
    ends = torch.cumsum(m_t, 0)
    i_t = torch.arange(total, device=dev)
    b_t = torch.searchsorted(ends, i_t, right=True)  # buffer of each perturbation (no host read-back)
    j_t = i_t - (ends - m_t)[b_t]
    sd_t = seed_t[b_t]
    base_t = off_t[b_t]
    h1 = _hash32(sd_t * 0x9E37 + j_t * 0x85EB + 1)
    h2 = _hash32(h1 + sd_t + 0x27D4EB2F)
    pos = base_t + j_t * block + (h1 % block)
    k = 1 + (h2 % kmax)
    k = torch.where(((h2 >> 20) & 1) == 1, -k, k)
    vals = arena[pos]
    if arena.dtype in FP8_TYPES:
        code_of_rank, rank_of_code = _fp8_tables_on(dev, arena.dtype)
        codes = vals.view(torch.uint8)
        rank = rank_of_code[codes.to(torch.int64)]
        r = (rank + k).clamp(0, len(code_of_rank) - 1)
        arena[pos] = torch.where(rank < 0, codes, code_of_rank[r]).view(arena.dtype)
        return
    if arena.dtype in INT_TYPES:
        info = torch.iinfo(arena.dtype)
        v = vals.to(torch.int64)
        o = v + k
        if arena.dtype == torch.int64:  # saturate instead of wrapping
            o = torch.where((k > 0) & (o < v), info.max, torch.where((k < 0) & (o > v), info.min, o))
        arena[pos] = o.clamp(info.min, info.max).to(arena.dtype)
        return
    nbits = 8 * arena.element_size()
    exp_bits = {torch.float64: 11, torch.float32: 8, torch.bfloat16: 8, torch.float16: 5}[arena.dtype]
    ibits = {8: torch.int8, 16: torch.int16, 32: torch.int32, 64: torch.int64}[nbits]
    sign = 1 << (nbits - 1)
    inf = ((1 << exp_bits) - 1) << (nbits - 1 - exp_bits)
    if nbits == 64:  # the int64 view holds the bits; work in it directly (no wider type)
        b = vals.view(torch.int64)
        mag = b & (sign - 1)
        neg = b < 0
    else:
        b = vals.view(ibits).to(torch.int64) & ((1 << nbits) - 1)
        mag = b & (sign - 1)
        neg = (b & sign) != 0
    o = torch.where(neg, -mag, mag) + k                    # sign-magnitude order, +0 and -0 both 0
    o = o.clamp(-inf, inf)
    out = torch.where(o < 0, (-o) | sign, o) if nbits < 64 else torch.where(o < 0, (-o) | (-(1 << 63)), o)
    out = torch.where(mag > inf, b, out)                   # NaNs unchanged
    if nbits == 64:
        arena[pos] = out.view(arena.dtype)
    else:
        arena[pos] = (out - ((out & sign) << 1)).to(ibits).view(arena.dtype)  # back to the signed view


def perturb_device(cand: torch.Tensor, dtype: int, seed: int, p_pert: float = 1e-4, kmax: int = 16) -> None:
    """``perturb_many`` on a single buffer."""
    perturb_many(cand.view(-1), dtype, [0], [cand.numel()], [seed], p_pert, kmax)


def materialize_candidate(gold: torch.Tensor, dtype: int, seed: int, p_pert: float = 1e-4,
                          kmax: int = 16) -> torch.Tensor:
    """A candidate output: the golden buffer with a seeded sparse set of
    elements moved by 1..kmax ULP (stand-in for a reproducer's output)."""
    rng = np.random.default_rng(seed)
    n = gold.numel()
    m = int(rng.binomial(n, p_pert)) if n else 0
    return perturb_pair(gold, dtype, rng, m, kmax).cand
