"""Independent (numpy / library) formulations used to pin the oracle and to
check the HIP path.  Nothing here calls the oracle or the HIP library."""
from __future__ import annotations

import numpy as np

PAGE = 4096


def bits_to_words(flags: np.ndarray) -> np.ndarray:
    """Bool per page -> u64 bitmap words, bit g%64 of word g//64."""
    n = len(flags)
    w = (n + 63) // 64
    padded = np.zeros(w * 64, dtype=bool)
    padded[:n] = flags
    return np.packbits(padded, bitorder="little").view("<u8").astype(np.uint64)


def words_to_bits(words: np.ndarray, n: int) -> np.ndarray:
    return np.unpackbits(np.ascontiguousarray(words, dtype="<u8").view(np.uint8),
                         bitorder="little")[:n].astype(bool)


def concat_pages(views) -> np.ndarray:
    if not views:
        return np.zeros((0, PAGE), dtype=np.uint8)
    return np.concatenate([v.reshape(-1, PAGE) for v in views])


def page_vas(ranges) -> np.ndarray:
    if not ranges:
        return np.zeros(0, dtype=np.uint64)
    return np.concatenate([np.uint64(b) + np.arange(s // PAGE, dtype=np.uint64) * np.uint64(PAGE)
                           for b, s in ranges])


def numpy_closure(ranges, views, lo: int, hi: int):
    """Vectorised closure scan: counts and the ordered (word_va, value) list."""
    bases = np.array([b for b, _ in ranges], dtype=np.uint64)
    ends = np.array([b + s for b, s in ranges], dtype=np.uint64)
    n_words = n_ptr = n_in = 0
    oob = []
    for (b, s), v in zip(ranges, views):
        w = v.view("<u8")
        n_words += len(w)
        ptr = (w >= np.uint64(lo)) & (w < np.uint64(hi))
        n_ptr += int(ptr.sum())
        idx = np.searchsorted(bases, w, side="right").astype(np.int64) - 1
        ok = idx >= 0
        inr = np.zeros(len(w), dtype=bool)
        inr[ok] = w[ok] < ends[idx[ok]]
        n_in += int((ptr & inr).sum())
        bad = np.nonzero(ptr & ~inr)[0]
        oob.extend((int(b) + 8 * int(i), int(w[i])) for i in bad)
    return dict(n_words=n_words, n_ptr_like=n_ptr, n_in_range=n_in, n_oob=len(oob)), oob
