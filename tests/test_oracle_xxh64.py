"""Pins the oracle's XXH64 against an independent implementation.

The hash is the public XXH64 definition (xxHash, Y. Collet); python-xxhash
(bundling libxxhash) is run as a library routine, never read.
"""
import os
import random

import numpy as np
import pytest

xxhash = pytest.importorskip("xxhash")


def test_short_and_page_lengths(oracle_lib):
    rnd = random.Random(11)
    for length in list(range(0, 300)) + [4095, 4096, 4097, 8192, 65536]:
        data = os.urandom(length)
        for seed in (0, 1, 2**64 - 1, rnd.getrandbits(64)):
            assert oracle_lib.xxh64(data, seed) == xxhash.xxh64_intdigest(data, seed), (length, seed)


def test_structured_pages(oracle_lib):
    pages = [bytes(4096), bytes([0xFF]) * 4096, bytes(i & 0xFF for i in range(4096)),
             np.arange(512, dtype=np.uint64).tobytes()]
    for p in pages:
        for seed in (0, 1, 0xDEADBEEF):
            assert oracle_lib.xxh64(p, seed) == xxhash.xxh64_intdigest(p, seed)


def test_seed_changes_zero_page_hash(oracle_lib):
    z = bytes(4096)
    assert oracle_lib.xxh64(z, 0) != oracle_lib.xxh64(z, 1)
