"""Pins the oracle's pointer graph between ranges and its reachable set.

Independent pins: the digraph the generator plants (each planted word records
its source range, target range and value), window restrictions applied to
those recorded values, hand-built graphs with known reachable sets, and a
transitive closure computed by repeated boolean matrix products (a different
algorithm from the oracle's breadth-first search)."""
import numpy as np
import pytest

from paper_2605_03208_amd import workloads as W


def _views(case):
    return W.host_views(case.layout, case.arena.host_copy())


@pytest.mark.parametrize("n,seed", [(1, 1), (7, 2), (64, 3), (130, 4)])
def test_planted_edges(oracle_lib, n, seed):
    o = oracle_lib
    case = W.graph_case(n_ranges=n, seed=seed)
    ranges = case.ranges()
    edge = o.pointer_graph(ranges, _views(case))
    assert edge.shape == (n, (n + 63) // 64)
    adj = o.edges_to_bool(edge, n)
    want = np.zeros((n, n), bool)
    for a, b in case.truth["edges"]:
        want[a, b] = True
    assert (adj == want).all()
    # bits past the last range in each row stay clear
    if n % 64:
        assert (edge[:, -1] >> np.uint64(n % 64) == 0).all()


def test_window_restricts_edges(oracle_lib):
    o = oracle_lib
    case = W.graph_case(n_ranges=20, seed=9)
    ranges = case.ranges()
    plants = case.truth["plants"]
    vals = sorted(v for _, _, v in plants)
    for lo, hi in ((vals[len(vals) // 3], vals[2 * len(vals) // 3]), (vals[0], vals[0] + 1),
                   (vals[-1], 2**64 - 1), (1, vals[0])):
        adj = o.edges_to_bool(o.pointer_graph(ranges, _views(case), lo, hi), len(ranges))
        want = np.zeros_like(adj)
        for a, b, v in plants:
            if lo <= v < hi:
                want[a, b] = True
        assert (adj == want).all(), (lo, hi)
    with pytest.raises(o.OracleError):
        o.pointer_graph(ranges, _views(case), 0, 5)
    with pytest.raises(o.OracleError):
        o.pointer_graph(ranges, _views(case), 9, 9)


def _edge_bm(adj):
    n = adj.shape[0]
    rw = (n + 63) // 64
    bits = np.zeros((n, rw * 64), np.uint8)
    bits[:, :n] = adj
    return np.packbits(bits, axis=1, bitorder="little").view(np.uint64).reshape(n, rw)


def test_reach_hand_built(oracle_lib):
    o = oracle_lib
    ranges = [(0x100000 + i * 0x10000, 0x2000) for i in range(6)]
    adj = np.zeros((6, 6), bool)
    adj[0, 1] = adj[1, 2] = adj[3, 0] = adj[4, 4] = True      # chain, a feeder, a self loop
    bm = _edge_bm(adj)
    inside = lambda r, off=0: ranges[r][0] + off
    cases = [([inside(0)], {0, 1, 2}), ([inside(3, 0x1FFF)], {3, 0, 1, 2}), ([inside(4)], {4}),
             ([inside(5)], {5}), ([], set()), ([inside(0) - 1, ranges[5][0] + 0x2000, 0, 7], set()),
             ([inside(2), inside(4, 8)], {2, 4})]
    for words, want in cases:
        got = o.graph_reach(ranges, bm, np.array(words, np.uint64))
        assert set(np.flatnonzero(got).tolist()) == want, (words, want)


def test_reach_matches_transitive_closure(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(3)
    for n in (1, 5, 63, 64, 65, 150):
        ranges = [(0x200000 + i * 0x3000, 0x1000) for i in range(n)]
        adj = rng.random((n, n)) < 1.2 / n
        bm = _edge_bm(adj)
        roots = rng.choice(n, size=min(n, 2), replace=False)
        words = np.array([ranges[r][0] + 8 for r in roots], np.uint64)
        got = o.graph_reach(ranges, bm, words)
        # closure by squaring (I + A) until it stops changing
        m = adj | np.eye(n, dtype=bool)
        while True:
            m2 = (m.astype(np.int64) @ m.astype(np.int64)) > 0
            if (m2 == m).all():
                break
            m = m2
        want = m[roots].any(axis=0)
        assert (got == want).all(), n


def test_graph_of_planted_case_reach(oracle_lib):
    o = oracle_lib
    case = W.graph_case(n_ranges=40, seed=12)
    ranges = case.ranges()
    edge = o.pointer_graph(ranges, _views(case))
    got = o.graph_reach(ranges, edge, case.truth["root_words"])
    reach, todo = set(case.truth["roots"]), list(case.truth["roots"])
    while todo:
        a = todo.pop()
        for x, b in case.truth["edges"]:
            if x == a and b not in reach:
                reach.add(b)
                todo.append(b)
    assert set(np.flatnonzero(got).tolist()) == reach
