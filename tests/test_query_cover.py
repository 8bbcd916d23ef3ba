"""The query-graph vertex cover behind PPSP_BATCH_VC (host logic of the
C-ABI library, no GPU): validity always; minimality against brute force on
small query graphs, undirected (components of up to 16 vertices are solved
exactly) and directed (bipartite sources/targets: Hopcroft-Karp matching and
Koenig's theorem give an exact minimum at any size)."""
import itertools

import numpy as np
import pytest


def _P():
    import paper_2506_16488_amd as P
    try:
        P.lib()
    except ImportError:
        from paper_2506_16488_amd import build
        build.build()
    return P


def _nodes(pairs, directed):
    """Query-graph vertices: (vertex, side) with side 1 for targets when directed."""
    out = []
    for s, t in pairs:
        if s == t:
            continue
        out.append((int(s), 0))
        out.append((int(t), 1 if directed else 0))
    return sorted(set(out))


def _brute_min_cover(pairs, directed):
    nodes = _nodes(pairs, directed)
    edges = [((int(s), 0), (int(t), 1 if directed else 0)) for s, t in pairs if s != t]
    for size in range(len(nodes) + 1):
        for c in itertools.combinations(nodes, size):
            cs = set(c)
            if all(a in cs or b in cs for a, b in edges):
                return size
    return len(nodes)


def _check_valid(pairs, root, ft, size, directed):
    roots = set()
    for q, (s, t) in enumerate(pairs):
        if s == t:
            assert root[q] == s and ft[q] == 0
            continue
        assert root[q] in (s, t)
        assert ft[q] == (1 if root[q] == t else 0)
        roots.add((int(root[q]), int(ft[q]) if directed else 0))
    assert size == len(roots)


@pytest.mark.parametrize("seed", range(40))
def test_directed_cover_is_minimum(seed):
    P = _P()
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(2, 8))
    k = int(rng.integers(1, 12))
    pairs = rng.integers(0, nv, (k, 2)).astype(np.uint32)
    root, ft, size = P.query_cover(pairs, directed=True)
    _check_valid(pairs, root, ft, size, True)
    assert size == _brute_min_cover(pairs, True), pairs.tolist()


@pytest.mark.parametrize("seed", range(40))
def test_undirected_cover_is_minimum_on_small_components(seed):
    P = _P()
    rng = np.random.default_rng(100 + seed)
    nv = int(rng.integers(2, 11))
    k = int(rng.integers(1, 14))
    pairs = rng.integers(0, nv, (k, 2)).astype(np.uint32)
    root, ft, size = P.query_cover(pairs, directed=False)
    _check_valid(pairs, root, ft, size, False)
    assert size == _brute_min_cover(pairs, False), pairs.tolist()


def test_patterns_and_large_graphs():
    P = _P()
    star = np.array([[0, v] for v in range(1, 9)], np.uint32)
    for directed in (False, True):
        root, ft, size = P.query_cover(star, directed=directed)
        assert size == 1 and set(root.tolist()) == {0}
    # reversed star on a directed graph: one backward search from the common target
    rstar = star[:, ::-1].copy()
    root, ft, size = P.query_cover(rstar, directed=True)
    assert size == 1 and set(root.tolist()) == {0} and ft.tolist() == [1] * 8
    # complete bipartite 3 x 4: the smaller side
    kb = np.array([[a, 10 + b] for a in range(3) for b in range(4)], np.uint32)
    for directed in (False, True):
        assert P.query_cover(kb, directed=directed)[2] == 3
    # large random query graphs: valid; directed ones exactly minimum (Koenig: = maximum matching)
    rng = np.random.default_rng(7)
    pairs = rng.integers(0, 400, (3000, 2)).astype(np.uint32)
    for directed in (False, True):
        root, ft, size = P.query_cover(pairs, directed=directed)
        _check_valid(pairs, root, ft, size, directed)
    src = rng.integers(0, 60, 500)
    dst = 1000 + rng.integers(0, 40, 500)
    pairs = np.stack([src, dst], 1).astype(np.uint32)
    root, ft, size = P.query_cover(pairs, directed=True)
    _check_valid(pairs, root, ft, size, True)
    assert size == _max_matching(pairs)


def _max_matching(pairs):
    """Maximum bipartite matching by simple augmenting paths (Kuhn), for the check."""
    adj = {}
    for s, t in pairs:
        adj.setdefault(int(s), set()).add(int(t))
    match = {}

    def try_(u, seen):
        for v in adj[u]:
            if v in seen:
                continue
            seen.add(v)
            if v not in match or try_(match[v], seen):
                match[v] = u
                return True
        return False
    return sum(1 for u in adj if try_(u, set()))


def test_self_pairs_and_errors():
    P = _P()
    root, ft, size = P.query_cover(np.array([[3, 3], [3, 5], [5, 5]], np.uint32))
    assert root.tolist()[0] == 3 and root.tolist()[2] == 5 and size == 1
    root, ft, size = P.query_cover(np.zeros((0, 2), np.uint32))
    assert size == 0
    import ctypes
    assert P.lib().ppsp_query_cover(None, 2, 0, None, None, ctypes.byref(ctypes.c_uint32())) == P.E_INVALID
