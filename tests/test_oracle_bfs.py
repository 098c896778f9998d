"""Pins of the oracle's BFS, parent rule, validator and TEPS count against
brute force on tiny graphs (CPU only)."""
import numpy as np
import pytest

import oracle


def _random_graph(rng, n, m, self_loops=True):
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    return src.astype(np.int64), dst.astype(np.int64)


def _apsp(n, src, dst):
    """All-pairs hop distances by repeated relaxation of a dense matrix."""
    INF = 10 ** 6
    D = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    A = np.zeros((n, n), dtype=bool)
    A[src, dst] = True
    A[dst, src] = True
    D[A] = np.minimum(D[A], 1)
    np.fill_diagonal(D, 0)
    for _ in range(n):
        D2 = np.minimum(D, (D[:, :, None] + D[None, :, :]).min(axis=1))
        if (D2 == D).all():
            break
        D = D2
    D[D >= INF] = -1
    return D, A


@pytest.mark.parametrize("seed", range(12))
def test_levels_and_parents_vs_apsp(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 48))
    m = int(rng.integers(0, 3 * n))
    src, dst = _random_graph(rng, n, m)
    D, A = _apsp(n, src, dst)
    adj = oracle.Adjacency(n, src, dst)
    for root in range(n):
        level = adj.bfs(root)
        assert level.tolist() == D[root].tolist()
        parent = adj.parents_max(level, root)
        # the highest-labelled vertex on any shortest path one hop before v
        for v in range(n):
            if v == root:
                assert parent[v] == root
            elif D[root, v] < 0:
                assert parent[v] == -1
            else:
                cands = [u for u in range(n) if A[u, v] and D[root, u] == D[root, v] - 1]
                assert parent[v] == max(cands)
        assert oracle.validate(n, src, dst, root, level, parent, D[root].astype(np.int32)) == 0


def test_self_loop_counts_twice_in_degree():
    adj = oracle.Adjacency(4, [0, 1, 2], [0, 2, 2])
    assert [adj.degree(v) for v in range(4)] == [2, 1, 3, 0]
    assert adj.bfs(0).tolist() == [0, -1, -1, -1]
    assert adj.bfs(1).tolist() == [-1, 0, 1, -1]


def test_teps_m_counts_component_tuples():
    rng = np.random.default_rng(3)
    n = 40
    src, dst = _random_graph(rng, n, 60)
    # add duplicates and self-loops explicitly
    src = np.r_[src, src[:5], [7, 7]]
    dst = np.r_[dst, dst[:5], [7, 7]]
    D, _ = _apsp(n, src, dst)
    adj = oracle.Adjacency(n, src, dst)
    for root in range(0, n, 7):
        level = adj.bfs(root)
        expect = sum(1 for a, b in zip(src, dst) if D[root, a] >= 0)
        assert oracle.teps_m(src, dst, level) == expect


def _tree(seed=5, n=30, m=70):
    rng = np.random.default_rng(seed)
    src, dst = _random_graph(rng, n, m, self_loops=False)
    adj = oracle.Adjacency(n, src, dst)
    level = adj.bfs(int(src[0]))
    parent = adj.parents_max(level, int(src[0]))
    return n, src, dst, int(src[0]), level, parent


def test_validator_accepts_any_valid_tree():
    n, src, dst, root, level, parent = _tree()
    assert oracle.validate(n, src, dst, root, level, parent) == 0
    # a min-rule tree is just as valid
    adj = oracle.Adjacency(n, src, dst)
    pmin = parent.copy()
    for v in range(n):
        if v != root and level[v] > 0:
            pmin[v] = min(u for u in range(n) if level[u] == level[v] - 1 and
                          (((src == u) & (dst == v)) | ((src == v) & (dst == u))).any())
    assert oracle.validate(n, src, dst, root, level, pmin) == 0


@pytest.mark.parametrize("plant,bit", [
    ("root_parent", 1), ("root_level", 1), ("missing_parent", 2), ("stray_parent", 2),
    ("non_edge", 4), ("level_skip", 8), ("edge_gap", 16), ("half_reached", 32),
])
def test_validator_catches_planted_mistakes(plant, bit):
    n, src, dst, root, level, parent = _tree()
    level, parent = level.copy(), parent.copy()
    reached = [v for v in range(n) if level[v] > 0]
    v = max(reached, key=lambda x: level[x])
    if plant == "root_parent":
        parent[root] = parent[v]
    elif plant == "root_level":
        level[root] = 1
    elif plant == "missing_parent":
        parent[v] = -1
    elif plant == "stray_parent":
        # four isolated vertices past the tree's graph: unreached, and one
        # of them is given a parent
        n += 4
        level = np.r_[level, [-1] * 4].astype(np.int32)
        parent = np.r_[parent, [-1] * 4].astype(np.int32)
        assert oracle.validate(n, src, dst, root, level, parent) == 0
        parent[n - 2] = root
    elif plant == "non_edge":
        nbrs = set(dst[src == v]) | set(src[dst == v])
        others = [u for u in range(n) if level[u] == level[v] - 1 and u not in nbrs]
        if not others:
            pytest.skip("no non-neighbour on the previous level")
        parent[v] = others[0]
    elif plant == "level_skip":
        level[v] += 1
    elif plant == "edge_gap":
        level[v] += 2
    elif plant == "half_reached":
        level[v] = -1
        parent[v] = -1
    got = oracle.validate(n, src, dst, root, level, parent)
    assert got & bit, (plant, got)
