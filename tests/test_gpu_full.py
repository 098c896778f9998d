"""Parity at full size: R-MAT scale 22 (edgefactor 16, 4 x 4 block grid) and
R-MAT scale 26 (8 x 8 block grid), from their seeded roots.

Levels are compared bit-exact with the oracle's queue BFS, parents exactly
with the (select, max) rule of Sec. III.A, the tree with the validity rules.
At scale 22 every level's every stream of every root is compared
byte-for-byte with the oracle's Algorithm 3 (Sec. V.B); at scale 26 sampled
streams of one root are recomputed one by one from the oracle's levels and
directory.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_5542_amd import inputs
from tests.gpu_util import log, require_gpu, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _setup(name, nroots):
    from paper_1208_5542_amd import csbfs
    wl = inputs.WORKLOADS[name]
    log(f"[full] generating {name}")
    src, dst = wl.tuples()
    roots = wl.roots(src, dst, nroots)
    log(f"[full] building graph p={wl.p}")
    g = csbfs.Graph(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), wl.n, wl.p)
    torch.cuda.synchronize()
    log("[full] oracle adjacency")
    adj = oracle.Adjacency(wl.n, src, dst)
    return wl, src, dst, roots, g, adj


def _check_tree(wl, src, dst, g, adj, r, root):
    n = wl.n
    lev = r.level.cpu().numpy()
    par = r.parent.cpu().numpy()
    log(f"[full] oracle queue BFS from {root}")
    ref = adj.bfs(root)
    assert (lev == ref).all(), "levels differ from the queue BFS"
    log("[full] oracle max-rule parents")
    assert (par == adj.parents_max(ref, root)).all(), "parents differ from the max rule"
    log("[full] oracle validity rules")
    assert oracle.validate(n, src, dst, root, lev, par, ref) == 0
    assert r.n_levels == int(ref.max()) + 1
    log("[full] traversed tuples")
    assert g.traversed_tuples(r.level) == oracle.teps_m(src, dst, ref)
    return ref


def test_rmat22_p4_full_parity():
    from paper_1208_5542_amd import csbfs
    wl, src, dst, roots, g, adj = _setup("rmat22_p4", 4)
    n, p = wl.n, wl.p
    eng = csbfs.Engine(g, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS)
    V = oracle.directory(n, p, src, dst)
    for root in roots[:4]:
        root = int(root)
        log(f"[full] root {root}")
        r = eng.bfs(root)
        ref = _check_tree(wl, src, dst, g, adj, r, root)
        log("[full] oracle Algorithm 3")
        a3 = adj.alg3(p, V.reshape(-1), root, dump=True)
        assert (a3.level == ref).all()
        assert (eng.stream_words(r.n_levels) == a3.words).all()
        for k in range(1, r.n_levels):
            for i in range(p):
                for j in range(p):
                    got = u64(eng.stream(k, i, j))
                    exp = a3.streams[k, i, j, : a3.words[k, i, j]]
                    assert got.tolist() == exp.tolist(), (root, k, i, j)
        lb = a3.level_bytes()
        for k in range(r.n_levels):
            assert r.stats[k]["wah_sieved_bytes"] == lb[k]["wah_sieved"]
            assert r.stats[k]["wah_unsieved_bytes"] == lb[k]["wah_unsieved"]
            assert r.stats[k]["self_bytes"] == lb[k]["self"]


def test_rmat26_p8_full_parity():
    """One root at scale 26 on the 8 x 8 grid (the oracle's share of it takes
    about a minute of host time): everything of the tree, and four sampled
    streams per level recomputed from the oracle's levels and directory."""
    from paper_1208_5542_amd import csbfs
    wl, src, dst, roots, g, adj = _setup("rmat26_p8", 1)
    n, p = wl.n, wl.p
    eng = csbfs.Engine(g, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS)
    rng = np.random.default_rng(0)
    root = int(roots[0])
    log(f"[full] root {root}")
    r = eng.bfs(root)
    ref = _check_tree(wl, src, dst, g, adj, r, root)
    log("[full] oracle directory")
    V = oracle.directory(n, p, src, dst)
    log("[full] sampled streams")
    for k in range(1, r.n_levels):
        for _ in range(4):
            i, j = (int(x) for x in rng.integers(0, p, 2))
            exp = oracle.stream_from_levels(ref, V, n, p, k, i, j)
            got = u64(eng.stream(k, i, j))
            assert got.tolist() == exp.tolist(), (root, k, i, j)
