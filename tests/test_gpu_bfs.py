"""GPU search against the oracle on small graphs: partition and directory,
levels bit-exact, (select, max) parents exact, per-level streams
byte-identical to the oracle's Algorithm 3, byte accounting, edge cases."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_5542_amd import inputs
from tests.gpu_util import from_words, log, require_gpu, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _graph(scale, ef=16, seed=None):
    src, dst = inputs.rmat_tuples(scale, ef, seed=seed)
    return 1 << scale, src, dst


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).cuda()


@pytest.mark.parametrize("scale,p", [(10, 1), (10, 2), (10, 4), (12, 8), (11, 4)])
def test_directory_and_blocks(scale, p):
    from paper_1208_5542_amd import csbfs
    n, src, dst = _graph(scale)
    log(f"graph build scale={scale} p={p}")
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    R = n // p
    assert g.info.nnz == 2 * len(src)
    V = oracle.directory(n, p, src, dst)
    dirw = g.directory()
    for i in range(p):
        for j in range(p):
            assert (from_words(dirw[i, j], R) == V[i, j]).all(), (i, j)
    # rows of every block as multisets: u in R_j -> its neighbours in R_i
    for i in range(p):
        for j in range(p):
            rp, col = g.block(i, j)
            rp, col = rp.cpu().numpy(), col.cpu().numpy()
            a = np.r_[src, dst]
            b = np.r_[dst, src]
            sel = (a // R == j) & (b // R == i)
            exp = {}
            for u, v in zip(a[sel] - j * R, b[sel] - i * R):
                exp.setdefault(int(u), []).append(int(v))
            assert rp[0] == 0 and rp[-1] == len(col)
            for u in range(R):
                row = col[rp[u]:rp[u + 1]].tolist()
                assert row == sorted(row, reverse=True), (i, j, u)  # decreasing ids
                assert sorted(row) == sorted(exp.get(u, [])), (i, j, u)


def _check_search(eng, g, n, p, src, dst, root, adj, V, keep=True, max_levels=64):
    r = eng.bfs(root)
    torch.cuda.synchronize()
    lev = r.level.cpu().numpy()
    par = r.parent.cpu().numpy()
    ref = adj.alg3(p, V, root, max_levels=max_levels, dump=keep)
    assert (lev == ref.level).all(), "level"
    assert (par == ref.parent).all(), "parent"
    assert r.n_levels == ref.n_levels
    assert oracle.validate(n, src, dst, root, lev, par, ref.level) == 0
    words = eng.stream_words(r.n_levels)
    assert (words == ref.words).all(), "stream lengths"
    if keep:
        for k in range(1, r.n_levels):
            for i in range(p):
                for j in range(p):
                    got = u64(eng.stream(k, i, j))
                    exp = ref.streams[k, i, j, : ref.words[k, i, j]]
                    assert got.tolist() == exp.tolist(), (k, i, j)
    # byte accounting
    lb = ref.level_bytes()
    for k in range(r.n_levels):
        s = r.stats[k]
        assert s["frontier"] == lb[k]["frontier"]
        assert s["wah_sieved_bytes"] == lb[k]["wah_sieved"]
        assert s["self_bytes"] == lb[k]["self"]
        assert s["raw_bytes"] == lb[k]["raw"]
        assert s["wah_unsieved_bytes"] == lb[k]["wah_unsieved"]
        assert s["max_rank_bytes"] == lb[k]["max_rank_volume"]
        if k > 0:
            off = ~np.eye(p, dtype=bool)
            assert s["sieved_bits"] == int(ref.sieved_bits[k][off].sum())
            assert s["unsieved_bits"] == (p - 1) * lb[k]["frontier"]
    # edges scanned when expanding level k: adjacency of every level-k vertex
    # inside the blocks whose view received it
    assert g.traversed_tuples(r.level) == oracle.teps_m(src, dst, lev)
    return r


def test_volume_p3_example(golden):
    """The hand-derived p = 3 example of Sec. VI.A's volume: stream lengths
    per level, per-level maximum of a processor's sent plus received bytes,
    and (from the word counts) every processor's volume over the search."""
    from paper_1208_5542_amd import csbfs
    gd = golden("volume_p3_example.json")
    n, p = gd["n"], gd["p"]
    g = csbfs.Graph(_dev(gd["src"]), _dev(gd["dst"]), n, p)
    for flags in (0, csbfs.FLAG_SPARSE_ONLY, csbfs.FLAG_BOTTOM_UP_ONLY):
        eng = csbfs.Engine(g, flags=flags)
        r = eng.bfs(gd["root"])
        lev = r.level.cpu().numpy()
        assert r.n_levels == gd["n_levels"]
        for k, vs in gd["levels"].items():
            assert sorted(np.flatnonzero(lev == int(k)).tolist()) == vs
        words = eng.stream_words(r.n_levels)
        assert words.tolist() == gd["words"]
        assert [s["wah_sieved_bytes"] for s in r.stats] == gd["wah_sieved_bytes"]
        assert [s["self_bytes"] for s in r.stats] == gd["self_bytes"]
        assert [s["max_rank_bytes"] for s in r.stats] == gd["per_level_max_rank_bytes"]
        sent = [8 * int(sum(words[k, i, j] for k in range(r.n_levels) for j in range(p) if j != i))
                for i in range(p)]
        recv = [8 * int(sum(words[k, i, j] for k in range(r.n_levels) for i in range(p) if j != i))
                for j in range(p)]
        assert sent == gd["rank_sent_bytes"] and recv == gd["rank_received_bytes"]


MODES = {"auto": 0, "sparse": 8, "dense": 16, "bottom_up": 32,
         # the binned push at every top-down level (default: wide levels only)
         "binned": 64, "binned_sparse": 8 | 64}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("scale,p,nroots", [(10, 1, 16), (10, 2, 4), (10, 4, 4), (11, 8, 3),
                                            (12, 4, 3), (13, 2, 2), (14, 4, 2)])
def test_search_matches_oracle(scale, p, nroots, mode):
    from paper_1208_5542_amd import csbfs
    n, src, dst = _graph(scale)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    eng = csbfs.Engine(g, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS | MODES[mode])
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    roots = inputs.pick_roots(n, src, dst, nroots, inputs.graph_seed(scale) + 2)
    for root in roots:
        log(f"search scale={scale} p={p} mode={mode} root={int(root)}")
        _check_search(eng, g, n, p, src, dst, int(root), adj, V)


@pytest.mark.parametrize("groups", [1024, 2048])
def test_encoder_segment_sizes(groups):
    """Both segment sizes of the search's encoder (1024 and 2048 groups), on
    pieces of several segments: R-MAT scale 20 on a 4 x 4 grid (2^18 bits per
    piece), streams byte-identical to the oracle's Algorithm 3; searched in a
    caller workspace whose config fixes the segment size."""
    from paper_1208_5542_amd import csbfs
    scale, p = 20, 4
    n, src, dst = _graph(scale)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    eng = csbfs.WorkspaceSearch(g, csbfs.search_config(flags=csbfs.FLAG_KEEP_STREAMS, max_levels=64,
                                                       segment_groups=groups))
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    for root in inputs.pick_roots(n, src, dst, 2, inputs.graph_seed(scale) + 2):
        log(f"search scale={scale} p={p} segment groups={groups} root={int(root)}")
        _check_search(eng, g, n, p, src, dst, int(root), adj, V)


def test_binned_push_bin_overflow():
    """Pairs past a bin segment's capacity go through the atomic push and the
    bin's resolve starts from what that left: 50 sources each push 400 of the
    same 2000 targets (rows of about 200 entries per block, so they go to the
    long-row kernel), all in the first of the two bins of a 2^16-vertex
    graph whose bin segments hold 48 pairs each, so most targets take their
    highest source from both paths; parents exact against the oracle."""
    from paper_1208_5542_amd import csbfs
    n, p = 1 << 16, 4
    rng = np.random.default_rng(31)
    root = 65000
    mids = rng.choice(np.arange(40000, 64000), 50, replace=False)
    targets = rng.choice(np.arange(0, 1 << 15), 2000, replace=False)
    src = [np.full(50, root), np.repeat(mids, 400)]
    dst = [mids, np.concatenate([rng.choice(targets, 400, replace=False) for _ in mids])]
    src.append(rng.integers(0, n, 3000))
    dst.append(rng.integers(0, n, 3000))
    src = np.concatenate(src).astype(np.int64)
    dst = np.concatenate(dst).astype(np.int64)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    for flags in (csbfs.FLAG_BINNED_PUSH, csbfs.FLAG_BINNED_PUSH | csbfs.FLAG_SPARSE_ONLY):
        eng = csbfs.WorkspaceSearch(g, csbfs.search_config(flags=csbfs.FLAG_KEEP_STREAMS | flags,
                                                           push_bin_pairs=24000))
        for r in (root, int(mids[0]), int(targets[0])):
            log(f"bin overflow flags={flags} root={r}")
            res = _check_search(eng, g, n, p, src, dst, r, adj, V)
            if r == root and flags & csbfs.FLAG_SPARSE_ONLY:
                # the expansion of f^1 (20000+ pairs, nearly all into one bin) was binned
                assert res.stats[1]["direction"] == csbfs.DIR_TOP_DOWN
                assert res.stats[1]["push"] == csbfs.PUSH_BINNED
                assert res.stats[1]["edges"] > 20000


def test_binned_push_default_choice():
    """By default a top-down level is binned only with at least 2^23
    adjacency entries, 64 per frontier vertex (and on this graph only with
    bins for all its entries); ATOMIC_PUSH never bins, BINNED_PUSH bins every
    top-down level that fits. Same results every way (R-MAT scale 20,
    4 x 4), checked against the oracle."""
    from paper_1208_5542_amd import csbfs
    scale, p = 20, 4
    n, src, dst = _graph(scale)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    cases = {
        "auto": csbfs.Engine(g, max_levels=64),
        "sparse": csbfs.WorkspaceSearch(g, csbfs.search_config(flags=csbfs.FLAG_SPARSE_ONLY,
                                                               push_bin_pairs=g.info.nnz)),
        "atomic": csbfs.Engine(g, max_levels=64, flags=csbfs.FLAG_ATOMIC_PUSH),
        "forced": csbfs.WorkspaceSearch(g, csbfs.search_config(flags=csbfs.FLAG_SPARSE_ONLY |
                                                               csbfs.FLAG_BINNED_PUSH,
                                                               push_bin_pairs=g.info.nnz)),
    }
    for name, eng in cases.items():
        for root in inputs.pick_roots(n, src, dst, 2, inputs.graph_seed(scale) + 2):
            log(f"push choice scale={scale} {name} root={int(root)}")
            r = _check_search(eng, g, n, p, src, dst, int(root), adj, V, keep=False)
            for k, s in enumerate(r.stats):
                binned = s["push"] == csbfs.PUSH_BINNED
                if name == "forced":
                    assert binned == (k > 0), k  # level 0 (the root alone) is set up unbinned
                elif binned:
                    assert name != "atomic"
                    assert s["direction"] == csbfs.DIR_TOP_DOWN and s["edges"] >= 1 << 23
                    assert s["edges"] >= 64 * s["frontier"]


def test_sparse_graph_many_levels():
    """A long path plus random chords: many levels, tiny frontiers."""
    from paper_1208_5542_amd import csbfs
    n, p = 4096, 4
    rng = np.random.default_rng(5)
    perm = rng.permutation(n)
    src = perm[:-1].astype(np.int64)
    dst = perm[1:].astype(np.int64)
    extra = rng.integers(0, n, (2, 40))
    src = np.r_[src, extra[0]].astype(np.int64)
    dst = np.r_[dst, extra[1]].astype(np.int64)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    for mode, flag in MODES.items():
        eng = csbfs.Engine(g, max_levels=4096, flags=flag)
        log(f"search long path mode={mode}")
        r = _check_search(eng, g, n, p, src, dst, int(perm[0]), adj, V, keep=False, max_levels=4096)
        assert r.n_levels > 50


def test_direction_choice_and_parameters():
    """Direction-optimizing levels: the default rule turns bottom-up on an
    R-MAT graph, the parameters force either direction, and every choice
    gives the oracle's levels, parents and streams."""
    from paper_1208_5542_amd import csbfs
    n, src, dst = _graph(14)
    p = 4
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    root = int(inputs.pick_roots(n, src, dst, 1, 21)[0])
    eng = csbfs.Engine(g, flags=csbfs.FLAG_KEEP_STREAMS)
    log("direction: default rule")
    r = _check_search(eng, g, n, p, src, dst, root, adj, V)
    dirs = [s["direction"] for s in r.stats]
    assert dirs[0] == csbfs.DIR_TOP_DOWN and csbfs.DIR_BOTTOM_UP in dirs, dirs
    for s in r.stats:
        if s["direction"] == csbfs.DIR_BOTTOM_UP:
            assert s["pulled"] > 0 and s["edges"] > 0
        else:
            assert s["pulled"] == 0
    log("direction: alpha = 0 (top-down only)")
    eng.set_direction(0.0, 64.0)
    r = _check_search(eng, g, n, p, src, dst, root, adj, V)
    assert all(s["direction"] == csbfs.DIR_TOP_DOWN for s in r.stats)
    log("direction: bottom-up from level 1 on")
    eng.set_direction(1e9, 1e9)
    r = _check_search(eng, g, n, p, src, dst, root, adj, V)
    assert [s["direction"] for s in r.stats] == [0] + [1] * (r.n_levels - 1)
    for bad in ((4.0, 0.0), (float("nan"), 1.0), (4.0, float("nan"))):
        with pytest.raises(csbfs.CsbfsError) as ei:
            eng.set_direction(*bad)
        assert ei.value.status == csbfs.EINVAL
    forced = csbfs.Engine(g, flags=csbfs.FLAG_BOTTOM_UP_ONLY)
    r = forced.bfs(root)
    assert all(s["direction"] == csbfs.DIR_BOTTOM_UP for s in r.stats)
    dense = csbfs.Engine(g, flags=csbfs.FLAG_DENSE_ONLY)
    r = dense.bfs(root)
    assert all(s["direction"] == csbfs.DIR_DENSE for s in r.stats)
    with pytest.raises(csbfs.CsbfsError) as ei:
        csbfs.Engine(g, flags=csbfs.FLAG_BOTTOM_UP_ONLY | csbfs.FLAG_SPARSE_ONLY)
    assert ei.value.status == csbfs.EINVAL


def test_stats_truncated_beyond_max_levels():
    from paper_1208_5542_amd import csbfs
    n, p = 1024, 2
    src = np.arange(0, n - 1, dtype=np.int64)
    dst = np.arange(1, n, dtype=np.int64)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    eng = csbfs.Engine(g, max_levels=8)
    r = eng.bfs(0)
    assert r.n_levels == n
    assert len(r.stats) == 8
    assert (r.level.cpu().numpy() == np.arange(n)).all()
    assert (r.parent.cpu().numpy()[1:] == np.arange(n - 1)).all()


def test_high_degree_rows_use_chunk_queue():
    """A star with a hub of degree >> the per-wave row limit."""
    from paper_1208_5542_amd import csbfs
    n, p = 1 << 14, 4
    rng = np.random.default_rng(9)
    hub = 77
    leaves = rng.permutation(np.arange(n))[:9000]
    leaves = leaves[leaves != hub]
    src = np.r_[np.full(len(leaves), hub), rng.integers(0, n, 3000)].astype(np.int64)
    dst = np.r_[leaves, rng.integers(0, n, 3000)].astype(np.int64)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    for mode, flag in MODES.items():
        eng = csbfs.Engine(g, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS | flag)
        for root in (hub, int(leaves[0])):
            log(f"star mode={mode} root={root}")
            _check_search(eng, g, n, p, src, dst, root, adj, V)


def test_isolated_root_and_empty_graph():
    from paper_1208_5542_amd import csbfs
    n, p = 256, 2
    src = np.array([1, 2, 5], dtype=np.int64)
    dst = np.array([2, 3, 5], dtype=np.int64)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    eng = csbfs.Engine(g)
    for root in (0, 5):  # no tuple at all / only a self-loop
        r = eng.bfs(root)
        lev = r.level.cpu().numpy()
        assert r.n_levels == 1 and lev[root] == 0 and (np.delete(lev, root) == -1).all()
        assert r.parent.cpu().numpy()[root] == root
        assert r.stats[0]["frontier"] == 1
    e = csbfs.Graph(torch.zeros(1, dtype=torch.int64, device="cuda")[:0],
                    torch.zeros(1, dtype=torch.int64, device="cuda")[:0], 128, 2)
    r = csbfs.Engine(e).bfs(127)
    assert r.n_levels == 1


def test_no_sieve_flag_gives_same_search():
    from paper_1208_5542_amd import csbfs
    n, src, dst = _graph(11)
    p = 4
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    a = csbfs.Engine(g)
    b = csbfs.Engine(g, flags=csbfs.FLAG_NO_SIEVE)
    adj = oracle.Adjacency(n, src, dst)
    ones = np.ones(p * n, dtype=np.uint8)
    root = int(inputs.pick_roots(n, src, dst, 1, 1)[0])
    ra, rb = a.bfs(root), b.bfs(root)
    assert torch.equal(ra.level, rb.level) and torch.equal(ra.parent, rb.parent)
    ref = adj.alg3(p, ones, root)
    assert (b.stream_words(rb.n_levels) == ref.words).all()
    for k in range(1, ra.n_levels):
        # the sieve only drops bits (WAH bytes need not shrink)
        assert ra.stats[k]["sieved_bits"] <= rb.stats[k]["sieved_bits"]
        assert rb.stats[k]["sieved_bits"] == rb.stats[k]["unsieved_bits"]
        assert rb.stats[k]["wah_sieved_bytes"] == rb.stats[k]["wah_unsieved_bytes"]


def test_deterministic_repeat():
    from paper_1208_5542_amd import csbfs
    n, src, dst = _graph(12)
    g = csbfs.Graph(_dev(src), _dev(dst), n, 4)
    eng = csbfs.Engine(g, flags=csbfs.FLAG_KEEP_STREAMS)
    root = int(inputs.pick_roots(n, src, dst, 1, 3)[0])
    r1 = eng.bfs(root)
    l1, p1, w1 = r1.level.clone(), r1.parent.clone(), eng.stream_words(r1.n_levels)
    s1 = [u64(eng.stream(k, 1, 2)).tolist() for k in range(1, r1.n_levels)]
    r2 = eng.bfs(root)
    assert torch.equal(l1, r2.level) and torch.equal(p1, r2.parent)
    assert (w1 == eng.stream_words(r2.n_levels)).all()
    assert s1 == [u64(eng.stream(k, 1, 2)).tolist() for k in range(1, r2.n_levels)]


def test_error_statuses():
    from paper_1208_5542_amd import csbfs
    n, src, dst = _graph(10)
    with pytest.raises(csbfs.CsbfsError) as ei:
        csbfs.Graph(_dev(np.r_[src, [n]]), _dev(np.r_[dst, [0]]), n, 2)
    assert ei.value.status == csbfs.ERANGE
    g = csbfs.Graph(_dev(src), _dev(dst), n, 2)
    eng = csbfs.Engine(g)
    for bad in (-1, n):
        with pytest.raises(csbfs.CsbfsError) as ei:
            eng.bfs(bad)
        assert ei.value.status == csbfs.ERANGE
    with pytest.raises(csbfs.CsbfsError) as ei:
        eng.stream(1, 0, 0)
    assert ei.value.status == csbfs.EINVAL
