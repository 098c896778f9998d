"""Batched searches (up to 64 roots at once) against the oracle, root by
root: levels bit-exact, every root's per-level streams byte-identical to the
oracle's Algorithm 3 for that root alone, byte accounting summed over the
roots, edges scanned once per level for the union of the frontiers, and
reuse of one engine across batches of different sizes."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).cuda()


def _expected_stats(refs, adj, p, n_levels):
    """Per-level sums over the roots whose level-k frontier is non-empty."""
    off = ~np.eye(p, dtype=bool)
    out = []
    for k in range(n_levels):
        e = dict(frontier=0, view_bits=0, sieved_bits=0, unsieved_bits=0, raw_bytes=0,
                 wah_unsieved_bytes=0, wah_sieved_bytes=0, self_bytes=0)
        send = np.zeros(p, dtype=np.int64)
        recv = np.zeros(p, dtype=np.int64)
        union = set()
        for ref in refs:
            if k >= ref.n_levels:
                continue
            verts = np.flatnonzero(ref.level == k)
            union.update(verts.tolist())
            lb = ref.level_bytes()[k]
            e["frontier"] += lb["frontier"]
            if k == 0:
                e["view_bits"] += p
                continue
            w = ref.words[k].astype(np.int64)
            e["view_bits"] += int(ref.sieved_bits[k].sum())
            e["sieved_bits"] += int(ref.sieved_bits[k][off].sum())
            e["unsieved_bits"] += (p - 1) * lb["frontier"]
            e["raw_bytes"] += lb["raw"]
            e["wah_unsieved_bytes"] += lb["wah_unsieved"]
            e["wah_sieved_bytes"] += lb["wah_sieved"]
            e["self_bytes"] += lb["self"]
            wo = np.where(off, w, 0)
            send += 8 * wo.sum(axis=1)
            recv += 8 * wo.sum(axis=0)
        e["max_rank_bytes"] = int((send + recv).max()) if k > 0 else 0
        e["edges"] = sum(adj.degree(int(u)) for u in union)
        out.append(e)
    return out


def _check_batch(eng, n, p, roots, adj, V, keep=True, max_levels=64, stream_roots=None):
    r = eng.bfs(roots)
    torch.cuda.synchronize()
    lev = r.level.cpu().numpy()
    refs = [adj.alg3(p, V, int(s), max_levels=max_levels, dump=keep) for s in roots]
    assert r.n_levels == max(ref.n_levels for ref in refs)
    for b, ref in enumerate(refs):
        assert (lev[b] == ref.level).all(), f"level of root {b} ({roots[b]})"
    words = eng.stream_words(r.n_levels)
    for b, ref in enumerate(refs):
        exp = np.zeros((r.n_levels, p, p), dtype=np.int64)
        exp[: ref.n_levels] = ref.words
        assert (words[:, b] == exp).all(), f"stream lengths of root {b}"
    if keep:
        for b in (range(len(roots)) if stream_roots is None else stream_roots):
            ref = refs[b]
            for k in range(1, r.n_levels):
                for i in range(p):
                    for j in range(p):
                        got = u64(eng.stream(k, b, i, j))
                        if k >= ref.n_levels:
                            assert len(got) == 0
                            continue
                        exp = ref.streams[k, i, j, : ref.words[k, i, j]]
                        assert got.tolist() == exp.tolist(), (b, k, i, j)
    exp_stats = _expected_stats(refs, adj, p, min(r.n_levels, max_levels))
    for k, e in enumerate(exp_stats):
        got = r.stats[k]
        for key, val in e.items():
            if key == "edges" and got["direction"] == 1:
                # bottom-up: the entries read before every missing root was found
                assert 0 <= got[key] <= 2 * adj_entries(adj, n), (k, key, got[key])
                continue
            assert got[key] == val, (k, key, got[key], val)
    return r


def adj_entries(adj, n):
    return sum(adj.degree(v) for v in range(n)) // 2


BATCH_MODES = {"auto": 0, "sparse": 8, "bottom_up": 32}


@pytest.mark.parametrize("mode", list(BATCH_MODES))
@pytest.mark.parametrize("scale,p,nroots", [(10, 1, 1), (10, 2, 7), (10, 4, 64), (11, 8, 33),
                                            (12, 4, 64), (12, 1, 64), (13, 2, 20)])
def test_batch_matches_oracle(scale, p, nroots, mode):
    """Each evaluation of the batched product (top-down push of root masks,
    bottom-up pull of frontier masks, or chosen per level) gives every root
    the levels and streams of its own search."""
    from paper_1208_5542_amd import csbfs
    n = 1 << scale
    src, dst = inputs.rmat_tuples(scale, 16)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    roots = [int(x) for x in inputs.pick_roots(n, src, dst, nroots, inputs.graph_seed(scale) + 2)]
    eng = csbfs.BatchEngine(g, max_roots=64, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS | BATCH_MODES[mode])
    log(f"batch scale={scale} p={p} roots={nroots} mode={mode}")
    r = _check_batch(eng, n, p, roots, adj, V, stream_roots=range(min(nroots, 6)))
    dirs = [s["direction"] for s in r.stats]
    if mode == "sparse":
        assert all(d == 0 for d in dirs)
    if mode == "bottom_up":
        assert all(d == 1 for d in dirs)


def test_batch_repeats_isolated_and_reuse():
    """Repeated roots, an isolated root, and one engine reused for a smaller
    batch right after a full one (no state may leak between batches)."""
    from paper_1208_5542_amd import csbfs
    scale, p = 11, 4
    n = 1 << scale
    src, dst = inputs.rmat_tuples(scale, 16)
    deg = np.bincount(np.r_[src, dst], minlength=n)
    isolated = int(np.flatnonzero(deg == 0)[0])
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    picked = [int(x) for x in inputs.pick_roots(n, src, dst, 40, 17)]
    roots = picked[:30] + [picked[0], picked[0], isolated] + picked[30:40] + [picked[5]] * 21
    assert len(roots) == 64
    eng = csbfs.BatchEngine(g, max_roots=64, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS)
    log("batch repeats + isolated root, 64 roots")
    r = _check_batch(eng, n, p, roots, adj, V, stream_roots=[0, 30, 31, 32])
    lev = r.level.cpu().numpy()
    assert (lev[30] == lev[0]).all() and (lev[31] == lev[0]).all()
    assert lev[32][isolated] == 0 and (np.delete(lev[32], isolated) == -1).all()
    log("batch reuse with 3 roots")
    _check_batch(eng, n, p, picked[10:13], adj, V)
    log("batch reuse with 1 root")
    r1 = _check_batch(eng, n, p, [isolated], adj, V)
    assert r1.n_levels == 1


def test_batch_single_root_equals_engine():
    from paper_1208_5542_amd import csbfs
    scale, p = 12, 4
    n = 1 << scale
    src, dst = inputs.rmat_tuples(scale, 16)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    single = csbfs.Engine(g, max_levels=64)
    batch = csbfs.BatchEngine(g, max_roots=8, max_levels=64)
    roots = [int(x) for x in inputs.pick_roots(n, src, dst, 8, 4)]
    rb = batch.bfs(roots)
    for b, s in enumerate(roots):
        rs = single.bfs(s)
        assert torch.equal(rs.level, rb.level[b]), b
    assert rb.n_levels == max(int(rb.level[b].max()) + 1 for b in range(len(roots)))


def test_batch_high_degree_hub_and_long_path():
    """Chunk-queue rows carrying root masks (a hub of degree ~9000), and a
    long path with many levels of tiny frontiers, including levels past
    max_levels (counters truncated, levels still exact)."""
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
    roots = [hub] + [int(x) for x in leaves[:40]]
    eng = csbfs.BatchEngine(g, max_roots=64, max_levels=64, flags=csbfs.FLAG_KEEP_STREAMS)
    log("batch star hub, 41 roots")
    _check_batch(eng, n, p, roots, adj, V, stream_roots=[0, 1])

    n, p = 4096, 4
    perm = rng.permutation(n)
    src = np.r_[perm[:-1], rng.integers(0, n, 40)].astype(np.int64)
    dst = np.r_[perm[1:], rng.integers(0, n, 40)].astype(np.int64)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    V = oracle.directory(n, p, src, dst).reshape(-1)
    roots = [int(perm[0]), int(perm[-1]), int(perm[n // 2])]
    eng = csbfs.BatchEngine(g, max_roots=4, max_levels=4096)
    log("batch long path, 3 roots")
    r = _check_batch(eng, n, p, roots, adj, V, keep=False, max_levels=4096)
    assert r.n_levels > 50
    small = csbfs.BatchEngine(g, max_roots=4, max_levels=8)
    rs = small.bfs(roots)
    assert rs.n_levels == r.n_levels and len(rs.stats) == 8
    assert torch.equal(rs.level, r.level)


def test_batch_no_sieve_flag():
    from paper_1208_5542_amd import csbfs
    scale, p = 11, 4
    n = 1 << scale
    src, dst = inputs.rmat_tuples(scale, 16)
    g = csbfs.Graph(_dev(src), _dev(dst), n, p)
    adj = oracle.Adjacency(n, src, dst)
    ones = np.ones(p * n, dtype=np.uint8)
    roots = [int(x) for x in inputs.pick_roots(n, src, dst, 5, 8)]
    eng = csbfs.BatchEngine(g, max_roots=8, flags=csbfs.FLAG_NO_SIEVE | csbfs.FLAG_KEEP_STREAMS)
    log("batch no sieve")
    _check_batch(eng, n, p, roots, adj, ones)


def test_batch_error_statuses():
    from paper_1208_5542_amd import csbfs
    n = 1 << 10
    src, dst = inputs.rmat_tuples(10, 16)
    g = csbfs.Graph(_dev(src), _dev(dst), n, 2)
    for bad in (0, 65):
        with pytest.raises(csbfs.CsbfsError) as ei:
            csbfs.BatchEngine(g, max_roots=bad)
        assert ei.value.status == csbfs.EINVAL
    with pytest.raises(csbfs.CsbfsError) as ei:
        csbfs.BatchEngine(g, flags=csbfs.FLAG_DENSE_ONLY)
    assert ei.value.status == csbfs.EINVAL
    eng = csbfs.BatchEngine(g, max_roots=4)
    with pytest.raises(csbfs.CsbfsError) as ei:
        eng.bfs([0, 1, 2, 3, 4])
    assert ei.value.status == csbfs.EINVAL
    with pytest.raises(csbfs.CsbfsError) as ei:
        eng.bfs([])
    assert ei.value.status == csbfs.EINVAL
    for bad in (-1, n):
        with pytest.raises(csbfs.CsbfsError) as ei:
            eng.bfs([0, bad])
        assert ei.value.status == csbfs.ERANGE
    eng.bfs([1, 2])
    with pytest.raises(csbfs.CsbfsError) as ei:
        eng.stream(1, 0, 0, 0)  # no KEEP_STREAMS
    assert ei.value.status == csbfs.EINVAL
