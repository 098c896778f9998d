"""Serving loop: queries over several resident graphs, continuously admitted
into concurrent single-root or batched searches under an HBM budget. Every
result must be identical to the same search alone (the single-root engine,
and a server that answers one request at a time) and to the oracle's
levels; both ways of answering are exercised."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_5542_amd import inputs
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).cuda()


@pytest.fixture(scope="module")
def pool():
    """Small stand-ins for the serving pool: R-MAT graphs of three scales and
    an Erdos-Renyi graph with 8 n tuples (average degree 16)."""
    from paper_1208_5542_amd import csbfs
    out = []
    for name, n, p, (src, dst) in [
        ("rmat10", 1 << 10, 1, inputs.rmat_tuples(10, 16)),
        ("rmat12", 1 << 12, 4, inputs.rmat_tuples(12, 16)),
        ("rmat13", 1 << 13, 2, inputs.rmat_tuples(13, 16)),
        ("er12", 1 << 12, 4, inputs.er_tuples(1 << 12, 8 << 12, 0xE12)),
    ]:
        g = csbfs.Graph(_dev(src), _dev(dst), n, p)
        roots = [int(r) for r in inputs.pick_roots(n, src, dst, 24, 7 + n)]
        out.append(dict(name=name, n=n, p=p, src=src, dst=dst, g=g, roots=roots,
                        adj=oracle.Adjacency(n, src, dst)))
    return out


def _requests(pool, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        gi = int(rng.integers(len(pool)))
        roots = pool[gi]["roots"]
        reqs.append((gi, roots[int(rng.integers(len(roots)))]))
    return reqs


def _serve(server, gids, pool, reqs):
    outs, ids = [], []
    for gi, root in reqs:
        out = torch.full((pool[gi]["n"],), -7, dtype=torch.int32, device="cuda")
        ids.append(server.submit(gids[gi], root, out))
        outs.append(out)
    infos = [server.wait(i) for i in ids]
    return outs, infos


def test_results_identical_alone_and_in_the_mix(pool):
    from paper_1208_5542_amd import csbfs
    reqs = _requests(pool, 96, 1)
    mix = csbfs.Server(slots=3, max_batch=8, max_levels=64, hbm_budget=1 << 30)
    gids = [mix.add_graph(e["g"]) for e in pool]
    log("serving: 96 mixed requests on 3 slots")
    outs, infos = _serve(mix, gids, pool, reqs)
    assert all(i["status"] == 0 for i in infos)
    assert max(i["batch_size"] for i in infos) > 1, "no request was taken together with another"
    assert all(i["t_submit"] <= i["t_start"] <= i["t_done"] for i in infos)
    # alone: one request at a time on a one-slot server, and the single-root engine
    alone = csbfs.Server(slots=1, max_batch=1, max_levels=64, hbm_budget=1 << 30)
    for e in pool:
        alone.add_graph(e["g"])
    log("serving: the same requests one at a time")
    outs1, infos1 = [], []
    for gi, root in reqs:
        o, inf = _serve(alone, list(range(len(pool))), pool, [(gi, root)])
        outs1.append(o[0])
        infos1.append(inf[0])
    assert all(i["batch_size"] == 1 for i in infos1)
    engines = [csbfs.Engine(e["g"], max_levels=64) for e in pool]
    for k, ((gi, root), a, b) in enumerate(zip(reqs, outs, outs1)):
        assert torch.equal(a, b), f"request {k}: mix differs from alone"
        single = engines[gi].bfs(root).level
        assert torch.equal(a, single), f"request {k}: differs from the single-root engine"
    for k in range(0, len(reqs), 12):
        gi, root = reqs[k]
        ref = pool[gi]["adj"].bfs(root)
        assert (outs[k].cpu().numpy() == ref).all(), f"request {k}: differs from the oracle"
    mix.close()
    alone.close()


def test_admission_under_a_small_budget(pool):
    """A budget that holds one engine at a time: requests for different
    graphs are served one engine after the other, never above the budget."""
    from paper_1208_5542_amd import csbfs
    probe = csbfs.Server(slots=1, max_batch=8, max_levels=64, hbm_budget=1 << 40)
    need = max(probe.graph_bytes(probe.add_graph(e["g"])) for e in pool)
    probe.close()
    server = csbfs.Server(slots=3, max_batch=8, max_levels=64, hbm_budget=need)
    gids = [server.add_graph(e["g"]) for e in pool]
    reqs = _requests(pool, 48, 2)
    log(f"serving under a budget of {need} bytes")
    outs, infos = [], []
    ids = []
    for gi, root in reqs:
        out = torch.empty(pool[gi]["n"], dtype=torch.int32, device="cuda")
        ids.append(server.submit(gids[gi], root, out))
        outs.append(out)
        assert server.bytes_held() <= need
    infos = [server.wait(i) for i in ids]
    assert server.bytes_held() <= need
    assert all(i["status"] == 0 for i in infos)
    engines = [csbfs.Engine(e["g"], max_levels=64) for e in pool]
    for (gi, root), o in zip(reqs, outs):
        assert torch.equal(o, engines[gi].bfs(root).level)
    server.close()


def test_both_answer_paths_match(pool):
    """Bursts of one graph's requests are answered by batched searches and
    lone requests by single-root searches; both equal the oracle."""
    from paper_1208_5542_amd import csbfs
    e = pool[1]
    server = csbfs.Server(slots=1, max_batch=16, max_levels=64, hbm_budget=1 << 30)
    gid = server.add_graph(e["g"])
    burst = [e["roots"][k % len(e["roots"])] for k in range(48)]
    outs = [torch.full((e["n"],), -7, dtype=torch.int32, device="cuda") for _ in burst]
    # a burst, queued much faster than one slot answers it
    ids = [server.submit(gid, root, out) for root, out in zip(burst, outs)]
    infos = [server.wait(i) for i in ids]
    # lone requests, each waited for before the next
    lone = e["roots"][:4]
    for root in lone:
        out = torch.full((e["n"],), -7, dtype=torch.int32, device="cuda")
        infos.append(server.wait(server.submit(gid, root, out)))
        outs.append(out)
    assert all(i["status"] == 0 for i in infos)
    assert any(i["batched"] == 1 for i in infos) and any(i["batched"] == 0 for i in infos)
    for root, o in zip(burst + lone, outs):
        assert (o.cpu().numpy() == e["adj"].bfs(root)).all()
    server.close()


def test_serving_errors(pool):
    from paper_1208_5542_amd import csbfs
    tiny = csbfs.Server(slots=1, max_batch=4, max_levels=16, hbm_budget=1024)
    with pytest.raises(csbfs.CsbfsError) as ei:
        tiny.add_graph(pool[0]["g"])
    assert ei.value.status == csbfs.ENOSPACE
    tiny.close()
    for bad in (dict(slots=0), dict(slots=17), dict(max_batch=65), dict(max_levels=0), dict(hbm_budget=0)):
        kw = dict(slots=1, max_batch=4, max_levels=16, hbm_budget=1 << 30)
        kw.update(bad)
        with pytest.raises(csbfs.CsbfsError) as ei:
            csbfs.Server(**kw)
        assert ei.value.status == csbfs.EINVAL
    s = csbfs.Server(slots=1, max_batch=4, max_levels=16, hbm_budget=1 << 30)
    gid = s.add_graph(pool[1]["g"])
    with pytest.raises(csbfs.CsbfsError) as ei:
        s.submit(gid + 5, 0)
    assert ei.value.status == csbfs.EINVAL
    with pytest.raises(csbfs.CsbfsError) as ei:
        s.submit(gid, pool[1]["n"])
    assert ei.value.status == csbfs.ERANGE
    with pytest.raises(csbfs.CsbfsError) as ei:
        s.wait(12345)
    assert ei.value.status == csbfs.EINVAL
    rid = s.submit(gid, pool[1]["roots"][0])  # no copy-out
    info = s.wait(rid)
    assert info["status"] == 0 and info["n_levels"] >= 2
    s.drain()
    s.close()


def test_concurrent_submitters_and_eviction(pool):
    """Four client threads submit at once to four slots whose budget holds
    two engines for four graphs, so engines are released and rebuilt while
    batches run; every result must still equal the single-root engine's."""
    import threading

    from paper_1208_5542_amd import csbfs
    probe = csbfs.Server(slots=1, max_batch=16, max_levels=64, hbm_budget=1 << 40)
    need = sorted(probe.graph_bytes(probe.add_graph(e["g"])) for e in pool)
    probe.close()
    budget = need[-1] + need[-2]
    server = csbfs.Server(slots=4, max_batch=16, max_levels=64, hbm_budget=budget)
    gids = [server.add_graph(e["g"]) for e in pool]
    results = {}
    errors = []

    def client(seed):
        try:
            reqs = _requests(pool, 40, seed)
            outs, ids = [], []
            for gi, root in reqs:
                out = torch.empty(pool[gi]["n"], dtype=torch.int32, device="cuda")
                ids.append(server.submit(gids[gi], root, out))
                outs.append(out)
            infos = [server.wait(i) for i in ids]
            results[seed] = (reqs, outs, infos)
        except Exception as exc:  # surfaced below
            errors.append(exc)

    log("serving: 4 client threads, budget of two engines")
    threads = [threading.Thread(target=client, args=(100 + k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=240)
    assert not errors, errors
    assert len(results) == 4
    assert server.bytes_held() <= budget
    engines = [csbfs.Engine(e["g"], max_levels=64) for e in pool]
    for reqs, outs, infos in results.values():
        assert all(i["status"] == 0 for i in infos)
        for (gi, root), o in zip(reqs, outs):
            assert torch.equal(o, engines[gi].bfs(root).level)
    server.close()
