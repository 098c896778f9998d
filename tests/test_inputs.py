"""The seeded input generator: determinism, sizes, initiator statistics,
permutation and root picking (CPU only)."""
import numpy as np

from paper_1208_5542_amd import inputs


def test_rng_is_counter_based_splitmix64():
    # SplitMix64 from state 0: first outputs of the published generator
    assert inputs.rng(0, 0) == 0xE220A8397B1DCDAF
    assert inputs.rng(0, 1) == 0x6E789E6AA1B965F4
    assert inputs.rng(0, 2) == 0x06C45D188009454F


def test_rmat_deterministic_and_sized():
    s1, d1 = inputs.rmat_tuples(10)
    s2, d2 = inputs.rmat_tuples(10)
    assert (s1 == s2).all() and (d1 == d2).all()
    assert len(s1) == 16 * 1024
    assert s1.min() >= 0 and s1.max() < 1024 and d1.min() >= 0 and d1.max() < 1024
    s3, _ = inputs.rmat_tuples(10, seed=inputs.graph_seed(10) + 99)
    assert not (s3 == s1).all()


def test_rmat_initiator_statistics():
    scale = 12
    src, dst = inputs.rmat_tuples(scale, 16, permute=False)
    # the top bit of (src, dst) picks the quadrant at the first recursion level
    top = scale - 1
    q = ((src >> top) & 1) * 2 + ((dst >> top) & 1)
    freq = np.bincount(q, minlength=4) / len(q)
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.01)
    # every level has the same statistics
    qb = ((src >> 3) & 1) * 2 + ((dst >> 3) & 1)
    assert np.allclose(np.bincount(qb, minlength=4) / len(qb), [0.57, 0.19, 0.19, 0.05], atol=0.01)


def test_permutation_is_a_permutation():
    p = inputs.permutation(10000, 5)
    assert (np.sort(p) == np.arange(10000)).all()
    assert not (p == np.arange(10000)).all()


def test_permuted_graph_is_relabelled_unpermuted_graph():
    s0, d0 = inputs.rmat_tuples(9, 4, permute=False)
    s1, d1 = inputs.rmat_tuples(9, 4, permute=True)
    perm = inputs.permutation(512, inputs.graph_seed(9) + 1)
    assert (perm[s0] == s1).all() and (perm[d0] == d1).all()


def test_roots_distinct_and_non_isolated():
    src, dst = inputs.rmat_tuples(10)
    roots = inputs.pick_roots(1024, src, dst, 64, 17)
    assert len(set(roots.tolist())) == len(roots) == 64
    nz = set(src[src != dst].tolist()) | set(dst[src != dst].tolist())
    assert all(int(r) in nz for r in roots)
    # a graph with only self-loops has no eligible root
    assert len(inputs.pick_roots(8, np.array([1, 2]), np.array([1, 2]), 4, 0)) == 0


def test_er_tuples():
    s, d = inputs.er_tuples(1 << 12, 8 << 12, 77)
    assert len(s) == 8 << 12 and s.max() < 4096 and d.min() >= 0
    assert abs(np.bincount(s, minlength=4096).mean() - 8) < 1e-9
