"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Only tuple lists, permutations and roots come from here; none of the BFS,
sieve or compression arithmetic does. The workloads mirror the paper's
experimental setup (Sec. VII.A): Kronecker/R-MAT graphs with 2^scale vertices
and edgefactor * 2^scale undirected tuples (edgefactor 16), self-loops and
duplicates kept.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librmat.so")
_lib = None

# Initiator of the recursive matrix generator (probabilities of the four
# quadrants); the fourth is 1 - A - B - C.
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def graph_seed(scale: int) -> int:
    """Seed of the tuple draws for an R-MAT graph of the given scale."""
    return 0x5EED0000 + scale


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing; run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    i64, u64, i32, dbl, p64 = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_void_p)
    lib.rmat_rng.argtypes = [u64, u64]
    lib.rmat_rng.restype = u64
    lib.rmat_permutation.argtypes = [i64, u64, p64]
    lib.rmat_permutation.restype = ctypes.c_int
    lib.rmat_edges.argtypes = [i32, i64, dbl, dbl, dbl, u64, p64, p64, p64]
    lib.rmat_edges.restype = ctypes.c_int
    lib.er_edges.argtypes = [i64, i64, u64, p64, p64]
    lib.er_edges.restype = ctypes.c_int
    lib.rmat_pick_roots.argtypes = [i64, i64, p64, p64, i64, u64, p64]
    lib.rmat_pick_roots.restype = i64
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def rng(seed: int, ctr: int) -> int:
    return int(_load().rmat_rng(seed, ctr))


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.int64)
    if _load().rmat_permutation(n, seed, _ptr(perm)) != 0:
        raise ValueError("bad permutation arguments")
    return perm


def rmat_tuples(scale: int, edgefactor: int = 16, *, seed: int | None = None,
                permute: bool = True, a: float = RMAT_A, b: float = RMAT_B,
                c: float = RMAT_C) -> tuple[np.ndarray, np.ndarray]:
    """R-MAT tuple list (src, dst) as int64 arrays of edgefactor * 2^scale entries.

    Ids are mapped through a seeded uniform permutation (seed + 1) unless
    ``permute`` is False.
    """
    if seed is None:
        seed = graph_seed(scale)
    n = 1 << scale
    m = edgefactor * n
    src = np.empty(m, dtype=np.int64)
    dst = np.empty(m, dtype=np.int64)
    perm = permutation(n, seed + 1) if permute else None
    rc = _load().rmat_edges(scale, m, a, b, c, seed,
                            _ptr(perm) if perm is not None else None,
                            _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("bad R-MAT arguments")
    return src, dst


def er_tuples(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Uniform random tuple list: m tuples with independent uniform endpoints."""
    src = np.empty(m, dtype=np.int64)
    dst = np.empty(m, dtype=np.int64)
    if _load().er_edges(n, m, seed, _ptr(src), _ptr(dst)) != 0:
        raise ValueError("bad Erdos-Renyi arguments")
    return src, dst


def pick_roots(n: int, src: np.ndarray, dst: np.ndarray, count: int,
               seed: int) -> np.ndarray:
    """Distinct roots, uniform over vertices with a non-self-loop tuple."""
    roots = np.empty(count, dtype=np.int64)
    got = _load().rmat_pick_roots(n, len(src), _ptr(src), _ptr(dst), count,
                                  seed, _ptr(roots))
    if got < 0:
        raise ValueError("bad root-picker arguments")
    return roots[:got].copy()


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: graph recipe, partition count and roots."""
    name: str
    scale: int
    p: int
    n_roots: int
    edgefactor: int = 16

    @property
    def n(self) -> int:
        return 1 << self.scale

    @property
    def m(self) -> int:
        return self.edgefactor << self.scale

    def tuples(self) -> tuple[np.ndarray, np.ndarray]:
        return rmat_tuples(self.scale, self.edgefactor)

    def roots(self, src: np.ndarray, dst: np.ndarray, count: int | None = None) -> np.ndarray:
        return pick_roots(self.n, src, dst, count or self.n_roots,
                          graph_seed(self.scale) + 2)


# The single-root workloads: a small parity case on one partition, a 4 x 4
# block grid at scale 22 and an 8 x 8 block grid at scale 26; and the batched
# one: 64 roots searched together at scale 24 on a 4 x 4 grid.
WORKLOADS = {
    "rmat10_p1": Workload("rmat10_p1", 10, 1, 16),
    "rmat22_p4": Workload("rmat22_p4", 22, 4, 64),
    "rmat26_p8": Workload("rmat26_p8", 26, 8, 64),
    "rmat24_p4": Workload("rmat24_p4", 24, 4, 64),
}
