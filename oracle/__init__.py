"""Oracle for the compression + sieve BFS: plain serial CPU code (oracle.c).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU path and must never be used as a fallback for it.

Bit vectors cross this interface as one uint8 per bit. Byte accounting per
level follows the paper's communication-volume discussion (Sec. VI.A):
raw bitmap bytes of the Allgatherv of Alg. 1, WAH bytes of Alg. 2 (no sieve)
and sieved WAH bytes of Alg. 3, all counted over messages between distinct
processors; the self stream of Alg. 3 is counted apart.

Parity pins: every function here is pinned by a test in ``tests/`` against
the paper's worked examples (Fig. 2 matrix, Table 3, Table 2 arithmetic),
brute force on tiny inputs, closed forms or invariants (Lemmas 1 and 2). The
64-bit WAH word layout beyond what Table 3 fixes (fill bit at bit 62,
single-group runs written as fills) is a stated reading, pinned by closed
forms and round trips only.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; run oracle/build.py or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_adj_build.argtypes = [i64, i64, vp, vp]
    lib.oracle_adj_build.restype = vp
    lib.oracle_adj_free.argtypes = [vp]
    lib.oracle_adj_free.restype = None
    lib.oracle_adj_n.argtypes = [vp]
    lib.oracle_adj_n.restype = i64
    lib.oracle_adj_degree.argtypes = [vp, i64]
    lib.oracle_adj_degree.restype = i64
    lib.oracle_bfs.argtypes = [vp, i64, vp]
    lib.oracle_bfs.restype = i64
    lib.oracle_parents_max.argtypes = [vp, vp, i64, vp]
    lib.oracle_parents_max.restype = ctypes.c_int
    lib.oracle_validate.argtypes = [i64, i64, vp, vp, i64, vp, vp, vp]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_directory.argtypes = [i64, i32, i64, vp, vp, vp]
    lib.oracle_directory.restype = ctypes.c_int
    lib.oracle_wah_encode.argtypes = [vp, i64, i32, i32, vp, i64]
    lib.oracle_wah_encode.restype = i64
    lib.oracle_wah_decode.argtypes = [vp, i64, i64, i32, i32, vp]
    lib.oracle_wah_decode.restype = ctypes.c_int
    lib.oracle_alg3_cap.argtypes = [i64, i32]
    lib.oracle_alg3_cap.restype = i64
    lib.oracle_alg3.argtypes = [vp, i32, vp, i64, i32, vp, vp, vp, vp, vp, vp]
    lib.oracle_alg3.restype = i64
    lib.oracle_teps_m.argtypes = [i64, vp, vp, vp]
    lib.oracle_teps_m.restype = i64
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"], "need a contiguous numpy array"
    return a.ctypes.data


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


class Adjacency:
    """Undirected adjacency of a tuple list (a self-loop appears twice)."""

    def __init__(self, n: int, src, dst):
        self.src = _i64(src)
        self.dst = _i64(dst)
        assert self.src.shape == self.dst.shape
        self.n = int(n)
        h = _load().oracle_adj_build(self.n, len(self.src), _p(self.src), _p(self.dst))
        if not h:
            raise ValueError("oracle_adj_build failed (bad sizes or ids out of range)")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_adj_free(h)
            self._h = None

    def degree(self, v: int) -> int:
        return int(_load().oracle_adj_degree(self._h, v))

    def bfs(self, root: int) -> np.ndarray:
        """Hop levels from root (-1 if unreachable), serial FIFO queue."""
        level = np.empty(self.n, dtype=np.int32)
        nl = _load().oracle_bfs(self._h, root, _p(level))
        if nl < 0:
            raise ValueError("oracle_bfs: bad root")
        return level

    def parents_max(self, level: np.ndarray, root: int) -> np.ndarray:
        """Parent by the (select, max) rule (Sec. III.A)."""
        level = np.ascontiguousarray(level, dtype=np.int32)
        parent = np.empty(self.n, dtype=np.int32)
        if _load().oracle_parents_max(self._h, _p(level), root, _p(parent)) != 0:
            raise ValueError("oracle_parents_max failed")
        return parent

    def alg3(self, p: int, V: np.ndarray, root: int, max_levels: int = 64, dump: bool = False):
        """Algorithm 3 level loop over p virtual processors; see Alg3Result."""
        lib = _load()
        n = self.n
        level = np.empty(n, dtype=np.int32)
        parent = np.empty(n, dtype=np.int32)
        words = np.zeros((max_levels, p, p), dtype=np.int64)
        sbits = np.zeros((max_levels, p, p), dtype=np.int64)
        uwords = np.zeros((max_levels, p), dtype=np.int64)
        cap = int(lib.oracle_alg3_cap(n, p))
        streams = np.zeros((max_levels, p, p, cap), dtype=np.uint64) if dump else None
        V = np.ascontiguousarray(V, dtype=np.uint8)
        assert V.size == p * n
        nl = lib.oracle_alg3(self._h, p, _p(V), root, max_levels, _p(level), _p(parent),
                             _p(words), _p(sbits), _p(uwords), _p(streams))
        if nl == -2:
            raise ValueError("oracle_alg3: max_levels too small")
        if nl < 0:
            raise ValueError(f"oracle_alg3 failed ({nl})")
        nl = int(nl)
        return Alg3Result(n=n, p=p, n_levels=nl, level=level, parent=parent,
                          words=words[:nl].copy(), sieved_bits=sbits[:nl].copy(),
                          unsieved_words=uwords[:nl].copy(),
                          streams=None if streams is None else streams[:nl].copy(), cap=cap)


@dataclass
class Alg3Result:
    n: int
    p: int
    n_levels: int
    level: np.ndarray
    parent: np.ndarray
    words: np.ndarray          # [levels, p, p]: stream words P_i -> P_j
    sieved_bits: np.ndarray    # [levels, p, p]: ones in f_i . V_{j,i}
    unsieved_words: np.ndarray  # [levels, p]: words of WAH-64(f_i), no sieve
    streams: np.ndarray | None  # [levels, p, p, cap]
    cap: int

    def level_bytes(self) -> list[dict]:
        """Per-level byte accounting (one dict per level)."""
        return [level_bytes(self.n, self.p, self.words[k], self.unsieved_words[k],
                            int((self.level == k).sum()))
                for k in range(self.n_levels)]

    def rank_volumes(self) -> dict:
        """Communication volume of every processor over the whole search."""
        return rank_volumes(self.p, self.words)


def raw_bitmap_bytes(nbits: int) -> int:
    """Bytes of an uncompressed bitmap of nbits bits held in 64-bit words."""
    return 8 * ((nbits + 63) // 64)


def bitmap_bytes(nbits: int) -> int:
    """Bytes of an nbits-bit bitmap packed into bytes (Table 2's bitmap column)."""
    return (nbits + 7) // 8


def sparse_vector_bytes(count: int) -> int:
    """Bytes of a sparse vector of count 64-bit vertex ids (Table 2)."""
    return 8 * count


def level_bytes(n: int, p: int, words, unsieved_words, frontier: int) -> dict:
    """Byte accounting for the messages that carry one frontier level."""
    words = np.asarray(words, dtype=np.int64).reshape(p, p)
    uw = np.asarray(unsieved_words, dtype=np.int64).reshape(p)
    R = n // p
    off = ~np.eye(p, dtype=bool)
    sent = int(8 * words[off].sum())
    self_b = int(8 * np.trace(words))
    if words.sum() == 0:  # level 0 is seeded, never sent
        raw = 0
        wah_unsieved = 0
    else:
        raw = p * (p - 1) * raw_bitmap_bytes(R)
        wah_unsieved = int(8 * (p - 1) * uw.sum())
    send = 8 * (words.sum(axis=1) - np.diag(words))
    recv = 8 * (words.sum(axis=0) - np.diag(words))
    # max_rank_volume: the largest bytes sent plus received by one processor
    # in this level alone (the whole-search volume is rank_volumes())
    return {"frontier": frontier, "raw": raw, "wah_unsieved": wah_unsieved,
            "wah_sieved": sent, "self": self_b,
            "max_rank_volume": int((send + recv).max()) if p > 1 else 0}


def rank_volumes(p: int, words) -> dict:
    """Communication volume of each processor (Sec. VI.A): V_i is the size of
    every message P_i takes part in over the whole algorithm, read here as
    the WAH bytes it sends plus the WAH bytes it receives, summed over all
    levels, with the self stream (never communicated) left out. The volume
    of the algorithm is V = max_i V_i.

    words: [levels, p, p] stream lengths, words[k, i, j] for P_i -> P_j.
    Returns sent[p], received[p], volume[p] (bytes) and max (bytes)."""
    w = np.asarray(words, dtype=np.int64).reshape(-1, p, p)
    sent = np.zeros(p, dtype=np.int64)
    received = np.zeros(p, dtype=np.int64)
    for k in range(w.shape[0]):
        for i in range(p):
            for j in range(p):
                if i != j:
                    sent[i] += 8 * w[k, i, j]
                    received[j] += 8 * w[k, i, j]
    volume = sent + received
    return {"sent": sent.tolist(), "received": received.tolist(), "volume": volume.tolist(),
            "max": int(volume.max()) if p > 1 else 0}


def validate(n: int, src, dst, root: int, level, parent, ref_level=None) -> int:
    """BFS tree validity rules; 0 if valid, else the OR of violated rule bits."""
    src, dst = _i64(src), _i64(dst)
    level = np.ascontiguousarray(level, dtype=np.int32)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    ref = None if ref_level is None else np.ascontiguousarray(ref_level, dtype=np.int32)
    rc = _load().oracle_validate(n, len(src), _p(src), _p(dst), root, _p(level), _p(parent), _p(ref))
    if rc < 0:
        raise ValueError("oracle_validate: bad arguments")
    return int(rc)


def directory(n: int, p: int, src, dst) -> np.ndarray:
    """Directory vectors as bytes, shape (p, p, n/p): V[i, j, k] of Eq. dir-vec."""
    src, dst = _i64(src), _i64(dst)
    V = np.empty(p * n, dtype=np.uint8)
    if _load().oracle_directory(n, p, len(src), _p(src), _p(dst), _p(V)) != 0:
        raise ValueError("oracle_directory: bad arguments")
    return V.reshape(p, p, n // p)


def wah_encode(bits, w: int = 64, fill_bit_field: bool = True) -> np.ndarray:
    """WAH words (uint64) of a 0/1 vector."""
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    g = w - 1
    cap = len(bits) // g + 2
    out = np.zeros(cap, dtype=np.uint64)
    nw = _load().oracle_wah_encode(_p(bits), len(bits), w, int(fill_bit_field), _p(out), cap)
    if nw < 0:
        raise ValueError(f"oracle_wah_encode failed ({nw})")
    return out[:nw].copy()


def wah_decode(words, nbits: int, w: int = 64, fill_bit_field: bool = True) -> np.ndarray:
    """0/1 vector of nbits decoded from WAH words; raises on an invalid stream."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    bits = np.zeros(max(nbits, 1), dtype=np.uint8)
    rc = _load().oracle_wah_decode(_p(words), len(words), nbits, w, int(fill_bit_field), _p(bits))
    if rc != 0:
        raise ValueError("invalid WAH stream")
    return bits[:nbits].copy()


def teps_m(src, dst, level) -> int:
    """Input tuples inside the traversed component (TEPS numerator)."""
    src, dst = _i64(src), _i64(dst)
    level = np.ascontiguousarray(level, dtype=np.int32)
    return int(_load().oracle_teps_m(len(src), _p(src), _p(dst), _p(level)))


def stream_from_levels(level, V, n: int, p: int, k: int, i: int, j: int) -> np.ndarray:
    """The stream P_i -> P_j carrying level k, from a level vector alone:
    WAH-64 of (level[R_i] == k) . V_{j,i} (Alg. 3, sieve then Compress)."""
    R = n // p
    piece = (np.asarray(level[i * R:(i + 1) * R]) == k).astype(np.uint8)
    piece &= np.asarray(V[j, i], dtype=np.uint8)
    return wah_encode(piece, 64, True)


def pack_bits(bits) -> np.ndarray:
    """0/1 vector -> uint64 words, bit k of the vector in bit k % 64 of word k // 64."""
    b = np.asarray(bits, dtype=np.uint8)
    pad = (-len(b)) % 64
    if pad:
        b = np.concatenate([b, np.zeros(pad, dtype=np.uint8)])
    return np.packbits(b, bitorder="little").view(np.uint64).copy()


def unpack_bits(words, nbits: int) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:nbits].copy()
