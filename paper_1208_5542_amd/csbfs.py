"""Thin ctypes binding of libcsbfs.so (include/csbfs.h).

Argument marshalling only: every step of the search runs in the library's HIP
kernels. torch provides device memory (tensors' data pointers) and the current
stream. Importing this module does not touch the GPU; the library is loaded
on first use and a missing library raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsbfs.so")

OK, EINVAL, ERANGE, ENOSPACE, EHIP, EOVERFLOW, ECORRUPT = 0, -1, -2, -3, -4, -5, -6
FLAG_TIMING, FLAG_KEEP_STREAMS, FLAG_NO_SIEVE, FLAG_SPARSE_ONLY, FLAG_DENSE_ONLY = 1, 2, 4, 8, 16
FLAG_BOTTOM_UP_ONLY, FLAG_BINNED_PUSH, FLAG_ATOMIC_PUSH = 32, 64, 128
DIR_TOP_DOWN, DIR_BOTTOM_UP, DIR_DENSE = 0, 1, 2
PUSH_ATOMIC, PUSH_BINNED = 0, 1

_lib = None


class CsbfsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("range", ctypes.c_int64), ("n_tuples", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("max_block_nnz", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class LevelStats(ctypes.Structure):
    _fields_ = [("frontier", ctypes.c_int64), ("edges", ctypes.c_int64),
                ("view_bits", ctypes.c_int64), ("sieved_bits", ctypes.c_int64), ("unsieved_bits", ctypes.c_int64),
                ("raw_bytes", ctypes.c_int64), ("wah_unsieved_bytes", ctypes.c_int64),
                ("wah_sieved_bytes", ctypes.c_int64), ("self_bytes", ctypes.c_int64),
                ("max_rank_bytes", ctypes.c_int64), ("pulled", ctypes.c_int64),
                ("ms_expand", ctypes.c_float), ("ms_update", ctypes.c_float),
                ("ms_compress", ctypes.c_float), ("ms_decode", ctypes.c_float),
                ("direction", ctypes.c_int32), ("ms_long_rows", ctypes.c_float),
                ("push", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class SearchConfig(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("max_levels", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("beta", ctypes.c_float), ("segment_groups", ctypes.c_int32), ("push_bin_pairs", ctypes.c_int32)]


class Sizes(ctypes.Structure):
    _fields_ = [("graph_bytes", ctypes.c_int64), ("build_scratch_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("alignment", ctypes.c_int64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("hbm_budget", ctypes.c_int64)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("root", ctypes.c_int64), ("graph_id", ctypes.c_int32),
                ("status", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("batched", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


def lib():
    """Load libcsbfs.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first "
                           "(there is no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                             ctypes.c_size_t)
    sig = {
        "csbfs_version": ([], ctypes.c_int),
        "csbfs_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "csbfs_last_error": ([], ctypes.c_char_p),
        "csbfs_graph_build": ([vp, vp, i64, i64, i32, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "csbfs_graph_build_into": ([vp, vp, i64, i64, i32, vp, sz, vp, sz, vp, ctypes.POINTER(vp)],
                                   ctypes.c_int),
        "csbfs_layout_query": ([i64, i64, i32, ctypes.POINTER(SearchConfig), ctypes.POINTER(Sizes)],
                               ctypes.c_int),
        "csbfs_bfs_ws": ([vp, i64, ctypes.POINTER(SearchConfig), vp, vp, ctypes.POINTER(LevelStats), i32,
                          ctypes.POINTER(i32), vp, sz, vp, vp], ctypes.c_int),
        "csbfs_ws_stream_words": ([vp, ctypes.POINTER(SearchConfig), vp, sz, i32, vp, i32, vp], ctypes.c_int),
        "csbfs_ws_copy_stream": ([vp, ctypes.POINTER(SearchConfig), vp, sz, i32, i32, i32, i32, vp, i64,
                                  ctypes.POINTER(i64), vp], ctypes.c_int),
        "csbfs_graph_free": ([vp], ctypes.c_int),
        "csbfs_graph_get_info": ([vp, ctypes.POINTER(GraphInfo)], ctypes.c_int),
        "csbfs_graph_copy_directory": ([vp, vp, i64, vp], ctypes.c_int),
        "csbfs_graph_copy_block": ([vp, i32, i32, vp, vp, i64, ctypes.POINTER(i64), vp], ctypes.c_int),
        "csbfs_count_traversed_tuples": ([vp, vp, ctypes.POINTER(i64), vp], ctypes.c_int),
        "csbfs_engine_create": ([vp, i32, u32, ctypes.POINTER(vp)], ctypes.c_int),
        "csbfs_engine_free": ([vp], ctypes.c_int),
        "csbfs_engine_set_direction": ([vp, ctypes.c_float, ctypes.c_float], ctypes.c_int),
        "csbfs_bfs": ([vp, i64, vp, vp, ctypes.POINTER(LevelStats), i32, ctypes.POINTER(i32), vp],
                      ctypes.c_int),
        "csbfs_engine_stream_words": ([vp, vp, i32], ctypes.c_int),
        "csbfs_engine_copy_stream": ([vp, i32, i32, i32, vp, i64, ctypes.POINTER(i64), vp],
                                     ctypes.c_int),
        "csbfs_batch_engine_create": ([vp, i32, i32, u32, ctypes.POINTER(vp)], ctypes.c_int),
        "csbfs_batch_engine_free": ([vp], ctypes.c_int),
        "csbfs_batch_bfs": ([vp, vp, i32, vp, ctypes.POINTER(LevelStats), i32, ctypes.POINTER(i32), vp],
                            ctypes.c_int),
        "csbfs_batch_stream_words": ([vp, vp, i32], ctypes.c_int),
        "csbfs_batch_copy_stream": ([vp, i32, i32, i32, i32, vp, i64, ctypes.POINTER(i64), vp],
                                    ctypes.c_int),
        "csbfs_batch_engine_bytes": ([vp, i32, i32, u32], i64),
        "csbfs_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)], ctypes.c_int),
        "csbfs_server_add_graph": ([vp, vp, ctypes.POINTER(i32)], ctypes.c_int),
        "csbfs_server_submit": ([vp, i32, i64, vp, vp, ctypes.POINTER(i64)], ctypes.c_int),
        "csbfs_server_wait": ([vp, i64, ctypes.POINTER(RequestInfo)], ctypes.c_int),
        "csbfs_server_drain": ([vp], ctypes.c_int),
        "csbfs_server_bytes_held": ([vp], i64),
        "csbfs_server_graph_bytes": ([vp, i32], i64),
        "csbfs_server_free": ([vp], ctypes.c_int),
        "csbfs_wah_capacity": ([i64], i64),
        "csbfs_wah_workspace_bytes": ([i64], sz),
        "csbfs_wah_encode": ([vp, vp, i64, vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "csbfs_wah_decode_or": ([vp, i64, i64, vp, vp, vp, sz, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != OK:
        L = lib()
        raise CsbfsError(rc, where, f"{L.csbfs_strerror(rc).decode()}: {L.csbfs_last_error().decode()}")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "need a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def version() -> int:
    return lib().csbfs_version()


def strerror(status: int) -> str:
    return lib().csbfs_strerror(status).decode()


def search_config(flags: int = 0, max_levels: int = 64, alpha: float = 0.0, beta: float = 0.0,
                  segment_groups: int = 0, push_bin_pairs: int = 0) -> SearchConfig:
    return SearchConfig(flags, max_levels, alpha, beta, segment_groups, push_bin_pairs)


def layout_query(n: int, n_tuples: int, p: int, config: SearchConfig | None = None) -> dict:
    """Exact byte sizes of the caller-owned buffers (csbfs_layout_query)."""
    out = Sizes()
    _check(lib().csbfs_layout_query(n, n_tuples, p, None if config is None else ctypes.byref(config),
                                    ctypes.byref(out)), "csbfs_layout_query")
    return {f[0]: int(getattr(out, f[0])) for f in Sizes._fields_}


def _bytes_tensor(nbytes: int) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


class Graph:
    """The p x p sub-block grid of an undirected graph.

    memory="library": csbfs_graph_build (the library allocates the graph);
    memory="caller": csbfs_graph_build_into with torch-allocated buffers of
    the sizes csbfs_layout_query gives (the tensor is kept as self.memory)."""

    def __init__(self, src: torch.Tensor, dst: torch.Tensor, n: int, p: int, stream=None,
                 memory: str = "library"):
        assert src.dtype == torch.int64 and dst.dtype == torch.int64 and src.shape == dst.shape
        h = ctypes.c_void_p()
        self.memory = None
        if memory == "caller":
            sz = layout_query(n, src.numel(), p)
            self.memory = _bytes_tensor(sz["graph_bytes"])
            scratch = _bytes_tensor(sz["build_scratch_bytes"])
            _check(lib().csbfs_graph_build_into(_ptr(src), _ptr(dst), src.numel(), n, p, _ptr(self.memory),
                                                self.memory.numel(), _ptr(scratch), scratch.numel(),
                                                _stream(stream), ctypes.byref(h)), "csbfs_graph_build_into")
            del scratch
        else:
            assert memory == "library", memory
            _check(lib().csbfs_graph_build(_ptr(src), _ptr(dst), src.numel(), n, p, _stream(stream),
                                           ctypes.byref(h)), "csbfs_graph_build")
        self._h = h
        self.n_tuples = int(src.numel())
        info = GraphInfo()
        _check(lib().csbfs_graph_get_info(h, ctypes.byref(info)), "csbfs_graph_get_info")
        self.info = info
        self.n, self.p, self.range = int(info.n), int(info.p), int(info.range)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().csbfs_graph_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def directory(self, stream=None) -> torch.Tensor:
        """V_{i,j} words, shape (p, p, n/p/64), uint64 bit patterns in int64."""
        W = self.range // 64
        out = torch.empty(self.p * self.p * W, dtype=torch.int64, device="cuda")
        _check(lib().csbfs_graph_copy_directory(self._h, _ptr(out), out.numel(), _stream(stream)),
               "csbfs_graph_copy_directory")
        return out.view(self.p, self.p, W)

    def block(self, i: int, j: int, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        """CSR of sub-block (i, j): (row_ptr int32[R+1], col int32 local ids)."""
        rp = torch.empty(self.range + 1, dtype=torch.int32, device="cuda")
        nnz = ctypes.c_int64()
        rc = lib().csbfs_graph_copy_block(self._h, i, j, _ptr(rp), None, 0, ctypes.byref(nnz),
                                          _stream(stream))
        if rc not in (OK, ENOSPACE):
            _check(rc, "csbfs_graph_copy_block")
        col = torch.empty(max(int(nnz.value), 1), dtype=torch.int32, device="cuda")
        _check(lib().csbfs_graph_copy_block(self._h, i, j, _ptr(rp), _ptr(col), col.numel(),
                                            ctypes.byref(nnz), _stream(stream)),
               "csbfs_graph_copy_block")
        return rp, col[: int(nnz.value)]

    def traversed_tuples(self, level: torch.Tensor, stream=None) -> int:
        m = ctypes.c_int64()
        _check(lib().csbfs_count_traversed_tuples(self._h, _ptr(level), ctypes.byref(m),
                                                  _stream(stream)), "csbfs_count_traversed_tuples")
        return int(m.value)


@dataclass
class BfsResult:
    level: torch.Tensor
    parent: torch.Tensor
    n_levels: int
    stats: list[dict]


class Engine:
    """Workspace for repeated searches on one graph (csbfs_engine_create)."""

    def __init__(self, graph: Graph, max_levels: int = 64, flags: int = 0):
        h = ctypes.c_void_p()
        _check(lib().csbfs_engine_create(graph.handle, max_levels, flags, ctypes.byref(h)),
               "csbfs_engine_create")
        self._h = h
        self.graph = graph
        self.max_levels = max_levels
        self.flags = flags
        self._stats = (LevelStats * max_levels)()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().csbfs_engine_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_direction(self, alpha: float, beta: float):
        """Parameters of the per-level top-down / bottom-up choice."""
        _check(lib().csbfs_engine_set_direction(self._h, alpha, beta), "csbfs_engine_set_direction")

    def bfs(self, root: int, level: torch.Tensor | None = None, parent: torch.Tensor | None = None,
            stream=None, with_stats: bool = True) -> BfsResult:
        n = self.graph.n
        if level is None:
            level = torch.empty(n, dtype=torch.int32, device="cuda")
        if parent is None:
            parent = torch.empty(n, dtype=torch.int32, device="cuda")
        nl = ctypes.c_int32()
        cap = self.max_levels if with_stats else 0
        _check(lib().csbfs_bfs(self._h, int(root), _ptr(level), _ptr(parent),
                               self._stats if with_stats else None, cap, ctypes.byref(nl),
                               _stream(stream)), "csbfs_bfs")
        n_levels = int(nl.value)
        stats = [self._stats[k].as_dict() for k in range(min(n_levels, cap))]
        return BfsResult(level, parent, n_levels, stats)

    def stream_words(self, n_levels: int):
        import numpy as np
        p = self.graph.p
        out = np.zeros(n_levels * p * p, dtype=np.int32)
        _check(lib().csbfs_engine_stream_words(self._h, out.ctypes.data_as(ctypes.c_void_p), n_levels),
               "csbfs_engine_stream_words")
        return out.reshape(n_levels, p, p)

    def stream(self, k: int, i: int, j: int, stream=None) -> torch.Tensor:
        cap = wah_capacity(self.graph.range)
        out = torch.zeros(cap, dtype=torch.int64, device="cuda")
        nw = ctypes.c_int64()
        _check(lib().csbfs_engine_copy_stream(self._h, k, i, j, _ptr(out), cap, ctypes.byref(nw),
                                              _stream(stream)), "csbfs_engine_copy_stream")
        return out[: int(nw.value)]


class WorkspaceSearch:
    """Searches on one graph in a caller-owned workspace (csbfs_bfs_ws): the
    workspace is a torch tensor of the size csbfs_layout_query gives and the
    frontier-size mailbox a pinned host tensor; the library allocates
    nothing."""

    def __init__(self, graph: Graph, config: SearchConfig | None = None, mailbox: bool = True):
        self.graph = graph
        self.config = config if config is not None else search_config()
        sz = layout_query(graph.n, graph.n_tuples, graph.p, self.config)
        self.workspace = _bytes_tensor(sz["workspace_bytes"])
        self.mailbox = torch.zeros(2, dtype=torch.int64, pin_memory=True) if mailbox else None
        self.max_levels = int(self.config.max_levels) or 64
        self._stats = (LevelStats * self.max_levels)()
        self.last_levels = 0

    def _ws(self):
        return _ptr(self.workspace), self.workspace.numel()

    def bfs(self, root: int, level: torch.Tensor | None = None, parent: torch.Tensor | None = None,
            stream=None, with_stats: bool = True) -> BfsResult:
        n = self.graph.n
        if level is None:
            level = torch.empty(n, dtype=torch.int32, device="cuda")
        if parent is None:
            parent = torch.empty(n, dtype=torch.int32, device="cuda")
        nl = ctypes.c_int32()
        cap = self.max_levels if with_stats else 0
        ws, wsb = self._ws()
        mb = None if self.mailbox is None else ctypes.c_void_p(self.mailbox.data_ptr())
        _check(lib().csbfs_bfs_ws(self.graph.handle, int(root), ctypes.byref(self.config), _ptr(level),
                                  _ptr(parent), self._stats if with_stats else None, cap, ctypes.byref(nl),
                                  ws, wsb, mb, _stream(stream)), "csbfs_bfs_ws")
        self.last_levels = int(nl.value)
        stats = [self._stats[k].as_dict() for k in range(min(self.last_levels, cap))]
        return BfsResult(level, parent, self.last_levels, stats)

    def stream_words(self, n_levels: int, stream=None):
        import numpy as np
        p = self.graph.p
        out = np.zeros(n_levels * p * p, dtype=np.int32)
        ws, wsb = self._ws()
        _check(lib().csbfs_ws_stream_words(self.graph.handle, ctypes.byref(self.config), ws, wsb,
                                           self.last_levels, out.ctypes.data_as(ctypes.c_void_p), n_levels,
                                           _stream(stream)), "csbfs_ws_stream_words")
        return out.reshape(n_levels, p, p)

    def stream(self, k: int, i: int, j: int, stream=None) -> torch.Tensor:
        cap = wah_capacity(self.graph.range)
        out = torch.zeros(cap, dtype=torch.int64, device="cuda")
        nw = ctypes.c_int64()
        ws, wsb = self._ws()
        _check(lib().csbfs_ws_copy_stream(self.graph.handle, ctypes.byref(self.config), ws, wsb, self.last_levels,
                                          k, i, j, _ptr(out), cap, ctypes.byref(nw), _stream(stream)),
               "csbfs_ws_copy_stream")
        return out[: int(nw.value)]


@dataclass
class BatchResult:
    level: torch.Tensor  # (n_roots, n) int32
    n_levels: int
    stats: list[dict]


class BatchEngine:
    """Workspace for batched searches of up to 64 roots (csbfs_batch_engine_create)."""

    def __init__(self, graph: Graph, max_roots: int = 64, max_levels: int = 64, flags: int = 0):
        h = ctypes.c_void_p()
        _check(lib().csbfs_batch_engine_create(graph.handle, max_roots, max_levels, flags, ctypes.byref(h)),
               "csbfs_batch_engine_create")
        self._h = h
        self.graph = graph
        self.max_roots = max_roots
        self.max_levels = max_levels
        self.flags = flags
        self.n_roots = 0
        self._stats = (LevelStats * max_levels)()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().csbfs_batch_engine_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bfs(self, roots, level: torch.Tensor | None = None, stream=None,
            with_stats: bool = True) -> BatchResult:
        roots = (ctypes.c_int64 * len(roots))(*[int(r) for r in roots])
        B, n = len(roots), self.graph.n
        if level is None:
            level = torch.empty((B, n), dtype=torch.int32, device="cuda")
        nl = ctypes.c_int32()
        cap = self.max_levels if with_stats else 0
        _check(lib().csbfs_batch_bfs(self._h, roots, B, _ptr(level), self._stats if with_stats else None,
                                     cap, ctypes.byref(nl), _stream(stream)), "csbfs_batch_bfs")
        self.n_roots = B
        n_levels = int(nl.value)
        stats = [self._stats[k].as_dict() for k in range(min(n_levels, cap))]
        return BatchResult(level.view(B, n), n_levels, stats)

    def stream_words(self, n_levels: int):
        """int32 (n_levels, n_roots, p, p) word counts of the last batch's streams."""
        import numpy as np
        p, B = self.graph.p, self.n_roots
        out = np.zeros(n_levels * B * p * p, dtype=np.int32)
        _check(lib().csbfs_batch_stream_words(self._h, out.ctypes.data_as(ctypes.c_void_p), n_levels),
               "csbfs_batch_stream_words")
        return out.reshape(n_levels, B, p, p)

    def stream(self, k: int, r: int, i: int, j: int, stream=None) -> torch.Tensor:
        cap = wah_capacity(self.graph.range)
        out = torch.zeros(cap, dtype=torch.int64, device="cuda")
        nw = ctypes.c_int64()
        _check(lib().csbfs_batch_copy_stream(self._h, k, r, i, j, _ptr(out), cap, ctypes.byref(nw),
                                             _stream(stream)), "csbfs_batch_copy_stream")
        return out[: int(nw.value)]


class Server:
    """Request loop over resident graphs (csbfs_server_*): continuous batching
    of queries into up to `slots` concurrent batched searches, engines admitted
    under an HBM budget."""

    def __init__(self, slots: int = 2, max_batch: int = 64, max_levels: int = 256,
                 hbm_budget: int = 32 << 30):
        cfg = ServerConfig(slots, max_batch, max_levels, 0, hbm_budget)
        h = ctypes.c_void_p()
        _check(lib().csbfs_server_create(ctypes.byref(cfg), ctypes.byref(h)), "csbfs_server_create")
        self._h = h
        self.graphs: list[Graph] = []

    def add_graph(self, graph: Graph) -> int:
        gid = ctypes.c_int32()
        _check(lib().csbfs_server_add_graph(self._h, graph.handle, ctypes.byref(gid)), "csbfs_server_add_graph")
        self.graphs.append(graph)
        return int(gid.value)

    def submit(self, graph_id: int, root: int, out: torch.Tensor | None = None, stream=None) -> int:
        """Queue a query; `out` (device int32[n]) receives the levels, after
        the work already queued on `stream` (default: torch's current
        stream)."""
        if out is not None:
            assert out.dtype == torch.int32 and out.numel() == self.graphs[graph_id].n
        rid = ctypes.c_int64()
        _check(lib().csbfs_server_submit(self._h, graph_id, int(root), _ptr(out),
                                         _stream(stream) if out is not None else None, ctypes.byref(rid)),
               "csbfs_server_submit")
        return int(rid.value)

    def wait(self, request_id: int) -> dict:
        info = RequestInfo()
        _check(lib().csbfs_server_wait(self._h, request_id, ctypes.byref(info)), "csbfs_server_wait")
        return info.as_dict()

    def drain(self):
        _check(lib().csbfs_server_drain(self._h), "csbfs_server_drain")

    def bytes_held(self) -> int:
        return int(lib().csbfs_server_bytes_held(self._h))

    def graph_bytes(self, graph_id: int) -> int:
        """Device bytes of one (slot, graph) block of a registered graph."""
        return int(lib().csbfs_server_graph_bytes(self._h, graph_id))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().csbfs_server_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wah_capacity(nbits: int) -> int:
    return int(lib().csbfs_wah_capacity(nbits))


def wah_workspace(nbits: int) -> torch.Tensor:
    nb = int(lib().csbfs_wah_workspace_bytes(nbits))
    return torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")


def wah_encode(bits: torch.Tensor, nbits: int, mask: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """WAH-64 stream (int64 words holding uint64 patterns) of bits AND mask."""
    cap = wah_capacity(nbits)
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    nw = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = workspace if workspace is not None else wah_workspace(nbits)
    _check(lib().csbfs_wah_encode(_ptr(bits), _ptr(mask), nbits, _ptr(out), cap, _ptr(nw),
                                  _ptr(ws), ws.numel(), _stream(stream)), "csbfs_wah_encode")
    return out[: int(nw.item())]


def wah_decode_or(words: torch.Tensor, nbits: int, dst: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None, stream=None) -> tuple[torch.Tensor, int]:
    """OR the decoded bits into dst (zeros if not given); returns (dst, status)."""
    if dst is None:
        dst = torch.zeros(max((nbits + 63) // 64, 1), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = workspace if workspace is not None else wah_workspace(nbits)
    _check(lib().csbfs_wah_decode_or(_ptr(words) if words.numel() else None, words.numel(), nbits,
                                     _ptr(dst), _ptr(status), _ptr(ws), ws.numel(), _stream(stream)),
           "csbfs_wah_decode_or")
    return dst, int(status.item())
