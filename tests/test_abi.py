"""The C ABI library loads, exports every entry point include/csbfs.h
declares, and rejects bad arguments on the host before touching a GPU
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(REPO, "include", "csbfs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csbfs_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1208_5542_amd import csbfs
    if not os.path.exists(csbfs.LIB_PATH):
        from paper_1208_5542_amd import _build
        _build.build_csbfs()
    return csbfs.lib()


def test_header_declares_the_expected_entry_points():
    names = _declared()
    for must in ("csbfs_graph_build", "csbfs_bfs", "csbfs_wah_encode", "csbfs_wah_decode_or",
                 "csbfs_engine_create", "csbfs_count_traversed_tuples"):
        assert must in names
    assert len(names) >= 18


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings(lib):
    from paper_1208_5542_amd import csbfs
    assert csbfs.version() == 10200
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert csbfs.strerror(code) != "unknown status"
    assert csbfs.strerror(-99) == "unknown status"


def test_host_side_argument_checks(lib):
    vp = ctypes.c_void_p
    h = vp()
    # graph build: null tuples, bad sizes, p not dividing n, n/p not a multiple of 64
    assert lib.csbfs_graph_build(None, None, 5, 1024, 4, None, ctypes.byref(h)) == -1
    assert lib.csbfs_graph_build(None, None, 0, 1000, 4, None, ctypes.byref(h)) == -2
    assert lib.csbfs_graph_build(None, None, 0, 1024, 3, None, ctypes.byref(h)) == -2
    assert b"p | n" in lib.csbfs_last_error()
    assert lib.csbfs_graph_build(None, None, 0, 2048, 64, None, ctypes.byref(h)) == -2
    assert lib.csbfs_graph_build(None, None, 0, 32, 1, None, ctypes.byref(h)) == -2
    assert lib.csbfs_graph_build(None, None, 0, 1 << 31, 1, None, ctypes.byref(h)) == -2
    assert lib.csbfs_graph_build(None, None, -1, 1024, 1, None, ctypes.byref(h)) == -1
    assert lib.csbfs_graph_build(None, None, 0, 1024, 1, None, None) == -1
    # engine and search on null handles
    assert lib.csbfs_engine_create(None, 64, 0, ctypes.byref(h)) == -1
    assert lib.csbfs_engine_set_direction(None, 4.0, 64.0) == -1
    assert lib.csbfs_batch_engine_create(None, 64, 64, 0, ctypes.byref(h)) == -1
    assert lib.csbfs_batch_bfs(None, None, 0, None, None, 0, None, None) == -1
    assert lib.csbfs_batch_stream_words(None, None, 0) == -1
    assert lib.csbfs_batch_engine_free(None) == 0
    assert lib.csbfs_batch_engine_bytes(None, 64, 64, 0) == -1
    # serving: configuration checks happen before any device call
    from paper_1208_5542_amd import csbfs as cb
    for bad in ((0, 64, 64, 0, 1 << 30), (17, 64, 64, 0, 1 << 30), (1, 0, 64, 0, 1 << 30),
                (1, 65, 64, 0, 1 << 30), (1, 64, 0, 0, 1 << 30), (1, 64, 64, 1, 1 << 30), (1, 64, 64, 0, 0)):
        cfg = cb.ServerConfig(*bad)
        assert lib.csbfs_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1, bad
    assert lib.csbfs_server_create(None, ctypes.byref(h)) == -1
    assert lib.csbfs_server_add_graph(None, None, None) == -1
    assert lib.csbfs_server_submit(None, 0, 0, None, None, None) == -1
    assert lib.csbfs_server_wait(None, 0, None) == -1
    assert lib.csbfs_server_drain(None) == -1
    assert lib.csbfs_server_bytes_held(None) == -1
    assert lib.csbfs_server_free(None) == 0
    assert lib.csbfs_bfs(None, 0, None, None, None, 0, None, None) == -1
    assert lib.csbfs_engine_stream_words(None, None, 0) == -1
    assert lib.csbfs_engine_copy_stream(None, 0, 0, 0, None, 0, None, None) == -1
    assert lib.csbfs_graph_get_info(None, None) == -1
    assert lib.csbfs_graph_free(None) == 0
    assert lib.csbfs_engine_free(None) == 0
    assert lib.csbfs_count_traversed_tuples(None, None, None, None) == -1
    # codec sizing and argument checks
    assert lib.csbfs_wah_capacity(0) == 1
    assert lib.csbfs_wah_capacity(63) == 2
    assert lib.csbfs_wah_capacity(1 << 20) == (1 << 20) // 63 + 1
    assert lib.csbfs_wah_capacity(-1) == -1
    assert lib.csbfs_wah_workspace_bytes(1 << 20) > 0
    assert lib.csbfs_wah_encode(None, None, 64, None, 0, None, None, 0, None) == -1
    lib.csbfs_wah_noalloc_max_bits.restype = ctypes.c_int64
    assert lib.csbfs_wah_noalloc_max_bits() > 4 * 10**9
    lib.csbfs_wah_encode_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.csbfs_wah_encode_noalloc(None, None, 64, None, 2, None, None) == -1
    assert lib.csbfs_wah_decode_or(None, 1, 64, None, None, None, 0, None) == -1


def test_package_import_does_not_need_a_gpu():
    import importlib
    import paper_1208_5542_amd.csbfs as m
    importlib.reload(m)
    assert m.FLAG_TIMING == 1 and m.FLAG_DENSE_ONLY == 16 and m.FLAG_BOTTOM_UP_ONLY == 32


def _struct_fields(name):
    text = open(HEADER).read()
    body = text[text.index(f"typedef struct {name} {{"):text.index(f"}} {name};")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return re.findall(r"\b(?:int64_t|int32_t|float|double)\s+(\w+);", body)


def test_server_structs_match_header():
    from paper_1208_5542_amd import csbfs
    assert _struct_fields("csbfs_server_config") == [f[0] for f in csbfs.ServerConfig._fields_]
    assert _struct_fields("csbfs_request_info") == [f[0] for f in csbfs.RequestInfo._fields_]
    assert ctypes.sizeof(csbfs.ServerConfig) == 24 and ctypes.sizeof(csbfs.RequestInfo) == 64
    assert csbfs.lib().csbfs_server_graph_bytes(None, 0) == -1


def test_level_stats_layout_matches_header():
    """The binding's struct has the header's field order and size."""
    from paper_1208_5542_amd import csbfs
    text = open(HEADER).read()
    body = text[text.index("typedef struct csbfs_level_stats {"):text.index("} csbfs_level_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b(?:int64_t|int32_t|float)\s+(\w+);", body)
    assert names == [f[0] for f in csbfs.LevelStats._fields_]
    assert ctypes.sizeof(csbfs.LevelStats) == 11 * 8 + 4 * 4 + 4 * 4


def test_layout_query_is_host_only_and_exact_in_its_inputs():
    """csbfs_layout_query needs no device, depends only on its arguments and
    grows with the config's kept levels and streams."""
    from paper_1208_5542_amd import csbfs
    a = csbfs.layout_query(1 << 22, 1 << 26, 4)
    assert a == csbfs.layout_query(1 << 22, 1 << 26, 4)
    assert a["alignment"] == 256
    for k in ("graph_bytes", "build_scratch_bytes", "workspace_bytes"):
        assert a[k] > 0 and a[k] % 256 == 0
    # the graph holds the column ids twice (blocks and merged pull rows)
    assert a["graph_bytes"] >= 2 * 4 * 2 * (1 << 26)
    keep = csbfs.layout_query(1 << 22, 1 << 26, 4, csbfs.search_config(flags=csbfs.FLAG_KEEP_STREAMS,
                                                                      max_levels=64))
    assert keep["graph_bytes"] == a["graph_bytes"] and keep["workspace_bytes"] > a["workspace_bytes"]
    deeper = csbfs.layout_query(1 << 22, 1 << 26, 4, csbfs.search_config(max_levels=1000))
    assert deeper["workspace_bytes"] > a["workspace_bytes"]
    with pytest.raises(csbfs.CsbfsError) as ei:
        csbfs.layout_query(1000, 10, 4)
    assert ei.value.status == csbfs.ERANGE
    with pytest.raises(csbfs.CsbfsError) as ei:
        csbfs.layout_query(1 << 12, -1, 4)
    assert ei.value.status == csbfs.EINVAL
    # the binned push's bins: none with ATOMIC_PUSH, nor by default on a graph
    # this small (no level could pass the threshold twice over); with
    # BINNED_PUSH 8 bytes per pair of capacity
    binned = csbfs.FLAG_BINNED_PUSH
    atomic = csbfs.layout_query(1 << 22, 1 << 26, 4, csbfs.search_config(flags=csbfs.FLAG_ATOMIC_PUSH))
    assert atomic["workspace_bytes"] == a["workspace_bytes"]
    small = csbfs.layout_query(1 << 22, 1 << 26, 4, csbfs.search_config(flags=binned, push_bin_pairs=1 << 20))
    big = csbfs.layout_query(1 << 22, 1 << 26, 4, csbfs.search_config(flags=binned, push_bin_pairs=1 << 24))
    assert atomic["workspace_bytes"] < small["workspace_bytes"] < big["workspace_bytes"]
    assert big["workspace_bytes"] - small["workspace_bytes"] >= 8 * ((1 << 24) - (1 << 20))
    # segments stay below the workgroups' 16-bit pair counts: a huge capacity
    # on a one-bin graph gives 512 segments of at most 65528 pairs
    huge = csbfs.layout_query(1 << 12, 100, 4, csbfs.search_config(flags=binned, push_bin_pairs=(1 << 31) - 1))
    none = csbfs.layout_query(1 << 12, 100, 4, csbfs.search_config(flags=csbfs.FLAG_ATOMIC_PUSH))
    assert 0 < huge["workspace_bytes"] - none["workspace_bytes"] <= 8 * 512 * 65528 + 4 * 512 + 2 * 256
    # a graph with 2^31 entries gets bins by default
    large = csbfs.layout_query(1 << 26, 1 << 30, 8)
    large_atomic = csbfs.layout_query(1 << 26, 1 << 30, 8, csbfs.search_config(flags=csbfs.FLAG_ATOMIC_PUSH))
    assert large["workspace_bytes"] - large_atomic["workspace_bytes"] >= 8 * (1 << 28)
    for bad in (csbfs.search_config(flags=csbfs.FLAG_TIMING), csbfs.search_config(flags=8 | 16),
                csbfs.search_config(max_levels=70000), csbfs.search_config(segment_groups=512),
                csbfs.search_config(flags=csbfs.FLAG_BINNED_PUSH | csbfs.FLAG_ATOMIC_PUSH),
                csbfs.SearchConfig(0, 64, 0.0, 0.0, 0, -1)):
        with pytest.raises(csbfs.CsbfsError) as ei:
            csbfs.layout_query(1 << 12, 100, 4, bad)
        assert ei.value.status == csbfs.EINVAL


def test_search_config_layout_matches_header():
    from paper_1208_5542_amd import csbfs
    assert _struct_fields("csbfs_sizes") == [f[0] for f in csbfs.Sizes._fields_]
    text = open(HEADER).read()
    body = text[text.index("typedef struct csbfs_search_config {"):text.index("} csbfs_search_config;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b(?:uint32_t|int32_t|float)\s+(\w+);", body)
    assert names == [f[0] for f in csbfs.SearchConfig._fields_]
    assert ctypes.sizeof(csbfs.SearchConfig) == 24 and ctypes.sizeof(csbfs.Sizes) == 32
