"""Compression + sieve BFS on MI355X (gfx950).

One level-synchronous breadth-first search over a p x p block grid of a
partitioned graph, with the p virtual processors held as buffers on one GPU:
top-down expansion of each block's frontier, the cross-directory sieve of
every outgoing message, word-aligned hybrid (WAH) compression, and
decompression into the receivers' frontier views, with message bytes counted.
Every step runs in hand-written HIP kernels behind the C ABI in
``include/csbfs.h``; ``csbfs`` is its thin Python binding and ``inputs`` the
seeded synthetic input generator.

Submodules are imported lazily so that the input generator stays usable on
machines without a GPU.
"""
__all__ = ["csbfs", "inputs"]
