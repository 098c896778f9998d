"""Helpers shared by the GPU tests (no method arithmetic here)."""
import time

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def to_words(bits01: np.ndarray) -> torch.Tensor:
    """0/1 numpy vector -> device int64 tensor of packed little-endian words."""
    b = np.asarray(bits01, dtype=np.uint8)
    pad = (-len(b)) % 64
    if pad:
        b = np.concatenate([b, np.zeros(pad, dtype=np.uint8)])
    w = np.packbits(b, bitorder="little").view(np.int64)
    if len(w) == 0:
        w = np.zeros(1, dtype=np.int64)
    return torch.from_numpy(w.copy()).cuda()


def from_words(words: torch.Tensor, nbits: int) -> np.ndarray:
    w = words.detach().cpu().numpy().astype(np.int64).view(np.uint8)
    return np.unpackbits(w, bitorder="little")[:nbits].astype(np.uint8)


def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.int64).view(np.uint64)


_T0 = time.perf_counter()


def log(msg: str):
    print(f"[{time.perf_counter() - _T0:7.1f}s] {msg}", flush=True)
