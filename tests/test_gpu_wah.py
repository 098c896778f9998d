"""GPU WAH-64 codec (sieve + compress, decompress) against the oracle codec:
streams byte-identical, round trips exact, corrupt streams flagged."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import from_words, log, require_gpu, to_words, u64

pytestmark = pytest.mark.gpu

ZF = np.uint64(1 << 63)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    from paper_1208_5542_amd import csbfs
    csbfs.lib()


def _patterns(nbits, rng):
    yield "zeros", np.zeros(nbits, np.uint8)
    yield "ones", np.ones(nbits, np.uint8)
    for d in (0.0005, 0.01, 0.3, 0.5, 0.97):
        yield f"rand{d}", (rng.random(nbits) < d).astype(np.uint8)
    b = np.zeros(nbits, np.uint8)
    b[::63] = 1
    yield "every63", b
    b = np.zeros(nbits, np.uint8)
    if nbits > 200000:
        b[70000:140000] = 1    # a 1-run across encoder segments
        b[150001] = 1
    if nbits > 4000000:
        b[300000:3000000] = 1  # a 1-run over about 20 segments
    b[-1] = 1
    yield "runs", b
    b = (rng.random(nbits) < 0.5).astype(np.uint8)
    b[nbits // 3: 2 * nbits // 3] = 0   # a long 0-run in the middle of random data
    yield "hole", b


# up to 66 encoder segments of 2048 groups: the last ones look back past 64
SIZES = [1, 10, 62, 63, 64, 126, 127, 1000, 4096, 64512, 64513, 129087, 1 << 18, (1 << 20) + 37,
         (1 << 23) + 12345]


@pytest.mark.parametrize("nbits", SIZES)
def test_encode_decode_parity(nbits):
    from paper_1208_5542_amd import csbfs
    rng = np.random.default_rng(nbits)
    ws = csbfs.wah_workspace(nbits)
    for name, bits in _patterns(nbits, rng):
        log(f"wah nbits={nbits} pattern={name}")
        ref = oracle.wah_encode(bits)
        got = u64(csbfs.wah_encode(to_words(bits), nbits, workspace=ws))
        assert got.tolist() == ref.tolist(), name
        back, status = csbfs.wah_decode_or(csbfs.wah_encode(to_words(bits), nbits, workspace=ws),
                                           nbits, workspace=ws)
        assert status == 0
        assert (from_words(back, nbits) == bits).all(), name


@pytest.mark.parametrize("nbits", [64, 4096, 1 << 20])
def test_sieve_mask_parity(nbits):
    from paper_1208_5542_amd import csbfs
    rng = np.random.default_rng(7 + nbits)
    for d_f, d_v in [(0.5, 0.1), (0.02, 0.5), (0.9, 0.9), (0.3, 0.0)]:
        f = (rng.random(nbits) < d_f).astype(np.uint8)
        v = (rng.random(nbits) < d_v).astype(np.uint8)
        ref = oracle.wah_encode(f & v)
        got = u64(csbfs.wah_encode(to_words(f), nbits, mask=to_words(v)))
        assert got.tolist() == ref.tolist()


def test_bits_past_nbits_are_ignored():
    from paper_1208_5542_amd import csbfs
    nbits = 100
    w = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    ref = oracle.wah_encode(np.ones(nbits, np.uint8))
    assert u64(csbfs.wah_encode(w, nbits)).tolist() == ref.tolist()


def test_decode_oracle_streams_and_or_semantics():
    from paper_1208_5542_amd import csbfs
    rng = np.random.default_rng(3)
    nbits = 200000
    a = (rng.random(nbits) < 0.01).astype(np.uint8)
    b = (rng.random(nbits) < 0.01).astype(np.uint8)
    words = torch.from_numpy(oracle.wah_encode(a).view(np.int64).copy()).cuda()
    dst = to_words(b)
    out, status = csbfs.wah_decode_or(words, nbits, dst=dst)
    assert status == 0
    assert (from_words(out, nbits) == (a | b)).all()


def _corrupt(words, nbits):
    from paper_1208_5542_amd import csbfs
    t = torch.from_numpy(np.asarray(words, dtype=np.uint64).view(np.int64).copy()).cuda()
    _, status = csbfs.wah_decode_or(t, nbits)
    return status


def test_decode_flags_corrupt_streams():
    nbits = 200  # G = 3, r = 11
    Z = 1 << 63
    assert _corrupt([Z | 3, 0], nbits) == 0
    assert _corrupt([Z | 0, 0], nbits) != 0            # zero-length fill
    assert _corrupt([Z | 4, 0], nbits) != 0            # too many groups
    assert _corrupt([Z | 2, 0], nbits) != 0            # too few groups
    assert _corrupt([Z | 3, 1 << 11], nbits) != 0      # active bits above r
    assert _corrupt([Z | 3, Z | 1], nbits) != 0        # fill in the active slot
    assert _corrupt([Z | 3], nbits) != 0               # missing active word
    assert _corrupt([Z | 1, Z | 1, Z | 1, 0, 0], nbits) != 0  # longer than capacity


def test_empty_stream():
    from paper_1208_5542_amd import csbfs
    got = csbfs.wah_encode(torch.zeros(1, dtype=torch.int64, device="cuda"), 0)
    assert got.numel() == 0
    _, status = csbfs.wah_decode_or(got, 0)
    assert status == 0
