"""Pins of the oracle's WAH codec: exhaustive round trips on tiny inputs,
closed forms of the 64-bit format, word-count structure and rejection of
invalid streams (CPU only)."""
import itertools

import numpy as np
import pytest

import oracle

ZF = 1 << 63          # 64-bit fill flag
OB = 1 << 62          # 64-bit fill bit


def _classes(bits, g, ones_fill):
    G = len(bits) // g
    out = []
    for x in range(G):
        s = int(sum(bits[x * g:(x + 1) * g]))
        if s == 0:
            out.append("Z")
        elif s == g and ones_fill:
            out.append("O")
        else:
            out.append("L")
    return out


def _expected_word_count(bits, g, ones_fill):
    """#literal groups + #maximal uniform runs + [active word]; a run longer
    than the count field holds is split into as many fills as it needs."""
    cls = _classes(bits, g, ones_fill)
    max_count = (1 << (g - 1 if ones_fill else g)) - 1  # w-2 or w-1 count bits
    n = 0
    for key, grp in itertools.groupby(cls):
        c = len(list(grp))
        n += c if key == "L" else -(-c // max_count)
    return n + (1 if len(bits) % g else 0)


@pytest.mark.parametrize("w,fb", [(4, False), (4, True), (5, True), (8, False), (8, True)])
def test_exhaustive_round_trip_tiny(w, fb):
    g = w - 1
    for nbits in range(0, 13):
        for x in range(1 << nbits):
            bits = np.array([(x >> t) & 1 for t in range(nbits)], dtype=np.uint8)
            words = oracle.wah_encode(bits, w, fb)
            assert len(words) == _expected_word_count(bits, g, fb), (nbits, x)
            assert all(int(v) < (1 << w) for v in words)
            assert len(words) <= nbits // g + 1
            assert oracle.wah_decode(words, nbits, w, fb).tolist() == bits.tolist(), (nbits, x)


@pytest.mark.parametrize("nbits", [63, 64, 126, 127, 1000, 1024, 4096, 65536])
def test_closed_forms_64(nbits):
    G, r = divmod(nbits, 63)
    zeros = np.zeros(nbits, dtype=np.uint8)
    exp = [ZF | G] + ([0] if r else [])
    assert oracle.wah_encode(zeros).tolist() == exp
    ones = np.ones(nbits, dtype=np.uint8)
    exp = [ZF | OB | G] + ([(1 << r) - 1] if r else [])
    assert oracle.wah_encode(ones).tolist() == exp
    for t in sorted({0, 1, 61, 62, 63, 64, 100, 63 * G - 1, nbits - 1} - {-1}):
        if t < 0 or t >= nbits:
            continue
        b = zeros.copy()
        b[t] = 1
        x, o = divmod(t, 63)
        if x < G:
            exp = ([ZF | x] if x else []) + [1 << (62 - o)]
            exp += ([ZF | (G - x - 1)] if G - x - 1 else []) + ([0] if r else [])
        else:  # the set bit sits in the active word, right-aligned
            exp = [ZF | G, 1 << (r - 1 - o)]
        assert oracle.wah_encode(b).tolist() == exp, t
        assert oracle.wah_decode(oracle.wah_encode(b), nbits).tolist() == b.tolist()


def test_literal_payload_is_msb_first():
    bits = np.zeros(126, dtype=np.uint8)
    bits[0] = 1          # first bit of group 0 -> bit 62
    bits[63 + 62] = 1    # last bit of group 1 -> bit 0
    bits[3] = 1
    w = oracle.wah_encode(bits)
    assert w.tolist() == [(1 << 62) | (1 << 59), 1]


def test_alternating_runs_64():
    # 0-run of 3 groups, literal, 1-run of 2 groups, 0-run of 1 group, then 10 active bits
    g = 63
    parts = [np.zeros(3 * g), np.r_[np.ones(5), np.zeros(58)], np.ones(2 * g), np.zeros(g),
             np.r_[np.ones(2), np.zeros(8)]]
    bits = np.concatenate(parts).astype(np.uint8)
    w = oracle.wah_encode(bits).tolist()
    assert w == [ZF | 3, (0b11111 << 58), ZF | OB | 2, ZF | 1, 0b1100000000]
    assert oracle.wah_decode(np.array(w, dtype=np.uint64), len(bits)).tolist() == bits.tolist()


@pytest.mark.parametrize("density", [0.0, 0.001, 0.02, 0.3, 0.5, 0.98, 1.0])
def test_random_round_trip_64(density):
    rng = np.random.default_rng(int(density * 1000) + 7)
    for nbits in [64, 640, 6400, 64 * 1000]:
        bits = (rng.random(nbits) < density).astype(np.uint8)
        # add runs so that fills of both kinds appear
        if nbits >= 640:
            bits[100:400] = 1
            bits[400:600] = 0
        w = oracle.wah_encode(bits)
        assert len(w) == _expected_word_count(bits, 63, True)
        assert len(w) <= nbits // 63 + 1
        assert oracle.wah_decode(w, nbits).tolist() == bits.tolist()


def test_decoder_rejects_invalid_streams():
    nbits = 200  # G = 3 groups, r = 11
    with pytest.raises(ValueError):
        oracle.wah_decode(np.array([ZF | 0, 0], dtype=np.uint64), nbits)  # zero-length fill
    with pytest.raises(ValueError):
        oracle.wah_decode(np.array([ZF | 4, 0], dtype=np.uint64), nbits)  # too many groups
    with pytest.raises(ValueError):
        oracle.wah_decode(np.array([ZF | 2, 0], dtype=np.uint64), nbits)  # too few groups
    with pytest.raises(ValueError):
        oracle.wah_decode(np.array([ZF | 3, 1 << 11], dtype=np.uint64), nbits)  # active padding
    with pytest.raises(ValueError):
        oracle.wah_decode(np.array([ZF | 3, ZF | 1], dtype=np.uint64), nbits)  # fill as active
    with pytest.raises(ValueError):
        oracle.wah_decode(np.array([ZF | 3], dtype=np.uint64), nbits)  # missing active
    assert oracle.wah_decode(np.array([ZF | 3, 0], dtype=np.uint64), nbits).sum() == 0
