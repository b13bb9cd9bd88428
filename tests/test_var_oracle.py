"""Pins of the oracle's variable-rate modes (Sec. 4.3: fixed precision and
fixed accuracy, Table 2) against what the definitions fix, on the CPU:

  lossless      32 planes in fixed precision decode exactly like the fixed-rate
                code at 64 bits/value (both keep every plane)
  embedded      a block's P-plane code is a bit prefix of its 32-plane code
  accuracy      fixed accuracy keeps every value within the tolerance (the
                mode's definition), on wide-range random blocks and on the
                synthetic matrix
  lengths       an all-zero block takes 1 bit, a block below the tolerance 9
                (header only); bits fall and errors rise as the tolerance grows
  index         offsets rise through the stream, and decoding from the index
                equals decoding block after block
"""
import numpy as np
import pytest

import oracle
from paper_1902_08018_amd import synth


def bits_of(stream, nbits):
    return np.unpackbits(np.asarray(stream, dtype=np.uint8), bitorder="little")[:nbits]


def wide_range(rows, cols, seed):
    rng = np.random.default_rng(seed)
    scale = np.exp2(rng.integers(-30, 10, size=(rows, 1)))
    return (rng.standard_normal((rows, cols)) * scale).astype(np.float32)


def test_32_planes_equal_fixed_rate_64():
    M = wide_range(16, 24, 1)
    s, idx, nb = oracle.encode_var(M, oracle.VAR_PRECISION, 32)
    D = oracle.decode_var(s, idx, 16, 24, oracle.VAR_PRECISION, 32)
    assert nb / M.size < 60  # every block fits the fixed-rate budget below
    F = oracle.decode(oracle.encode(M, 64), 16, 24, 64)
    assert np.array_equal(D.view(np.uint32), F.view(np.uint32))


@pytest.mark.parametrize("seed", range(6))
def test_precision_code_is_embedded(seed):
    blk = wide_range(4, 4, 10 + seed)
    s32, _, n32 = oracle.encode_var(blk, oracle.VAR_PRECISION, 32)
    full = bits_of(s32, n32)
    prev = 0
    for p in (1, 2, 5, 8, 13, 20, 27, 31, 32):
        s, _, n = oracle.encode_var(blk, oracle.VAR_PRECISION, p)
        assert n >= prev and np.array_equal(bits_of(s, n), full[:n])
        prev = n


@pytest.mark.parametrize("minexp", [-30, -20, -12, -4, 0, 6])
def test_accuracy_bound(minexp):
    M = wide_range(40, 36, 3)
    s, idx, nb = oracle.encode_var(M, oracle.VAR_ACCURACY, minexp)
    D = oracle.decode_var(s, idx, 40, 36, oracle.VAR_ACCURACY, minexp)
    err = np.abs(D.astype(np.float64) - M)
    # per block, the bound holds where the planes were not clamped at 32
    blocks_ok = np.ones((10, 9), bool)
    for bi in range(10):
        for bj in range(9):
            b = M[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4]
            e = np.frexp(np.abs(b).max())[1] if np.any(b) else -200
            blocks_ok[bi, bj] = e - minexp <= 25
    mask = np.kron(blocks_ok, np.ones((4, 4), bool))
    assert mask.any()
    assert np.all(err[mask] <= 2.0 ** minexp)


def test_accuracy_on_the_synthetic_matrix():
    M = synth.matrix_rows(synth.SMALL, 0, 128)
    prev_bits, prev_err = None, None
    for minexp in (-26, -20, -16, -12):
        s, idx, nb = oracle.encode_var(M, oracle.VAR_ACCURACY, minexp)
        D = oracle.decode_var(s, idx, 128, 4096, oracle.VAR_ACCURACY, minexp)
        err = float(np.abs(D.astype(np.float64) - M).max())
        assert err <= 2.0 ** minexp
        if prev_bits is not None:
            assert nb < prev_bits and err >= prev_err
        prev_bits, prev_err = nb, err


def test_block_lengths():
    Z = np.zeros((8, 12), np.float32)
    s, idx, nb = oracle.encode_var(Z, oracle.VAR_ACCURACY, -10)
    assert nb == 6  # six all-zero blocks, one bit each
    small = np.full((8, 12), 2.0 ** -20, np.float32)
    s, idx, nb = oracle.encode_var(small, oracle.VAR_ACCURACY, -10)
    assert nb == 6 * 9  # emax - minexp + 7 < 0: header only
    assert np.all(oracle.decode_var(s, idx, 8, 12, oracle.VAR_ACCURACY, -10) == 0)


@pytest.mark.parametrize("shape", [(10, 300), (37, 133), (4, 4)])
def test_index(shape):
    rows, cols = shape
    M = wide_range(rows, cols, 5)
    for mode, param in ((oracle.VAR_PRECISION, 11), (oracle.VAR_ACCURACY, -18)):
        s, idx, nb = oracle.encode_var(M, mode, param)
        assert idx.size == ((rows + 3) // 4) * oracle.var_groups(cols)
        assert idx[0] == 0 and np.all(np.diff(idx.astype(np.int64)) > 0) and idx[-1] < nb
        A = oracle.decode_var(s, idx, rows, cols, mode, param)
        B = oracle.decode_var(s, None, rows, cols, mode, param)
        assert np.array_equal(A.view(np.uint32), B.view(np.uint32))


@pytest.mark.parametrize("planes", [1, 8, 17, 25, 32])
def test_block_bits_bound(planes):
    """A block coded to P planes takes at most 25 + 17 P bits: the 9-bit
    header, at most 16 verbatim bits a plane after the first, one ending
    group bit a plane, and over all planes at most 16 run-starting group bits
    and 16 run bits (a run passes each coefficient once).  The GPU decoder
    stages 20 words a block on this bound."""
    rng = np.random.default_rng(100 + planes)
    blocks = [rng.standard_normal((4, 4)) * np.exp2(rng.integers(-40, 40)) for _ in range(300)]
    blocks += [np.full((4, 4), 1.0), np.eye(4) * 3.0 - 1.0, np.indices((4, 4)).sum(0) % 2 - 0.5,
               np.where(rng.random((4, 4)) < 0.5, -1.0, 1.0) * rng.integers(1, 1 << 20, (4, 4)),
               rng.standard_normal((4, 4)) * np.exp2(rng.integers(-30, 30, (4, 4)))]
    worst = 0
    for b in blocks:
        _, _, nb = oracle.encode_var(np.asarray(b, np.float32), oracle.VAR_PRECISION, planes)
        worst = max(worst, nb)
    assert worst <= 25 + 17 * planes
    if planes == 32:
        assert worst > 16 * 31  # white noise reaches the verbatim-dominated regime the bound covers
