"""Pins of the reduced-precision quantisers (oracle/quant.py) and of the
Table 2 error metrics (oracle/metrics.py), CPU only.

The quantisers are checked against what the number formats fix -- codes
derived by hand from the OCP e4m3 layout (bias 7, 3 mantissa bits, largest
finite 448 = 1.75 * 2^8, smallest subnormal 2^-9), the round-to-nearest-even
tie rule, and saturation -- and against torch's own conversions, which are an
implementation independent of both the oracle and the GPU library.  The
metrics are checked against values computed by hand on 3-5 element arrays.
"""
import math

import numpy as np
import pytest
import torch

from oracle import metrics, quant


# --------------------------------------------------------------- e4m3
# (input, code) pairs derived by hand from the format
E4M3_HAND = [
    (448.0, 0x7E),            # largest finite: S=0 E=1111 M=110
    (500.0, 0x7E),            # beyond it: saturates (reading: RNE_sat)
    (1.0e6, 0x7E),
    (-448.0, 0xFE),
    (-1.0e9, 0xFE),
    (2.0 ** -9, 0x01),        # smallest subnormal
    (2.0 ** -6, 0x08),        # smallest normal: E=0001 M=000
    (1.0, 0x38),              # E=0111 (bias 7)
    (-1.0, 0xB8),
    (1.0625, 0x38),           # midway 1.0 (0x38) / 1.125 (0x39): even code
    (1.1875, 0x3A),           # midway 1.125 (0x39) / 1.25 (0x3A): even code
    (432.0, 0x7E),            # midway 416 (0x7D) / 448 (0x7E)
    (400.0, 0x7C),            # midway 384 (0x7C) / 416 (0x7D)
    (2.5 * 2.0 ** -9, 0x02),  # subnormal midway 2 / 3 units: even
    (3.5 * 2.0 ** -9, 0x04),  # subnormal midway 3 / 4 units: even
    (7.5 * 2.0 ** -9, 0x08),  # midway largest subnormal / smallest normal
    (2.0 ** -10, 0x00),       # half the smallest subnormal: tie to code 0
    (2.0 ** -10 * 1.001, 0x01),
    (2.0 ** -11, 0x00),       # below half of the smallest subnormal
    (-2.0 ** -11, 0x00),      # a negative value rounding to 0 gives code 0, never 0x80
    (0.0, 0x00),
    (-0.0, 0x00),
    (3.0, 0x44),              # 1.5 * 2^1: E=1000 M=100
    (0.3, 0x2A),              # 0.3 = 1.2 * 2^-2 -> M = 1.6 -> 2 (1.25 * 2^-2 = 0.3125)
]


@pytest.mark.parametrize("x,code", E4M3_HAND)
def test_e4m3_hand_codes(x, code):
    got = int(quant.e4m3_rne_sat(np.array([x]))[0])
    assert got == code, (x, hex(got), hex(code))


def test_e4m3_value_table_from_format():
    # value of each code from sign / exponent / mantissa, written out here
    assert quant.e4m3_value(0x7E) == 448.0
    assert quant.e4m3_value(0x01) == 2.0 ** -9
    assert quant.e4m3_value(0x07) == 7 * 2.0 ** -9
    assert quant.e4m3_value(0x08) == 2.0 ** -6
    assert quant.e4m3_value(0x38) == 1.0
    assert quant.e4m3_value(0xC4) == -3.0
    assert math.isnan(quant.e4m3_value(0x7F)) and math.isnan(quant.e4m3_value(0xFF))
    pos = [quant.e4m3_value(c) for c in range(0x7F)]
    assert all(a < b for a, b in zip(pos, pos[1:])), "codes 0..126 ascend"


def test_e4m3_round_trip_and_midpoints():
    # every finite code maps back to itself; the exact midpoint between two
    # neighbours goes to the even code; a hair either side goes to the
    # nearer one
    for c in range(0x7E + 1):
        v = quant.e4m3_value(c)
        assert int(quant.e4m3_rne_sat(np.array([v]))[0]) == c
        if c > 0:
            assert int(quant.e4m3_rne_sat(np.array([-v]))[0]) == c | 0x80
    for c in range(0x7E):
        a, b = quant.e4m3_value(c), quant.e4m3_value(c + 1)
        mid = (a + b) / 2
        even = c if c % 2 == 0 else c + 1
        assert int(quant.e4m3_rne_sat(np.array([mid]))[0]) == even, (c, mid)
        eps = (b - a) * 1e-3
        assert int(quant.e4m3_rne_sat(np.array([mid - eps]))[0]) == c
        assert int(quant.e4m3_rne_sat(np.array([mid + eps]))[0]) == c + 1


def test_e4m3_against_torch_cast():
    # torch's float8_e4m3fn cast rounds to nearest even but does not
    # saturate and keeps -0; on every value it maps to a nonzero finite
    # code the two must agree
    rng = np.random.default_rng(7)
    x = np.concatenate([
        rng.uniform(-448, 448, 20000),
        rng.uniform(-1, 1, 20000) * 2.0 ** rng.integers(-12, 9, 20000),
        np.array([quant.e4m3_value(c) for c in range(1, 0x7E)]) * 1.0000001,
    ]).astype(np.float32)
    t = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    o = quant.e4m3_rne_sat(x.astype(np.float64))
    keep = (t & 0x7F) != 0
    assert keep.sum() > 30000
    np.testing.assert_array_equal(o[keep], t[keep])
    # where torch gives +-0 the oracle gives code 0
    assert np.all(o[~keep] == 0)


def test_fp8_block_scale_hand_block():
    # one 4x4 block with amax 7: s = 7/448 = 1/64, codes of f * 64
    blk = np.array([[7.0, -3.5, 0.0, 1.0],
                    [0.25, 6.0, -7.0, 2.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [1.5, -1.5, 3.0, 0.5]], dtype=np.float32)
    codes, s = quant.fp8_block_scaled(blk)
    assert s[0] == np.float32(7.0 / 448.0)
    want = quant.e4m3_rne_sat(blk.reshape(-1).astype(np.float64) * 64.0)
    np.testing.assert_array_equal(codes[0], want)
    assert codes[0][0] == 0x7E and codes[0][6] == 0xFE     # +-7 -> +-448
    deq = quant.fp8_dequant(codes, s, 4, 4)
    assert deq[0, 0] == 7.0 and deq[1, 2] == -7.0
    zc, zs = quant.fp8_block_scaled(np.zeros((4, 4), np.float32))
    assert zs[0] == 0.0 and not zc.any()


# --------------------------------------------------------------- BF16 / FP16
def test_bf16_hand_ties():
    # 1 + 2^-8 is midway between 1 (0x3F80) and 1 + 2^-7 (0x3F81): even 0x3F80
    # 1 + 3 * 2^-8 is midway between 0x3F81 and 0x3F82: even 0x3F82
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -2.0, 3.0e38],
                 dtype=np.float32)
    got = quant.bf16_bits(x)
    assert [hex(v) for v in got] == ["0x3f80", "0x3f80", "0x3f82", "0x3f81", "0xc000", "0x7f62"]


def test_bf16_against_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.standard_normal(50000) * 10.0 ** rng.integers(-30, 30, 50000),
        # exact ties: a random BF16 value plus half a BF16 ulp
        ((rng.integers(0x0080, 0x7F00, 20000).astype(np.uint32) << 16) | 0x8000).view(np.float32),
    ]).astype(np.float32)
    t = torch.from_numpy(x).bfloat16().view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(quant.bf16_bits(x), t)
    np.testing.assert_array_equal(quant.bf16_values(t), torch.from_numpy(t.view(np.int16)).view(torch.bfloat16).float().numpy())


def test_f16_against_torch():
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(50000) * 10.0 ** rng.integers(-8, 5, 50000)).astype(np.float32)
    np.testing.assert_array_equal(quant.to_f16(x), torch.from_numpy(x).half().numpy())


# --------------------------------------------------------------- metrics
def test_metrics_hand_values():
    src = np.array([0.0, 1.0, 2.0, 3.0])
    dec = np.array([0.0, 1.0, 2.0, 5.0])
    # differences (0, 0, 0, 2): RMSE = sqrt(4 / 4) = 1, range 3, max 2
    assert metrics.rmse(src, dec) == 1.0
    assert metrics.nrmse(src, dec) == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert metrics.max_pointwise_error(src, dec) == 2.0
    assert metrics.psnr(src, dec) == pytest.approx(20.0 * math.log10(3.0 / 2.0), rel=1e-14)

    src = np.array([[1.0, -2.0], [4.0, 0.5]])
    dec = np.array([[1.5, -2.5], [3.0, 0.5]])
    # differences (0.5, -0.5, -1, 0): RMSE = sqrt(1.5 / 4), range 6, max 1
    assert metrics.rmse(src, dec) == pytest.approx(math.sqrt(0.375), rel=1e-15)
    assert metrics.nrmse(src, dec) == pytest.approx(math.sqrt(0.375) / 6.0, rel=1e-15)
    assert metrics.max_pointwise_error(src, dec) == 1.0

    # a sign error must not cancel: RMSE of (+1, -1, +1) is 1, not 1/3
    assert metrics.rmse(np.zeros(3), np.array([1.0, -1.0, 1.0])) == 1.0
    # the range is the source's, not the decoded matrix's
    assert metrics.nrmse(np.array([0.0, 10.0, 5.0]), np.array([0.0, 10.0, 35.0])) == pytest.approx(
        math.sqrt(300.0) / 10.0, rel=1e-15)


def test_rel_l2_hand_values():
    assert metrics.rel_l2(np.array([3.0, 4.0]), np.array([0.0, 4.0])) == pytest.approx(3.0 / 4.0, rel=1e-15)
    assert metrics.rel_l2(np.array([1.0, 2.0, 2.0]), np.array([1.0, 2.0, 4.0])) == pytest.approx(
        2.0 / math.sqrt(21.0), rel=1e-15)
