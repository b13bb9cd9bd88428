"""The library's host encoder for the variable-rate formats (fixed precision,
fixed accuracy; Sec. 4.3) against the oracle's, on the CPU: the same index
and the same code bits, for partial edge blocks, both modes and wide-range
data.  No GPU is needed (the encoder is host code of the library)."""
import numpy as np
import pytest

import oracle
from paper_1902_08018_amd import wh


def wide_range(rows, cols, seed):
    rng = np.random.default_rng(seed)
    scale = np.exp2(rng.integers(-24, 8, size=(rows, 1)))
    return (rng.standard_normal((rows, cols)) * scale).astype(np.float32)


@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (37, 133), (64, 520)])
@pytest.mark.parametrize("fmt,param", [(wh.WH_FMT_ZFP_FIXED_PRECISION, 1), (wh.WH_FMT_ZFP_FIXED_PRECISION, 17),
                                       (wh.WH_FMT_ZFP_FIXED_PRECISION, 32), (wh.WH_FMT_ZFP_FIXED_ACCURACY, -26),
                                       (wh.WH_FMT_ZFP_FIXED_ACCURACY, -8), (wh.WH_FMT_ZFP_FIXED_ACCURACY, 12)])
def test_encoder_matches_oracle(shape, fmt, param):
    M = wide_range(*shape, seed=sum(shape))
    M[0, :min(3, shape[1])] = 0.0  # zero values inside blocks
    omode = oracle.VAR_PRECISION if fmt == wh.WH_FMT_ZFP_FIXED_PRECISION else oracle.VAR_ACCURACY
    rate = param if fmt == wh.WH_FMT_ZFP_FIXED_PRECISION else wh.accuracy_rate(param)
    buf = wh.wh_encode_var(M, fmt, rate)
    s, idx, nbits = oracle.encode_var(M, omode, param)
    ib = wh.wh_var_index_bytes(*shape)
    assert ib == idx.size * 8
    assert buf.size % 8 == 0 and buf.size >= ib + (nbits + 7) // 8 + 16
    assert np.array_equal(buf[:ib].view(np.uint64), idx)
    code = buf[ib:]
    assert np.array_equal(code[:s.size], s) and not code[s.size:].any()


def test_encoder_errors():
    with pytest.raises(wh.WhError) as ei:
        wh.wh_encode_var(np.array([[np.nan]], np.float32), wh.WH_FMT_ZFP_FIXED_PRECISION, 8)
    assert ei.value.status == wh.WH_ERR_INVALID
    with pytest.raises(wh.WhError) as ei:
        wh.wh_encode_var(np.ones((4, 4), np.float32), wh.WH_FMT_ZFP_FIXED_PRECISION, 33)
    assert ei.value.status == wh.WH_ERR_FORMAT
    with pytest.raises(wh.WhError) as ei:
        wh.wh_encode_var(np.ones((4, 4), np.float32), wh.WH_FMT_ZFP_FIXED_RATE, 8)
    assert ei.value.status == wh.WH_ERR_FORMAT
