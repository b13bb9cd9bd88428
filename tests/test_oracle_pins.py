"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against a closed form, a hand derivation, a
printed number of the paper, an algebraic identity, or brute force, so that
a plausible slip (dropped term, wrong sign, swapped index, transposed
operand, wrong bit order) fails at least one of them:

  hand-derived stream   a constant block's 80 bits (bit order, header,
                        lift of constants, negabinary, group tests)
  hand-derived ramps    which sequency positions a ramp along c / along r
                        lights up (catches a transposed lift or order)
  lift = A v / 16       exact on multiples of 16; inverse lift undoes it;
                        the inverse matrix is A^-1 (computed by numpy)
  order rule            the sequency order obeys its stated sort key
  coder                 lossless at 36 bits/value for arbitrary blocks;
                        embedded (a lower rate is a prefix); fixed size
  zero / constant       closed forms: +0, exact at every rate >= 5
  rank-1                M = w v^T with small integers: y = (v.u) w exactly
  brute force           math.fsum of exact products bounds the FP64 sum
  twin                  C oracle == independent pure-Python twin, bit for
                        bit, on tiny matrices and on random byte strings
  Table 2 / Fig. 11     metric definitions and pipeline formulas reproduce
                        the paper's printed numbers
  Sec. 4.4 claim        FP32 accumulation of a 256000-term row loses most
                        of its bits; the FP64 and Fig. 7 reductions do not
  edge padding          a partial block codes the matrix padded by its last
                        row / column (numpy's "edge" pad); decoding drops
                        the padding; the GEMV sums the real columns only
"""
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from oracle import metrics, twin
from paper_1902_08018_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
A = np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]], dtype=np.int64)


def read_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]


def block_matrix(blocks16):
    """(n, 16) blocks in local order -> a 4 x 4n matrix (one block-row)."""
    n = blocks16.shape[0]
    return blocks16.reshape(n, 4, 4).transpose(1, 0, 2).reshape(4, 4 * n).astype(np.float32)


# --------------------------------------------------------- hand derivations
def test_constant_block_stream_matches_hand_derivation():
    expect = bytes.fromhex(read_golden("constant_block_rate5.txt")[0].replace(" ", ""))
    M = np.ones((4, 4), dtype=np.float32)
    s = oracle.encode(M, 5)
    assert bytes(s) == expect
    assert bytes(twin.encode_matrix(M, 5)) == expect
    assert np.array_equal(oracle.decode(s, 4, 4, 5), M)


def _coefficients(f16, rate=36):
    """Transform coefficients (sequency order, int32) from the oracle's own
    stream: decode its plane code at the lossless budget."""
    M = block_matrix(np.asarray(f16, dtype=np.float32).reshape(1, 16))
    s = oracle.encode(M, rate)
    bits = np.unpackbits(s, bitorder="little")
    # strip the 9 header bits: repack from bit 9
    tail = np.packbits(bits[9:], bitorder="little")
    n16, _ = oracle.decode_planes(tail, 16 * rate - 9)
    return np.array([twin.from_negabinary(int(v)) for v in n16])


def test_ramp_coefficients_match_hand_derivation():
    lines = dict(ln.split(" ", 1) for ln in read_golden("ramp_blocks.txt"))
    ramp_c = np.tile(np.arange(4, dtype=np.float32), 4)           # f[r][c] = c
    ramp_r = np.repeat(np.arange(4, dtype=np.float32), 4)         # f[r][c] = r
    for name, f in (("ramp_c", ramp_c), ("ramp_r", ramp_r)):
        want = np.zeros(16, dtype=np.int64)
        for tok in lines[name].split():
            pos, val = tok.split(":")
            want[int(pos)] = int(val)
        assert np.array_equal(_coefficients(f), want), name


# ---------------------------------------------------------------- transform
def test_lift_is_A_over_16_on_multiples_of_16():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        v = rng.integers(-2 ** 25, 2 ** 25, size=4) * 16
        assert np.array_equal(oracle.fwd_lift4(v), (A @ v) // 16)
        assert np.array_equal(np.asarray(twin.lift(*[int(x) for x in v])), (A @ v) // 16)


def test_inverse_lift_is_inverse_matrix():
    Ainv16 = np.rint(np.linalg.inv(A / 16.0) * 16).astype(np.int64)  # 16 * A^-1, integral
    assert np.allclose(np.linalg.inv(A / 16.0) * 16, Ainv16)
    rng = np.random.default_rng(1)
    for _ in range(2000):
        v = rng.integers(-2 ** 25, 2 ** 25, size=4) * 16
        c = (A @ v) // 16
        assert np.array_equal(oracle.inv_lift4(c), v)
        assert np.array_equal((Ainv16 @ c) // 16, v)
        assert np.array_equal(np.asarray(twin.unlift(*[int(x) for x in c])), v)


def test_2d_transform_rows_then_columns():
    rng = np.random.default_rng(2)
    for _ in range(300):
        b = rng.integers(-2 ** 20, 2 ** 20, size=(4, 4)) * 256
        want = ((A @ ((b @ A.T) // 16)) // 16)  # rows (over c) first, then columns (over r)
        got = oracle.fwd_xform(b.reshape(16)).reshape(4, 4)
        assert np.array_equal(got, want)
        assert np.array_equal(oracle.inv_xform(got.reshape(16)).reshape(4, 4), b)


def test_lift_wraps_modulo_2_32():
    # the decoder must be total: sums that overflow int32 wrap
    v = np.array([2 ** 31 - 1, 2 ** 31 - 1, -2 ** 31, -2 ** 31])
    out = oracle.inv_lift4(v)
    out_twin = np.asarray(twin.unlift(*[int(x) for x in v]))
    assert np.array_equal(out, out_twin)


def test_sequency_order_obeys_its_rule():
    order = oracle.sequency_order()
    assert sorted(order) == list(range(16))
    keys = [((v & 3) + (v >> 2), (v & 3) ** 2 + (v >> 2) ** 2, -(v & 3)) for v in order]
    assert keys == sorted(keys)
    assert order[0] == 0 and order[-1] == 15
    assert order == twin.sequency_order()


# --------------------------------------------------------------------- coder
def test_coder_lossless_at_rate_36_for_any_coefficients():
    rng = np.random.default_rng(3)
    budget = 16 * 36 - 9
    worst = 0
    cases = [rng.integers(0, 2 ** 32, size=16, dtype=np.uint64).astype(np.uint32) for _ in range(3000)]
    cases += [np.full(16, 0xFFFFFFFF, np.uint32), np.full(16, 0x55555555, np.uint32),
              np.array([1 << 31] + [0] * 15, np.uint32), np.array([0] * 15 + [1], np.uint32)]
    for n16 in cases:
        buf, used = oracle.encode_planes(n16, budget)
        back, used2 = oracle.decode_planes(buf, budget)
        assert used == used2
        assert np.array_equal(back, n16)
        worst = max(worst, used)
    assert worst <= budget


@pytest.mark.parametrize("lo,hi", [(8, 16), (4, 8), (2, 12)])
def test_code_is_embedded(lo, hi):
    """The rate-lo block is the first 16*lo bits of the rate-hi block."""
    M = synth.matrix_rows(synth.SMALL, 0, 8)[:, :512]
    s_lo = np.unpackbits(oracle.encode(M, lo), bitorder="little").reshape(-1, 16 * lo)
    s_hi = np.unpackbits(oracle.encode(M, hi), bitorder="little").reshape(-1, 16 * hi)
    assert np.array_equal(s_hi[:, :16 * lo], s_lo)


def test_fixed_size_and_random_access():
    M = synth.matrix_rows(synth.SMALL, 0, 16)[:, :256]
    for rate in (3, 8, 16):
        s = oracle.encode(M, rate)
        assert s.size * 8 == (16 // 4) * (256 // 4) * 16 * rate
        full = oracle.decode_blocks(s, rate, 0, 256)
        for b in (0, 17, 255):
            assert np.array_equal(oracle.decode_blocks(s, rate, b, 1)[0].view(np.uint32), full[b].view(np.uint32))


# ---------------------------------------------------------- closed forms
@pytest.mark.parametrize("rate", [1, 2, 8, 16])
def test_zero_block(rate):
    M = np.zeros((4, 8), dtype=np.float32)
    M[:, 4:] = -0.0
    s = oracle.encode(M, rate)
    assert not s.any()
    d = oracle.decode(s, 4, 8, rate)
    assert np.array_equal(d.view(np.uint32), np.zeros((4, 8), np.uint32))  # +0 (not -0)


@pytest.mark.parametrize("rate", [5, 6, 8, 16, 32])
def test_constant_blocks_exact_at_rate_5_and_up(rate):
    rng = np.random.default_rng(rate)
    consts = (rng.standard_normal(64) * np.exp2(rng.integers(-120, 120, size=64))).astype(np.float32)
    blocks = np.repeat(consts[:, None], 16, axis=1)
    M = block_matrix(blocks)
    assert np.array_equal(oracle.decode(oracle.encode(M, rate), 4, M.shape[1], rate), M)


def test_constant_block_codes_in_73_bits():
    """The hand derivation's bit count: the plane code of a lone DC
    coefficient 2^29 (negabinary 0x60000000) is 64 bits when the budget does
    not cut it, so the block needs 9 + 64 = 73 bits; the coder stops reading
    at the same place."""
    n16 = np.zeros(16, dtype=np.uint32)
    n16[0] = twin.negabinary(2 ** 29)
    assert n16[0] == 0x60000000
    buf, used = oracle.encode_planes(n16, 1000)
    assert used == 64
    back, used2 = oracle.decode_planes(buf, 1000)
    assert used2 == 64 and np.array_equal(back, n16)
    assert twin.code_planes([int(v) for v in n16], 1000) == [int(b) for b in np.unpackbits(
        buf, bitorder="little")[:64]]


def test_error_bound_at_lossless_coder_rate():
    """At 36 bits/value only block-floating-point truncation and the lift's
    floors remain: |f - fhat| <= c * 2^(emax - 30) with a small c."""
    rng = np.random.default_rng(4)
    blocks = rng.standard_normal((4096, 16)) * np.exp2(rng.integers(-60, 60, size=(4096, 1)))
    blocks = blocks.astype(np.float32)
    M = block_matrix(blocks)
    d = oracle.decode(oracle.encode(M, 36), 4, M.shape[1], 36)
    db = d.reshape(4, -1, 4).transpose(1, 0, 2).reshape(-1, 16)
    emax = np.array([max(math.frexp(float(v))[1] for v in b if v != 0) for b in blocks])
    err = np.abs(db.astype(np.float64) - blocks) / np.exp2(emax - 30.0)[:, None]
    # the float result also carries one FP32 rounding: allow 2^-24 relative
    err_excess = err - np.abs(blocks) * 2.0 ** -24 / np.exp2(emax - 30.0)[:, None]
    assert err_excess.max() <= 8.0


def test_rank1_closed_form():
    """M = w v^T with |w|,|v| <= 15 is reproduced exactly at 36 bits/value,
    so y = (v . u) w exactly for integer u and within FP64 rounding for
    u in [0, 1)."""
    rng = np.random.default_rng(5)
    rows, cols = 64, 256
    w = rng.integers(-15, 16, size=rows).astype(np.float64)
    v = rng.integers(-15, 16, size=cols).astype(np.float64)
    M = np.outer(w, v).astype(np.float32)
    s = oracle.encode(M, 36)
    assert np.array_equal(oracle.decode(s, rows, cols, 36), M)
    ui = rng.integers(0, 100, size=cols).astype(np.float32)
    assert np.array_equal(oracle.gemv_fp64(s, rows, cols, 36, ui), (v @ ui) * w)
    u = synth.uniform(cols, seed=5)
    y = oracle.gemv_fp64(s, rows, cols, 36, u)
    exact = np.array([math.fsum(float(v[j]) * float(u[j]) for j in range(cols))]) * w
    assert np.allclose(y, exact, rtol=1e-13, atol=1e-12)


def test_gemv_brute_force_fsum():
    M = synth.matrix_rows(synth.MatrixSpec(16, 64, 8, 3.0), 0, 16)
    u = synth.uniform(64, seed=9)
    for rate in (8, 16):
        s = oracle.encode(M, rate)
        Mhat = oracle.decode(s, 16, 64, rate)
        y = oracle.gemv_fp64(s, 16, 64, rate, u)
        exact = np.array(twin.gemv_exact(Mhat, u))
        bound = 64 * 2.0 ** -53 * (np.abs(Mhat).astype(np.float64) @ np.abs(u).astype(np.float64))
        assert np.all(np.abs(y - exact) <= bound)
        # paper-MP: FP32 products, FP64 sum, one final rounding
        ymp = oracle.gemv_paper_mp(s, 16, 64, rate, u)
        prods = Mhat.astype(np.float32) * u.astype(np.float32)  # FP32 products
        want = np.array([np.float32(math.fsum(float(p) for p in row)) for row in prods])
        assert np.array_equal(ymp, want)


def test_threads_do_not_change_results():
    M = synth.matrix_rows(synth.SMALL, 0, 64)
    u = synth.u_vector(synth.SMALL)
    s = oracle.encode(M, 8)
    assert np.array_equal(oracle.gemv_fp64(s, 64, 4096, 8, u, nthreads=1),
                          oracle.gemv_fp64(s, 64, 4096, 8, u, nthreads=5))


def test_row_range_matches_full():
    M = synth.matrix_rows(synth.SMALL, 0, 64)
    u = synth.u_vector(synth.SMALL)
    s = oracle.encode(M, 8)
    full = oracle.gemv_fp64(s, 64, 4096, 8, u)
    assert np.array_equal(oracle.gemv_fp64(s, 64, 4096, 8, u, 20, 40), full[20:40])


# ----------------------------------------------------------------- the twin
@pytest.mark.parametrize("rate", [1, 2, 3, 5, 8, 11, 16, 36])
def test_twin_matches_oracle_on_matrices(rate):
    M = synth.matrix_rows(synth.MatrixSpec(8, 16, 4, 2.0), 0, 8)
    s = oracle.encode(M, rate)
    assert bytes(s) == twin.encode_matrix(M, rate)
    d1 = oracle.decode(s, 8, 16, rate)
    d2 = twin.decode_matrix(bytes(s), 8, 16, rate)
    assert np.array_equal(d1.view(np.uint32), d2.view(np.uint32))


@pytest.mark.parametrize("rate", [1, 2, 4, 7, 8, 16, 33])
def test_twin_matches_oracle_on_random_bytes(rate):
    rng = np.random.default_rng(rate)
    s = rng.integers(0, 256, size=2 * rate * 24, dtype=np.uint8)
    d1 = oracle.decode(s, 8, 12, rate)
    d2 = twin.decode_matrix(bytes(s), 8, 12, rate)
    assert np.array_equal(d1.view(np.uint32), d2.view(np.uint32))


finite_f32 = st.floats(width=32, allow_nan=False, allow_infinity=False)


@settings(max_examples=150, deadline=None)
@given(vals=st.lists(finite_f32, min_size=16, max_size=16), rate=st.integers(1, 36),
       shift=st.integers(-140, 120))
def test_twin_matches_oracle_property(vals, rate, shift):
    f = np.array(vals, dtype=np.float64) * 2.0 ** shift
    with np.errstate(over="ignore"):
        f = np.clip(f, -3.4e38, 3.4e38).astype(np.float32)
    M = block_matrix(f.reshape(1, 16))
    s = oracle.encode(M, rate)
    assert bytes(s) == twin.encode_matrix(M, rate)
    d1 = oracle.decode(s, 4, 4, rate)
    d2 = twin.decode_matrix(bytes(s), 4, 4, rate)
    assert np.array_equal(d1.view(np.uint32), d2.view(np.uint32))


def test_nonfinite_rejected():
    M = np.ones((4, 4), dtype=np.float32)
    M[1, 2] = np.inf
    with pytest.raises(oracle.OracleError):
        oracle.encode(M, 8)
    with pytest.raises(ValueError):
        twin.encode_matrix(M, 8)


def test_shape_rejected():
    with pytest.raises(oracle.OracleError):  # an empty matrix has no blocks to code
        oracle.encode(np.ones((0, 4), dtype=np.float32), 8)


# ----------------------------------------------- the paper's printed numbers
def test_table2_metric_relations():
    for ln in read_golden("table2_zfp_errors.csv"):
        mode, axis, bpv, ratio, rmse, nrmse, maxerr, psnr = ln.split(",")
        assert metrics.compression_ratio(float(bpv)) == pytest.approx(float(ratio), abs=0.01)
        assert metrics.psnr_from_nrmse(float(nrmse)) == pytest.approx(float(psnr), abs=0.05)


def test_fig11_pipeline_arithmetic():
    rows = dict((r.split(",")[0], (float(r.split(",")[1]), float(r.split(",")[2])))
                for r in read_golden("fig11_breakdown.txt"))
    t_comp, t_tr, t_dec = rows["computation"][0], rows["transfer"][0], rows["decompression"][1]
    ratio = t_tr / rows["transfer"][1]
    assert ratio == pytest.approx(10.0, abs=0.01)
    before = metrics.pipeline_latency(t_tr, t_comp)
    after = metrics.pipeline_latency(t_tr, t_comp, t_dec, ratio)
    assert before == pytest.approx(100.0)
    assert after == pytest.approx(53.28, abs=0.01)
    assert 1 - after / before == pytest.approx(0.47, abs=0.01)       # Sec. 5.2: latency cut by about 47 %
    assert t_dec / after == pytest.approx(0.52, abs=0.01)            # Sec. 5.2: decode is 52 % of the time
    # Table 1 period: transfer-bound before, decode+compute-bound after
    assert metrics.pipeline_period(t_tr, t_comp) == t_tr
    assert metrics.pipeline_period(t_tr, t_comp, t_dec, ratio) == pytest.approx(t_comp + t_dec)


def test_gemv_cost_formulas():
    # Sec. 2.1: M(2N-1) FLOP and MN + N + M values for an M x N GEMV
    assert metrics.gemv_flops(378, 256000) == 378 * 511999
    assert metrics.gemv_ios(378, 256000) == 378 * 256000 + 256000 + 378
    # the paper's 198.3 GFLOP/s on 378 x 256K is one GEMV in ~0.976 ms
    assert metrics.gemv_flops(378, 256000) / 198.3e9 == pytest.approx(0.976e-3, rel=1e-3)


def test_long_fp32_reduction_loses_bits():
    """Sec. 4.4: a 256000-term FP32 running sum is badly contaminated, an FP64
    reduction of the FP32 products is not."""
    cols = 256000
    spec = synth.MatrixSpec(4, cols, 512, 64.0, seed=7)
    M = synth.matrix_rows(spec, 0, 4)
    u = synth.uniform(cols, seed=7)
    exact = np.array([math.fsum(float(a) * float(b) for a, b in zip(M[i], u)) for i in range(4)])
    naive = oracle.dense_gemv_fp32_naive(M, u).astype(np.float64)
    mp = oracle.dense_gemv_paper_mp(M, u).astype(np.float64)
    f64 = oracle.dense_gemv_fp64(M, u)
    rel_naive = np.abs(naive - exact) / np.abs(exact)
    rel_mp = np.abs(mp - exact) / np.abs(exact)
    assert rel_naive.max() > 1e-5                    # far above FP32's 6e-8
    assert rel_mp.max() <= 2.0 ** -24                # one final rounding
    assert np.abs(f64 - exact).max() <= 1e-12 * np.abs(exact).max()


# ------------------------------------------------------- quality (unpinned)
def test_compression_error_decreases_with_rate():
    """Parity unpinned (the paper's C_d is not public): only plausibility --
    error falls with rate, and rate 8 is in the same decade band as the
    paper's fixed-rate-8 NRMSE (~2e-5, Table 2) or better."""
    M = synth.matrix_rows(synth.SMALL, 0, 256)
    errs = [metrics.rmse(M, oracle.decode(oracle.encode(M, r), 256, 4096, r)) for r in (4, 8, 12, 16)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    nr8 = metrics.nrmse(M, oracle.decode(oracle.encode(M, 8), 256, 4096, 8))
    assert nr8 < 1e-3


# ---------------------------------------------------- partial blocks (edge padding)
@pytest.mark.parametrize("rows,cols", [(1, 1), (3, 5), (7, 13), (38, 22), (9, 38)])
@pytest.mark.parametrize("rate", [4, 8, 16])
def test_partial_blocks_are_edge_padded(rows, cols, rate):
    """A matrix whose sides are not multiples of 4 is coded as the matrix
    padded by repeating its last row and column (numpy's "edge" padding);
    decoding drops the padding, and the GEMV sums over the real columns."""
    rng = np.random.default_rng(rows * 1000 + cols)
    M = (rng.standard_normal((rows, cols)) * np.exp2(rng.integers(-3, 4, size=(rows, 1)))).astype(np.float32)
    P = np.pad(M, ((0, -rows % 4), (0, -cols % 4)), mode="edge")
    s = oracle.encode(M, rate)
    assert s.size == oracle.stream_nbytes(rows, cols, rate) == P.size // 16 * 2 * rate
    assert np.array_equal(s, oracle.encode(P, rate))
    D = oracle.decode(s, rows, cols, rate)
    Dp = oracle.decode(s, P.shape[0], P.shape[1], rate)
    assert np.array_equal(D.view(np.uint32), Dp[:rows, :cols].view(np.uint32))
    u = rng.random(cols).astype(np.float32)
    y = oracle.gemv_fp64(s, rows, cols, rate, u)
    ref = np.array([math.fsum(float(a) * float(b) for a, b in zip(row, u)) for row in D])
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-300)
    for rb, re in [(0, rows), (rows // 2, rows), (0, (rows + 1) // 2), (rows // 3, rows - rows // 3)]:
        # any range of rows: the same values as the whole product's slice
        yr = oracle.gemv_fp64(s, rows, cols, rate, u, row_begin=rb, row_end=re)
        assert np.array_equal(yr, y[rb:re])
        ym = oracle.gemv_paper_mp(s, rows, cols, rate, u, row_begin=rb, row_end=re)
        assert np.array_equal(ym, oracle.gemv_paper_mp(s, rows, cols, rate, u)[rb:re])


def test_row_range_bounds():
    M = np.ones((9, 8), np.float32)
    s = oracle.encode(M, 8)
    u = np.ones(8, np.float32)
    assert oracle.gemv_fp64(s, 9, 8, 8, u, row_begin=5, row_end=5).size == 0
    for rb, re in [(3, 2), (0, 10), (10, 10)]:
        with pytest.raises(oracle.OracleError):
            oracle.gemv_fp64(s, 9, 8, 8, u, row_begin=rb, row_end=re)
