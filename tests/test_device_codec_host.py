"""The GPU codec's source (whz_device.hpp), built for the host, against the
oracle: bit-exact decode and byte-exact encode at every compiled block size,
with and without idle lanes in the wave, under AddressSanitizer so that a
read past a staged block's zero padding fails the test.

The AMDGPU builtins the header uses (alignbit, bfe, perm, wave vote) are
emulated from their ISA definitions; the GPU tests check the same source on
the hardware."""
import os
import shutil
import subprocess
import warnings

import numpy as np
import pytest

import oracle
from paper_1902_08018_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host_codec", "device_codec_host.cpp")
WORDS = [1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 16]  # the decoder's compiled block sizes (rate = 2 * words)


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("codec") / "device_codec_host")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:  # no sanitizer runtime: plain build, padding reads unchecked
        warnings.warn("AddressSanitizer unavailable: reads past the staged padding go unchecked")
        r = subprocess.run([gxx, "-std=c++17", "-O2", SRC, "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def run(exe, tmp_path, mode, nw, data, n, idle=0):
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    fin.write_bytes(np.ascontiguousarray(data).tobytes())
    r = subprocess.run([exe, mode, str(nw), str(n), str(fin), str(fout), str(idle)], capture_output=True, text=True,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    assert r.returncode < 64, f"host codec failed ({r.returncode}):\n{r.stderr[-3000:]}"
    return fout.read_bytes(), r.returncode


def blocks_of(M):
    R, C = M.shape
    return M.reshape(R // 4, 4, C // 4, 4).transpose(0, 2, 1, 3).reshape(-1, 16)


def extreme_matrix(rng, n=1024):
    """n blocks (n/4 block-rows x 4 block-cols) spanning the whole exponent range."""
    vals = rng.standard_normal((n, 16)) * np.exp2(rng.integers(-149, 127, size=(n, 1)).astype(np.float64))
    vals = vals.astype(np.float32)
    vals[rng.random((n, 16)) < 0.2] = 0.0
    vals[:16] = np.float32(1e-45) * rng.integers(-3, 4, size=(16, 16))   # subnormal blocks
    vals[16:32] = np.float32(3.4e38) * rng.choice([-1, 1], size=(16, 16))  # at the top of the range
    vals[32:48] = 0.0                                                     # zero blocks
    return vals.reshape(n // 4, 4, 4, 4).transpose(0, 2, 1, 3).reshape(n, 16)


@pytest.mark.parametrize("nw", WORDS)
def test_decode_arbitrary_bits(exe, tmp_path, nw):
    """Any bit string decodes, and exactly as the oracle decodes it."""
    rate = 2 * nw
    rng = np.random.default_rng(100 + nw)
    n = 3000
    g = rng.integers(0, 256, size=2 * rate * n, dtype=np.uint8)
    g[: 2 * rate * 64] &= np.uint8(0x0F)  # many sparse blocks (long runs, early budget ends)
    want = oracle.decode_blocks(g, rate, 0, n)
    for idle in (0, 1):
        got, _ = run(exe, tmp_path, "decode", nw, g, n, idle)
        assert np.array_equal(np.frombuffer(got, np.uint32).reshape(n, 16), want.view(np.uint32)), f"idle={idle}"


@pytest.mark.parametrize("nw", WORDS)
def test_encode_then_decode_matches_oracle(exe, tmp_path, nw):
    rate = 2 * nw
    rng = np.random.default_rng(200 + nw)
    for M in (synth.matrix_rows(synth.SMALL, 0, 16)[:, :1024], extreme_matrix(rng)):
        stream = oracle.encode(M, rate)
        blocks = blocks_of(M).astype(np.float32)
        n = blocks.shape[0]
        got, bad = run(exe, tmp_path, "encode", nw, blocks, n)
        assert bad == 0
        assert got == stream.tobytes()
        want = oracle.decode_blocks(stream, rate, 0, n)
        for idle in (0, 1):
            got, _ = run(exe, tmp_path, "decode", nw, stream, n, idle)
            assert np.array_equal(np.frombuffer(got, np.uint32).reshape(n, 16), want.view(np.uint32))


def test_encode_rejects_non_finite(exe, tmp_path):
    blocks = np.ones((4, 16), np.float32)
    blocks[1, 3] = np.nan
    blocks[3, 0] = np.inf
    got, bad = run(exe, tmp_path, "encode", 4, blocks, 4)
    assert bad == 2
    w = np.frombuffer(got, np.uint32).reshape(4, 4)
    assert np.all(w[1] == 0) and np.all(w[3] == 0)  # encoded as zero blocks


def test_linear_row_sums_match_integer_inverse(exe, tmp_path):
    """The fused kernels take a block's row sums against u as B (C (B^T u)),
    B the inverse lift without its two floor halvings.  That differs from the
    integer inverse transform only by those halvings: a few units of the
    block's last integer bit per value.  The coefficients are those of value
    blocks the encoder accepts (|value| < 2^30 after block scaling), with low
    bits dropped as a fixed rate drops bit planes."""
    rng = np.random.default_rng(7)
    n = 6000
    vals = rng.integers(-(2 ** 30) + 1, 2 ** 30, size=(n, 16), dtype=np.int64)
    smooth = rng.integers(-(2 ** 30) + 2 ** 22, 2 ** 30 - 2 ** 22, size=(n // 2, 1))
    vals[: n // 2] = smooth + rng.integers(-(2 ** 20), 2 ** 20, size=(n // 2, 16))  # smooth blocks
    vals[:100] = rng.integers(-3, 4, size=(100, 16))                            # tiny values
    cf = np.stack([oracle.fwd_xform(v) for v in vals]).astype(np.int64)
    drop = rng.integers(0, 24, size=(n, 1))
    cf = (cf >> drop) << drop                                                   # lost low planes
    u = rng.random((n, 4)).astype(np.float32)
    u[:50] *= -1.0
    rec = np.zeros(n, dtype=[("c", "<i4", 16), ("u", "<f4", 4)])
    rec["c"] = cf.astype(np.int32)
    rec["u"] = u
    got, _ = run(exe, tmp_path, "linear", 0, rec, n)
    out = np.frombuffer(got, np.float64).reshape(n, 8)
    exact, lin = out[:, :4], out[:, 4:]
    bound = 8.0 * np.abs(u).astype(np.float64).sum(axis=1, keepdims=True)
    assert np.all(np.abs(exact - lin) <= bound), float(np.max(np.abs(exact - lin) / bound))
