"""CPU tests of the host side: the C-ABI library loads and exports every
entry point its header declares, argument checking and sizes work without a
GPU, and the seeded input generator is pinned to its published definitions."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1902_08018_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wh.h")
LIB = os.path.join(ROOT, "paper_1902_08018_amd", "libwh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wh_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libwh.so not built")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} declared in wh.h but not exported"


def test_status_strings(lib):
    lib.wh_status_str.restype = ctypes.c_char_p
    for st in range(-7, 2):
        s = lib.wh_status_str(st)
        assert s and s != b"unknown status"
    assert lib.wh_status_str(-99) == b"unknown status"


class Desc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint32), ("cols", ctypes.c_uint32), ("fmt", ctypes.c_int32),
                ("rate", ctypes.c_uint32)]


@pytest.mark.parametrize("rows,cols,fmt,rate,want", [
    (4096, 4096, 1, 8, 4096 * 4096),              # 1 byte per value at rate 8
    (4096, 4096, 1, 16, 2 * 4096 * 4096),
    (65536, 65536, 1, 8, 65536 * 65536),
    (8, 12, 1, 2, 6 * 4),                         # 6 blocks x 4 bytes
    (6, 8, 1, 8, 4 * 16),                         # partial block-row: 2 x 2 blocks
    (378, 256000, 1, 8, 95 * 64000 * 16),         # the paper's slit matrix, edge-padded to 380 rows
    (1, 1, 1, 16, 32),
    (64, 64, 2, 0, 64 * 64 * 4),
    (64, 64, 3, 0, 64 * 64 * 2),
    (64, 64, 4, 0, 64 * 64 * 2),
    (64, 64, 5, 0, 256 * 16 + 256 * 4),
])
def test_storage_bytes(lib, rows, cols, fmt, rate, want):
    n = ctypes.c_uint64()
    d = Desc(rows, cols, fmt, rate)
    assert lib.wh_storage_bytes(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value == want


@pytest.mark.parametrize("rows,cols,fmt,rate,code", [
    (6, 8, 2, 0, -2), (8, 6, 3, 0, -2), (0, 8, 1, 8, -2),   # shape (dense formats: whole 4 x 4 tiles)
    (8, 8, 1, 7, -3), (8, 8, 1, 34, -3), (8, 8, 9, 0, -3),  # odd / too large rate, unknown format
])
def test_storage_bytes_errors(lib, rows, cols, fmt, rate, code):
    n = ctypes.c_uint64(12345)
    d = Desc(rows, cols, fmt, rate)
    assert lib.wh_storage_bytes(ctypes.byref(d), ctypes.byref(n)) == code
    assert n.value == 12345  # out-param untouched on error


def test_null_arguments_rejected(lib):
    assert lib.wh_create(0, 0, None) == -1
    assert lib.wh_destroy(None) == -1
    assert lib.wh_gemv(None, ctypes.c_uint64(1), None, None, 0, 0, 0, None) == -1
    assert lib.wh_submit(None, None, None) == -1
    assert lib.wh_poll(None, ctypes.c_uint64(1), None) == -1


def test_create_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert lib.wh_create(0, 0, ctypes.byref(ctx)) == -6  # WH_ERR_DEVICE
    assert ctx.value is None


# ------------------------------------------------------------- generator
def test_splitmix64_published_output():
    # SplitMix64 (Steele, Lea, Flood 2014) seeded with 0: its first output is
    # the output function applied to the golden gamma, 0xE220A8397B1DCDAF.
    L = synth._hostlib()
    # key(seed, stream) is mix64((seed << 8) | stream); recover mix64 through
    # hash(k=-1): mix64(key + 0) = mix64(mix64(stream)); with a known key path
    # instead check the output function on the gamma via the twin below.
    def mix64(z):
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & 0xFFFFFFFFFFFFFFFF
        z = (z ^ (z >> 27)) * 0x94D049BB133111EB & 0xFFFFFFFFFFFFFFFF
        return z ^ (z >> 31)
    assert mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    for seed, stream, k in [(0, 0, 0), (0, 1, 5), (7, 3, 123456789)]:
        key = mix64((seed << 8) | stream)
        want = mix64((key + (k + 1) * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF)
        assert int(L.whs_hash(seed, stream, k)) == want


def test_uniform_vectors_exact_24_bit():
    u = synth.uniform(100000, seed=0)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))
    assert abs(u.mean() - 0.5) < 0.005
    assert abs(u.var() - 1 / 12) < 0.002


def test_matrix_follows_its_definition():
    spec = synth.MatrixSpec(64, 64, 8, 2.0, sigma=0.0)
    M = synth.matrix(spec)
    for i, j in [(0, 0), (3, 5), (63, 0), (10, 50)]:
        d = math.hypot(i % 8 - j % 8, i // 8 - j // 8)
        assert M[i, j] == np.float32(math.exp(-d / 2.0))
    # noise: Irwin-Hall(12) has mean 0, variance 1
    spec_n = synth.MatrixSpec(64, 4096, 64, 8.0, sigma=1.0)
    base = synth.matrix(synth.MatrixSpec(64, 4096, 64, 8.0, sigma=0.0)).astype(np.float64)
    z = synth.matrix(spec_n).astype(np.float64) - base
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.02
    assert np.abs(z).max() <= 6.0


def test_matrix_rows_are_slices():
    spec = synth.MatrixSpec(64, 256, 16, 4.0)
    full = synth.matrix(spec)
    assert np.array_equal(synth.matrix_rows(spec, 20, 28), full[20:28])
