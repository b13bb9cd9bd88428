"""GPU parity of the thermal step (Sec. 2.1, Eq. 1) against the FP64 oracle.

  one step      the GPU rounds the FP64 row sum once to FP32, as the oracle's
                stored state does: bit-equal but for rare last-bit ties of
                summation order (at most 1 FP32 ulp), on the 608 x 608 mesh
                (about 3.7e5 temperatures, the paper's size) and small meshes
                down to one cell
  runs          64 steps with a moving source (even and odd counts: the
                ping-pong ends in either buffer) within 1e-6 relative L2
  heat content  c^T T grows by dt * sum(u) per step on the GPU's own output
  errors        in-place step, short leading dimension; out-of-range CSR
                entries are skipped by the kernel's own bounds checks
"""
import math

import numpy as np
import pytest
import torch

from oracle import thermal
from paper_1902_08018_amd import synth, wh

pytestmark = pytest.mark.gpu


def system(spec):
    row_ptr, col, val, b = synth.thermal_system(spec)
    return (row_ptr, col, val, b), wh.ThermalSystem(row_ptr, col, val, b)


@pytest.mark.parametrize("spec", [synth.ThermalSpec(1, 1), synth.ThermalSpec(5, 1), synth.ThermalSpec(1, 4),
                                  synth.ThermalSpec(4, 3), synth.ThermalSpec(9, 7, seed=3),
                                  synth.ThermalSpec(257, 131, seed=1), synth.THERMAL])
def test_one_step(gpu_ctx, spec):
    host, dev = system(spec)
    T = synth.thermal_initial(spec)
    u = synth.thermal_source(spec, 5)
    want = thermal.thermal_step(*host, T, u).astype(np.float32)
    Td, ud = torch.from_numpy(T).cuda(), torch.from_numpy(u).cuda()
    out = torch.full((spec.n + 1,), -7.0, device="cuda")
    wh.wh_thermal_step(gpu_ctx, dev, Td, ud, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got[spec.n] == -7.0
    got = got[:spec.n]
    ulp = np.spacing(np.abs(want))
    assert np.all(np.abs(got - want) <= ulp)
    assert np.mean(got == want) >= 0.9999


@pytest.mark.parametrize("steps", [64, 63, 1])
def test_run(gpu_ctx, steps):
    spec = synth.ThermalSpec(128, 96, seed=2)
    host, dev = system(spec)
    T0 = synth.thermal_initial(spec)
    U = np.stack([synth.thermal_source(spec, k) for k in range(steps)])
    want = thermal.thermal_run(*host, T0, U)
    Ud = torch.zeros((steps, spec.n + 3), device="cuda")  # leading dimension > n
    Ud[:, :spec.n] = torch.from_numpy(U)
    Td = torch.from_numpy(T0).cuda()
    work = torch.empty(spec.n, device="cuda")
    wh.wh_thermal_run(gpu_ctx, dev, Td, Ud, work)
    torch.cuda.synchronize()
    got = Td.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= 1e-6
    # heat content on the GPU's own output
    c = synth.thermal_capacity(spec)
    gain = spec.dt * math.fsum(U.astype(np.float64).ravel())
    before, after = math.fsum(c * T0.astype(np.float64)), math.fsum(c * got)
    assert abs(after - (before + gain)) <= 1e-6 * before


def test_zero_steps_and_errors(gpu_ctx):
    spec = synth.ThermalSpec(4, 3)
    host, dev = system(spec)
    T = torch.from_numpy(synth.thermal_initial(spec)).cuda()
    T_copy = T.clone()
    U = torch.zeros((0, spec.n), device="cuda")
    work = torch.empty(spec.n, device="cuda")
    wh.wh_thermal_run(gpu_ctx, dev, T, U, work)
    torch.cuda.synchronize()
    assert torch.equal(T, T_copy)
    u = torch.zeros(spec.n, device="cuda")
    with pytest.raises(wh.WhError) as ei:
        wh.wh_thermal_step(gpu_ctx, dev, T, u, T)  # in place
    assert ei.value.status == wh.WH_ERR_INVALID
    with pytest.raises(wh.WhError) as ei:
        wh.wh_thermal_run(gpu_ctx, dev, T, torch.zeros((2, spec.n), device="cuda"), T)  # work is T
    assert ei.value.status == wh.WH_ERR_INVALID


def test_out_of_range_entries_are_skipped(gpu_ctx):
    """A row pointer past nnz and a column >= n: the kernel's bounds checks
    skip those entries (the arrays themselves have their stated lengths)."""
    n = 4
    row_ptr = np.array([0, 2, 9, 9, 3], np.uint32)  # row 1 claims entries up to 9 > nnz = 3
    col = np.array([0, 7, 2], np.uint32)             # column 7 >= n
    val = np.array([1.0, 5.0, 2.0], np.float32)
    b = np.zeros(n, np.float32)
    dev = wh.ThermalSystem(row_ptr, col, val, b)
    assert dev.nnz == 3
    T = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda")
    out = torch.full((n,), -7.0, device="cuda")
    wh.wh_thermal_step(gpu_ctx, dev, T, torch.zeros(n, device="cuda"), out)
    torch.cuda.synchronize()
    # row 0: entries 0..1 -> 1*T0 (col 7 skipped); row 1: entries 2..2 (clamped to nnz) -> 2*T2;
    # row 2: empty; row 3: row_ptr 9 > 3 clamps to [3, 3): empty
    assert out.cpu().tolist() == [1.0, 6.0, 0.0, 0.0]
