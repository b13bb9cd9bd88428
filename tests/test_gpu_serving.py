"""GPU tests of the serving loop (wh_submit / wh_poll).

  alone vs mix   a request's result is the same (relative L2 2e-6) whether it
                 runs by itself or batched with a stream of other requests
                 against several matrices, and within 1e-6 of the FP64 oracle
  admission      a request that cannot fit the HBM budget (or k > 64) is
                 rejected at submit with WH_ERR_BUDGET
  deadline       a late result is still delivered and flagged missed
  tickets        unknown tickets give WH_ERR_NOT_FOUND; a ticket retires
                 after its result is read
  row chunks     with WH_SERVE_CHUNK_VALUES small, every pass runs as many
                 row-chunk launches (the last one ragged): results still
                 within 1e-6 of the oracle, k = 1 and multi-RHS
  cyclic scan    a request submitted during another's pass joins it at the
                 next chunk launch (starts before that pass ends)
  columns        a request takes any free columns of its matrix's slot
  buffers        pageable host U or Y is refused at submit
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1902_08018_amd import synth, wh

pytestmark = pytest.mark.gpu

SPECS = [synth.MatrixSpec(1024, 1024, 32, 8.0, seed=21), synth.MatrixSpec(2048, 1024, 32, 8.0, seed=22),
         synth.MatrixSpec(512, 2048, 32, 8.0, seed=23)]


def wait(ctx, tickets, timeout=30.0):
    res = {}
    t_end = time.monotonic() + timeout
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            st, r = wh.wh_poll(ctx, t)
            if st == wh.WH_OK:
                res[t] = (r.status, r.t_arrive_ns, r.t_start_ns, r.t_done_ns, r.missed, r.batch_size)
        assert time.monotonic() < t_end, "requests did not complete"
        time.sleep(0.0002)
    return res


def make_request(mat, U, Y, deadline_ns=5_000_000):
    return wh.wh_request(mat=mat, U=U.data_ptr(), u_on_device=int(U.is_cuda), k=U.shape[0], Y=Y.data_ptr(),
                         y_on_device=int(Y.is_cuda), deadline_ns=deadline_ns, arrival_ns=0)


@pytest.fixture(scope="module")
def serving():
    ctx = wh.wh_create(0, 256 << 20)
    mats, streams, refs = [], [], []
    for sp in SPECS:
        M = synth.matrix(sp)
        s = oracle.encode(M, 8)
        d = torch.from_numpy(s).cuda()
        streams.append(d)
        mats.append(wh.wh_load_compressed(ctx, sp.rows, sp.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d))
        refs.append(oracle.decode(s, sp.rows, sp.cols, 8).astype(np.float64))
    yield ctx, mats, refs
    wh.wh_destroy(ctx)


def test_alone_and_in_the_mix(serving):
    ctx, mats, refs = serving
    rng = np.random.default_rng(7)
    # the probe request: matrix 1, k = 3, host (pinned) buffers
    Up = torch.from_numpy(synth.uniform(3 * SPECS[1].cols, seed=99).reshape(3, -1)).pin_memory()
    Y_alone = torch.zeros((3, SPECS[1].rows), dtype=torch.float32).pin_memory()
    t = wh.wh_submit(ctx, make_request(mats[1], Up, Y_alone))
    wait(ctx, [t])
    ref = Up.numpy().astype(np.float64) @ refs[1].T
    err_alone = np.linalg.norm(Y_alone.numpy() - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err_alone.max() <= 1e-6
    # the same request inside a burst of 60 others (host and device buffers)
    keep, tickets, checks = [], [], []
    for i in range(61):
        if i == 30:
            Y_mix = torch.zeros_like(Y_alone).pin_memory()
            tickets.append(wh.wh_submit(ctx, make_request(mats[1], Up, Y_mix)))
            continue
        j = int(rng.integers(0, 3))
        k = int(rng.integers(1, 9))
        on_dev = bool(rng.integers(0, 2))
        U = torch.from_numpy(synth.uniform(k * SPECS[j].cols, seed=1000 + i).reshape(k, -1))
        Y = torch.zeros((k, SPECS[j].rows), dtype=torch.float32)
        if on_dev:
            U, Y = U.cuda(), Y.cuda()
        else:
            U, Y = U.pin_memory(), Y.pin_memory()
        keep.append((U, Y))
        tickets.append(wh.wh_submit(ctx, make_request(mats[j], U, Y)))
        checks.append((j, U, Y))
    res = wait(ctx, tickets)
    assert all(r[0] == wh.WH_OK for r in res.values())
    assert max(r[5] for r in res.values()) > 1, "no batching happened"
    torch.cuda.synchronize()
    rel = np.linalg.norm(Y_mix.numpy() - Y_alone.numpy(), axis=1) / np.linalg.norm(Y_alone.numpy(), axis=1)
    print(f"alone vs mix: worst rel-L2 {rel.max():.3e}")
    assert rel.max() <= 2e-6
    for j, U, Y in checks:
        r = U.cpu().numpy().astype(np.float64) @ refs[j].T
        e = np.linalg.norm(Y.cpu().numpy() - r, axis=1) / np.linalg.norm(r, axis=1)
        assert e.max() <= 1e-6


def test_deadline_flag_and_ticket_retire(serving):
    ctx, mats, _ = serving
    U = torch.rand((1, SPECS[0].cols), device="cuda")
    Y = torch.zeros((1, SPECS[0].rows), device="cuda")
    t = wh.wh_submit(ctx, make_request(mats[0], U, Y, deadline_ns=1))
    res = wait(ctx, [t])[t]
    assert res[0] == wh.WH_OK and res[4] == 1           # late, but delivered
    assert res[1] <= res[2] <= res[3]
    assert torch.count_nonzero(Y) > 0
    with pytest.raises(wh.WhError) as ei:
        wh.wh_poll(ctx, t)                               # retired
    assert ei.value.status == wh.WH_ERR_NOT_FOUND


def test_admission_rejects_what_cannot_fit():
    # 1 MiB: less than one 64-vector slot of a 1024^2 matrix (512 KiB of U and
    # Y, plus the FP64 partials of its 16-slab multi-RHS plan, 8 MiB)
    ctx = wh.wh_create(0, 1 << 20)
    try:
        M = synth.matrix(SPECS[0])
        d = torch.from_numpy(oracle.encode(M, 8)).cuda()
        mat = wh.wh_load_compressed(ctx, 1024, 1024, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
        U = torch.rand((1, 1024), device="cuda")
        Y = torch.zeros((1, 1024), device="cuda")
        with pytest.raises(wh.WhError) as ei:
            wh.wh_submit(ctx, make_request(mat, U, Y))
        assert ei.value.status == wh.WH_ERR_BUDGET
    finally:
        wh.wh_destroy(ctx)


def test_k_limit_and_unknown(serving):
    ctx, mats, _ = serving
    U = torch.rand((65, SPECS[0].cols), device="cuda")
    Y = torch.zeros((65, SPECS[0].rows), device="cuda")
    with pytest.raises(wh.WhError) as ei:
        wh.wh_submit(ctx, make_request(mats[0], U, Y))
    assert ei.value.status == wh.WH_ERR_BUDGET
    with pytest.raises(wh.WhError) as ei:
        wh.wh_submit(ctx, make_request(12345, U[:1], Y[:1]))
    assert ei.value.status == wh.WH_ERR_NOT_FOUND
    with pytest.raises(wh.WhError) as ei:
        wh.wh_poll(ctx, 987654321)
    assert ei.value.status == wh.WH_ERR_NOT_FOUND


def test_unload_while_served():
    """Unloading a served matrix finishes its batches in flight, fails its
    queued requests with WH_ERR_NOT_FOUND, frees its slots for others, and
    later requests for it are unknown."""
    # 20 MiB: one slot of the 2048 x 1024 matrix (16.75 MiB: U, Y and the FP64
    # partials of its 16-slab multi-RHS plan), but not that and a slot of the
    # 512 x 2048 one (8.6 MiB) together
    ctx = wh.wh_create(0, 20 << 20)
    try:
        M = synth.matrix(SPECS[1])
        d = torch.from_numpy(oracle.encode(M, 8)).cuda()
        mat = wh.wh_load_compressed(ctx, SPECS[1].rows, SPECS[1].cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
        U = torch.rand((8, SPECS[1].cols), device="cuda")
        keep, tickets = [], []
        for _ in range(40):
            Y = torch.zeros((8, SPECS[1].rows), device="cuda")
            keep.append(Y)
            tickets.append(wh.wh_submit(ctx, make_request(mat, U, Y)))
        wh.wh_unload(ctx, mat)
        codes = []
        for t in tickets:
            try:
                st, r = wh.wh_poll(ctx, t)
                codes.append(st)
            except wh.WhError as e:
                codes.append(e.status)
        assert all(c in (wh.WH_OK, wh.WH_ERR_NOT_FOUND) for c in codes), codes
        assert wh.WH_PENDING not in codes
        with pytest.raises(wh.WhError) as ei:
            wh.wh_submit(ctx, make_request(mat, U[:1], keep[0][:1]))
        assert ei.value.status == wh.WH_ERR_NOT_FOUND
        # the budget it held serves the other matrix now
        M2 = synth.matrix(SPECS[2])
        d2 = torch.from_numpy(oracle.encode(M2, 8)).cuda()
        mat2 = wh.wh_load_compressed(ctx, SPECS[2].rows, SPECS[2].cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d2)
        U2 = torch.rand((2, SPECS[2].cols), device="cuda")
        Y2 = torch.zeros((2, SPECS[2].rows), device="cuda")
        t2 = wh.wh_submit(ctx, make_request(mat2, U2, Y2))
        assert wait(ctx, [t2])[t2][0] == wh.WH_OK
        ref = U2.double().cpu().numpy() @ oracle.decode(oracle.encode(M2, 8), SPECS[2].rows, SPECS[2].cols, 8).astype(np.float64).T
        err = np.linalg.norm(Y2.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= 1e-6
    finally:
        wh.wh_destroy(ctx)


def test_row_chunked_passes(monkeypatch):
    monkeypatch.setenv("WH_SERVE_CHUNK_VALUES", str(69632))  # 68 rows of 1024 columns, 32 rows of 2048
    ctx = wh.wh_create(0, 256 << 20)
    try:
        mats, refs = [], []
        keep = []
        for sp in SPECS:
            s = oracle.encode(synth.matrix(sp), 8)
            d = torch.from_numpy(s).cuda()
            keep.append(d)
            mats.append(wh.wh_load_compressed(ctx, sp.rows, sp.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d))
            refs.append(oracle.decode(s, sp.rows, sp.cols, 8).astype(np.float64))
        tickets, checks = [], []
        for i, k in enumerate([1, 5, 1, 17, 3, 64]):
            j = i % 3
            U = torch.from_numpy(synth.uniform(k * SPECS[j].cols, seed=500 + i).reshape(k, -1)).pin_memory()
            Y = torch.full((k, SPECS[j].rows), -7.0, dtype=torch.float32).pin_memory()
            tickets.append(wh.wh_submit(ctx, make_request(mats[j], U, Y)))
            checks.append((j, U, Y))
        res = wait(ctx, tickets)
        assert all(r[0] == wh.WH_OK for r in res.values())
        for j, U, Y in checks:
            r = U.numpy().astype(np.float64) @ refs[j].T
            e = np.linalg.norm(Y.numpy() - r, axis=1) / np.linalg.norm(r, axis=1)
            assert e.max() <= 1e-6, (j, U.shape[0], e.max())
    finally:
        wh.wh_destroy(ctx)


def test_load_shedding(monkeypatch):
    """WH_SERVE_SHED=1: while a matrix's oldest queued request has waited
    longer than its deadline, new requests for it are rejected at submit
    with WH_ERR_BUDGET; once the queue drains they are admitted again, and
    every admitted request completes with a correct result.  Deadlines of 1
    ns make any queued request overdue at once."""
    monkeypatch.setenv("WH_SERVE_SHED", "1")
    ctx = wh.wh_create(0, 256 << 20)
    try:
        sp = SPECS[1]
        s = oracle.encode(synth.matrix(sp), 8)
        d = torch.from_numpy(s).cuda()
        mat = wh.wh_load_compressed(ctx, sp.rows, sp.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
        ref_M = oracle.decode(s, sp.rows, sp.cols, 8).astype(np.float64)
        bufs = [(torch.from_numpy(synth.uniform(8 * sp.cols, seed=700 + i).reshape(8, -1)).cuda(),
                 torch.full((8, sp.rows), -7.0, device="cuda")) for i in range(200)]
        reqs = [make_request(mat, U, Y, deadline_ns=1) for U, Y in bufs]
        torch.cuda.synchronize()
        tickets, rejected = [], 0
        for req, (U, Y) in zip(reqs, bufs):  # a tight loop: the queue backs up
            try:
                tickets.append((wh.wh_submit(ctx, req), U, Y))
            except wh.WhError as e:
                assert e.status == wh.WH_ERR_BUDGET
                rejected += 1
        assert rejected > 0 and tickets, (rejected, len(tickets))
        res = wait(ctx, [t for t, _, _ in tickets])
        assert all(r[0] == wh.WH_OK for r in res.values())
        torch.cuda.synchronize()
        for _, U, Y in tickets:
            r = U.cpu().numpy().astype(np.float64) @ ref_M.T
            e = np.linalg.norm(Y.cpu().numpy() - r, axis=1) / np.linalg.norm(r, axis=1)
            assert e.max() <= 1e-6
        # drained: admitted again
        U = torch.from_numpy(synth.uniform(sp.cols, seed=999).reshape(1, -1)).cuda()
        Y = torch.empty((1, sp.rows), device="cuda")
        t = wh.wh_submit(ctx, make_request(mat, U, Y, deadline_ns=1))
        wait(ctx, [t])
    finally:
        wh.wh_destroy(ctx)


def test_requests_join_a_pass_in_progress(monkeypatch):
    """The scan over a matrix's row chunks takes new requests at the next
    chunk launch: a request submitted while another's pass is under way
    starts before that pass ends, and both results are right."""
    monkeypatch.setenv("WH_SERVE_CHUNK_VALUES", str(8 * 1024))  # 8 rows a chunk: 256 chunks of 2048 x 1024
    ctx = wh.wh_create(0, 256 << 20)
    try:
        sp = SPECS[1]
        s = oracle.encode(synth.matrix(sp), 8)
        d = torch.from_numpy(s).cuda()
        mat = wh.wh_load_compressed(ctx, sp.rows, sp.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
        ref_M = oracle.decode(s, sp.rows, sp.cols, 8).astype(np.float64)
        # warm the slot (graphs built on the first request)
        U0 = torch.from_numpy(synth.uniform(sp.cols, seed=800).reshape(1, -1)).cuda()
        Y0 = torch.empty((1, sp.rows), device="cuda")
        t0 = wh.wh_submit(ctx, make_request(mat, U0, Y0))
        wait(ctx, [t0])
        UA = torch.from_numpy(synth.uniform(2 * sp.cols, seed=801).reshape(2, -1)).cuda()
        UB = torch.from_numpy(synth.uniform(3 * sp.cols, seed=802).reshape(3, -1)).cuda()
        YA = torch.full((2, sp.rows), -7.0, device="cuda")
        YB = torch.full((3, sp.rows), -7.0, device="cuda")
        torch.cuda.synchronize()
        ta = wh.wh_submit(ctx, make_request(mat, UA, YA, deadline_ns=1))  # late at once: not held back
        time.sleep(0.0005)
        tb = wh.wh_submit(ctx, make_request(mat, UB, YB))
        res = wait(ctx, [ta, tb])
        a, b = res[ta], res[tb]
        assert a[0] == wh.WH_OK and b[0] == wh.WH_OK
        print(f"A: start {(a[2] - a[1]) * 1e-6:.3f} ms done {(a[3] - a[1]) * 1e-6:.3f} ms; "
              f"B: start {(b[2] - a[1]) * 1e-6:.3f} ms done {(b[3] - a[1]) * 1e-6:.3f} ms")
        assert b[2] < a[3], "B waited for A's pass to end"
        assert b[3] >= a[3]
        torch.cuda.synchronize()
        for U, Y in ((UA, YA), (UB, YB)):
            r = U.cpu().numpy().astype(np.float64) @ ref_M.T
            e = np.linalg.norm(Y.cpu().numpy() - r, axis=1) / np.linalg.norm(r, axis=1)
            assert e.max() <= 1e-6
    finally:
        wh.wh_destroy(ctx)


def test_pageable_host_buffers_are_refused(serving):
    """Host buffers must be page-locked (their copies are then asynchronous
    and the loop never waits on one); pageable ones are refused at submit."""
    ctx, mats, _ = serving
    U = torch.rand((1, SPECS[0].cols))       # pageable
    Y = torch.zeros((1, SPECS[0].rows))
    with pytest.raises(wh.WhError) as ei:
        wh.wh_submit(ctx, make_request(mats[0], U, Y.pin_memory()))
    assert ei.value.status == wh.WH_ERR_INVALID
    with pytest.raises(wh.WhError) as ei:
        wh.wh_submit(ctx, make_request(mats[0], U.pin_memory(), Y))
    assert ei.value.status == wh.WH_ERR_INVALID


def test_requests_take_scattered_columns(monkeypatch):
    """A request takes any free right-hand-side columns of the matrix's slot,
    not only a consecutive run: C joins while B still holds columns in the
    middle of those A freed, and every result is right."""
    monkeypatch.setenv("WH_SERVE_CHUNK_VALUES", str(8 * 1024))  # 256 chunks of 2048 x 1024
    ctx = wh.wh_create(0, 256 << 20)
    try:
        sp = SPECS[1]
        s = oracle.encode(synth.matrix(sp), 8)
        d = torch.from_numpy(s).cuda()
        mat = wh.wh_load_compressed(ctx, sp.rows, sp.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
        ref_M = oracle.decode(s, sp.rows, sp.cols, 8).astype(np.float64)
        U0 = torch.from_numpy(synth.uniform(sp.cols, seed=900).reshape(1, -1)).cuda()
        Y0 = torch.empty((1, sp.rows), device="cuda")
        wait(ctx, [wh.wh_submit(ctx, make_request(mat, U0, Y0, deadline_ns=1))])  # slot built, pass timed
        bufs = {}
        for name, k, seed in (("A", 3, 901), ("B", 2, 902), ("C", 5, 903)):
            bufs[name] = (torch.from_numpy(synth.uniform(k * sp.cols, seed=seed).reshape(k, -1)).cuda(),
                          torch.full((k, sp.rows), -7.0, device="cuda"))
        torch.cuda.synchronize()
        ta = wh.wh_submit(ctx, make_request(mat, *bufs["A"], deadline_ns=1))
        time.sleep(0.004)  # B joins part of the way through A's pass
        tb = wh.wh_submit(ctx, make_request(mat, *bufs["B"], deadline_ns=1))
        ra = wait(ctx, [ta])[ta]
        tc = wh.wh_submit(ctx, make_request(mat, *bufs["C"], deadline_ns=1))
        res = wait(ctx, [tb, tc])
        rb, rc = res[tb], res[tc]
        print(f"A done {(ra[3] - ra[1]) * 1e-6:.2f} ms, B start {(rb[2] - ra[1]) * 1e-6:.2f} done "
              f"{(rb[3] - ra[1]) * 1e-6:.2f}, C start {(rc[2] - ra[1]) * 1e-6:.2f}")
        assert rc[2] < rb[3], "C did not join while B was under way"
        torch.cuda.synchronize()
        for U, Y in bufs.values():
            r = U.cpu().numpy().astype(np.float64) @ ref_M.T
            e = np.linalg.norm(Y.cpu().numpy() - r, axis=1) / np.linalg.norm(r, axis=1)
            assert e.max() <= 1e-6
    finally:
        wh.wh_destroy(ctx)
