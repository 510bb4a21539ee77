"""Helpers for the GPU parity tests: run the HIP path through the C-ABI
binding, and compare its output with the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np


def gpu_pipeline(knots3, p, ctrl_np, coef=None, which=3, precision=0, stream=None):
    """wq_bind -> wq_setup (-> wq_qp_physical -> wq_set_coefficient) ->
    wq_pattern -> wq_assemble -> wq_sync.  Returns (plan, row_ptr, col_idx,
    mass, stiff) as device tensors."""
    import torch
    from paper_1605_01238_amd import Plan
    plan = Plan(knots3, p, precision)
    plan.bind(stream)
    ctrl = torch.from_numpy(np.ascontiguousarray(ctrl_np)).cuda()
    plan.setup(ctrl, None, stream)
    if coef is not None:
        x = plan.qp_physical(stream).cpu().numpy().reshape(-1, plan.d)
        a = torch.from_numpy(np.ascontiguousarray(coef(x))).cuda()
        plan.set_coefficient(a, stream)
    row_ptr, col_idx = plan.pattern(stream=stream)
    mass, stiff = plan.assemble(which, stream=stream)
    plan.sync(stream)
    return plan, row_ptr, col_idx, mass, stiff


def gather_rows(row_ptr, values, rows):
    """Values of the given rows (host numpy), gathered on the device."""
    import torch
    rp = row_ptr.cpu().numpy()
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    t = torch.from_numpy(idx).to(values.device)
    return rp, values.index_select(0, t).cpu().numpy().astype(np.float64)


def compare_rows(problem, rows, rp, vals_flat, which):
    """Row-normwise (max|d| / max|row|) and matrix-normwise errors of the
    given rows against the oracle's sum-factorized rows."""
    pos = 0
    row_err, max_abs_d, max_abs = 0.0, 0.0, 0.0
    worst = -1
    for r in rows:
        L = int(rp[r + 1] - rp[r])
        got = vals_flat[pos:pos + L]
        pos += L
        ref = problem.row(int(r), which)
        assert ref.shape == got.shape, (r, ref.shape, got.shape)
        d = np.abs(got - ref).max()
        s = np.abs(ref).max()
        if d / s > row_err:
            row_err, worst = d / s, int(r)
        max_abs_d = max(max_abs_d, d)
        max_abs = max(max_abs, s)
    return row_err, max_abs_d / max_abs, worst


# ---- oracle rows in parallel (spawned CPU workers; the oracle only) -------

_WORKER = {}


def _worker_init(knots, p, ctrl, coef):
    from oracle.assembly import Problem
    _WORKER["P"] = Problem(knots, p, ctrl, coef=coef)


def _worker_rows(args):
    rows, whichs = args
    P = _WORKER["P"]
    return [(int(r), w, P.row(int(r), w)) for r in rows for w in whichs]


def oracle_rows_parallel(knots, p, ctrl, coef, rows, whichs, nproc=None):
    """Oracle rows {(which, row): values} computed by `nproc` spawned worker
    processes (each builds its own Problem; nothing there touches the GPU)."""
    import multiprocessing as mp
    import os
    import time
    nproc = nproc or max(1, min(16, os.cpu_count() or 1))
    rows = [int(r) for r in rows]
    chunks = [(rows[k::nproc * 4], tuple(whichs)) for k in range(nproc * 4)]
    chunks = [c for c in chunks if c[0]]
    t0 = time.time()
    out = {}
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc, initializer=_worker_init, initargs=(list(knots), p, ctrl, coef)) as pool:
        for k, res in enumerate(pool.imap_unordered(_worker_rows, chunks)):
            for r, w, v in res:
                out[(w, r)] = v
            if k % 8 == 0:
                print(f"[oracle] {len(out)}/{len(rows) * len(whichs)} rows ({time.time() - t0:.0f} s)", flush=True)
    return out
