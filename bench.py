#!/usr/bin/env python3
"""Benchmark: weighted-quadrature formation of the isogeometric stiffness (and
mass) matrix on one MI355X.

One step = one pass of the whole device path over one synthetic patch:
  wq_setup    univariate rules (B-splines, exact integrals, minimum-norm
              weights) and the coefficient field at every quadrature point,
  wq_pattern  the CSR pattern (row_ptr, col_idx),
  wq_assemble the sum-factorized rows written into their CSR slots.
Inputs (knots, control net, coefficient at the quadrature points) are
resident in device memory before timing starts.

Prints ONE JSON line (rank 0).  Default workload: p = 4, 32^3 elements,
perturbed map, non-constant coefficient, stiffness, FP64.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="p4_32el_perturbed_coef")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--which", choices=["stiff", "mass", "both"], default=None,
                    help="matrices to form (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU budget of the oracle baseline (0 disables)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per wq_assemble (rocprofv3 --pmc FETCH_SIZE and "
                         "WRITE_SIZE, scaled by a plain copy); ignored once the contraction "
                         "source has changed since the counters were taken")
    return ap.parse_args()


def cpu_baseline(w, which_names, budget_s):
    """The oracle's sum-factorized row formation (Algorithm 3), as it
    stands, on a bounded sample of rows of the same workload, one thread."""
    from threadpoolctl import threadpool_limits
    from oracle.assembly import Problem
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        P = Problem(w.knots(), w.p, w.ctrl(), coef=w.coefficient())
        t_rules = time.perf_counter() - t0
        rng = np.random.default_rng(0)
        N = int(np.prod(w.n_dof()))
        nnz, rows = 0, 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            r = int(rng.integers(0, N))
            for name in which_names:
                nnz += P.row(r, name).size
            rows += 1
        dt = time.perf_counter() - t0
    return {"value": nnz / dt / 1e9, "unit": "GNNZ/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} random rows of the same workload ({'+'.join(which_names)}), "
                      f"sum-factorized FP64 oracle rows incl. per-row geometry, {dt:.1f} s; "
                      f"one-time exact-rational rule setup {t_rules:.1f} s not included"}


def contraction_source_digest():
    import hashlib
    src = os.path.join(ROOT, "paper_1605_01238_amd", "csrc", "wq_contract.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(path, key):
    """HBM bytes per wq_assemble from the committed counter summary, or None
    when there is none for this workload or the kernels changed since."""
    try:
        entry = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not entry or entry.get("source_digest") != contraction_source_digest():
        return None
    return entry.get("bytes_per_launch")


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "one GPU only: rows would shard across GPUs without "
                          "communication, but no multi-GPU path is built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1605_01238_amd import WQ_FP32, WQ_FP64, Plan
    from workloads import WORKLOADS

    w = WORKLOADS[args.workload]
    which_names = {"stiff": ("stiff",), "mass": ("mass",), "both": ("mass", "stiff")}[args.which] \
        if args.which else tuple(w.which)
    which = (1 if "mass" in which_names else 0) | (2 if "stiff" in which_names else 0)
    prec = WQ_FP64 if args.precision == "fp64" else WQ_FP32
    bv = 8 if prec == WQ_FP64 else 4

    # ---- inputs resident in HBM (untimed) ----
    plan = Plan(w.knots(), w.p, prec)
    plan.bind()
    ctrl = torch.from_numpy(w.ctrl()).cuda()
    coef = None
    cf = w.coefficient()
    if cf is not None:
        plan.setup(ctrl)
        x = plan.qp_physical().cpu().numpy().reshape(-1, plan.d)
        coef = torch.from_numpy(np.ascontiguousarray(cf(x))).cuda()
    row_ptr = torch.empty(plan.n_rows + 1, dtype=torch.int64, device="cuda")
    col_idx = torch.empty(plan.nnz, dtype=torch.int32, device="cuda")
    mass = torch.empty(plan.nnz, dtype=plan.value_dtype, device="cuda") if which & 1 else None
    stiff = torch.empty(plan.nnz, dtype=plan.value_dtype, device="cuda") if which & 2 else None
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    ea = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]

    def step(i=None):
        if i is not None:
            ev[2 * i].record(stream)
        plan.setup(ctrl, coef)
        plan.pattern(row_ptr, col_idx)
        plan.assemble(which, mass, stiff)
        if i is not None:
            ev[2 * i + 1].record(stream)

    for _ in range(args.warmup):
        step()
    plan.sync()
    torch.cuda.synchronize()
    # throughput: K plain steps between two synchronizations
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.sync()
    # per-step latency: K more steps, each bracketed by events on the stream
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    plan.sync()

    n_mat = len(which_names)
    ms_per_step = dt / args.steps * 1e3
    value = plan.nnz * n_mat / (dt / args.steps) / 1e9
    t_step = np.array([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps)])    # ms
    # the contraction alone (its inputs complete), for the roofline: the same
    # number of wq_assemble launches, each bracketed by events on the stream
    # the kernels run on
    for i in range(args.steps):
        ea[2 * i].record(stream)
        plan.assemble(which, mass, stiff)
        ea[2 * i + 1].record(stream)
    torch.cuda.synchronize()
    plan.sync()
    t_asm = np.array([ea[2 * i].elapsed_time(ea[2 * i + 1]) for i in range(args.steps)])  # ms
    # algorithmic bytes of one contraction launch: the values written plus one
    # read of the coefficient-field channels it uses
    chans = (6 if which & 2 else 0) + (1 if which & 1 else 0)
    algo_bytes = plan.nnz * bv * n_mat + plan.n_qp_total * chans * bv
    achieved = algo_bytes / (t_asm.mean() * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic_json, f"{w.name}:{args.precision}:{'+'.join(which_names)}")
    out = {
        "metric": "assembled nonzeros/s (GNNZ/s) + % HBM-write roofline, 3D p=4..6; p99 latency",
        "value": round(value, 4),
        "unit": "GNNZ/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == WQ_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "p": w.p, "n_el": list(w.n_el), "matrices": list(which_names),
                   "nnz_per_matrix": plan.nnz, "n_dof": plan.n_rows, "n_qp": plan.n_qp_total,
                   "step": "wq_setup + wq_pattern + wq_assemble", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "wq_assemble = k_first + k_push (two launches)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launch_ms_mean": round(float(t_asm.mean()), 4),
                     "algorithmic_bytes_per_launch": int(algo_bytes)},
        "latency_ms": {"step_p50": round(float(np.percentile(t_step, 50)), 4),
                       "step_p99": round(float(np.percentile(t_step, 99)), 4),
                       "assemble_p50": round(float(np.percentile(t_asm, 50)), 4),
                       "assemble_p99": round(float(np.percentile(t_asm, 99)), 4)},
    }
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(w, which_names, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
