#!/usr/bin/env python3
"""Benchmark: weighted-quadrature formation of the isogeometric mass and
stiffness matrices on one MI355X.

One step = one pass of the whole device path over one synthetic patch:
  wq_setup    univariate rules (B-splines, exact integrals, minimum-norm
              weights) and the coefficient field at every quadrature point,
  wq_pattern  the CSR pattern (row_ptr, col_idx),
  wq_assemble the sum-factorized rows written into their CSR slots.
Inputs (knots, control net, coefficient at the quadrature points) are
resident in device memory before timing starts.

Prints ONE JSON line.  Default workload: p = 6, 64^3 elements, twisted and
perturbed map, mass + stiffness, FP64 (the large single-patch case, whose
5.2 GB per matrix is far beyond the 256 MB last-level cache).  Extra keys
give the same patch in FP32 bulk (speed-up and error against the FP64 run)
and the p = 4, 32^3 stiffness case.
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
MAX_CPU_WORKERS = 16    # host-core share of one GPU


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="p6_64el_twisted")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--which", choices=["stiff", "mass", "both"], default=None,
                    help="matrices to form (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the oracle baseline on the host cores (0 disables)")
    ap.add_argument("--extras", type=int, default=1,
                    help="also time the FP32-bulk form of the workload and the p=4 32^3 case")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per wq_assemble (rocprofv3 --pmc FETCH_SIZE and "
                         "WRITE_SIZE, scaled by a plain copy); ignored once the contraction "
                         "source has changed since the counters were taken")
    return ap.parse_args()


# ---------------------------------------------------------------- CPU leg --
_CPU_PROBLEM = None


def _cpu_worker(args):
    """Rows of the oracle (sum-factorized, Algorithm 3) for `budget` seconds,
    one thread; returns (rows, nonzeros, seconds)."""
    seed, budget, which_names, n_rows = args
    from threadpoolctl import threadpool_limits
    rng = np.random.default_rng(seed)
    nnz, rows = 0, 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            r = int(rng.integers(0, n_rows))
            for name in which_names:
                nnz += _CPU_PROBLEM.row(r, name).size
            rows += 1
        dt = time.perf_counter() - t0
    return rows, nnz, dt


def cpu_baseline(w, which_names, budget_s):
    """The oracle as it stands (its sum-factorized rows, including the
    per-row geometry) on random rows of the same workload: one thread for
    a short while, then one process per host core (at most 16) for
    `budget_s` seconds.  Runs before the GPU is touched (worker processes
    are forked)."""
    import multiprocessing as mp
    from oracle.assembly import Problem
    global _CPU_PROBLEM
    t0 = time.perf_counter()
    _CPU_PROBLEM = Problem(w.knots(), w.p, w.ctrl(), coef=w.coefficient())
    t_rules = time.perf_counter() - t0
    n_rows = int(np.prod(w.n_dof()))
    r1, z1, d1 = _cpu_worker((12345, min(4.0, budget_s), which_names, n_rows))
    cores = max(1, min(MAX_CPU_WORKERS, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(s, budget_s, which_names, n_rows) for s in range(cores)])
    wall = time.perf_counter() - t0
    rows = sum(r for r, _, _ in res)
    nnz = sum(z for _, z, _ in res)
    return {"value": nnz / wall / 1e9, "unit": "GNNZ/s", "cores": cores, "kind": "oracle",
            "single_thread_value": z1 / d1 / 1e9,
            "sample": f"{rows} random rows of the same workload ({'+'.join(which_names)}) on {cores} "
                      f"processes for {wall:.1f} s wall (one-thread run: {r1} rows, {d1:.1f} s); "
                      f"sum-factorized FP64 oracle rows incl. per-row geometry; one-time "
                      f"exact-rational rule setup {t_rules:.1f} s not included"}


# ---------------------------------------------------------------- GPU leg --
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


class Run:
    """Device state of one workload at one precision: plan, inputs and
    outputs resident in HBM."""

    def __init__(self, w, prec, which_names):
        import torch
        from paper_1605_01238_amd import Plan
        self.w, self.which_names = w, which_names
        self.which = (1 if "mass" in which_names else 0) | (2 if "stiff" in which_names else 0)
        self.plan = plan = Plan(w.knots(), w.p, prec)
        plan.bind()
        self.ctrl = torch.from_numpy(w.ctrl()).cuda()
        self.coef = None
        cf = w.coefficient()
        if cf is not None:
            plan.setup(self.ctrl)
            x = plan.qp_physical().cpu().numpy().reshape(-1, plan.d)
            self.coef = torch.from_numpy(np.ascontiguousarray(cf(x))).cuda()
        self.row_ptr = torch.empty(plan.n_rows + 1, dtype=torch.int64, device="cuda")
        self.col_idx = torch.empty(plan.nnz, dtype=torch.int32, device="cuda")
        self.mass = torch.empty(plan.nnz, dtype=plan.value_dtype, device="cuda") if self.which & 1 else None
        self.stiff = torch.empty(plan.nnz, dtype=plan.value_dtype, device="cuda") if self.which & 2 else None
        self.stream = torch.cuda.current_stream()

    def step(self):
        self.plan.setup(self.ctrl, self.coef)
        self.plan.pattern(self.row_ptr, self.col_idx)
        self.plan.assemble(self.which, self.mass, self.stiff)

    def time_steps(self, steps, warmup):
        """Throughput over `steps` back-to-back steps between two device
        synchronizations; then per-step latencies (each step bracketed by
        events) and per-assemble durations (events on the stream the
        kernels run on)."""
        import torch
        for _ in range(warmup):
            self.step()
        self.plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        self.plan.sync()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        for i in range(steps):
            ev[2 * i].record(self.stream)
            self.step()
            ev[2 * i + 1].record(self.stream)
        torch.cuda.synchronize()
        self.plan.sync()
        t_step = np.array([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)])
        ea = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        for i in range(steps):
            ea[2 * i].record(self.stream)
            self.plan.assemble(self.which, self.mass, self.stiff)
            ea[2 * i + 1].record(self.stream)
        torch.cuda.synchronize()
        self.plan.sync()
        t_asm = np.array([ea[2 * i].elapsed_time(ea[2 * i + 1]) for i in range(steps)])
        return dt / steps * 1e3, t_step, t_asm

    def value_bytes(self):
        return self.plan.sizes.value_bytes * len(self.which_names)


def batch_extra(steps, warmup, n_patches=64, seed=4):
    """The batched form: n_patches independent 3D patches, p uniform in
    {2..6}, 8..40 elements per direction (independently), each with its own
    seeded perturbed geometry and coefficient field; FP32 bulk (FP64 weights
    and Jacobians), schedules from the library's autotuner, the whole launch
    sequence replayed from a captured HIP graph.  Set beside the plain FP64
    form (one wq_assemble per patch) on the same GPU: speed-up and the
    matrix-normwise difference of the values."""
    import torch
    from paper_1605_01238_amd import WQ_FP32, WQ_FP64, Batch, Plan
    from workloads import batch_patches
    ws = batch_patches(n_patches, seed=seed)

    def make(prec):
        plans, mass, stiff = [], [], []
        for w in ws:
            plan = Plan(w.knots(), w.p, prec)
            plan.bind()
            plan.setup(torch.from_numpy(w.ctrl()).cuda())
            x = plan.qp_physical().reshape(-1, plan.d)
            plan.set_coefficient(w.coefficient().torch(x).contiguous())
            plans.append(plan)
            mass.append(torch.empty(plan.nnz, dtype=plan.value_dtype, device="cuda"))
            stiff.append(torch.empty(plan.nnz, dtype=plan.value_dtype, device="cuda"))
        return plans, mass, stiff

    p32, m32, s32 = make(WQ_FP32)
    batch = Batch(p32)
    batch.bind(m32, s32)
    batch.tune(3)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(max(1, warmup)):
            batch.assemble(3, use_graph=True, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            batch.assemble(3, use_graph=True, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t32 = e0.elapsed_time(e1) / steps
    nnz = sum(p.nnz for p in p32)
    # the same FP32 plans, one wq_assemble per patch (batching at equal precision)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record()
    for _ in range(steps):
        for plan, m, s in zip(p32, m32, s32):
            plan.assemble(3, m, s)
    g1.record()
    torch.cuda.synchronize()
    t32p = g0.elapsed_time(g1) / steps
    p64, m64, s64 = make(WQ_FP64)
    for plan, m, s in zip(p64, m64, s64):
        plan.assemble(3, m, s)
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    for _ in range(steps):
        for plan, m, s in zip(p64, m64, s64):
            plan.assemble(3, m, s)
    f1.record()
    torch.cuda.synchronize()
    t64 = f0.elapsed_time(f1) / steps
    err = {"mass": 0.0, "stiff": 0.0}
    for a, b_ in ((m32, m64), (s32, s64)):
        key = "mass" if a is m32 else "stiff"
        for x, y in zip(a, b_):
            err[key] = max(err[key], float((x.double() - y).abs().max() / y.abs().max()))
    out = {"workload": f"{n_patches} patches, p in 2..6, 8..40 elements/dir, mass+stiff",
           "nnz_per_matrix": nnz, "value": round(2 * nnz / (t32 * 1e-3) / 1e9, 3), "unit": "GNNZ/s",
           "ms_per_batch": round(t32, 4), "dtype": "f32",
           "frac": round(2 * nnz * 4 / (t32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "fp64_per_patch_ms": round(t64, 4),
           "speedup_vs_fp64_per_patch": round(t64 / t32, 3),
           "fp32_per_patch_ms": round(t32p, 4),
           "speedup_vs_fp32_per_patch": round(t32p / t32, 3),
           "matrix_normwise_diff_vs_fp64": err,
           "schedule": batch.schedule()}
    del batch, p32, m32, s32, p64, m64, s64
    torch.cuda.empty_cache()
    return out


def serving_extra(n_requests=2000, n_geoms=16, seed=5):
    """The serving loop: n_geoms resident geometries (p uniform in {2..6},
    8..48 elements per direction, 2D with probability 0.3), each set up once
    (weights, det J, J^{-1}, pattern resident); n_requests requests, each a
    new seeded coefficient field on one of them (stiffness, FP32 bulk),
    arriving as a seeded Poisson stream; continuous batching over 4 streams
    with at most 32 requests and 32 GiB in flight.  First all requests at
    once (capacity), then Poisson rates of 0.5 and 0.8 of that capacity."""
    import torch
    from paper_1605_01238_amd import WQ_FP32, WQ_STIFF
    from paper_1605_01238_amd.serving import Geometry, Server, poisson_requests, summarize
    from workloads import batch_patches, coefficient_field
    ws = batch_patches(n_geoms, seed=seed, nel_range=(8, 48), d_choices=(2, 3), p2d=0.3)
    geoms = [Geometry(w.knots(), w.p, w.ctrl(), WQ_FP32, WQ_STIFF) for w in ws]

    def coef(req, xq):
        return coefficient_field(req.coef_seed).torch(xq).contiguous()

    srv = Server(geoms, coef, n_streams=4, max_inflight=32, hbm_budget=32 << 30)
    srv.run(poisson_requests(64, 0.0, n_geoms, seed + 1))          # warm-up
    torch.cuda.synchronize()
    cap = summarize(srv.run(poisson_requests(n_requests, 0.0, n_geoms, seed + 2)))
    runs = {"all_at_once": cap}
    for frac in (0.5, 0.8):
        rate = frac * cap["requests_per_s"]
        runs[f"poisson_{frac}x"] = dict(summarize(srv.run(poisson_requests(n_requests, rate, n_geoms,
                                                                         seed + 3))),
                                        rate_per_s=round(rate, 1))
    torch.cuda.synchronize()
    out = {"workload": f"{n_requests} requests on {n_geoms} resident geometries (p 2..6, 8..48 el/dir, "
                       f"30% 2D), new coefficient each, stiffness, FP32 bulk",
           "geometries": [(w.p, list(w.n_el)) for w in ws], "runs": runs,
           "peak_inflight": srv.peak_inflight, "peak_gib_inflight": round(srv.peak_bytes / 2**30, 2)}
    del srv, geoms
    torch.cuda.empty_cache()
    return out


def fill_rate_gbs(nbytes, reps=5):
    """Write-only streaming fill of `nbytes` on the same GPU (torch fill_),
    GB/s: the practical write ceiling beside the nominal peak."""
    import torch
    buf = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    buf.fill_(1.0)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = []
    for _ in range(reps):
        s.record()
        buf.fill_(0.0)
        e.record()
        torch.cuda.synchronize()
        best.append(s.elapsed_time(e))
    del buf
    torch.cuda.empty_cache()
    return buf_bytes_gbs(nbytes, float(np.median(best)))


def buf_bytes_gbs(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "one GPU only: rows would shard across GPUs without "
                          "communication, but no multi-GPU path is built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    from workloads import MID_P4, WORKLOADS
    w = WORKLOADS[args.workload]
    which_names = {"stiff": ("stiff",), "mass": ("mass",), "both": ("mass", "stiff")}[args.which] \
        if args.which else tuple(w.which)

    # CPU leg first, before anything initialises the GPU (its workers are forked)
    cpu = cpu_baseline(w, which_names, args.cpu_seconds) if args.cpu_seconds > 0 else None

    import torch
    from paper_1605_01238_amd import WQ_FP32, WQ_FP64
    prec = WQ_FP64 if args.precision == "fp64" else WQ_FP32
    run = Run(w, prec, which_names)
    plan = run.plan
    ms_per_step, t_step, t_asm = run.time_steps(args.steps, args.warmup)
    n_mat = len(which_names)
    value = plan.nnz * n_mat / (ms_per_step * 1e-3) / 1e9
    vbytes = run.value_bytes()
    bv = vbytes // (plan.nnz * n_mat)
    # field channels the contraction reads: the stiffness K11..K23 (only
    # K11, K22, K12 on a plane patch), the mass det J
    chans = ((6 if plan.d == 3 else 3) if run.which & 2 else 0) + (1 if run.which & 1 else 0)
    read_bytes = plan.n_qp_total * chans * bv
    achieved = buf_bytes_gbs(vbytes, float(t_asm.mean()))
    fill = fill_rate_gbs(vbytes)
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
        "roofline": {"bound": "hbm",
                     "kernel": "wq_assemble (" + ("k_first + k_push" if plan.d == 3 else "k_plane") + " per matrix)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launch_ms_mean": round(float(t_asm.mean()), 4),
                     "algorithmic_bytes_per_launch": int(vbytes),
                     "field_read_bytes_per_launch": int(read_bytes),
                     "fill_gbs": round(fill, 1), "frac_of_fill": round(achieved / fill, 4),
                     "assemble_gnnz_s": round(plan.nnz * n_mat / (t_asm.mean() * 1e-3) / 1e9, 2)},
        "latency_ms": {"step_p50": round(float(np.percentile(t_step, 50)), 4),
                       "step_p99": round(float(np.percentile(t_step, 99)), 4),
                       "assemble_p50": round(float(np.percentile(t_asm, 50)), 4),
                       "assemble_p99": round(float(np.percentile(t_asm, 99)), 4)},
    }
    if args.extras:
        extras = {}
        if prec == WQ_FP64:
            # the same patch in FP32 bulk: speed-up and matrix-normwise
            # difference against the FP64 values just formed
            ref = {"mass": run.mass, "stiff": run.stiff}
            r32 = Run(w, WQ_FP32, which_names)
            ms32, _, ta32 = r32.time_steps(args.steps, args.warmup)
            errs = {}
            for name in which_names:
                a64 = ref[name]
                a32 = r32.mass if name == "mass" else r32.stiff
                errs[name] = float((a32.double() - a64).abs().max() / a64.abs().max())
            vb32 = r32.value_bytes()
            extras["fp32_bulk"] = {
                "value": round(plan.nnz * n_mat / (ms32 * 1e-3) / 1e9, 4), "ms_per_step": round(ms32, 4),
                "assemble_ms_mean": round(float(ta32.mean()), 4),
                "frac": round(buf_bytes_gbs(vb32, float(ta32.mean())) / HBM_PEAK_GBS, 4),
                "speedup_vs_fp64_step": round(ms_per_step / ms32, 3),
                "speedup_vs_fp64_assemble": round(float(t_asm.mean() / ta32.mean()), 3),
                "matrix_normwise_diff_vs_fp64": errs}
            del r32
        del run
        torch.cuda.empty_cache()
        if w.name != MID_P4.name:
            r4 = Run(MID_P4, prec, tuple(MID_P4.which))
            ms4, _, ta4 = r4.time_steps(args.steps, args.warmup)
            vb4 = r4.value_bytes()
            extras[MID_P4.name] = {
                "value": round(r4.plan.nnz / (ms4 * 1e-3) / 1e9, 4), "ms_per_step": round(ms4, 4),
                "assemble_ms_mean": round(float(ta4.mean()), 4),
                "frac": round(buf_bytes_gbs(vb4, float(ta4.mean())) / HBM_PEAK_GBS, 4),
                "note": "225 MB of values: fits the 256 MB last-level cache"}
            del r4
        extras["batch_64"] = batch_extra(args.steps, args.warmup)
        extras["serving"] = serving_extra()
        sv = extras["serving"]["runs"]["poisson_0.8x"]
        out["latency_ms"]["serving_p50"] = sv["latency_ms_p50"]
        out["latency_ms"]["serving_p99"] = sv["latency_ms_p99"]
        out["extra"] = extras
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
