"""Batches of patches (wq_batch_*): per-class persistent launches over a
device work queue, autotuned schedules, captured graphs.  Every patch's
values must equal its own wq_assemble bit for bit (same kernels, same
arithmetic per row), for every schedule and on every graph replay; sampled
rows are also checked against the oracle."""
import numpy as np
import pytest

from parity_helpers import compare_rows, gather_rows
from workloads import batch_patches, sample_rows

pytestmark = pytest.mark.gpu


def _make(ws, precision):
    """Bound and set-up plans of the workloads, the per-patch reference values
    from wq_assemble, and empty outputs for the batch."""
    import torch
    from paper_1605_01238_amd import Plan
    plans, refs, outs = [], [], []
    for w in ws:
        plan = Plan(w.knots(), w.p, precision)
        plan.bind()
        ctrl = torch.from_numpy(w.ctrl()).cuda()
        plan.setup(ctrl)
        x = plan.qp_physical().reshape(-1, plan.d)
        plan.set_coefficient(w.coefficient().torch(x).contiguous())
        m, s = plan.assemble(3)
        plan.sync()
        plans.append(plan)
        refs.append((m, s))
        outs.append((torch.full_like(m, float("nan")), torch.full_like(s, float("nan"))))
    return plans, refs, outs


def _equal_all(refs, outs):
    import torch
    for k, ((m, s), (m2, s2)) in enumerate(zip(refs, outs)):
        assert torch.equal(m, m2), f"patch {k}: mass differs"
        assert torch.equal(s, s2), f"patch {k}: stiffness differs"


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_patch_assembly(precision):
    import torch
    from paper_1605_01238_amd import Batch
    ws = batch_patches(12, seed=7, nel_range=(4, 12), d_choices=(2, 3), p2d=0.3)
    plans, refs, outs = _make(ws, precision)
    b = Batch(plans)
    b.bind([o[0] for o in outs], [o[1] for o in outs])
    print(f"[batch prec={precision}] {len(ws)} patches, {b.n_classes} classes: "
          f"{[(w.p, w.n_el) for w in ws]}", flush=True)
    b.assemble(3)
    torch.cuda.synchronize()
    _equal_all(refs, outs)
    # the autotuner tries every candidate schedule (each must be exact too)
    for o in outs:
        o[0].fill_(float("nan"))
        o[1].fill_(float("nan"))
    b.tune(3)
    print(f"[batch prec={precision}] tuned: {b.schedule()}", flush=True)
    b.assemble(3)
    torch.cuda.synchronize()
    _equal_all(refs, outs)


def test_batch_graph_replays():
    """Captured launch sequence replayed three times with eager work and
    synchronizations between the replays; each replay equals the eager
    per-patch result (the work-queue counters are reset by a kernel inside
    the graph)."""
    import torch
    from paper_1605_01238_amd import Batch
    ws = batch_patches(8, seed=11, nel_range=(5, 10))
    plans, refs, outs = _make(ws, 1)
    b = Batch(plans)
    b.bind([o[0] for o in outs], [o[1] for o in outs])
    side = torch.cuda.Stream()
    for rep in range(3):
        for o in outs:
            o[0].fill_(float("nan"))
            o[1].fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            b.assemble(3, use_graph=True, stream=side)
        side.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        _equal_all(refs, outs)
        print(f"[batch graph] replay {rep} equal ({float(junk):.1f})", flush=True)
    # after tuning (schedules may now launch the single-patch kernels patch
    # after patch, masses and stiffnesses on separate side streams) the
    # graph is captured again; its replays must still be exact
    b.tune(3)
    print(f"[batch graph] tuned: {b.schedule()}", flush=True)
    for rep in range(2):
        for o in outs:
            o[0].fill_(float("nan"))
            o[1].fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            b.assemble(3, use_graph=True, stream=side)
        side.synchronize()
        _equal_all(refs, outs)
        print(f"[batch graph] tuned replay {rep} equal", flush=True)


def test_batch_sampled_rows_against_oracle():
    """FP32 bulk batch: sampled rows (uniform and boundary) of every patch
    against the FP64 oracle, matrix-normwise within 1e-5."""
    import torch
    from oracle.assembly import Problem
    from paper_1605_01238_amd import Batch
    ws = batch_patches(5, seed=13, nel_range=(4, 9))
    plans, refs, outs = _make(ws, 1)
    b = Batch(plans)
    b.bind([o[0] for o in outs], [o[1] for o in outs])
    b.assemble(3)
    torch.cuda.synchronize()
    for k, (w, plan) in enumerate(zip(ws, plans)):
        P = Problem(w.knots(), w.p, w.ctrl(), coef=w.coefficient())
        row_ptr, _ = plan.pattern()
        rows = sample_rows(plan.n, w.p, 12, 12, seed=k)
        for name, vals in (("mass", outs[k][0]), ("stiff", outs[k][1])):
            rp, v = gather_rows(row_ptr, vals, rows)
            _, mat_err, _ = compare_rows(P, rows, rp, v, name)
            print(f"[batch oracle] patch {k} p={w.p} n_el={w.n_el} {name}: {mat_err:.2e}", flush=True)
            assert mat_err <= 1e-5


def test_batch_rejects_repeated_plan_and_unbound_use():
    from paper_1605_01238_amd import Batch, Plan, WQError
    from workloads import open_uniform_knots
    kn = [open_uniform_knots(3, 5)] * 3
    a = Plan(kn, 3)
    with pytest.raises(WQError):
        Batch([a, a])
    b = Batch([a])
    with pytest.raises(WQError):
        b.assemble(3)   # not bound
