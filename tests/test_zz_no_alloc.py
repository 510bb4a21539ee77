"""The allocation-free assembly (wq_assemble_static), called through the
C-ABI, against wq_assemble on the same plan: the values must be identical
bit for bit (same kernels, same arithmetic; only the home of the
first-contraction buffer differs).  Two calls in a row, the second with a
smaller patch; the first patch needs several slabs of the static scratch."""
import ctypes as C

import numpy as np
import pytest

from parity_helpers import gpu_pipeline
from workloads import coefficient_field, control_net, open_uniform_knots, random_open_knots

pytestmark = pytest.mark.gpu


def _static(plan, which, mass, stiff):
    import torch
    from paper_1605_01238_amd import _wq
    st = _wq.wq_assemble_static(plan._h, which, mass.data_ptr() if mass is not None else None,
                                stiff.data_ptr() if stiff is not None else None,
                                torch.cuda.current_stream().cuda_stream)
    _wq.check(st, plan._h)
    plan.sync()


def _case(p, nel, seed, precision, coef_seed=None, uniform=False):
    import torch
    if uniform:
        kn = [open_uniform_knots(p, e) for e in nel]
    else:
        kn = [random_open_knots(p, e, seed=seed + k) for k, e in enumerate(nel)]
    ctrl = control_net(kn, p, seed=seed, twist_deg=15.0 if len(nel) == 3 else 0.0)
    cf = coefficient_field(coef_seed) if coef_seed is not None else None
    plan, _, _, mass, stiff = gpu_pipeline(kn, p, ctrl, cf, which=3, precision=precision)
    nan = float("nan")
    m2 = torch.full_like(mass, nan)
    s2 = torch.full_like(stiff, nan)
    return plan, mass, stiff, m2, s2


@pytest.mark.parametrize("precision", [0, 1])
def test_static_scratch_matches_workspace_assembly(precision):
    import torch
    from paper_1605_01238_amd import WQ_STATIC_SCRATCH_BYTES
    # first call: p = 4 on 64 x 60 x 40 spans; one stiffness plane of the
    # first-contraction buffer is 135 * 127 * 9 * 8 values, so the 64 MiB
    # scratch holds 6 (FP64) or 13 (FP32) of the 44 planes
    p, nel = 4, (64, 60, 40)
    plan, mass, stiff, m2, s2 = _case(p, nel, 5, precision, coef_seed=6, uniform=True)
    ebytes = 8 if precision == 0 else 4
    plane = plan.n_qp[0] * plan.n_qp[1] * (2 * p + 1) * 8 * ebytes
    assert WQ_STATIC_SCRATCH_BYTES // plane < plan.n[2], "the first case must need several slabs"
    print(f"[no-alloc] p={p} n_el={nel} prec={precision}: {plan.n[2]} planes, "
          f"{WQ_STATIC_SCRATCH_BYTES // plane} per slab", flush=True)
    _static(plan, 3, m2, s2)
    assert torch.equal(m2, mass) and torch.equal(s2, stiff)
    # second call, smaller: p = 3 on a ragged non-uniform patch, stiffness then mass
    plan_b, mass_b, stiff_b, m2b, s2b = _case(3, (9, 7, 11), 8, precision)
    print(f"[no-alloc] p=3 n_el=(9, 7, 11) prec={precision}", flush=True)
    _static(plan_b, 2, None, s2b)
    _static(plan_b, 1, m2b, None)
    assert torch.equal(s2b, stiff_b) and torch.equal(m2b, mass_b)


def test_static_scratch_plane_patch():
    """A plane patch has no first contraction: the static call uses no
    scratch and gives wq_assemble's values."""
    import torch
    plan, mass, stiff, m2, s2 = _case(5, (40, 33), 12, 0, coef_seed=13)
    print("[no-alloc] plane p=5 n_el=(40, 33)", flush=True)
    _static(plan, 3, m2, s2)
    assert torch.equal(m2, mass) and torch.equal(s2, stiff)


def test_static_scratch_refuses_oversized_plane():
    """A plan whose single first-contraction plane exceeds the scratch is
    refused before any device work (host check)."""
    from paper_1605_01238_amd import Plan, WQ_STATIC_SCRATCH_BYTES, _wq
    import torch
    p = 6
    # n_qp = 2 n_el + 11; (2 n_el + 11)^2 * 13 * 8 * 8 > 64 MiB for n_el >= 145
    kn = [open_uniform_knots(p, 150), open_uniform_knots(p, 150), open_uniform_knots(p, p + 2)]
    plan = Plan(kn, p)
    plan.bind()
    plan.setup(torch.from_numpy(control_net(kn, p, seed=None)).cuda())
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    st = _wq.wq_assemble_static(plan._h, 2, None, out.data_ptr(), None)
    assert st == _wq.WQ_ENOSPACE
    assert b"static scratch" in _wq.wq_last_error(plan._h)
    plan.sync()
