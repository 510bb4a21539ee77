"""GPU parity of NURBS set-ups (wq_setup_nurbs) against the oracle: rational
maps with B-spline test/trial functions (both matrices) and rational
test/trial functions (mass, values scaled by w_i w_j), on the exact quarter
annulus, a thick quarter cylinder and random weights in 1D, 2D and 3D;
every row, FP64 within 1e-12 row-normwise; FP32 bulk within 1e-5
matrix-normwise; the stiffness of rational functions is refused."""
import numpy as np
import pytest

from parity_helpers import compare_rows, gather_rows
from test_oracle_nurbs import quarter_annulus
from workloads import coefficient_field, control_net, greville, open_uniform_knots, random_open_knots

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def nurbs_pipeline(knots, p, ctrl, weights, coef, which, basis, precision=0):
    import torch
    from paper_1605_01238_amd import Plan
    plan = Plan(knots, p, precision)
    plan.bind()
    c = torch.from_numpy(np.ascontiguousarray(ctrl)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(weights, dtype=np.float64)).cuda()
    plan.setup_nurbs(c, w, None, basis)
    if coef is not None:
        x = plan.qp_physical().cpu().numpy().reshape(-1, plan.d)
        plan.setup_nurbs(c, w, torch.from_numpy(np.ascontiguousarray(coef(x))).cuda(), basis)
    row_ptr, col_idx = plan.pattern()
    mass, stiff = plan.assemble(which)
    plan.sync()
    return plan, row_ptr, col_idx, mass, stiff


def thick_cylinder(n_rad, n_ang, n_z):
    kn2, ctrl2, w2 = quarter_annulus(n_rad, n_ang)
    k3 = open_uniform_knots(2, n_z)
    z = 0.5 * greville(k3, 2)
    n3 = len(z)
    ctrl = np.concatenate([np.broadcast_to(ctrl2[None], (n3,) + ctrl2.shape),
                           np.broadcast_to(z[:, None, None, None], (n3,) + ctrl2.shape[:2] + (1,))], axis=-1)
    return kn2 + [k3], np.ascontiguousarray(ctrl), np.broadcast_to(w2[None], (n3,) + w2.shape).copy()


def random_nurbs(p, nel, seed):
    kn = [random_open_knots(p, e, seed=seed + k) for k, e in enumerate(nel)]
    ctrl = control_net(kn, p, seed=seed, amp_h=0.1 if len(nel) > 1 else 0.3 / p)
    rng = np.random.default_rng(seed)
    return kn, ctrl, rng.uniform(0.5, 1.5, ctrl.shape[:-1])


CASES = {
    "annulus": lambda: (2,) + tuple(quarter_annulus(4, 5)),
    "cylinder": lambda: (2,) + tuple(thick_cylinder(4, 5, 4)),
    "random1d_p3": lambda: (3,) + tuple(random_nurbs(3, (11,), 70)),
    "random2d_p6": lambda: (6,) + tuple(random_nurbs(6, (8, 9), 71)),
    "random3d_p4": lambda: (4,) + tuple(random_nurbs(4, (6, 7, 6), 72)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("basis", [0, 1])
def test_nurbs_all_rows(name, basis):
    from oracle.assembly import Problem
    p, kn, ctrl, w = CASES[name]()
    cf = coefficient_field(73) if name in ("cylinder", "random2d_p6") else None
    which = 3 if basis == 0 else 1
    print(f"[nurbs {name} basis={basis}] running", flush=True)
    plan, row_ptr, col_idx, mass, stiff = nurbs_pipeline(kn, p, ctrl, w, cf, which, basis)
    P = Problem(kn, p, ctrl, coef=cf, weights=w, basis="nurbs" if basis else "bspline")
    rp_ref, ci_ref = P.csr_pattern()
    assert np.array_equal(row_ptr.cpu().numpy(), rp_ref)
    assert np.array_equal(col_idx.cpu().numpy(), ci_ref)
    rows = np.arange(plan.n_rows)
    for nm, vals in (("mass", mass), ("stiff", stiff)):
        if vals is None:
            continue
        rp, v = gather_rows(row_ptr, vals, rows)
        row_err, _, worst = compare_rows(P, rows, rp, v, nm)
        print(f"  {nm}: row-normwise {row_err:.2e} (row {worst})", flush=True)
        assert row_err <= FP64_TOL


def test_nurbs_fp32_bulk_and_physical_points():
    import torch
    from oracle.assembly import Problem
    from oracle.geometry import rational_map_and_jacobian
    p, kn, ctrl, w = CASES["random3d_p4"]()
    plan, row_ptr, _, mass, stiff = nurbs_pipeline(kn, p, ctrl, w, None, 3, 0, precision=1)
    P = Problem(kn, p, ctrl, weights=w)
    rows = np.arange(plan.n_rows)
    for nm, vals in (("mass", mass), ("stiff", stiff)):
        rp, v = gather_rows(row_ptr, vals, rows)
        _, mat_err, _ = compare_rows(P, rows, rp, v, nm)
        print(f"[nurbs fp32] {nm}: matrix-normwise {mat_err:.2e}", flush=True)
        assert mat_err <= 1e-5
    x = plan.qp_physical().cpu().numpy()          # [q3][q2][q1][3]
    X = [P.rules[k].x for k in range(3)]
    F = rational_map_and_jacobian(kn, p, ctrl, w, [np.asarray(t, dtype=np.float64) for t in X])[0]
    F = np.transpose(F.astype(np.float64), (2, 1, 0, 3))
    assert np.abs(x - F).max() < 1e-13


def test_nurbs_basis_refuses_stiffness_and_batches():
    import torch
    from paper_1605_01238_amd import Batch, WQError
    p, kn, ctrl, w = CASES["annulus"]()
    plan, _, _, mass, _ = nurbs_pipeline(kn, p, ctrl, w, None, 1, 1)
    with pytest.raises(WQError):
        plan.assemble(2)
    b = Batch([plan])
    b.bind([torch.empty_like(mass)], [torch.empty_like(mass)])
    with pytest.raises(WQError):
        b.assemble(1)


def test_nurbs_through_static_request_and_batch():
    """The other entry points on NURBS set-ups give wq_assemble's values bit
    for bit: wq_assemble_static and wq_assemble_request with rational
    test/trial functions (mass), and a batch of rational-map plans with
    B-spline functions (both matrices)."""
    import torch
    from paper_1605_01238_amd import Batch, _wq
    p, kn, ctrl, w = CASES["cylinder"]()
    plan, _, _, mass, _ = nurbs_pipeline(kn, p, ctrl, w, None, 1, 1)
    m2 = torch.full_like(mass, float("nan"))
    st = _wq.wq_assemble_static(plan._h, 1, m2.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    _wq.check(st, plan._h)
    plan.sync()
    assert torch.equal(m2, mass)
    ctx = torch.empty(plan.request_bytes() + 256, dtype=torch.uint8, device="cuda")
    m3, _ = plan.assemble_request(ctx, None, 1)
    plan.sync()
    assert torch.equal(m3, mass)
    plans, refs = [], []
    for name in ("annulus", "random3d_p4", "cylinder"):
        p, kn, ctrl, w = CASES[name]()
        pl, _, _, m, s = nurbs_pipeline(kn, p, ctrl, w, None, 3, 0)
        plans.append(pl)
        refs.append((m, s))
    outs = [(torch.full_like(m, float("nan")), torch.full_like(s, float("nan"))) for m, s in refs]
    b = Batch(plans)
    b.bind([o[0] for o in outs], [o[1] for o in outs])
    b.assemble(3)
    torch.cuda.synchronize()
    for (m, s), (m2, s2) in zip(refs, outs):
        assert torch.equal(m, m2) and torch.equal(s, s2)
