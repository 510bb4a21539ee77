"""Requests on resident geometries (wq_assemble_request) and the serving
loop (continuous batching, admission by memory budget).  A request's values
equal the plan's own assembly for that coefficient up to the rounding of
a * K (one product), match the oracle on sampled rows, and are the same bit
for bit whether the request runs alone or in a mix of overlapping requests."""
import numpy as np
import pytest

from parity_helpers import compare_rows, gather_rows
from workloads import batch_patches, coefficient_field, control_net, random_open_knots, sample_rows

pytestmark = pytest.mark.gpu


def _coef(req, xq):
    return coefficient_field(req.coef_seed).torch(xq).contiguous()


def test_request_equals_assembly_with_coefficient():
    import torch
    from oracle.assembly import Problem
    from paper_1605_01238_amd import Plan
    p, nel = 4, (9, 11, 8)
    kn = [random_open_knots(p, e, seed=40 + k) for k, e in enumerate(nel)]
    ctrl = control_net(kn, p, seed=41, twist_deg=20.0)
    cf = coefficient_field(42)
    a = Plan(kn, p)
    a.bind()
    a.setup(torch.from_numpy(ctrl).cuda())             # a = 1: the resident geometry
    x = a.qp_physical().reshape(-1, 3)
    coef = cf.torch(x).contiguous()
    ctx = torch.empty(a.request_bytes() + 256, dtype=torch.uint8, device="cuda")
    m1, s1 = a.assemble_request(ctx, coef, 3)
    b = Plan(kn, p)
    b.bind()
    b.setup(torch.from_numpy(ctrl).cuda(), coef)      # the coefficient inside the setup
    m2, s2 = b.assemble(3)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2)                        # det J only: identical
    rel = float((s1 - s2).abs().max() / s2.abs().max())
    print(f"[request] stiffness vs setup with the coefficient: {rel:.2e}", flush=True)
    assert rel <= 1e-14
    P = Problem(kn, p, ctrl, coef=cf)
    row_ptr, _ = a.pattern()
    rows = sample_rows(a.n, p, 20, 20, seed=3)
    rp, v = gather_rows(row_ptr, s1, rows)
    err, _, _ = compare_rows(P, rows, rp, v, "stiff")
    assert err <= 1e-12


def test_request_needs_unit_field():
    import torch
    from paper_1605_01238_amd import Plan, WQError
    from workloads import open_uniform_knots
    kn = [open_uniform_knots(3, 6)] * 3
    a = Plan(kn, 3)
    a.bind()
    ctrl = torch.from_numpy(control_net(kn, 3, seed=5)).cuda()
    coef = torch.ones(a.n_qp_total, dtype=torch.float64, device="cuda")
    a.setup(ctrl, coef)
    ctx = torch.empty(a.request_bytes() + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(WQError):
        a.assemble_request(ctx, coef, 2)
    a.set_coefficient(None)
    a.assemble_request(ctx, coef, 2)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(WQError):
        a.assemble_request(small, coef, 2)
    a.sync()


def _geoms(n, seed, precision, which):
    from paper_1605_01238_amd.serving import Geometry
    ws = batch_patches(n, seed=seed, nel_range=(6, 14), d_choices=(2, 3), p2d=0.3)
    return ws, [Geometry(w.knots(), w.p, w.ctrl(), precision, which) for w in ws]


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_in_the_mix(precision):
    """60 requests on 6 geometries arriving faster than they are served (so
    that many are in flight together on 4 streams); each result equals the
    same request served alone, bit for bit."""
    import torch
    from paper_1605_01238_amd.serving import Server, poisson_requests
    ws, geoms = _geoms(6, 21, precision, 3)
    srv = Server(geoms, _coef, n_streams=4, max_inflight=12, hbm_budget=8 << 30)
    reqs = poisson_requests(60, rate=20000.0, n_geoms=len(geoms), seed=5)
    res = srv.run(reqs, keep={r.rid for r in reqs})
    torch.cuda.synchronize()
    print(f"[serving prec={precision}] {len(res['records'])} requests, peak in flight "
          f"{srv.peak_inflight}, peak bytes {srv.peak_bytes / 2**20:.1f} MiB", flush=True)
    assert len(res["records"]) == 60 and srv.peak_inflight > 1
    for r in reqs:
        m_mix, s_mix = res["outputs"][r.rid]
        m_one, s_one = srv.serve_alone(r)
        assert torch.equal(m_mix, m_one) and torch.equal(s_mix, s_one), r


def test_admission_respects_budget():
    """A budget of about two requests: never more in flight than fits, and
    every request completes."""
    import torch
    from paper_1605_01238_amd import WQ_STIFF
    from paper_1605_01238_amd.serving import Server, poisson_requests
    ws, geoms = _geoms(4, 23, 1, WQ_STIFF)
    budget = 2 * max(g.bytes_per_request for g in geoms)
    srv = Server(geoms, _coef, n_streams=4, max_inflight=16, hbm_budget=budget)
    reqs = poisson_requests(40, rate=0.0, n_geoms=len(geoms), seed=9)   # all at once
    res = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(res["records"]) == 40
    assert srv.peak_bytes <= budget
    print(f"[serving budget] peak {srv.peak_bytes} of {budget} bytes, peak in flight {srv.peak_inflight}", flush=True)


def test_served_requests_match_oracle():
    """Sampled rows of served FP32 requests against the FP64 oracle with the
    request's own coefficient (matrix-normwise 1e-5)."""
    import torch
    from oracle.assembly import Problem
    from paper_1605_01238_amd.serving import Server, poisson_requests
    ws, geoms = _geoms(3, 27, 1, 3)
    srv = Server(geoms, _coef, n_streams=2, max_inflight=8)
    reqs = poisson_requests(6, rate=5000.0, n_geoms=len(geoms), seed=11)
    res = srv.run(reqs, keep={r.rid for r in reqs})
    torch.cuda.synchronize()
    for r in reqs:
        w, g = ws[r.geom], geoms[r.geom]
        P = Problem(w.knots(), w.p, w.ctrl(), coef=coefficient_field(r.coef_seed))
        n3 = g.plan.n if g.plan.d == 3 else (g.plan.n[0], g.plan.n[1], 1)
        rows = sample_rows(n3, w.p, 6, 6, seed=r.rid)
        m, s = res["outputs"][r.rid]
        for name, vals in (("mass", m), ("stiff", s)):
            rp, v = gather_rows(g.row_ptr, vals, rows)
            _, mat_err, _ = compare_rows(P, rows, rp, v, name)
            print(f"[serving oracle] request {r.rid} p={w.p} n_el={w.n_el} {name}: {mat_err:.2e}", flush=True)
            assert mat_err <= 1e-5
