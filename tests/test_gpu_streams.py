"""Ordering of the device work: the univariate stage of wq_setup runs on a
stream of the plan and is joined by the calls that read its tables.  These
tests re-run setups back to back and assemble on other streams, and require
bit-identical values to a fresh plan on the default stream."""
import numpy as np
import pytest

from parity_helpers import gpu_pipeline
from workloads import control_net, random_open_knots

pytestmark = pytest.mark.gpu

P = 3
NEL = (6, 7, 8)


def _case(seed):
    kn = [random_open_knots(P, e, seed=seed + k) for k, e in enumerate(NEL)]
    return kn, control_net(kn, P, seed=seed, twist_deg=20.0)


def test_setup_twice_then_again():
    """setup(A) assemble, setup(B) assemble, setup(A) assemble on one plan:
    every result equals a fresh plan's, so a setup never overwrites tables
    that an earlier assembly still reads, nor is read before it is done."""
    import torch
    from paper_1605_01238_amd import Plan
    kn, ctrl_a = _case(31)
    ctrl_b = control_net(kn, P, seed=32, twist_deg=-15.0)
    ref_a = gpu_pipeline(kn, P, ctrl_a, None, which=3)
    ref_b = gpu_pipeline(kn, P, ctrl_b, None, which=3)
    plan = Plan(kn, P)
    plan.bind()
    out = []
    for c in (ctrl_a, ctrl_b, ctrl_a):
        plan.setup(torch.from_numpy(c).cuda())
        m, s = plan.assemble(3)
        out.append((m, s))          # no sync in between: ordering only
    plan.sync()
    for (m, s), ref in zip(out, (ref_a, ref_b, ref_a)):
        assert torch.equal(m, ref[3]) and torch.equal(s, ref[4])
    assert not torch.equal(out[0][1], out[1][1])


def test_assemble_on_another_stream():
    """setup on stream s1, assemble on s2 (s2 waits for s1's geometry as any
    caller must): the plan's own join covers the univariate stage."""
    import torch
    from paper_1605_01238_amd import Plan
    kn, ctrl = _case(41)
    ref = gpu_pipeline(kn, P, ctrl, None, which=3)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    plan = Plan(kn, P)
    with torch.cuda.stream(s1):
        plan.bind(s1)
        c = torch.from_numpy(ctrl).cuda()
        plan.setup(c, None, s1)
    s2.wait_stream(s1)
    with torch.cuda.stream(s2):
        m, s = plan.assemble(3, stream=s2)
        plan.sync(s2)
    torch.cuda.synchronize()
    assert torch.equal(m, ref[3]) and torch.equal(s, ref[4])


def test_weights_read_joins_setup():
    """wq_weights right after wq_setup (no sync) returns the new weights."""
    import torch
    from paper_1605_01238_amd import Plan
    from oracle.rules import rules_for
    kn, ctrl = _case(51)
    plan = Plan(kn, P)
    plan.bind()
    plan.setup(torch.from_numpy(ctrl).cuda())
    w, qs, qc = plan.weights(1, 2)     # pairing (alpha, beta) = (0, 1)
    w, qc = w.cpu().numpy(), qc.cpu().numpy()
    R = rules_for(list(kn[1]), P)
    for i in range(R.n):
        ref = R.w64[(0, 1)][i]
        assert np.abs(w[i, :qc[i]] - ref).max() <= 1e-15 * np.abs(ref).max()


def test_set_geometry_keeps_rules_and_matches_setup():
    """wq_set_geometry (new net, same knots, rules kept) gives the values of
    a fresh wq_setup with that net, bit for bit, also after a NURBS set-up
    (it returns the plan to a polynomial map)."""
    import torch
    from paper_1605_01238_amd import Plan
    from workloads import coefficient_field, control_net, random_open_knots
    p, nel = 4, (6, 7, 6)
    kn = [random_open_knots(p, e, seed=90 + k) for k, e in enumerate(nel)]
    nets = [torch.from_numpy(control_net(kn, p, seed=s, amp_h=0.1)).cuda() for s in (91, 92)]
    ref = Plan(kn, p)
    ref.bind()
    ref.setup(nets[1])
    m_ref, s_ref = ref.assemble(3)
    ref.sync()
    plan = Plan(kn, p)
    plan.bind()
    plan.setup(nets[0])
    m0, s0 = plan.assemble(3)
    plan.set_geometry(nets[1])
    m1, s1 = plan.assemble(3)
    w = torch.full((plan.n_rows,), 1.3, dtype=torch.float64, device="cuda")
    plan.setup_nurbs(nets[0], w, None, 1)
    plan.set_geometry(nets[1])
    m2, s2 = plan.assemble(3)
    plan.sync()
    assert torch.equal(m1, m_ref) and torch.equal(s1, s_ref)
    assert torch.equal(m2, m_ref) and torch.equal(s2, s_ref)
    assert not torch.equal(s0, s_ref)
