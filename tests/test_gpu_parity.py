"""GPU parity of the HIP path (through the C-ABI) against the CPU oracle.

Tolerances: FP64 row-normwise max|d|/max|row| <= 1e-12; FP32 bulk
matrix-normwise max|d|/max|A| <= 1e-5; pattern bit-exact.
"""
import numpy as np
import pytest

from parity_helpers import compare_rows, gather_rows, gpu_pipeline
from workloads import (SMALL_P2, coefficient_field, control_net, open_uniform_knots,
                       random_open_knots)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def small_case():
    from oracle.assembly import Problem
    w = SMALL_P2
    kn, ctrl = w.knots(), w.ctrl()
    P = Problem(kn, w.p, ctrl)
    out = gpu_pipeline(kn, w.p, ctrl, None, which=3)
    return P, out


def test_small_pattern_bit_exact(small_case):
    P, (plan, row_ptr, col_idx, _, _) = small_case
    rp, ci = P.csr_pattern()
    assert plan.nnz == ci.size == SMALL_P2.exact_nnz()
    assert np.array_equal(row_ptr.cpu().numpy(), rp)
    assert np.array_equal(col_idx.cpu().numpy(), ci)


@pytest.mark.parametrize("which", ["mass", "stiff"])
def test_small_values_all_rows(small_case, which):
    P, (plan, row_ptr, _, mass, stiff) = small_case
    vals = (mass if which == "mass" else stiff).cpu().numpy()
    rp = row_ptr.cpu().numpy()
    rows = np.arange(plan.n_rows)
    row_err, mat_err, worst = compare_rows(P, rows, rp, vals, which)
    print(f"[c1 {which}] row-normwise {row_err:.3e} (row {worst}), matrix-normwise {mat_err:.3e}")
    assert row_err <= FP64_TOL


def test_small_weights_match_exact_oracle(small_case):
    from oracle.rules import PAIRINGS
    P, (plan, *_) = small_case
    worst = 0.0
    for d in range(3):
        R = P.rules[d]
        for (al, be) in PAIRINGS:
            w, qs, qc = plan.weights(d, 2 * be + al)
            w, qs, qc = w.cpu().numpy(), qs.cpu().numpy(), qc.cpu().numpy()
            for i in range(R.n):
                assert qs[i] == R.Q[i][0] and qc[i] == len(R.Q[i])
                ref = R.w64[(al, be)][i]
                got = w[i, :qc[i]]
                assert np.all(w[i, qc[i]:] == 0)
                worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    print(f"[c1 weights] max relative error vs exact {worst:.3e}")
    assert worst <= 1e-12


def test_small_field_matches_oracle_geometry(small_case):
    from oracle.geometry import coefficients_from_jacobian, map_and_jacobian
    P, (plan, *_) = small_case
    f = plan.field().cpu().numpy()            # (7, nq3, nq2, nq1)
    X = [P.rules[k].x for k in range(3)]           # exact points
    F, J = map_and_jacobian(P.knots3, P.p, P.ctrl, *X)
    det, K = coefficients_from_jacobian(J)
    F = F.astype(np.float64)
    det = det.astype(np.float64).transpose(2, 1, 0)
    K = K.astype(np.float64).transpose(2, 1, 0, 3, 4)
    chans = [det, K[..., 0, 0], K[..., 1, 1], K[..., 2, 2], K[..., 0, 1], K[..., 0, 2], K[..., 1, 2]]
    for c, ref in enumerate(chans):
        err = np.abs(f[c] - ref).max() / np.abs(ref).max()
        print(f"[c1 field] channel {c} max relative error {err:.2e}")
        assert err <= 1e-14, c
    xp = plan.qp_physical().cpu().numpy()
    assert np.abs(xp - F.transpose(2, 1, 0, 3)).max() <= 1e-14


@pytest.mark.parametrize("p,nel,seed", [(3, (5, 6, 7), 11), (5, (7, 8, 9), 12)])
def test_nonuniform_ragged_with_coefficient(p, nel, seed):
    """Non-uniform knots, different sizes per direction, twisted perturbed
    map, non-constant coefficient: every row, both matrices, FP64."""
    from oracle.assembly import Problem
    kn = [random_open_knots(p, e, seed=seed + k) for k, e in enumerate(nel)]
    ctrl = control_net(kn, p, seed=seed, twist_deg=25.0)
    coef = coefficient_field(seed)
    P = Problem(kn, p, ctrl, coef=coef)
    plan, row_ptr, col_idx, mass, stiff = gpu_pipeline(kn, p, ctrl, coef, which=3)
    rp, ci = P.csr_pattern()
    assert np.array_equal(row_ptr.cpu().numpy(), rp)
    assert np.array_equal(col_idx.cpu().numpy(), ci)
    rows = np.arange(plan.n_rows)
    for which, vals in (("mass", mass), ("stiff", stiff)):
        row_err, mat_err, worst = compare_rows(P, rows, rp, vals.cpu().numpy(), which)
        print(f"[p{p} nonuniform {which}] row-normwise {row_err:.3e} (row {worst})")
        assert row_err <= FP64_TOL


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_minimum_size_each_degree(p):
    """Smallest allowed patch (p+2 spans per direction): every row is a
    boundary row."""
    from oracle.assembly import Problem
    kn = [open_uniform_knots(p, p + 2)] * 3
    ctrl = control_net(kn, p, seed=p)
    P = Problem(kn, p, ctrl)
    plan, row_ptr, _, mass, stiff = gpu_pipeline(kn, p, ctrl, None, which=3)
    rp = row_ptr.cpu().numpy()
    rows = np.arange(plan.n_rows)
    for which, vals in (("mass", mass), ("stiff", stiff)):
        row_err, _, worst = compare_rows(P, rows, rp, vals.cpu().numpy(), which)
        print(f"[min size p={p} {which}] {len(rows)} rows, row-normwise {row_err:.3e}", flush=True)
        assert row_err <= FP64_TOL, (which, row_err, worst)


def test_fp32_bulk_small(small_case):
    from oracle.assembly import Problem
    P, _ = small_case
    w = SMALL_P2
    plan, row_ptr, _, mass, stiff = gpu_pipeline(w.knots(), w.p, w.ctrl(), None, which=3, precision=1)
    rp = row_ptr.cpu().numpy()
    rows = np.arange(plan.n_rows)
    for which, vals in (("mass", mass), ("stiff", stiff)):
        assert vals.dtype.itemsize == 4
        row_err, mat_err, _ = compare_rows(P, rows, rp, vals.cpu().numpy(), which)
        print(f"[c1 fp32 {which}] matrix-normwise {mat_err:.3e} row-normwise {row_err:.3e}")
        assert mat_err <= FP32_TOL


def test_deterministic_and_every_slot_written(small_case):
    import torch
    P, (plan, row_ptr, col_idx, mass, stiff) = small_case
    m2 = torch.full_like(mass, float("nan"))
    s2 = torch.full_like(stiff, float("nan"))
    plan.assemble(3, m2, s2)
    plan.sync()
    assert not torch.isnan(m2).any() and not torch.isnan(s2).any()
    assert torch.equal(m2, mass) and torch.equal(s2, stiff)


def test_bad_geometry_reports_egeom():
    from paper_1605_01238_amd import WQError, _wq
    p = 2
    kn = [open_uniform_knots(p, 5)] * 3
    ctrl = control_net(kn, p, None).copy()
    ctrl[..., 0] = ctrl[..., 0][:, :, ::-1]          # mirror x: det J < 0 everywhere
    with pytest.raises(WQError) as ei:
        gpu_pipeline(kn, p, ctrl, None, which=2)
    assert ei.value.status == _wq.WQ_EGEOM


@pytest.mark.parametrize("p,nel,uniform", [(6, 64, True), (5, 9, False), (4, 32, True)])
def test_weights_equal_exact_rationals(p, nel, uniform):
    """The device weights (double-double data, refined KKT solve) equal the
    exact rational minimum-norm weights rounded to FP64, to a few ulps."""
    import torch
    from oracle.rules import PAIRINGS, rules_for
    from paper_1605_01238_amd import Plan
    kn = open_uniform_knots(p, nel) if uniform else random_open_knots(p, nel, seed=9)
    R = rules_for(list(kn), p)
    plan = Plan([kn, kn, kn], p)
    plan.bind()
    plan.setup(torch.from_numpy(control_net([kn] * 3, p, None)).cuda())
    plan.sync()
    worst = 0.0
    for (al, be) in PAIRINGS:
        w, qs, qc = plan.weights(0, 2 * be + al)
        w, qc = w.cpu().numpy(), qc.cpu().numpy()
        for i in range(R.n):
            ref = R.w64[(al, be)][i]
            worst = max(worst, np.abs(w[i, :qc[i]] - ref).max() / np.abs(ref).max())
    print(f"[weights p={p} nel={nel} uniform={uniform}] max relative error vs exact {worst:.2e}")
    assert worst <= 1e-15
