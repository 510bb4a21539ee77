"""GPU parity at the full benchmark sizes, on sampled rows the oracle can
compute one by one, plus properties checked on every row.

Workloads: p = 4 on 32^3 elements with a non-constant coefficient (stiffness,
FP64 and FP32 bulk) and p = 6 on 64^3 elements with a twisted perturbed map
(stiffness and mass, FP64 and FP32 bulk).
"""
import numpy as np
import pytest

from parity_helpers import compare_rows, gather_rows, gpu_pipeline, oracle_rows_parallel
from workloads import LARGE_P6, MID_P4, sample_rows

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5
U32 = 2.0 ** -24


def s1_tol(precision, p):
    """Bound on max_i |sum_j s_ij| / sum_j |s_ij| (exactly 0 in exact
    arithmetic).  FP64: 1e-13.  FP32: the row sum adds up (2p+1)^3 entries
    whose rounding errors are independent, each below ~16 units of FP32
    roundoff relative to the row's absolute sum: a random walk gives
    16 u32 sqrt((2p+1)^3)."""
    return 1e-13 if precision == 0 else 16 * U32 * ((2 * p + 1) ** 3) ** 0.5


def check_structure(plan, row_ptr, col_idx, rows, problem):
    import torch
    rp = row_ptr.cpu().numpy()
    assert rp[0] == 0 and rp[-1] == plan.nnz
    assert np.all(np.diff(rp) > 0)
    # columns strictly increasing inside every row
    d = col_idx[1:] - col_idx[:-1]
    starts = torch.zeros(plan.nnz, dtype=torch.bool, device=col_idx.device)
    starts[row_ptr[:-1]] = True
    assert bool(((d > 0) | starts[1:]).all())
    for r in rows[:64]:
        got = col_idx[int(rp[r]):int(rp[r + 1])].cpu().numpy()
        assert np.array_equal(got, problem.row_columns(int(r)))


def stiffness_kills_constants(row_ptr, vals):
    """max over rows of |sum_j s_ij| / sum_j |s_ij| (S 1 = 0, all rows)."""
    import torch
    lengths = (row_ptr[1:] - row_ptr[:-1])
    v = vals.double()
    s = torch.segment_reduce(v, "sum", lengths=lengths)
    a = torch.segment_reduce(v.abs(), "sum", lengths=lengths)
    return float((s.abs() / a).max())


def run_case(w, which_names, rows, precision):
    from oracle.assembly import Problem
    which = (1 if "mass" in which_names else 0) | (2 if "stiff" in which_names else 0)
    return gpu_pipeline(w.knots(), w.p, w.ctrl(), w.coefficient(), which=which, precision=precision)


@pytest.fixture(scope="module")
def mid_oracle():
    from oracle.assembly import Problem
    w = MID_P4
    P = Problem(w.knots(), w.p, w.ctrl(), coef=w.coefficient())
    rows = sample_rows(w.n_dof(), w.p, 512, 512, seed=21)
    got = oracle_rows_parallel(w.knots(), w.p, w.ctrl(), w.coefficient(), rows, ("stiff",))
    ref = {r: got[("stiff", r)] for r in (int(x) for x in rows)}
    return w, P, rows, ref


class _Cached:
    def __init__(self, P, ref):
        self.P, self.ref = P, ref

    def row(self, r, which):
        return self.ref[r]

    def row_columns(self, r):
        return self.P.row_columns(r)


@pytest.mark.parametrize("precision", [0, 1])
def test_mid_p4_stiffness(mid_oracle, precision):
    import torch
    w, P, rows, ref = mid_oracle
    plan, row_ptr, col_idx, _, stiff = run_case(w, ("stiff",), rows, precision)
    assert plan.nnz == w.exact_nnz() == 28094464
    check_structure(plan, row_ptr, col_idx, rows, P)
    rp, vals = gather_rows(row_ptr, stiff, rows)
    row_err, mat_err, worst = compare_rows(_Cached(P, ref), rows, rp, vals, "stiff")
    s1 = stiffness_kills_constants(row_ptr, stiff)
    print(f"[p4 32^3 stiff prec={precision}] rows={len(rows)} row-normwise {row_err:.3e} "
          f"(row {worst}) matrix-normwise {mat_err:.3e}  max|S1|/sum|S| {s1:.2e}")
    assert not bool(torch.isnan(stiff).any())
    if precision == 0:
        assert row_err <= FP64_TOL
    else:
        assert mat_err <= FP32_TOL
    assert s1 <= s1_tol(precision, w.p)
    del stiff, col_idx, row_ptr, plan
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def large_oracle():
    from oracle.assembly import Problem
    w = LARGE_P6
    P = Problem(w.knots(), w.p, w.ctrl(), coef=None)
    rows = sample_rows(w.n_dof(), w.p, 512, 512, seed=22)
    ref = oracle_rows_parallel(w.knots(), w.p, w.ctrl(), None, rows, ("stiff", "mass"))
    return w, P, rows, ref


class _Cached2:
    def __init__(self, P, ref):
        self.P, self.ref = P, ref

    def row(self, r, which):
        return self.ref[(which, r)]


@pytest.mark.parametrize("precision", [0, 1])
def test_large_p6_mass_and_stiffness(large_oracle, precision):
    import torch
    w, P, rows, ref = large_oracle
    plan, row_ptr, col_idx, mass, stiff = run_case(w, ("mass", "stiff"), rows, precision)
    assert plan.nnz == w.exact_nnz() == 653972032
    check_structure(plan, row_ptr, col_idx, rows, P)
    for name, vals_dev in (("stiff", stiff), ("mass", mass)):
        rp, vals = gather_rows(row_ptr, vals_dev, rows)
        row_err, mat_err, worst = compare_rows(_Cached2(P, ref), rows, rp, vals, name)
        print(f"[p6 64^3 {name} prec={precision}] rows={len(rows)} row-normwise {row_err:.3e} "
              f"(row {worst}) matrix-normwise {mat_err:.3e}")
        if precision == 0:
            assert row_err <= FP64_TOL
        else:
            assert mat_err <= FP32_TOL
    s1 = stiffness_kills_constants(row_ptr, stiff)
    print(f"[p6 64^3 prec={precision}] max|S1|/sum|S| {s1:.2e}")
    assert s1 <= s1_tol(precision, w.p)
    # total mass ~ volume of the mapped domain (not exact for a non-affine map)
    tot = float(mass.double().sum())
    print(f"[p6 64^3 prec={precision}] total mass {tot:.12f}")
    assert abs(tot - 1.0) < 0.05
    del mass, stiff, col_idx, row_ptr, plan
    torch.cuda.empty_cache()
