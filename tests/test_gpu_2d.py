"""GPU parity of the 2D path (plane patches) against the oracle: the pattern
bit-exact, FP64 values within 1e-12 row-normwise on every row (small cases)
or on sampled rows, FP32 bulk within the rounding model of the 3D tests."""
import numpy as np
import pytest

from parity_helpers import compare_rows, gather_rows, gpu_pipeline, oracle_rows_parallel
from workloads import coefficient_field, control_net, open_uniform_knots, random_open_knots

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _case(p, nel, seed, uniform):
    kn = [open_uniform_knots(p, e) if uniform else random_open_knots(p, e, seed=seed + k)
          for k, e in enumerate(nel)]
    return kn, control_net(kn, p, seed=seed, amp_h=0.15)


@pytest.mark.parametrize("p,nel,uniform,coef", [
    (2, (6, 9), True, None), (3, (7, 5), False, 3), (4, (9, 8), False, None),
    (5, (8, 11), True, 5), (6, (9, 10), False, 6)])
def test_2d_all_rows(p, nel, uniform, coef):
    import torch
    from oracle.assembly import Problem
    kn, ctrl = _case(p, nel, 20 + p, uniform)
    cf = None if coef is None else coefficient_field(coef)
    P = Problem(kn, p, ctrl, coef=cf)
    print(f"[2d p={p} nel={nel} coef={coef}] running", flush=True)
    plan, row_ptr, col_idx, mass, stiff = gpu_pipeline(kn, p, ctrl, cf, which=3)
    rp_ref, ci_ref = P.csr_pattern()
    assert np.array_equal(row_ptr.cpu().numpy(), rp_ref)
    assert np.array_equal(col_idx.cpu().numpy(), ci_ref)
    rows = np.arange(plan.n_rows)
    for which, vals in (("mass", mass), ("stiff", stiff)):
        rp, v = gather_rows(row_ptr, vals, rows)
        row_err, mat_err, worst = compare_rows(P, rows, rp, v, which)
        print(f"  {which}: row-normwise {row_err:.2e} (row {worst})", flush=True)
        assert row_err <= FP64_TOL
    lengths = row_ptr[1:] - row_ptr[:-1]
    s1 = (torch.segment_reduce(stiff, "sum", lengths=lengths).abs()
          / torch.segment_reduce(stiff.abs(), "sum", lengths=lengths)).max().item()
    assert s1 <= 1e-13


@pytest.mark.parametrize("p", [2, 4, 6])
def test_2d_fp32_bulk(p):
    from oracle.assembly import Problem
    kn, ctrl = _case(p, (8, 9), 40 + p, False)
    P = Problem(kn, p, ctrl)
    plan, row_ptr, _, mass, stiff = gpu_pipeline(kn, p, ctrl, None, which=3, precision=1)
    rows = np.arange(plan.n_rows)
    tol = 16 * 2.0 ** -24 * np.sqrt((2 * p + 1) ** 2)
    for which, vals in (("mass", mass), ("stiff", stiff)):
        rp, v = gather_rows(row_ptr, vals, rows)
        _, mat_err, _ = compare_rows(P, rows, rp, v, which)
        print(f"[2d fp32 p={p}] {which}: matrix-normwise {mat_err:.2e} (bound {tol:.2e})", flush=True)
        assert mat_err <= min(tol, 1e-5)


def test_2d_large_sampled_rows():
    """p = 4 on 128 x 96 elements: about 130 sampled rows (boundary layers of
    both directions, corners and uniform rows)."""
    from oracle.assembly import Problem
    p, nel = 4, (128, 96)
    kn = [open_uniform_knots(p, e) for e in nel]
    ctrl = control_net(kn, p, seed=77)
    cf = coefficient_field(78)
    P = Problem(kn, p, ctrl, coef=cf)
    plan, row_ptr, col_idx, mass, stiff = gpu_pipeline(kn, p, ctrl, cf, which=3)
    n1, n2 = P.n
    rng = np.random.default_rng(5)
    picks = [(0, 0), (1, 0), (n1 - 1, n2 - 1), (p, 3), (n1 - 2, 1), (2, n2 - 3)]
    # the boundary layers of both directions, then uniform rows
    lay1 = [0, 1, p - 1, p, n1 - p - 1, n1 - 2, n1 - 1]
    lay2 = [0, 1, p - 1, p, n2 - p - 1, n2 - 2, n2 - 1]
    picks += [(int(rng.choice(lay1)), int(b)) for b in rng.integers(0, n2, 32)]
    picks += [(int(a), int(rng.choice(lay2))) for a in rng.integers(0, n1, 32)]
    picks += [(int(a), int(b)) for a, b in zip(rng.integers(0, n1, 64), rng.integers(0, n2, 64))]
    rows = np.array(sorted({i1 + n1 * i2 for i1, i2 in picks}))
    ref = oracle_rows_parallel(kn, p, ctrl, cf, rows, ("mass", "stiff"))
    rp, _ = gather_rows(row_ptr, stiff, rows)
    for r in rows[:6]:
        assert np.array_equal(col_idx[int(rp[r]):int(rp[r + 1])].cpu().numpy(), P.row_columns(int(r)))

    class _Cached:
        def row(self, r, which):
            return ref[(which, r)]
    for which, vals in (("mass", mass), ("stiff", stiff)):
        rp, v = gather_rows(row_ptr, vals, rows)
        row_err, _, worst = compare_rows(_Cached(), rows, rp, v, which)
        print(f"[2d 128x96 p=4] {which}: row-normwise {row_err:.2e} (row {worst})", flush=True)
        assert row_err <= FP64_TOL


@pytest.mark.parametrize("name", ["p4_512el_plane", "p6_256el_plane"])
def test_2d_bench_workloads_sampled_rows(name):
    """The plane workloads of the benchmark, at their full size and with the
    launch the benchmark times: sampled rows (corners, both boundary layers,
    uniform rows; strips and runs of rows split at many places) against the
    oracle, every matrix the workload forms, FP64 within 1e-12."""
    import time
    from oracle.assembly import Problem
    from workloads import WORKLOADS, sample_rows
    w = WORKLOADS[name]
    kn, p, ctrl, cf = w.knots(), w.p, w.ctrl(), w.coefficient()
    which = (1 if "mass" in w.which else 0) | (2 if "stiff" in w.which else 0)
    plan, row_ptr, col_idx, mass, stiff = gpu_pipeline(kn, p, ctrl, cf, which=which)
    print(f"[2d {name}] GPU done; oracle rules ...", flush=True)
    t0 = time.time()
    P = Problem(kn, p, ctrl, coef=cf)
    n1, n2 = P.n
    rows = sample_rows((n1, n2, 1), p, 40, 24, seed=9)
    print(f"[2d {name}] oracle set up in {time.time() - t0:.0f} s; {len(rows)} rows", flush=True)
    for wname, vals in (("mass", mass), ("stiff", stiff)):
        if wname not in w.which:
            continue
        rp, v = gather_rows(row_ptr, vals, rows)
        row_err, _, worst = compare_rows(P, rows, rp, v, wname)
        print(f"[2d {name}] {wname}: row-normwise {row_err:.2e} (row {worst})", flush=True)
        assert row_err <= FP64_TOL


def test_2d_setup_twice_then_again():
    """setup(A) assemble, setup(B) assemble, setup(A) assemble on one plane
    plan, no synchronization in between: each result equals a fresh plan's."""
    import torch
    from paper_1605_01238_amd import Plan
    p, nel = 3, (7, 9)
    kn = [random_open_knots(p, e, seed=60 + k) for k, e in enumerate(nel)]
    nets = [control_net(kn, p, seed=s, amp_h=0.15) for s in (61, 62)]
    refs = [gpu_pipeline(kn, p, c, None, which=3) for c in nets]
    plan = Plan(kn, p)
    plan.bind()
    out = []
    for c in (nets[0], nets[1], nets[0]):
        plan.setup(torch.from_numpy(c).cuda())
        out.append(plan.assemble(3))
    plan.sync()
    for (m, s), ref in zip(out, (refs[0], refs[1], refs[0])):
        assert torch.equal(m, ref[3]) and torch.equal(s, ref[4])
    assert not torch.equal(out[0][1], out[1][1])
