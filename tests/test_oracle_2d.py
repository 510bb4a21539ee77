"""Pins for the 2D forms of the oracle (CPU only): the same definitions as in
3D with two directions (Section 3, d = 2; Algorithm 3 with two mode
products)."""
import numpy as np
import pytest

from oracle.assembly import Problem
from oracle.geometry import coefficients_from_jacobian_2d, map_and_jacobian_2d
from workloads import coefficient_field, control_net, open_uniform_knots, random_open_knots

A2 = np.array([[1.3, 0.25], [-0.15, 0.8]])


def to_dense(P, vals):
    rp, ci = P.csr_pattern()
    N = rp.size - 1
    D = np.zeros((N, N))
    for r in range(N):
        D[r, ci[rp[r]:rp[r + 1]]] = vals[rp[r]:rp[r + 1]]
    return D


def test_identity_and_affine_map_2d():
    p = 3
    kn = [open_uniform_knots(p, 4), random_open_knots(p, 5, seed=2)]
    rng = np.random.default_rng(0)
    X = [np.sort(rng.uniform(0.02, 0.98, 6)) for _ in range(2)]
    F, J = (t.astype(np.float64) for t in map_and_jacobian_2d(kn, p, control_net(kn, p, None), *X))
    G = np.stack(np.meshgrid(*X, indexing="ij"), -1)
    assert np.abs(F - G).max() < 1e-14 and np.abs(J - np.eye(2)).max() < 1e-13
    s = np.array([0.2, -0.1])
    F, J = (t.astype(np.float64) for t in map_and_jacobian_2d(kn, p, control_net(kn, p, None, affine=A2, shift=s), *X))
    assert np.abs(F - (G @ A2.T + s)).max() < 1e-13
    assert np.abs(J - A2).max() < 1e-13


def test_jacobian_finite_differences_and_coefficients_2d():
    p = 2
    kn = [open_uniform_knots(p, 5)] * 2
    ctrl = control_net(kn, p, seed=4, amp_h=0.2)
    x = [np.array([0.31, 0.62]), np.array([0.27, 0.71])]
    _, J = map_and_jacobian_2d(kn, p, ctrl, *x)
    J = J.astype(np.float64)
    h = 1e-6
    for b in range(2):
        xp = [v.copy() for v in x]
        xm = [v.copy() for v in x]
        xp[b] = xp[b] + h
        xm[b] = xm[b] - h
        Fp = map_and_jacobian_2d(kn, p, ctrl, *xp)[0].astype(np.float64)
        Fm = map_and_jacobian_2d(kn, p, ctrl, *xm)[0].astype(np.float64)
        assert np.abs((Fp - Fm) / (2 * h) - J[..., :, b]).max() < 1e-7
    a = np.full(J.shape[:2], 1.7)
    det, K = coefficients_from_jacobian_2d(J, a)
    Ji = np.linalg.inv(J)
    ref = 1.7 * np.linalg.det(J)[..., None, None] * Ji @ np.swapaxes(Ji, -1, -2)
    assert np.abs(det - np.linalg.det(J)).max() < 1e-14
    assert np.abs(K - ref).max() < 1e-13


@pytest.mark.parametrize("which", ["mass", "stiff"])
def test_direct_equals_sum_factorized_2d(which):
    p = 3
    kn = [open_uniform_knots(p, 5), random_open_knots(p, 6, seed=7)]
    P = Problem(kn, p, control_net(kn, p, seed=5, amp_h=0.15), coef=coefficient_field(6))
    a = P.assemble(which, "direct")
    b = P.assemble(which, "sumfact")
    rp, _ = P.csr_pattern()
    for r in range(rp.size - 1):
        s = slice(rp[r], rp[r + 1])
        assert np.abs(a[s] - b[s]).max() <= 1e-13 * np.abs(a[s]).max()


def kron_closed_form_2d(P, which, A):
    """Exact Galerkin matrix of x = A zeta + s, a = 1, from the exact 1D
    integral tables (eq. 4.2) as Kronecker products."""
    R = P.rules
    detA = np.linalg.det(A)
    Ai = np.linalg.inv(A)
    K = detA * Ai @ Ai.T

    def table(k, al, be):
        n = R[k].n
        T = np.zeros((n, n))
        for i in range(n):
            for j in R[k].I[i]:
                T[i, j] = float(R[k].integ[(al, be)][i][j])
        return T
    if which == "mass":
        return detA * np.kron(table(1, 0, 0), table(0, 0, 0))
    S = 0
    for l in range(2):
        for m in range(2):
            T = [table(k, int(k == m), int(k == l)) for k in range(2)]
            S = S + K[l, m] * np.kron(T[1], T[0])
    return S


@pytest.mark.parametrize("p,n_el,uniform", [(2, (4, 5), True), (4, (6, 7), False)])
def test_affine_exactness_2d(p, n_el, uniform):
    kn = [open_uniform_knots(p, e) for e in n_el] if uniform else \
        [random_open_knots(p, e, seed=e) for e in n_el]
    P = Problem(kn, p, control_net(kn, p, None, affine=A2, shift=[0.3, -0.4]))
    for which in ("mass", "stiff"):
        wq = to_dense(P, P.assemble(which))
        ref = kron_closed_form_2d(P, which, A2)
        sgq = P.sgq_matrices(which)
        scale = np.abs(ref).max()
        assert np.abs(wq - ref).max() <= 1e-12 * scale
        assert np.abs(sgq - ref).max() <= 1e-12 * scale
    M = to_dense(P, P.assemble("mass"))
    detA = np.linalg.det(A2)
    assert abs(M.sum() - detA) <= 1e-12 * detA            # total mass = area
    for r in range(M.shape[0]):                           # row sums = det A int B_i
        i = P.multi(r)
        expect = detA
        for k in range(2):
            kk = P.knots3[k]
            expect *= (kk[i[k] + p + 1] - kk[i[k]]) / (p + 1)
        assert abs(M[r].sum() - expect) <= 1e-13


def test_stiffness_kills_constants_2d():
    p = 4
    kn = [open_uniform_knots(p, 6), random_open_knots(p, 7, seed=3)]
    P = Problem(kn, p, control_net(kn, p, seed=8, amp_h=0.2), coef=coefficient_field(9))
    rp, _ = P.csr_pattern()
    for r in range(0, rp.size - 1, 3):
        s = P.row(r, "stiff")
        assert abs(s.sum()) <= 1e-12 * np.abs(s).max()


def test_pattern_brute_force_and_nnz_2d():
    p = 3
    kn = [open_uniform_knots(p, 5), random_open_knots(p, 6, seed=1)]
    P = Problem(kn, p, control_net(kn, p, None))
    rp, ci = P.csr_pattern()
    n1, n2 = P.n
    assert ci.size == ((2 * p + 1) * n1 - p * (p + 1)) * ((2 * p + 1) * n2 - p * (p + 1))
    sup = [[(kn[k][i], kn[k][i + p + 1]) for i in range(P.n[k])] for k in range(2)]
    for r in range(rp.size - 1):
        i = P.multi(r)
        cols = [c for c in range(n1 * n2)
                if all(max(sup[k][i[k]][0], sup[k][P.multi(c)[k]][0]) <
                       min(sup[k][i[k]][1], sup[k][P.multi(c)[k]][1]) for k in range(2))]
        assert list(ci[rp[r]:rp[r + 1]]) == cols
