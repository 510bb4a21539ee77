"""Pins for oracle/assembly.py (CPU only)."""
import numpy as np
import pytest

from oracle.assembly import Problem
from workloads import (SMALL_P2, coefficient_field, control_net, open_uniform_knots,
                       random_open_knots)

A_MAP = np.array([[1.2, 0.3, 0.1], [0.2, 0.9, -0.2], [0.05, 0.1, 1.1]])


def to_dense(P, vals):
    rp, ci = P.csr_pattern()
    N = rp.size - 1
    D = np.zeros((N, N))
    for r in range(N):
        D[r, ci[rp[r]:rp[r + 1]]] = vals[rp[r]:rp[r + 1]]
    return D


def kron_closed_form(P, which, A):
    """Exact Galerkin matrix of an affine map x = A zeta + s with a = 1, as
    Kronecker products of the exact 1D integral tables (eq. 4.2)."""
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
        return detA * np.kron(table(2, 0, 0), np.kron(table(1, 0, 0), table(0, 0, 0)))
    S = 0
    for l in range(3):
        for m in range(3):
            T = [table(k, int(k == m), int(k == l)) for k in range(3)]
            S = S + K[l, m] * np.kron(T[2], np.kron(T[1], T[0]))
    return S


@pytest.mark.parametrize("which", ["mass", "stiff"])
def test_direct_equals_sum_factorized(which):
    p = 2
    kn = [open_uniform_knots(p, 3), random_open_knots(p, 4, seed=2), open_uniform_knots(p, 2)]
    P = Problem(kn, p, control_net(kn, p, seed=9, twist_deg=20), coef=coefficient_field(4))
    a = P.assemble(which, "direct")
    b = P.assemble(which, "sumfact")
    rp, _ = P.csr_pattern()
    for r in range(rp.size - 1):
        s = slice(rp[r], rp[r + 1])
        assert np.abs(a[s] - b[s]).max() <= 1e-13 * np.abs(a[s]).max()


@pytest.mark.parametrize("p,n_el,uniform", [(2, (3, 4, 3), True), (3, (2, 3, 4), False)])
def test_affine_exactness(p, n_el, uniform):
    if uniform:
        kn = [open_uniform_knots(p, e) for e in n_el]
    else:
        kn = [random_open_knots(p, e, seed=e) for e in n_el]
    ctrl = control_net(kn, p, None, affine=A_MAP, shift=[0.1, -0.2, 0.3])
    P = Problem(kn, p, ctrl)
    for which in ("mass", "stiff"):
        wq = to_dense(P, P.assemble(which))
        ref = kron_closed_form(P, which, A_MAP)
        sgq = P.sgq_matrices(which)
        scale = np.abs(ref).max()
        assert np.abs(wq - ref).max() <= 1e-12 * scale
        assert np.abs(sgq - ref).max() <= 1e-12 * scale
        assert np.abs(wq - wq.T).max() <= 1e-12 * scale   # exact => symmetric
    M = to_dense(P, P.assemble("mass"))
    detA = np.linalg.det(A_MAP)
    assert abs(M.sum() - detA) <= 1e-12 * detA           # total mass = volume
    n1, n2, n3 = P.n
    for r in range(M.shape[0]):                          # row sums = det A int B_i
        i = P.multi(r)
        expect = detA
        for k in range(3):
            kk = P.knots3[k]
            expect *= (kk[i[k] + p + 1] - kk[i[k]]) / (p + 1)
        assert abs(M[r].sum() - expect) <= 1e-13


def test_stiffness_kills_constants_and_mass_rowsum():
    p = 3
    kn = [open_uniform_knots(p, 3), open_uniform_knots(p, 4), random_open_knots(p, 3, seed=5)]
    P = Problem(kn, p, control_net(kn, p, seed=3, twist_deg=30), coef=coefficient_field(8))
    rp, _ = P.csr_pattern()
    for r in range(0, rp.size - 1, 7):
        s = P.row(r, "stiff")
        assert abs(s.sum()) <= 1e-12 * np.abs(s).max()
        # mass row sum = Q_i(c) = sum_q prod_k w00 * det J
        m = P.row(r, "mass")
        i = P.multi(r)
        det, _, _ = P.row_fields(r)
        w = [P.rules[k].w64[(0, 0)][i[k]] for k in range(3)]
        qi = np.einsum("x,y,z,xyz->", w[0], w[1], w[2], det)
        assert abs(m.sum() - qi) <= 1e-13 * abs(qi)


def test_nonsymmetric_for_nonconstant_coefficient():
    p = 2
    kn = [open_uniform_knots(p, 3)] * 3
    P = Problem(kn, p, control_net(kn, p, seed=1, twist_deg=30), coef=coefficient_field(2))
    M = to_dense(P, P.assemble("mass"))
    assert np.abs(M - M.T).max() > 1e-8 * np.abs(M).max()


def test_pattern_brute_force_and_nnz():
    w = SMALL_P2
    kn = w.knots()
    P = Problem(kn, w.p, w.ctrl())
    rp, ci = P.csr_pattern()
    assert ci.size == w.exact_nnz() == 85184
    n1, n2, n3 = P.n
    p = w.p
    sup = [[(kn[k][i], kn[k][i + p + 1]) for i in range(P.n[k])] for k in range(3)]
    rng = np.random.default_rng(0)
    for r in rng.integers(0, rp.size - 1, 40):
        i = P.multi(int(r))
        cols = []
        for c in range(n1 * n2 * n3):
            j = P.multi(c)
            if all(max(sup[k][i[k]][0], sup[k][j[k]][0]) < min(sup[k][i[k]][1], sup[k][j[k]][1])
                   for k in range(3)):
                cols.append(c)
        assert list(ci[rp[r]:rp[r + 1]]) == cols


@pytest.mark.slow
def test_wq_approaches_galerkin_under_refinement():
    """Not parity: WQ - Galerkin (high-order SGQ) shrinks with h (the paper
    reports optimal convergence, Section 7.1)."""
    p = 2
    errs = []
    for ne in (2, 4):
        kn = [open_uniform_knots(p, ne)] * 3
        P = Problem(kn, p, control_net(kn, p, seed=None, twist_deg=40), coef=None)
        wq = to_dense(P, P.assemble("mass"))
        ref = P.sgq_matrices("mass", n_gauss=8)
        errs.append(np.abs(wq - ref).max() / np.abs(ref).max())
    assert errs[1] < errs[0]
