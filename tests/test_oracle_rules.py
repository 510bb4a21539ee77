"""Pins for oracle/rules.py (CPU only)."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.rules import PAIRINGS, UnivariateRules, quadrature_points, rules_for
from oracle.splines import basis_and_derivs
from workloads import open_uniform_knots, random_open_knots

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def exact_uniform(p, n_el, a=Fr(0), b=Fr(1)):
    return [a] * (p + 1) + [a + (b - a) * Fr(k, n_el) for k in range(1, n_el)] + [b] * (p + 1)


@pytest.mark.parametrize("p,key", [(1, "cavalieri_simpson_p1"), (2, "weights_p2"), (3, "weights_p3")])
def test_printed_interior_weights(p, key):
    h = Fr(1, 12)
    r = UnivariateRules(exact_uniform(p, 12), p)
    i = 6  # interior function
    got = [w / h for w in r.w[(0, 0)][i]]
    assert got == [Fr(s) for s in GOLD[key]["weights_over_h"]]


def test_printed_integrals_p2():
    h = Fr(1, 12)
    r = UnivariateRules(exact_uniform(2, 12), 2)
    i = 6
    got = [r.integ[(0, 0)][i][j] / h for j in r.I[i]]
    assert got == [Fr(s) for s in GOLD["integrals_p2"]["values_over_h"]]


def test_printed_nonsymmetry_example():
    g = GOLD["nonsymmetry_p3"]
    kn = exact_uniform(3, 12, Fr(-8), Fr(16))          # h = 2
    r = UnivariateRules(kn, 3)
    i = [k for k in range(r.n) if kn[k] == 0 and kn[k + 4] == 8][0]
    j = i + 1

    def Q(test, trial):
        tot = Fr(0)
        for w, q in zip(r.w[(0, 0)][test], r.Q[test]):
            x = r.x[q]
            tot += w * x * r.Bq[0][trial][q]
        return float(tot)
    assert [float(r.x[q]) for q in r.Q[i]] == [1, 2, 3, 4, 5, 6, 7]
    assert abs(Q(i, j) - g["Qi_cBj"]) <= g["abs_tol"]
    assert abs(Q(j, i) - g["Qj_cBi"]) <= g["abs_tol"]


@pytest.mark.parametrize("p,n_el", [(2, 8), (3, 5), (4, 9), (5, 6), (6, 10), (3, 2), (2, 1)])
def test_point_counts(p, n_el):
    r = rules_for(list(open_uniform_knots(p, n_el)), p)
    expect = 2 * n_el + 2 * p - 1 if n_el >= 2 else p + 1
    assert len(r.x) == expect
    assert all(r.x[k] < r.x[k + 1] for k in range(len(r.x) - 1))
    assert r.x[0] > 0 and r.x[-1] < 1
    for i in range(r.n):
        assert len(r.Q[i]) >= len(r.I[i])          # eq. numb_nodes
        if n_el >= p + 2:                           # no support holds both boundary spans
            assert len(r.Q[i]) <= 3 * p + 1
        assert r.Q[i] == list(range(r.Q[i][0], r.Q[i][-1] + 1))   # contiguous
    if n_el >= 2 * p + 2:
        mid = r.n // 2
        assert len(r.Q[mid]) == 2 * p + 1          # interior: knots + midpoints


@pytest.mark.parametrize("p,n_el,uniform", [(2, 6, True), (3, 7, False), (4, 9, True), (6, 14, True), (5, 8, False)])
def test_moments_and_exactness(p, n_el, uniform):
    kn = list(open_uniform_knots(p, n_el)) if uniform else list(random_open_knots(p, n_el, seed=p))
    r = rules_for(kn, p)
    for i in range(r.n):
        # int B_i = (xi_{i+p+1} - xi_i)/(p+1)
        assert sum(r.w[(0, 0)][i]) == (r.knots[i + p + 1] - r.knots[i]) / (p + 1)
        # int B_i' = B_i(1) - B_i(0) in {-1, 0, 1} (open knots)
        expect = (1 if i == r.n - 1 else 0) - (1 if i == 0 else 0)
        assert sum(r.w[(0, 1)][i]) == expect
        for (al, be) in PAIRINGS:
            A = np.array([[float(r.Bq[al][j][q]) for q in r.Q[i]] for j in r.I[i]])
            b = np.array([float(r.integ[(al, be)][i][j]) for j in r.I[i]])
            res = A @ r.w64[(al, be)][i] - b
            assert np.abs(res).max() <= 1e-14 * max(1.0, np.abs(b).max()) * len(r.Q[i])


@pytest.mark.parametrize("p,n_el", [(2, 6), (3, 8), (4, 10)])
def test_min_norm_against_svd_lstsq(p, n_el):
    """Independent route: numpy's SVD-based least squares returns the
    minimum-norm solution of a consistent (possibly rank-deficient) system."""
    r = rules_for(list(open_uniform_knots(p, n_el)), p)
    for i in range(r.n):
        for (al, be) in PAIRINGS:
            A = np.array([[float(r.Bq[al][j][q]) for q in r.Q[i]] for j in r.I[i]])
            b = np.array([float(r.integ[(al, be)][i][j]) for j in r.I[i]])
            w, _, rank, sv = np.linalg.lstsq(A, b, rcond=1e-12)
            assert rank == len(r.I[i]) - al         # derivative systems lose exactly one rank
            scale = np.abs(w).max()
            assert np.abs(w - r.w64[(al, be)][i]).max() <= 1e-9 * scale
            # minimum norm: orthogonal to the null space of A
            _, s, Vt = np.linalg.svd(A)
            null = Vt[rank:]
            if len(null):
                assert np.abs(null @ r.w64[(al, be)][i]).max() <= 1e-10 * scale


@pytest.mark.parametrize("p", [2, 3, 5])
def test_integrals_vs_gauss(p):
    """Exact rational integrals against FP64 element-wise Gauss-Legendre."""
    kn = list(random_open_knots(p, 6, seed=3))
    r = rules_for(kn, p)
    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    chi = np.unique(kn)
    pts, wts = [], []
    for a, b in zip(chi[:-1], chi[1:]):
        pts += list(0.5 * (a + b) + 0.5 * (b - a) * gx)
        wts += list(0.5 * (b - a) * gw)
    V = np.array([basis_and_derivs(kn, p, x)[0] for x in pts])
    D = np.array([basis_and_derivs(kn, p, x)[1] for x in pts])
    tab = {0: V, 1: D}
    wts = np.array(wts)
    for (al, be) in PAIRINGS:
        for i in range(r.n):
            for j in r.I[i]:
                g = float(np.sum(wts * tab[be][:, i] * tab[al][:, j]))
                assert abs(g - float(r.integ[(al, be)][i][j])) <= 1e-13 * (1 + abs(g))


def test_interior_positivity_soft():
    """Section 2 observes positive (0,0) weights for interior functions."""
    for p in (2, 3, 4, 5, 6):
        r = rules_for(list(open_uniform_knots(p, 3 * p + 3)), p)
        i = r.n // 2
        assert all(w > 0 for w in r.w[(0, 0)][i])


@pytest.mark.parametrize("p,n_el", [(2, 6), (4, 9), (6, 12)])
def test_boundary_points_reading_and_mirror_symmetry(p, n_el):
    """Reading of Remark 4.1 used here: in each boundary span [a, b] the
    p+1 points together with a and b are equally spaced.  Points and weights
    of symmetric knot vectors are mirror symmetric."""
    kn = exact_uniform(p, n_el)
    r = UnivariateRules(kn, p)
    h = Fr(1, n_el)
    left = [Fr(0)] + r.x[:p + 1] + [h]
    right = [1 - h] + r.x[-(p + 1):] + [Fr(1)]
    for seq in (left, right):
        d = [seq[k + 1] - seq[k] for k in range(len(seq) - 1)]
        assert all(v == h / (p + 2) for v in d)
    nq = len(r.x)
    assert all(r.x[q] == 1 - r.x[nq - 1 - q] for q in range(nq))
    for (al, be) in PAIRINGS:
        sign = (-1) ** be           # B_i(x) = B_{n-1-i}(1-x); only the test derivative flips the sign
        for i in range(r.n):
            assert r.w[(al, be)][i] == [sign * v for v in reversed(r.w[(al, be)][r.n - 1 - i])]
