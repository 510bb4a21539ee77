"""Pins for oracle/splines.py (CPU only)."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.splines import basis_and_derivs, overlap_set
from workloads import open_uniform_knots, random_open_knots

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def exact_uniform(p, n_el, a=Fr(0), b=Fr(1)):
    return [a] * (p + 1) + [a + (b - a) * Fr(k, n_el) for k in range(1, n_el)] + [b] * (p + 1)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_partition_of_unity_exact(p):
    kn = exact_uniform(p, 7)
    rng = np.random.default_rng(p)
    for _ in range(20):
        x = Fr(int(rng.integers(0, 10**6)), 10**6)
        v, d = basis_and_derivs(kn, p, x)
        assert sum(v) == 1
        assert sum(d) == 0
        assert all(t >= 0 for t in v)


def test_printed_quadratic_values():
    g = GOLD["bspline_values_p2"]
    h = Fr(1, 10)
    kn = exact_uniform(2, 10)
    i = 5                       # interior: support [xi_5, xi_8] = [3h, 6h]
    start = kn[i]
    for t, val in zip(g["points_in_units_of_h_from_support_start"], g["values"]):
        v, _ = basis_and_derivs(kn, 2, start + Fr(t) * h)
        assert v[i] == Fr(val)


def test_printed_cubic_values():
    g = GOLD["bspline_values_p3"]
    # h = 2 knots at even integers on [-8, 16]; B_j with support [2, 10]
    kn = exact_uniform(3, 12, Fr(-8), Fr(16))
    j = [k for k in range(len(kn) - 4) if kn[k] == 2 and kn[k + 4] == 10][0]
    for t, val in zip(g["points"], g["values"]):
        v, _ = basis_and_derivs(kn, 3, Fr(t))
        assert v[j] == Fr(val)


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_derivative_vs_finite_difference(p):
    kn = list(random_open_knots(p, 9, seed=p))
    rng = np.random.default_rng(10 + p)
    for _ in range(10):
        x = float(rng.uniform(0.01, 0.99))
        eps = 1e-6
        vp, _ = basis_and_derivs(kn, p, x + eps)
        vm, _ = basis_and_derivs(kn, p, x - eps)
        _, d = basis_and_derivs(kn, p, x)
        fd = (np.array(vp) - np.array(vm)) / (2 * eps)
        assert np.allclose(fd, d, atol=1e-5 * max(1.0, np.abs(d).max()))


@pytest.mark.parametrize("p", [2, 5])
def test_mirror_symmetry(p):
    kn = exact_uniform(p, 6)
    n = len(kn) - p - 1
    for x in (Fr(1, 7), Fr(2, 5), Fr(1, 2), Fr(5, 6)):
        v, d = basis_and_derivs(kn, p, x)
        w, e = basis_and_derivs(kn, p, 1 - x)
        for i in range(n):
            assert v[i] == w[n - 1 - i]
            assert d[i] == -e[n - 1 - i]


@pytest.mark.parametrize("p,n_el", [(1, 5), (2, 8), (3, 4), (6, 10), (4, 1), (3, 2)])
def test_overlap_sets_band_and_nnz(p, n_el):
    kn = list(open_uniform_knots(p, n_el))
    n = n_el + p
    total = 0
    for i in range(n):
        I = overlap_set(kn, p, i)
        assert I == list(range(max(0, i - p), min(n - 1, i + p) + 1))
        total += len(I)
    # Section 3: N_NZ = (2p+1) N_DOF - p(p+1) in 1D with maximal regularity
    assert total == (2 * p + 1) * n - p * (p + 1)
