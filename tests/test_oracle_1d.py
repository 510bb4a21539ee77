"""Pins for the 1D forms of the oracle (CPU only): Section 3 with one
direction, where J = dF/dzeta, the mass carries c = J and the stiffness
K = a / J (the setting of the test problem of Section 7.1)."""
import math
from itertools import combinations

import numpy as np
import pytest

from oracle.assembly import Problem
from oracle.geometry import map_and_jacobian_1d
from oracle.splines import basis_and_derivs
from workloads import (arcsin_curve_net, control_net, greville, open_uniform_knots,
                       random_open_knots)


def to_dense(P, vals):
    rp, ci = P.csr_pattern()
    N = rp.size - 1
    D = np.zeros((N, N))
    for r in range(N):
        D[r, ci[rp[r]:rp[r + 1]]] = vals[rp[r]:rp[r + 1]]
    return D


def quadratic_net(knots, p, gamma):
    """Control points of x(t) = t + gamma t^2 in closed form (Marsden's
    identity: the coefficient of t^2 on B_i is the mean of the pairwise
    products of the knots xi_{i+1} .. xi_{i+p}; that of t is their mean)."""
    n = len(knots) - p - 1
    C = np.empty((n, 1))
    for i in range(n):
        inner = [float(k) for k in knots[i + 1:i + p + 1]]
        e2 = sum(a * b for a, b in combinations(inner, 2)) / math.comb(p, 2)
        C[i, 0] = sum(inner) / p + gamma * e2
    return C


def test_identity_affine_and_quadratic_maps_1d():
    p = 3
    kn = random_open_knots(p, 6, seed=4)
    X = np.sort(np.random.default_rng(1).uniform(0.01, 0.99, 9))
    F, J = (t.astype(np.float64) for t in map_and_jacobian_1d([kn], p, control_net([kn], p, None), X))
    assert np.abs(F[:, 0] - X).max() < 1e-15 and np.abs(J[:, 0, 0] - 1).max() < 1e-13
    F, J = (t.astype(np.float64) for t in map_and_jacobian_1d([kn], p, 1.7 * greville(kn, p)[:, None] - 0.3, X))
    assert np.abs(F[:, 0] - (1.7 * X - 0.3)).max() < 1e-14 and np.abs(J[:, 0, 0] - 1.7).max() < 1e-13
    F, J = (t.astype(np.float64) for t in map_and_jacobian_1d([kn], p, quadratic_net(kn, p, 0.4), X))
    assert np.abs(F[:, 0] - (X + 0.4 * X * X)).max() < 1e-14
    assert np.abs(J[:, 0, 0] - (1 + 0.8 * X)).max() < 1e-12


def test_jacobian_finite_differences_1d():
    p = 4
    kn = open_uniform_knots(p, 7)
    ctrl = control_net([kn], p, seed=9, amp_h=0.1)
    X = np.array([0.11, 0.37, 0.52, 0.93])
    hstep = 1e-6
    Fp = map_and_jacobian_1d([kn], p, ctrl, X + hstep)[0][:, 0].astype(np.float64)
    Fm = map_and_jacobian_1d([kn], p, ctrl, X - hstep)[0][:, 0].astype(np.float64)
    J = map_and_jacobian_1d([kn], p, ctrl, X)[1][:, 0, 0].astype(np.float64)
    assert np.abs((Fp - Fm) / (2 * hstep) - J).max() < 1e-8


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_affine_exactness_1d(p):
    """x = alpha t + beta: every rule is exact for the products B_i B_j and
    B_i' B_j' (eq. exact), so M = alpha G0 and S = G1 / alpha exactly; the
    reference is Gauss quadrature with p+1 points per span (exact for these
    degree-2p piecewise polynomials)."""
    kn = random_open_knots(p, 7, seed=p)
    ctrl = 0.8 * greville(kn, p)[:, None] + 0.25
    P = Problem([kn], p, ctrl)
    for which in ("mass", "stiff"):
        D = to_dense(P, P.assemble(which))
        G = P.sgq_matrices(which)
        assert np.abs(D - G).max() <= 1e-13 * np.abs(G).max(), which


def test_kronecker_relation_with_2d():
    """The plane patch F(t, s) = (x(t), s) has det J = x'(t) and
    K = diag(1 / x', x'), so its matrices are Kronecker products of 1D ones:
    M2 = Ms (x) M1 and S2 = Ms (x) S1 + Ss (x) M1, where (M1, S1) are the 1D
    matrices of x(t) and (Ms, Ss) those of the identity map in s (rows with
    i1 fastest).  This ties the 1D forms to the independently pinned 2D ones."""
    p = 3
    k1 = random_open_knots(p, 6, seed=5)
    ks = open_uniform_knots(p, 4)
    c1 = control_net([k1], p, seed=3, amp_h=0.1)
    gs = greville(ks, p)
    ctrl2 = np.stack(np.broadcast_arrays(c1[None, :, 0], gs[:, None]), axis=-1)
    P1, Ps = Problem([k1], p, c1), Problem([ks], p, gs[:, None])
    P2 = Problem([k1, ks], p, ctrl2)
    M1, S1 = (to_dense(P1, P1.assemble(w)) for w in ("mass", "stiff"))
    Ms, Ss = (to_dense(Ps, Ps.assemble(w)) for w in ("mass", "stiff"))
    M2, S2 = (to_dense(P2, P2.assemble(w)) for w in ("mass", "stiff"))
    assert np.abs(M2 - np.kron(Ms, M1)).max() <= 1e-13 * np.abs(M2).max()
    assert np.abs(S2 - (np.kron(Ms, S1) + np.kron(Ss, M1))).max() <= 1e-13 * np.abs(S2).max()


def test_coefficient_enters_as_a_over_j():
    """On x(t) = t + gamma t^2 the coefficient a(x) = sqrt(1 + 4 gamma x)
    equals x'(t) at x = x(t), so K = a / J = 1 at every point and the
    stiffness equals that of the identity map; a evaluated at t instead of
    x, or multiplied instead of divided by J, breaks this."""
    p, gamma = 3, 0.6
    kn = open_uniform_knots(p, 9)
    coef = lambda x: np.sqrt(1.0 + 4.0 * gamma * x[:, 0])
    Pq = Problem([kn], p, quadratic_net(kn, p, gamma), coef=coef)
    Pi = Problem([kn], p, greville(kn, p)[:, None])
    S, S0 = Pq.assemble("stiff"), Pi.assemble("stiff")
    assert np.abs(S - S0).max() <= 1e-12 * np.abs(S0).max()
    # S 1 = 0 for any map and coefficient (the B_j' sum to zero)
    rp, _ = Pq.csr_pattern()
    assert np.abs(np.add.reduceat(S, rp[:-1])).max() <= 1e-12 * np.abs(S).max()


# ---- the 1D test problem of Section 7.1 on a spline curve map ------------

LEN = math.pi / 6
f_of = lambda x: (5.0 * np.exp(2.0 * x) - 1.0) / 4.0
u_of = lambda x: (np.exp(2.0 * x) - 1.0) / 4.0
du_of = lambda x: np.exp(2.0 * x) / 2.0


def curve_tables(knots, p, ng=8):
    """Gauss points and weights (ng per span) with the dense basis values and
    derivatives there (test infrastructure for load vectors and errors)."""
    gx, gw = np.polynomial.legendre.leggauss(ng)
    chi = np.unique(knots)
    T, W, V, D = [], [], [], []
    for e in range(len(chi) - 1):
        a, b = chi[e], chi[e + 1]
        for g, w in zip(0.5 * (a + b) + 0.5 * (b - a) * gx, 0.5 * (b - a) * gw):
            v, d = basis_and_derivs(list(knots), p, float(g))
            T.append(g), W.append(w), V.append(np.asarray(v, np.float64)), D.append(np.asarray(d, np.float64))
    return np.array(T), np.array(W), np.array(V), np.array(D)


def solve_curve_problem(knots, p, ctrl, M, S):
    """u'' + u = f on the physical interval x(t), t in [0, 1]: Galerkin
    system (M - S) u = F with Dirichlet values u(0) = 0, u(pi/6) = u_of(pi/6)
    (the exact solution's value), load by Gauss quadrature.  Returns the L2
    and H1-seminorm errors in physical coordinates."""
    _, W, V, D = curve_tables(knots, p)
    x, xd = V @ ctrl[:, 0], D @ ctrl[:, 0]
    F = V.T @ (W * f_of(x) * xd)
    A = M - S
    n = A.shape[0]
    ub = np.zeros(n)
    ub[-1] = u_of(LEN)
    inner = np.arange(1, n - 1)
    u = ub.copy()
    u[inner] = np.linalg.solve(A[np.ix_(inner, inner)], F[inner] - A[inner] @ ub)
    e0 = np.sqrt(np.sum(W * xd * (V @ u - u_of(x)) ** 2))
    e1 = np.sqrt(np.sum(W * xd * ((D @ u) / xd - du_of(x)) ** 2))
    return e0, e1


@pytest.mark.parametrize("p", [2, 3])
def test_curve_problem_converges_optimally(p):
    """Section 7.1's problem with the map given as a spline curve (Schoenberg
    control points of x = arcsin(t/2)): the WQ Galerkin solution converges
    at the optimal rates, h^{p+1} in L2 and h^p in H1."""
    errs = []
    for ne in (8, 16, 32):
        kn = open_uniform_knots(p, ne)
        ctrl = arcsin_curve_net(kn, p)
        P = Problem([kn], p, ctrl)
        M, S = (to_dense(P, P.assemble(w)) for w in ("mass", "stiff"))
        errs.append(solve_curve_problem(kn, p, ctrl, M, S))
    E = np.array(errs)
    rate = lambda k: math.log2(E[-2, k] / E[-1, k])
    print(f"p={p} L2 {E[:, 0]} H1 {E[:, 1]}")
    assert rate(0) >= p + 1 - 0.3 and rate(1) >= p - 0.3
