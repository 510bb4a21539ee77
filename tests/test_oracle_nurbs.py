"""Pins for the NURBS forms of the oracle (CPU only): a rational map
(homogeneous net and quotient rule) and, for the mass, rational test and
trial functions with the denominator folded into the factor c (Section 3).

The exact quarter annulus used here is built independently of the oracle:
the quadratic quarter circle (control points (1,0), (1,1), (0,1), weights
1, sqrt(2)/2, 1) refined by Boehm's knot insertion in homogeneous
coordinates, written out below."""
import math

import numpy as np
import pytest

from oracle.assembly import Problem
from oracle.geometry import map_and_jacobian_2d, rational_map_and_jacobian
from workloads import control_net, greville, open_uniform_knots, random_open_knots


def insert_knot(knots, p, Pw, u):
    """Boehm's algorithm: insert u once into `knots` (homogeneous control
    points Pw, shape (n, k)); the curve is unchanged."""
    knots = list(knots)
    s = max(i for i in range(len(knots) - 1) if knots[i] <= u < knots[i + 1])
    Q = []
    for i in range(len(Pw) + 1):
        if i <= s - p:
            Q.append(Pw[i])
        elif i > s:
            Q.append(Pw[i - 1])
        else:
            a = (u - knots[i]) / (knots[i + p] - knots[i])
            Q.append((1 - a) * Pw[i - 1] + a * Pw[i])
    return knots[:s + 1] + [u] + knots[s + 1:], np.array(Q)


def quarter_circle(n_el):
    """Open uniform knots of degree 2 with n_el spans and the homogeneous
    control points (x w, y w, w) of the exact unit quarter circle."""
    h = math.sqrt(0.5)
    knots = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    Pw = np.array([[1.0, 0.0, 1.0], [h, h, h], [0.0, 1.0, 1.0]])
    for k in range(1, n_el):
        knots, Pw = insert_knot(knots, 2, Pw, k / n_el)
    return np.array(knots), Pw


def quarter_annulus(n_rad, n_ang, r0=1.0, r1=2.0):
    """Degree-2 plane patch of the quarter annulus r0 <= r <= r1: direction 1
    radial (linear in r), direction 2 angular (exact circle).  Returns
    (knots, ctrl (n2, n1, 2), weights (n2, n1))."""
    k1 = open_uniform_knots(2, n_rad)
    r = r0 + (r1 - r0) * greville(k1, 2)
    k2, Pw = quarter_circle(n_ang)
    w = Pw[:, 2]
    xy = Pw[:, :2] / w[:, None]
    ctrl = r[None, :, None] * xy[:, None, :]
    weights = np.broadcast_to(w[:, None], (len(w), len(r))).copy()
    return [k1, k2], ctrl, weights


def test_constant_weights_reduce_to_bsplines():
    """w = const: the rational map is the polynomial one, and the NURBS
    functions are the B-splines (w_i w_j / W^2 = 1), so every row agrees."""
    p = 3
    kn = [open_uniform_knots(p, 5), random_open_knots(p, 6, seed=3)]
    ctrl = control_net(kn, p, seed=4, amp_h=0.15)
    w = np.full(ctrl.shape[:-1], 2.5)
    X = [np.linspace(0.03, 0.97, 7)] * 2
    F0, J0 = (t.astype(np.float64) for t in map_and_jacobian_2d(kn, p, ctrl, *X))
    F1, J1, W = rational_map_and_jacobian(kn, p, ctrl, w, X)
    assert np.abs(F1.astype(np.float64) - F0).max() < 1e-14
    assert np.abs(J1.astype(np.float64) - J0).max() < 1e-12
    assert np.abs(W.astype(np.float64) - 2.5).max() < 1e-15
    P0 = Problem(kn, p, ctrl)
    Pr = Problem(kn, p, ctrl, weights=w)
    Pn = Problem(kn, p, ctrl, weights=w, basis="nurbs")
    for r in (0, 7, 19, 40):
        for which in ("mass", "stiff"):
            a, b = P0.row(r, which), Pr.row(r, which)
            assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
        a, b = P0.row(r, "mass"), Pn.row(r, "mass")
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_exact_quarter_annulus_map():
    """|F| is the radius, linear in the radial parameter; J agrees with
    central differences of F; the area is pi/4 (r1^2 - r0^2)."""
    kn, ctrl, w = quarter_annulus(3, 4)
    rng = np.random.default_rng(0)
    X = [np.sort(rng.uniform(0.01, 0.99, 6)) for _ in range(2)]
    F, J, _ = rational_map_and_jacobian(kn, 2, ctrl, w, X)
    F = F.astype(np.float64)
    assert np.abs(np.linalg.norm(F, axis=-1) - (1.0 + X[0])[:, None]).max() < 1e-14
    hstep = 1e-6
    for b in range(2):
        Xp = [x.copy() for x in X]
        Xm = [x.copy() for x in X]
        Xp[b] = Xp[b] + hstep
        Xm[b] = Xm[b] - hstep
        Fp = rational_map_and_jacobian(kn, 2, ctrl, w, Xp)[0].astype(np.float64)
        Fm = rational_map_and_jacobian(kn, 2, ctrl, w, Xm)[0].astype(np.float64)
        assert np.abs((Fp - Fm) / (2 * hstep) - J[..., :, b].astype(np.float64)).max() < 1e-8
    # area by a 12-point Gauss rule per span of the determinant
    gx, gw = np.polynomial.legendre.leggauss(12)
    pts, wts = [], []
    for k in kn:
        chi = np.unique(k)
        pts.append(np.concatenate([0.5 * (a + b) + 0.5 * (b - a) * gx for a, b in zip(chi[:-1], chi[1:])]))
        wts.append(np.concatenate([0.5 * (b - a) * gw for a, b in zip(chi[:-1], chi[1:])]))
    _, J, _ = rational_map_and_jacobian(kn, 2, ctrl, w, pts)
    det = (J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]).astype(np.float64)
    area = float(wts[0] @ det @ wts[1])
    assert abs(area - math.pi / 4 * 3.0) < 1e-12


def test_nurbs_mass_partition_of_unity():
    """The rational functions sum to one, so all entries of the NURBS mass
    matrix add up to the area: exactly (to rounding) with 10-point Gauss
    quadrature, and to the WQ rules' accuracy with the rows (the factor c
    is not a polynomial)."""
    kn, ctrl, w = quarter_annulus(4, 6)
    P = Problem(kn, 2, ctrl, weights=w, basis="nurbs")
    area = math.pi / 4 * 3.0
    M = P.sgq_matrices("mass", n_gauss=10)
    assert abs(M.sum() - area) < 1e-11
    tot = P.assemble("mass").sum()
    assert abs(tot - area) < 2e-4 * area
    # the factors matter: without w_i w_j the entries sum to int det J / W^2
    wf = w.ravel()
    assert abs((M / np.outer(wf, wf)).sum() - area) > 1e-2
    # B-spline functions on the same map also sum to one
    Pb = Problem(kn, 2, ctrl, weights=w)
    assert abs(Pb.sgq_matrices("mass", n_gauss=10).sum() - area) < 1e-11


def test_nurbs_rows_direct_equals_sumfact_and_stiffness_refused():
    kn, ctrl, w = quarter_annulus(4, 5)
    P = Problem(kn, 2, ctrl, weights=w, basis="nurbs")
    for r in (0, 5, 13, 29):
        a, b = P.row(r, "mass", "direct"), P.row(r, "mass", "sumfact")
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    with pytest.raises(NotImplementedError):
        P.row(3, "stiff")


def test_thick_cylinder_volume_3d():
    """The quarter annulus extruded linearly in z to height 0.5 (degree 2 in
    all directions): the volume of the rational 3D map is 0.5 pi/4 (r1^2 - r0^2)."""
    kn2, ctrl2, w2 = quarter_annulus(2, 3)
    k3 = open_uniform_knots(2, 2)
    z = 0.5 * greville(k3, 2)
    n3 = len(z)
    ctrl = np.concatenate([np.broadcast_to(ctrl2[None], (n3,) + ctrl2.shape),
                           np.broadcast_to(z[:, None, None, None], (n3,) + ctrl2.shape[:2] + (1,))], axis=-1)
    w = np.broadcast_to(w2[None], (n3,) + w2.shape).copy()
    kn = kn2 + [k3]
    gx, gw = np.polynomial.legendre.leggauss(8)
    pts, wts = [], []
    for k in kn:
        chi = np.unique(k)
        pts.append(np.concatenate([0.5 * (a + b) + 0.5 * (b - a) * gx for a, b in zip(chi[:-1], chi[1:])]))
        wts.append(np.concatenate([0.5 * (b - a) * gw for a, b in zip(chi[:-1], chi[1:])]))
    _, J, _ = rational_map_and_jacobian(kn, 2, np.ascontiguousarray(ctrl), w, pts)
    det = np.linalg.det(J.astype(np.float64))
    vol = float(np.einsum("a,b,c,abc->", wts[0], wts[1], wts[2], det))
    assert abs(vol - 0.5 * math.pi / 4 * 3.0) < 1e-12
