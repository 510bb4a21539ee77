"""Geometry map and PDE coefficients at points, for the oracle (test
infrastructure only).

Section 3: the domain is a single spline patch F(zeta) = sum_i C_i B_i(zeta);
the mass integrand carries c = det DF (eq. mass2) and the stiffness carries
c_lm = { [DF^{-1} DF^{-T}] det DF }_lm (eq. coef_stiff), here multiplied by a
scalar diffusion coefficient a(F(zeta)) ("non-constant coefficients could be
included as well", Section 3).

Everything is evaluated directly from the definition: at each point, the sum
over the (p+1)^3 tensor-product B-splines that are nonzero there.  The
inverse is the explicit adjugate formula.

Precision: DF = sum_i C_i grad B_i cancels strongly (the B_i' sum to zero and
are O(1/h)), so a plain FP64 evaluation carries O(eps/h) error.  To serve as
a reference, the oracle evaluates the same sums in x87 extended precision
(numpy longdouble, 64-bit significand); at rational points (the quadrature
points) the univariate B-spline values and derivatives are exact rationals
before conversion.  Results are rounded to FP64 by the callers.

The 2D forms (``map_and_jacobian_2d``, ``coefficients_from_jacobian_2d``)
follow the same definitions with (p+1)^2 functions per point and a 2x2 J;
the 1D forms (``map_and_jacobian_1d``, ``coefficients_from_jacobian_1d``)
with p+1 functions per point, J = dF/dzeta, det J = J and K = a / J (the
one-direction case of eq. coef_stiff, as in the problem of Section 7.1).
``rational_map_and_jacobian`` evaluates a NURBS map through its homogeneous
net (the same sums, then the quotient rule).

Pins (tests/test_oracle_geometry.py): Greville control points give the
identity map (J = I, K = I); an affine control net gives J = A everywhere;
J agrees with central finite differences of F; K agrees with an
independently computed det(J) inv(J) inv(J)^T (numpy.linalg); the same for
the 2D forms.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np

from fractions import Fraction

from .splines import basis_and_derivs, exact_knots, find_span


LD = np.longdouble


def to_ld(v) -> np.longdouble:
    """A float or an exact Fraction as longdouble (two-term split of a
    Fraction, so the conversion is correctly rounded to 64 bits)."""
    if isinstance(v, Fraction):
        hi = float(v)
        return LD(hi) + LD(float(v - Fraction(hi)))
    return LD(v)


def local_basis(knots: Sequence, p: int, pts: Sequence):
    """For each point: first index of the p+1 nonzero B-splines, and their
    values and derivatives there.  Points given as Fractions are evaluated
    exactly (exact knots); floats in FP64.  Returns (first[np], V[np,p+1],
    D[np,p+1]) with V, D in longdouble."""
    exact = len(pts) > 0 and isinstance(pts[0], Fraction)
    kn = exact_knots(knots) if exact else [float(k) for k in knots]
    n = len(kn) - p - 1
    first = np.zeros(len(pts), dtype=np.int64)
    V = np.zeros((len(pts), p + 1), dtype=LD)
    D = np.zeros((len(pts), p + 1), dtype=LD)
    for k, x in enumerate(pts):
        x = x if exact else float(x)
        s = find_span(kn, x)
        vals, ders = basis_and_derivs(kn, p, x)
        f = min(max(s - p, 0), n - p - 1)
        first[k] = f
        V[k] = [to_ld(t) for t in vals[f:f + p + 1]]
        D[k] = [to_ld(t) for t in ders[f:f + p + 1]]
    return first, V, D


def map_and_jacobian(knots3, p: int, ctrl: np.ndarray, X1, X2, X3):
    """F and J = dF/dzeta on the tensor grid X1 x X2 x X3.

    ctrl: (n3, n2, n1, k) control points (linear index i1 + n1(i2 + n2 i3)),
    k = 3 (or 4 for a homogeneous net).  Returns F with shape
    (len(X1), len(X2), len(X3), k) and J with shape
    (len(X1), len(X2), len(X3), k, 3), J[..., a, b] = dF_a / dzeta_b, in
    longdouble."""
    ctrl = np.asarray(ctrl).astype(LD)
    f1, V1, D1 = local_basis(knots3[0], p, X1)
    f2, V2, D2 = local_basis(knots3[1], p, X2)
    f3, V3, D3 = local_basis(knots3[2], p, X3)
    r = np.arange(p + 1)
    n1, n2, n3 = len(X1), len(X2), len(X3)
    k = ctrl.shape[-1]   # components (3, or 4 for a homogeneous net)
    F = np.zeros((n1, n2, n3, k), dtype=LD)
    J = np.zeros((n1, n2, n3, k, 3), dtype=LD)
    # gather the local (p+1)^3 control blocks for every grid point
    i1 = (f1[:, None] + r[None, :])            # (n1, p+1)
    i2 = (f2[:, None] + r[None, :])
    i3 = (f3[:, None] + r[None, :])
    for c in range(n3):                         # one z-plane of points at a time
        # Cloc[a, b, l3, l2, l1, :] = ctrl[i3[c,l3], i2[b,l2], i1[a,l1], :]
        Cloc = ctrl[i3[c][None, None, :, None, None],
                    i2[None, :, None, :, None],
                    i1[:, None, None, None, :], :]
        def contract(A1, A2, A3c):
            # sum over the local functions of the product basis value times C
            W = (A3c[None, None, :, None, None] * A2[None, :, None, :, None]
                 * A1[:, None, None, None, :])
            return np.einsum("abxyz,abxyzd->abd", W, Cloc)
        F[:, :, c, :] = contract(V1, V2, V3[c])
        J[:, :, c, :, 0] = contract(D1, V2, V3[c])
        J[:, :, c, :, 1] = contract(V1, D2, V3[c])
        J[:, :, c, :, 2] = contract(V1, V2, D3[c])
    return F, J


def coefficients_from_jacobian(J: np.ndarray, a: Optional[np.ndarray] = None):
    """Mass factor c = det J and stiffness coefficient
    K = a det(J) J^{-1} J^{-T} = a adj(J) adj(J)^T / det(J) (eq. coef_stiff).

    Returns (detJ[...], K[..., 3, 3])."""
    j = J
    c00 = j[..., 1, 1] * j[..., 2, 2] - j[..., 1, 2] * j[..., 2, 1]
    c01 = j[..., 1, 2] * j[..., 2, 0] - j[..., 1, 0] * j[..., 2, 2]
    c02 = j[..., 1, 0] * j[..., 2, 1] - j[..., 1, 1] * j[..., 2, 0]
    c10 = j[..., 0, 2] * j[..., 2, 1] - j[..., 0, 1] * j[..., 2, 2]
    c11 = j[..., 0, 0] * j[..., 2, 2] - j[..., 0, 2] * j[..., 2, 0]
    c12 = j[..., 0, 1] * j[..., 2, 0] - j[..., 0, 0] * j[..., 2, 1]
    c20 = j[..., 0, 1] * j[..., 1, 2] - j[..., 0, 2] * j[..., 1, 1]
    c21 = j[..., 0, 2] * j[..., 1, 0] - j[..., 0, 0] * j[..., 1, 2]
    c22 = j[..., 0, 0] * j[..., 1, 1] - j[..., 0, 1] * j[..., 1, 0]
    det = j[..., 0, 0] * c00 + j[..., 0, 1] * c01 + j[..., 0, 2] * c02
    # adj(J) = cofactor matrix transposed
    adj = np.stack([np.stack([c00, c10, c20], -1),
                    np.stack([c01, c11, c21], -1),
                    np.stack([c02, c12, c22], -1)], -2)
    K = np.einsum("...ik,...jk->...ij", adj, adj) / det[..., None, None]
    if a is not None:
        K = K * np.asarray(a)[..., None, None]
    return det, K


def map_and_jacobian_2d(knots2, p: int, ctrl: np.ndarray, X1, X2):
    """F and J = dF/dzeta of a bivariate map on the grid X1 x X2.

    ctrl: (n2, n1, 2) control points (linear index i1 + n1 i2).  Returns F
    with shape (len(X1), len(X2), 2) and J with shape (len(X1), len(X2), 2, 2),
    J[..., a, b] = dF_a / dzeta_b, in longdouble."""
    ctrl = np.asarray(ctrl).astype(LD)
    f1, V1, D1 = local_basis(knots2[0], p, X1)
    f2, V2, D2 = local_basis(knots2[1], p, X2)
    r = np.arange(p + 1)
    i1 = f1[:, None] + r[None, :]              # (n1, p+1)
    i2 = f2[:, None] + r[None, :]
    # Cloc[a, b, l2, l1, :] = ctrl[i2[b, l2], i1[a, l1], :]
    Cloc = ctrl[i2[None, :, :, None], i1[:, None, None, :], :]

    def contract(A1, A2):
        W = A2[None, :, :, None] * A1[:, None, None, :]
        return np.einsum("abyz,abyzd->abd", W, Cloc)
    F = contract(V1, V2)
    J = np.stack([contract(D1, V2), contract(V1, D2)], axis=-1)
    return F, J


def coefficients_from_jacobian_2d(J: np.ndarray, a: Optional[np.ndarray] = None):
    """2D forms of eq. mass2 and eq. coef_stiff: c = det J and
    K = a det(J) J^{-1} J^{-T} = a adj(J) adj(J)^T / det(J) with
    adj(J) = [[J11, -J01], [-J10, J00]].  Returns (detJ[...], K[..., 2, 2])."""
    j = J
    det = j[..., 0, 0] * j[..., 1, 1] - j[..., 0, 1] * j[..., 1, 0]
    adj = np.stack([np.stack([j[..., 1, 1], -j[..., 0, 1]], -1),
                    np.stack([-j[..., 1, 0], j[..., 0, 0]], -1)], -2)
    K = np.einsum("...ik,...jk->...ij", adj, adj) / det[..., None, None]
    if a is not None:
        K = K * np.asarray(a)[..., None, None]
    return det, K


def map_and_jacobian_1d(knots1, p: int, ctrl: np.ndarray, X1):
    """F and J = dF/dzeta of a univariate map at the points X1.

    ctrl: (n1, k) control points (k components, 1 for a curve in the line).
    Returns F with shape (len(X1), k) and J with shape (len(X1), k, 1), in
    longdouble."""
    ctrl = np.asarray(ctrl).astype(LD)
    f1, V1, D1 = local_basis(knots1[0], p, X1)
    i1 = f1[:, None] + np.arange(p + 1)[None, :]
    C = ctrl[i1]                                   # (n_pts, p+1, k)
    F = np.einsum("ar,ark->ak", V1, C)
    J = np.einsum("ar,ark->ak", D1, C)
    return F, J[:, :, None]


def coefficients_from_jacobian_1d(J: np.ndarray, a: Optional[np.ndarray] = None):
    """1D forms of eq. mass2 and eq. coef_stiff: c = J and K = a / J.
    Returns (J[...], K[..., 1, 1])."""
    det = J[..., 0, 0]
    K = 1 / J
    if a is not None:
        K = K * np.asarray(a)[..., None, None]
    return det, K


def rational_map_and_jacobian(knots, p: int, ctrl: np.ndarray, weights: np.ndarray, X):
    """A NURBS map F = sum_i w_i C_i B_i / W, W = sum_i w_i B_i (the rational
    generalisation Section 3 allows through the factor c), on the tensor grid
    of the points X (one array per direction, d = len(knots)).

    The spline map of the homogeneous net (w C, w) gives N = sum w_i C_i B_i,
    W and their derivatives; then F = N / W and, by the quotient rule,
    J = (dN - F dW^T) / W.  Returns (F[..., d], J[..., d, d], W[...]) in
    longdouble, indexed like the polynomial forms."""
    d = len(knots)
    C = np.asarray(ctrl).astype(LD)
    w = np.asarray(weights).astype(LD)[..., None]
    H = np.concatenate([C * w, w], axis=-1)        # homogeneous net
    if d == 3:
        Fh, Jh = map_and_jacobian(knots, p, H, X[0], X[1], X[2])
    elif d == 2:
        Fh, Jh = map_and_jacobian_2d(knots, p, H, X[0], X[1])
    else:
        Fh, Jh = map_and_jacobian_1d(knots, p, H, X[0])
    N, W = Fh[..., :d], Fh[..., d]
    F = N / W[..., None]
    J = (Jh[..., :d, :] - F[..., :, None] * Jh[..., d, None, :]) / W[..., None, None]
    return F, J, W
