"""Univariate weighted-quadrature rules for the oracle (test infrastructure only).

* ``quadrature_points`` -- the global point layout of Remark 4.1 (choice of
  quadrature points): all interior knots, the midpoints of the internal
  knot-spans, and p+1 equally spaced points in each of the two boundary
  knot-spans.  Reading used (the remark does not say whether the boundary
  points include the span ends): the p+1 points are strictly inside the span,
  a + k (b - a)/(p + 2), k = 1..p+1, and the domain end points are never
  quadrature points.  With one single knot-span the p+1 strictly interior
  equally spaced points are used.
* ``point_set`` -- Q_i of Section 4: points inside the open support of B_i.
* ``exact_integrals`` -- the four families of eq. (4.2) (label
  eq:integrals): int_0^1 B_i^(beta) B_j^(alpha), beta = derivative order on
  the test function B_i, alpha = derivative order on the trial function B_j,
  computed exactly per knot-span with the closed Newton-Cotes rule on 2p+1
  equispaced points (exact for the degree <= 2p integrand) in rationals.
* ``wq_weights`` -- Algorithm 2: for every test index i and every pairing,
  the minimum-Euclidean-norm solution of the exactness conditions of
  eq. (4.4) (label eq:exact) restricted to Q_i (eq. 4.5, label eq:support).

Reading of the pairing labels (the paper's labels of eq:integrals and of
eq:quadrule/eq:exact are swapped with respect to each other): a rule
w^(alpha,beta)_{i} integrates against B_i^(beta) (test) and is exact on the
trial functions B_j^(alpha), i.e.
    sum_{q in Q_i} w^(alpha,beta)_{i,q} B_j^(alpha)(x_q) = int B_i^(beta) B_j^(alpha),
for all j in I_i.  This is the only reading under which the rules reproduce
the exact Galerkin matrices for constant coefficients (eq. 4.4's purpose).

The minimum-norm solution is the plain definition: w in range(A^T) with
A w = b, obtained as w = A^T y from any exact solution y of (A A^T) y = b.
Every system is solved in exact rational arithmetic, then rounded to FP64.

Pins (tests/test_oracle_rules.py): the interior weights printed in Section 2
for p = 1, 2, 3 (h/3 [1,1,1]; h/30 [2,7,12,7,2]; h [1/105, 3/35, 5/21, 1/3,
...]), the p = 2 integrals h/120 [1, 26, 66, 26, 1], the printed
non-symmetry example (2.3647 vs 2.3615), moment identities, an independent
SVD-based least-squares solve, and the number of points of Remark 4.1.
"""
from __future__ import annotations

import functools
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .splines import basis_and_derivs, cox_de_boor, distinct_knots, exact_knots, n_basis, overlap_set

PAIRINGS = ((0, 0), (1, 0), (0, 1), (1, 1))  # (alpha = trial order, beta = test order)


def quadrature_points(knots: Sequence, p: int) -> list:
    """Global quadrature points in increasing order (Remark 4.1, reading above).
    Exact if ``knots`` are Fractions."""
    chi = distinct_knots(knots)
    n_el = len(chi) - 1
    if n_el == 1:
        a, b = chi
        return [a + (b - a) * k / (p + 2) for k in range(1, p + 2)]
    pts = []
    a, b = chi[0], chi[1]
    pts += [a + (b - a) * k / (p + 2) for k in range(1, p + 2)]
    for k in range(1, n_el):
        pts.append(chi[k])
        if k < n_el - 1:                       # internal span [chi_k, chi_{k+1}]
            pts.append((chi[k] + chi[k + 1]) / 2)
    a, b = chi[n_el - 1], chi[n_el]
    pts += [a + (b - a) * k / (p + 2) for k in range(1, p + 2)]
    return pts


def point_set(knots: Sequence, p: int, pts: Sequence, i: int) -> List[int]:
    """Q_i: indices q with x_q in the open support (xi_i, xi_{i+p+1})."""
    a, b = knots[i], knots[i + p + 1]
    return [q for q, x in enumerate(pts) if a < x < b]


def newton_cotes_weights(m: int) -> List[Fraction]:
    """Closed Newton-Cotes weights on [0, 1] with m+1 equispaced nodes k/m:
    the exact solution of sum_k c_k (k/m)^e = 1/(e+1), e = 0..m."""
    nodes = [Fraction(k, m) for k in range(m + 1)]
    A = [[t ** e for t in nodes] for e in range(m + 1)]
    rhs = [Fraction(1, e + 1) for e in range(m + 1)]
    return _solve_square(A, rhs)


def _solve_square(A, b):
    """Exact Gauss-Jordan elimination with pivot search (nonsingular A)."""
    n = len(A)
    M = [list(A[r]) + [b[r]] for r in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def min_norm_solve(A: List[list], b: list) -> list:
    """Exact minimum-Euclidean-norm solution of the consistent system A w = b:
    w = A^T y with (A A^T) y = b solved by exact row reduction (free
    variables set to 0).  Raises if the system is inconsistent."""
    r = len(A)
    c = len(A[0])
    G = [[sum(A[a][k] * A[bb][k] for k in range(c)) for bb in range(r)] for a in range(r)]
    M = [G[a][:] + [b[a]] for a in range(r)]
    pivcols = []
    row = 0
    for col in range(r):
        piv = next((k for k in range(row, r) if M[k][col] != 0), None)
        if piv is None:
            continue
        M[row], M[piv] = M[piv], M[row]
        inv = 1 / M[row][col]
        M[row] = [v * inv for v in M[row]]
        for k in range(r):
            if k != row and M[k][col] != 0:
                f = M[k][col]
                M[k] = [vk - f * vr for vk, vr in zip(M[k], M[row])]
        pivcols.append(col)
        row += 1
    for k in range(row, r):
        if M[k][r] != 0:
            raise ValueError("inconsistent exactness system")
    y = [Fraction(0)] * r
    for k, col in enumerate(pivcols):
        y[col] = M[k][r]
    w = [sum(A[a][q] * y[a] for a in range(r)) for q in range(c)]
    for a in range(r):  # exactness check, in exact arithmetic
        if sum(A[a][q] * w[q] for q in range(c)) != b[a]:
            raise ValueError("minimum-norm solve failed the exactness check")
    return w


class UnivariateRules:
    """Everything Algorithms 1-2 compute for one direction, in exact
    arithmetic (Fractions) plus FP64 copies.

    Attributes (0-based indices):
      n, p, knots (Fractions), x (Fractions), x64 (np.float64 array)
      I[i]  list of j in I_i        Q[i]  list of q in Q_i
      B0[i][q], B1[i][q] -- exact values/derivatives of B_i at x_q, q in Q_i
      integ[(alpha,beta)][i][j] -- int B_i^(beta) B_j^(alpha), j in I_i
      w[(alpha,beta)][i] -- exact weights on Q_i (list of Fractions)
      w64[(alpha,beta)][i] -- the same rounded to FP64 (np.ndarray)
    """

    def __init__(self, knots: Sequence, p: int):
        self.p = p
        self.knots = exact_knots(knots)
        self.n = n_basis(self.knots, p)
        self.x = quadrature_points(self.knots, p)
        self.x64 = np.array([float(v) for v in self.x], dtype=np.float64)
        self.I = [overlap_set(self.knots, p, i) for i in range(self.n)]
        self.Q = [point_set(self.knots, p, self.x, i) for i in range(self.n)]
        vals = [basis_and_derivs(self.knots, p, xq) for xq in self.x]  # per point
        # tables of Algorithm 1 at the quadrature points: valsQ[d][j][q]
        self.Bq = [[[vals[q][d][j] for q in range(len(self.x))] for j in range(self.n)]
                   for d in (0, 1)]
        self.integ = exact_integrals(self.knots, p)
        self.w: Dict[Tuple[int, int], list] = {}
        self.w64: Dict[Tuple[int, int], list] = {}
        for (al, be) in PAIRINGS:
            ws, ws64 = [], []
            for i in range(self.n):
                A = [[self.Bq[al][j][q] for q in self.Q[i]] for j in self.I[i]]
                b = [self.integ[(al, be)][i][j] for j in self.I[i]]
                wi = min_norm_solve(A, b)
                ws.append(wi)
                ws64.append(np.array([float(v) for v in wi], dtype=np.float64))
            self.w[(al, be)] = ws
            self.w64[(al, be)] = ws64

    def table64(self, deriv: int) -> np.ndarray:
        """Dense FP64 table B^(deriv)_j(x_q), shape (n, n_qp)."""
        return np.array([[float(v) for v in row] for row in self.Bq[deriv]], dtype=np.float64)


def exact_integrals(knots: Sequence, p: int) -> Dict[Tuple[int, int], List[dict]]:
    """int_0^1 B_i^(beta) B_j^(alpha) for all i and j in I_i, exactly.

    Per knot-span [a, b] the integrand is a polynomial of degree <= 2p, which
    the closed Newton-Cotes rule with 2p+1 equispaced nodes integrates
    exactly; B-splines are evaluated exactly at the rational nodes."""
    knots = exact_knots(knots)
    n = n_basis(knots, p)
    chi = distinct_knots(knots)
    m = max(2 * p, 1)
    cw = newton_cotes_weights(m)
    out = {pr: [dict() for _ in range(n)] for pr in PAIRINGS}
    I = [overlap_set(knots, p, i) for i in range(n)]
    for e in range(len(chi) - 1):
        a, b = chi[e], chi[e + 1]
        nodes = [a + (b - a) * Fraction(k, m) for k in range(m + 1)]
        V = [_span_values(knots, p, a, b, t) for t in nodes]
        for i in range(n):
            if not (knots[i] <= a and b <= knots[i + p + 1]):
                continue
            for j in I[i]:
                if not (knots[j] <= a and b <= knots[j + p + 1]):
                    continue
                for (al, be) in PAIRINGS:
                    s = sum(cw[k] * V[k][be][i] * V[k][al][j] for k in range(m + 1))
                    out[(al, be)][i][j] = out[(al, be)][i].get(j, Fraction(0)) + (b - a) * s
    for pr in PAIRINGS:
        for i in range(n):
            for j in I[i]:
                out[pr][i].setdefault(j, Fraction(0))
    return out


def _span_values(knots, p, a, b, t):
    """Values and derivatives at t of the polynomial pieces the B-splines
    have on the span [a, b]; at the span ends these are the one-sided limits
    from inside the span, as exact integration per span requires."""
    m = len(knots) - 1
    span = max(k for k in range(m) if knots[k] == a and knots[k + 1] == b)
    return cox_de_boor(knots, p, span, t)


@functools.lru_cache(maxsize=16)
def _rules_cached(key: Tuple, p: int) -> UnivariateRules:
    return UnivariateRules([Fraction(n, d) for (n, d) in key], p)


def rules_for(knots: Sequence, p: int) -> UnivariateRules:
    """Cached ``UnivariateRules`` keyed by the exact knot values."""
    key = tuple((f.numerator, f.denominator) for f in exact_knots(list(knots)))
    return _rules_cached(key, p)
