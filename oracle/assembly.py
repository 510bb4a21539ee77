"""Row-by-row formation of the WQ mass and stiffness matrices, for the oracle
(test infrastructure only).

Conventions (0-based): the row index is the test function i, the column the
trial function j (the weights belong to the test function, Section 2); the
linear index of (i1, i2, i3) is i1 + n1 (i2 + n2 i3) (Section 3, direction 1
fastest); columns of a row are in increasing linear order.  No symmetrisation
and no boundary conditions.

* ``Problem.row(..., method="direct")`` -- the plain nested WQ sum of
  eq. (6.2) (label eq:massquadrature): for every j in I_i, the sum over
  q in Q_i of the product over directions of w_{k,i_k,q_k} B_{j_k}(x_{q_k})
  times the coefficient at x_q, written as one unfactorized sum.  For the
  stiffness, the analogue from eq. (3.3) (label eq:stiff): the sum over the
  d^2 pairs (l, m) (l = derivative direction of the test function, m = of the
  trial function) where direction k uses the rule w^(alpha_k, beta_k) with
  alpha_k = [k == m] (trial) and beta_k = [k == l] (test), the trial factor
  B^(alpha_k)_{j_k}, and the coefficient c_lm.
* ``Problem.row(..., method="sumfact")`` -- Algorithm 3 (eq. 6.3, label
  eq:sumfactorization): C_i x_3 (B W)_3 x_2 (B W)_2 x_1 (B W)_1 as successive
  mode products; the stiffness is the sum of the d^2 such products.
* ``Problem.sgq_matrices`` -- element-wise standard Gauss quadrature (SGQ,
  Section 1) with p+1 Gauss-Legendre points per direction and element; exact
  for affine maps and constant coefficients, used by the exactness pins.

The same definitions in d = 2 (two directions, d^2 = 4 stiffness terms) are
taken when two knot vectors are given, and in d = 1 (one direction, one
stiffness term with K = a / J: the problem of Section 7.1) when one is.

NURBS (the generalisation Section 3 names, with the polynomial denominator
in the factor c): a rational map (weights given) changes only J; with
basis="nurbs" the mass of the rational functions R_i = w_i B_i / W is the
B-spline row with c = det J / W^2, scaled by w_i w_j.

Pins (tests/test_oracle_assembly.py): direct == sum-factorized (the identity
between eq:massquadrature and eq:sumfactorization), affine exactness against
a closed Kronecker formula of exact 1D integrals and against SGQ, S 1 = 0,
mass row sums, total mass = volume, the nnz formula of Section 3.
"""
from __future__ import annotations

from typing import Callable, Optional, Sequence

import numpy as np

from .geometry import (coefficients_from_jacobian, coefficients_from_jacobian_1d, coefficients_from_jacobian_2d,
                       map_and_jacobian, map_and_jacobian_1d, map_and_jacobian_2d, rational_map_and_jacobian)
from .rules import rules_for


def mode_product(X: np.ndarray, A: np.ndarray, m: int) -> np.ndarray:
    """(X x_m A)[..., k_m, ...] = sum_j A[k_m, j] X[..., j, ...]  (Section 6)."""
    return np.moveaxis(np.tensordot(A, X, axes=(1, m)), 0, m)


class Problem:
    """One single-patch problem in d = 3 (or d = 2, or d = 1) dimensions:
    knots, degree, control net, coefficient."""

    def __init__(self, knots3: Sequence, p: int, ctrl: np.ndarray,
                 coef: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                 weights: Optional[np.ndarray] = None, basis: str = "bspline"):
        """weights: NURBS weights of the control points (shape of the net
        without its last axis) for a rational map, else None.  basis:
        "bspline" (test and trial functions B_i, on any map) or "nurbs" (the
        rational functions R_i = w_i B_i / W of the same net, mass only:
        m_ij = w_i w_j int B_i B_j det J / W^2, the denominator folded into
        the factor c as Section 3 describes)."""
        d = len(knots3)
        if d not in (1, 2, 3):
            raise ValueError("1D, 2D or 3D problems only")
        self.d = d
        self.p = p
        self.knots3 = [np.asarray(k, dtype=np.float64) for k in knots3]
        self.rules = [rules_for(list(k), p) for k in self.knots3]
        self.n = tuple(r.n for r in self.rules)
        self.ctrl = np.asarray(ctrl, dtype=np.float64)
        if self.ctrl.shape != tuple(reversed(self.n)) + (d,):
            raise ValueError("control net shape must be (n_d, ..., n1, d)")
        self.coef = coef
        self.weights = None if weights is None else np.asarray(weights, dtype=np.float64)
        if self.weights is not None and self.weights.shape != self.ctrl.shape[:-1]:
            raise ValueError("weights must have the shape of the control net without its last axis")
        if basis not in ("bspline", "nurbs") or (basis == "nurbs" and self.weights is None):
            raise ValueError("basis 'nurbs' needs weights")
        self.basis = basis
        self.B = [(r.table64(0), r.table64(1)) for r in self.rules]

    # ---- indices ---------------------------------------------------------
    def multi(self, row: int):
        out = []
        for nk in self.n:
            out.append(row % nk)
            row //= nk
        return tuple(out)

    def linear(self, idx) -> int:
        r, s = 0, 1
        for k, nk in enumerate(self.n):
            r += idx[k] * s
            s *= nk
        return r

    def row_columns(self, row: int) -> np.ndarray:
        i = self.multi(row)
        I = [self.rules[k].I[i[k]] for k in range(self.d)]
        # direction 1 fastest: iterate the last direction outermost
        cols = [0]
        stride = 1
        strides = []
        for nk in self.n:
            strides.append(stride)
            stride *= nk
        for k in reversed(range(self.d)):
            cols = [c + j * strides[k] for c in cols for j in I[k]]
        return np.array(cols, dtype=np.int64)

    def csr_pattern(self):
        N = int(np.prod(self.n))
        cols = [self.row_columns(r) for r in range(N)]
        row_ptr = np.zeros(N + 1, dtype=np.int64)
        row_ptr[1:] = np.cumsum([len(c) for c in cols])
        return row_ptr, np.concatenate(cols).astype(np.int32)

    # ---- per-row data ----------------------------------------------------
    def operator(self, k: int, ik: int, alpha: int, beta: int) -> np.ndarray:
        """B^(k,ik) W^(k,ik) of Section 6 for pairing (alpha, beta):
        T[j, q] = B^(alpha)_j(x_q) w^(alpha,beta)_{ik,q}, j in I_ik, q in Q_ik."""
        r = self.rules[k]
        Bt = self.B[k][alpha][np.ix_(r.I[ik], r.Q[ik])]
        return Bt * r.w64[(alpha, beta)][ik][None, :]

    GRID_LIMIT = 100_000   # quadrature grids up to this size are evaluated once

    def _geometry(self, X):
        """(F, J) at the grid X; for a rational map also W (else None)."""
        if self.weights is not None:
            return rational_map_and_jacobian(self.knots3, self.p, self.ctrl, self.weights, X)
        return self._polynomial_geometry(X) + (None,)

    def _polynomial_geometry(self, X):
        if self.d == 3:
            return map_and_jacobian(self.knots3, self.p, self.ctrl, X[0], X[1], X[2])
        if self.d == 2:
            return map_and_jacobian_2d(self.knots3, self.p, self.ctrl, X[0], X[1])
        return map_and_jacobian_1d(self.knots3, self.p, self.ctrl, X[0])

    def _coefficients(self, J, a):
        return {3: coefficients_from_jacobian, 2: coefficients_from_jacobian_2d,
                1: coefficients_from_jacobian_1d}[self.d](J, a)

    def _fields_on(self, X):
        F, J, W = self._geometry(X)
        F = F.astype(np.float64)
        d = self.d
        a = None if self.coef is None else self.coef(F.reshape(-1, d)).reshape(F.shape[:d])
        det, K = self._coefficients(J, a)
        if self.basis == "nurbs":
            det = det / (W * W)
        return det.astype(np.float64), K.astype(np.float64), F

    def row_fields(self, row: int):
        """Coefficients on the block Q_i1 x ... x Q_id (arrays indexed
        [q1, ..., qd]): mass factor det J, stiffness K (d x d), and F,
        evaluated at the exact quadrature points (on the whole grid at once
        when it is small, else on the row's block)."""
        i = self.multi(row)
        Q = [self.rules[k].Q[i[k]] for k in range(self.d)]
        last = getattr(self, "_last", None)
        if last is not None and last[0] == row:
            return last[1]
        if np.prod([len(r.x) for r in self.rules]) <= self.GRID_LIMIT:
            if getattr(self, "_grid", None) is None:
                self._grid = self._fields_on([r.x for r in self.rules])
            det, K, F = self._grid
            s = tuple(slice(q[0], q[-1] + 1) for q in Q)
            return det[s], K[s], F[s]
        out = self._fields_on([[self.rules[k].x[q] for q in Q[k]] for k in range(self.d)])
        self._last = (row, out)
        return out

    # ---- formation ---------------------------------------------------------
    def row(self, row: int, which: str, method: str = "sumfact") -> np.ndarray:
        """Values of the row in increasing column order."""
        d = self.d
        i = self.multi(row)
        det, K, _ = self.row_fields(row)
        if which == "mass":
            terms = [((0,) * d, (0,) * d, det)]
        elif which == "stiff" and self.basis == "nurbs":
            raise NotImplementedError("stiffness with NURBS test and trial functions")
        elif which == "stiff":
            terms = []
            for l in range(d):          # test-function derivative direction
                for m in range(d):      # trial-function derivative direction
                    al = tuple(int(k == m) for k in range(d))
                    be = tuple(int(k == l) for k in range(d))
                    terms.append((al, be, K[..., l, m]))
        else:
            raise ValueError(which)
        out = None
        for al, be, field in terms:
            T = [self.operator(k, i[k], al[k], be[k]) for k in range(d)]
            if method == "direct":
                if d == 3:
                    v = np.einsum("ax,by,cz,xyz->abc", T[0], T[1], T[2], field, optimize=False)
                elif d == 2:
                    v = np.einsum("ax,by,xy->ab", T[0], T[1], field, optimize=False)
                else:
                    v = np.einsum("ax,x->a", T[0], field, optimize=False)
            elif method == "sumfact":
                v = field
                for k in reversed(range(d)):
                    v = mode_product(v, T[k], k)
            else:
                raise ValueError(method)
            out = v if out is None else out + v
        # [j1, ..., jd] -> increasing linear column order (j1 fastest)
        vals = np.ascontiguousarray(out.transpose(tuple(reversed(range(d))))).ravel()
        if self.basis == "nurbs":   # R_i R_j = w_i w_j B_i B_j / W^2
            w = self.weights.ravel()
            vals = vals * w[row] * w[self.row_columns(row)]
        return vals

    def assemble(self, which: str, method: str = "sumfact") -> np.ndarray:
        N = int(np.prod(self.n))
        return np.concatenate([self.row(r, which, method) for r in range(N)])

    # ---- element-wise standard Gauss quadrature (SGQ) -------------------
    def sgq_matrices(self, which: str, n_gauss: Optional[int] = None) -> np.ndarray:
        """Dense N x N Galerkin matrix by element-wise Gauss-Legendre quadrature
        with n_gauss (default p+1) points per direction per element."""
        d = self.d
        ng = self.p + 1 if n_gauss is None else n_gauss
        gx, gw = np.polynomial.legendre.leggauss(ng)
        pts, wts = [], []
        for k in range(d):
            chi = np.unique(self.knots3[k])
            P, W = [], []
            for e in range(len(chi) - 1):
                a, b = chi[e], chi[e + 1]
                P.append(0.5 * (a + b) + 0.5 * (b - a) * gx)
                W.append(0.5 * (b - a) * gw)
            pts.append(np.concatenate(P))
            wts.append(np.concatenate(W))
        F, J, W = self._geometry(pts)
        F = F.astype(np.float64)
        a = None if self.coef is None else self.coef(F.reshape(-1, d)).reshape(F.shape[:d])
        det, K = self._coefficients(J, a)
        if self.basis == "nurbs":
            if which != "mass":
                raise NotImplementedError("stiffness with NURBS test and trial functions")
            det = det / (W * W)
        det, K = det.astype(np.float64), K.astype(np.float64)
        if d == 3:
            Wq = wts[0][:, None, None] * wts[1][None, :, None] * wts[2][None, None, :]
        elif d == 2:
            Wq = wts[0][:, None] * wts[1][None, :]
        else:
            Wq = wts[0]
        # dense basis tables at Gauss points
        from .splines import basis_and_derivs
        tabs = []
        for k in range(d):
            V = np.array([basis_and_derivs(list(self.knots3[k]), self.p, float(x))[0] for x in pts[k]])
            D = np.array([basis_and_derivs(list(self.knots3[k]), self.p, float(x))[1] for x in pts[k]])
            tabs.append((V.T, D.T))   # (n_k, n_gauss_total)
        N = int(np.prod(self.n))

        def phi(dirs_deriv):
            # values of all N tensor basis functions at all points, flattened
            A = [tabs[k][dirs_deriv[k]] for k in range(d)]
            if d == 3:
                T = np.einsum("ix,jy,kz->kjixyz", A[0], A[1], A[2])
            elif d == 2:
                T = np.einsum("ix,jy->jixy", A[0], A[1])
            else:
                T = A[0]
            return T.reshape(N, -1)
        if which == "mass":
            P0 = phi((0,) * d)
            M = (P0 * (Wq * det).ravel()[None, :]) @ P0.T
            if self.basis == "nurbs":
                w = self.weights.ravel()
                M = M * w[:, None] * w[None, :]
            return M
        G = [phi(tuple(int(k == dd) for k in range(d))) for dd in range(d)]
        S = np.zeros((N, N))
        for l in range(d):
            for m in range(d):
                S += (G[l] * (Wq * K[..., l, m]).ravel()[None, :]) @ G[m].T
        return S
