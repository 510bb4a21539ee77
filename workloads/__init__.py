"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module only *generates inputs*: knot vectors, control nets of the
geometry map, and the scalar diffusion coefficient a(x).  It contains none
of the weighted-quadrature arithmetic (no quadrature points, no weights, no
assembly), so both the CPU oracle and the HIP path can consume its output
without sharing any of the method's code.

Shapes follow the paper's 3D timing workloads (single tensor-product patch,
maximal regularity C^{p-1}, uniform open knot vectors on [0,1]); the paper
measures on no public dataset, so every input here is synthetic and seeded.

Array conventions
-----------------
* knots: float64, open (end knots repeated p+1 times), length n + p + 1.
* control net: float64 array of shape (n3, n2, n1, 3) in C order, i.e. the
  linear DOF index is i1 + n1*(i2 + n2*i3) (direction 1 fastest, as in the
  paper's linear numbering of multi-indices, Section 3), 3 physical coords.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


def open_uniform_knots(p: int, n_el: int, a: float = 0.0, b: float = 1.0) -> np.ndarray:
    """Open uniform knot vector with n_el equal spans on [a, b] and simple
    interior knots (continuity C^{p-1})."""
    if p < 0 or n_el < 1:
        raise ValueError("need p >= 0 and n_el >= 1")
    inner = [a + (b - a) * k / n_el for k in range(1, n_el)]
    return np.array([a] * (p + 1) + inner + [b] * (p + 1), dtype=np.float64)


def random_open_knots(p: int, n_el: int, seed: int, min_ratio: float = 0.3) -> np.ndarray:
    """Open knot vector on [0,1] with n_el spans of seeded random lengths.

    Span lengths are drawn in [min_ratio, 1] (relative) and normalised, so no
    span is degenerate.  Used to exercise non-uniform knots."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.uniform(min_ratio, 1.0, size=n_el)
    cuts = np.cumsum(lens) / lens.sum()
    inner = list(cuts[:-1])
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1), dtype=np.float64)


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae (averages of p consecutive interior knots of each
    basis function); control points placed there reproduce the identity."""
    n = len(knots) - p - 1
    if p == 0:
        return 0.5 * (knots[:-1] + knots[1:])
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(n)], dtype=np.float64)


def control_net(knots3, p: int, seed: Optional[int], amp_h: float = 0.05,
                twist_deg: float = 0.0, affine: Optional[np.ndarray] = None,
                shift: Optional[np.ndarray] = None) -> np.ndarray:
    """Control net of a trivariate (or, given two knot vectors, bivariate;
    given one, univariate) spline map on the given knots.

    Recipe: Greville points (identity map); optionally an affine map
    x -> A x + s; optionally (3D only) a twist of the (x, y) coordinates
    about the axis (1/2, 1/2, z) by an angle growing linearly in z up to
    ``twist_deg`` degrees at z = 1; then a seeded uniform perturbation
    U(-amp_h*h, amp_h*h) of every coordinate of every control point, h being
    the smallest span length.  ``seed=None`` disables the perturbation.
    Returns float64 of shape (n3, n2, n1, 3), (n2, n1, 2) in 2D or (n1, 1)
    in 1D (a 1D perturbation below h/(2p) keeps the points increasing, so
    that J > 0)."""
    g = [greville(np.asarray(k, dtype=np.float64), p) for k in knots3]
    if len(g) == 1:
        if twist_deg:
            raise ValueError("the twist is defined for 3D nets only")
        P = g[0][:, None].astype(np.float64)
    elif len(g) == 2:
        if twist_deg:
            raise ValueError("the twist is defined for 3D nets only")
        X2, X1 = np.meshgrid(g[1], g[0], indexing="ij")
        P = np.stack([X1, X2], axis=-1).astype(np.float64)
    else:
        X3, X2, X1 = np.meshgrid(g[2], g[1], g[0], indexing="ij")
        P = np.stack([X1, X2, X3], axis=-1).astype(np.float64)
    if affine is not None:
        A = np.asarray(affine, dtype=np.float64)
        P = P @ A.T
        if shift is not None:
            P = P + np.asarray(shift, dtype=np.float64)
    if twist_deg:
        th = np.deg2rad(twist_deg) * P[..., 2]
        cx, cy = P[..., 0] - 0.5, P[..., 1] - 0.5
        P = P.copy()
        P[..., 0] = 0.5 + np.cos(th) * cx - np.sin(th) * cy
        P[..., 1] = 0.5 + np.sin(th) * cx + np.cos(th) * cy
    if seed is not None and amp_h > 0:
        h = min(float(np.min(np.diff(np.unique(np.asarray(k))))) for k in knots3)
        rng = np.random.Generator(np.random.PCG64(seed))
        P = P + rng.uniform(-amp_h * h, amp_h * h, size=P.shape)
    return np.ascontiguousarray(P, dtype=np.float64)


def arcsin_curve_net(knots: np.ndarray, p: int) -> np.ndarray:
    """Control points of the curve map of the 1D test problem (the inverse
    of t = 2 sin x: x(t) = arcsin(t / 2), t in [0, 1], x in [0, pi/6]).

    Recipe: the de Boor-Fix dual functionals applied to the degree-p Taylor
    polynomial of x at the Greville abscissa g_i,
        C_i = (1/p!) sum_r (-1)^r psi_i^(p-r)(g_i) x^(r)(g_i),
        psi_i(y) = prod_{j=1..p} (y - xi_{i+j}),
    a local quasi-interpolant that reproduces polynomials of degree p and
    approximates x to O(h^{p+1}) (O(h^{p+1-k}) in the k-th derivative), and
    keeps both end points.  The derivatives come in closed form:
    x' = (4 - t^2)^{-1/2} and x^(k+1) = P_k(t) (4 - t^2)^{-1/2-k} with
    P_0 = 1, P_{k+1} = (4 - t^2) P_k' + (2k + 1) t P_k.
    Returns float64 (n1, 1)."""
    kn = np.asarray(knots, dtype=np.float64)
    n = kn.size - p - 1
    g = greville(kn, p)
    polys = [np.polynomial.Polynomial([1.0])]
    four = np.polynomial.Polynomial([4.0, 0.0, -1.0])
    tpoly = np.polynomial.Polynomial([0.0, 1.0])
    for k in range(p):
        Pk = polys[-1]
        polys.append(four * Pk.deriv() + (2 * k + 1) * tpoly * Pk)
    C = np.empty((n, 1))
    for i in range(n):
        t = g[i]
        deriv = [math.asin(t / 2.0)] + [polys[k](t) * (4.0 - t * t) ** (-0.5 - k) for k in range(p)]
        psi = np.polynomial.Polynomial.fromroots(kn[i + 1:i + p + 1])
        C[i, 0] = sum((-1) ** r * psi.deriv(p - r)(t) * deriv[r] for r in range(p + 1)) / math.factorial(p)
    return np.ascontiguousarray(C)


@dataclasses.dataclass(frozen=True)
class CoefficientField:
    """a(x) = 1 + 0.5 sin(g(x)), g a low-frequency Fourier sum with seeded
    N(0,1)/|k|^2 amplitudes over k in {0,1,2}^3 minus the origin; a in [0.5, 1.5]."""
    ks: np.ndarray      # (m, 3) integer wave vectors
    alpha: np.ndarray   # (m,)
    beta: np.ndarray    # (m,)

    def torch(self, x):
        """The same field evaluated with torch on x's device (input
        generation on the GPU for large point sets)."""
        import torch
        if x.shape[-1] < 3:
            x = torch.cat([x, torch.zeros(x.shape[:-1] + (3 - x.shape[-1],), dtype=x.dtype, device=x.device)], dim=-1)
        ks = torch.as_tensor(self.ks, dtype=torch.float64, device=x.device)
        ph = 2.0 * math.pi * (x.to(torch.float64) @ ks.T)
        a = torch.as_tensor(self.alpha, device=x.device)
        b = torch.as_tensor(self.beta, device=x.device)
        g = torch.cos(ph) @ a + torch.sin(ph) @ b
        return 1.0 + 0.5 * torch.sin(g)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        if x.shape[-1] < 3:    # a plane or a line: the field on z = 0 (and y = 0)
            x = np.concatenate([x, np.zeros(x.shape[:-1] + (3 - x.shape[-1],))], axis=-1)
        ph = 2.0 * math.pi * (x @ self.ks.T.astype(np.float64))
        g = np.cos(ph) @ self.alpha + np.sin(ph) @ self.beta
        return 1.0 + 0.5 * np.sin(g)


def coefficient_field(seed: int) -> CoefficientField:
    ks = np.array([(a, b, c) for c in range(3) for b in range(3) for a in range(3)
                   if (a, b, c) != (0, 0, 0)], dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    k2 = (ks.astype(np.float64) ** 2).sum(axis=1)
    alpha = rng.standard_normal(len(ks)) / k2
    beta = rng.standard_normal(len(ks)) / k2
    return CoefficientField(ks=ks, alpha=alpha, beta=beta)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic single-patch problem (3D, or 2D when n_el has two
    entries)."""
    name: str
    p: int
    n_el: tuple
    geom_seed: Optional[int]
    coef_seed: Optional[int]     # None => a(x) = 1
    twist_deg: float = 0.0
    which: tuple = ("mass", "stiff")

    def knots(self):
        return [open_uniform_knots(self.p, ne) for ne in self.n_el]

    def ctrl(self):
        return control_net(self.knots(), self.p, self.geom_seed, twist_deg=self.twist_deg)

    def coefficient(self) -> Optional[CoefficientField]:
        return None if self.coef_seed is None else coefficient_field(self.coef_seed)

    def n_dof(self):
        return tuple(ne + self.p for ne in self.n_el)

    def exact_nnz(self) -> int:
        """nnz of the tensor-product pattern: product of the 1D counts
        (2p+1) n - p(p+1) (maximal regularity, open knots)."""
        out = 1
        for n in self.n_dof():
            out *= (2 * self.p + 1) * n - self.p * (self.p + 1)
        return out


# The three single-patch workloads (small oracle-sized case, the p=4
# benchmark case, and the large p=6 twisted case).
SMALL_P2 = Workload("p2_8el_perturbed", 2, (8, 8, 8), geom_seed=1, coef_seed=None,
                    which=("mass", "stiff"))
MID_P4 = Workload("p4_32el_perturbed_coef", 4, (32, 32, 32), geom_seed=2, coef_seed=3,
                  which=("stiff",))
LARGE_P6 = Workload("p6_64el_twisted", 6, (64, 64, 64), geom_seed=4, coef_seed=None,
                    twist_deg=30.0, which=("stiff", "mass"))

# the p = 4..6 x {32^3, 64^3} sweep (same recipe as MID_P4: perturbed
# Greville net, smooth coefficient, stiffness)
SWEEP = tuple(Workload(f"p{p}_{e}el_perturbed_coef", p, (e, e, e), geom_seed=10 + p, coef_seed=20 + p,
                       which=("stiff",))
              for p, e in ((4, 64), (5, 32), (5, 64), (6, 32)))

# plane patches (2D): perturbed Greville nets of the same recipe
PLANE = (Workload("p4_512el_plane", 4, (512, 512), geom_seed=30, coef_seed=31, which=("stiff",)),
         Workload("p6_256el_plane", 6, (256, 256), geom_seed=32, coef_seed=None, which=("stiff", "mass")))

WORKLOADS = {w.name: w for w in (SMALL_P2, MID_P4, LARGE_P6) + SWEEP + PLANE}


def batch_patches(n: int, seed: int, p_range=(2, 6), nel_range=(8, 40), d_choices=(3,), p2d: float = 0.0):
    """n independent single-patch problems of mixed degree and size (a
    batch): p uniform in p_range, elements per direction uniform in
    nel_range (independently per direction), dimension from d_choices (2 with
    probability p2d when both are allowed), each with its own seeded
    perturbed geometry and coefficient field."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        d = 2 if (2 in d_choices and rng.random() < p2d) else 3
        # at least p+2 knot-spans per direction (the method's minimum patch)
        nel = tuple(max(p + 2, int(rng.integers(nel_range[0], nel_range[1] + 1))) for _ in range(d))
        out.append(Workload(f"batch{seed}_{k}", p, nel, geom_seed=1000 * seed + 2 * k + 1,
                            coef_seed=1000 * seed + 2 * k + 2, which=("mass", "stiff")))
    return out


def sample_rows(n_dof3, p: int, n_uniform: int, n_boundary: int, seed: int) -> np.ndarray:
    """Seeded row sample: uniform rows plus rows touching the boundary layers
    (some i_l in {0, 1, p-1, p, n-p-1, n-2, n-1}).  Returns sorted unique
    linear row indices (i1 fastest)."""
    n1, n2, n3 = n_dof3
    rng = np.random.Generator(np.random.PCG64(seed))
    N = n1 * n2 * n3
    rows = set(int(r) for r in rng.integers(0, N, size=n_uniform))
    layers = []
    for n in (n1, n2, n3):
        cand = {0, 1, p - 1, p, n - p - 1, n - 2, n - 1}
        layers.append(sorted(c for c in cand if 0 <= c < n))
    for _ in range(n_boundary):
        idx = [int(rng.integers(0, n)) for n in (n1, n2, n3)]
        d = int(rng.integers(0, 3))
        idx[d] = int(rng.choice(layers[d]))
        if rng.random() < 0.3:   # edges/corners
            d2 = (d + 1 + int(rng.integers(0, 2))) % 3
            idx[d2] = int(rng.choice(layers[d2]))
        rows.add(idx[0] + n1 * (idx[1] + n2 * idx[2]))
    return np.array(sorted(rows), dtype=np.int64)
