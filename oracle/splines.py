"""Univariate B-splines for the oracle (test infrastructure only).

Cox-de Boor recursion for the values and first derivatives of all degree-p
B-splines of an open knot vector (Section 2 and Section 3 of the paper use
the standard B-spline properties; Algorithm 1 evaluates B and B' at the
quadrature points).  Written generically: the same code runs on Python
floats and on ``fractions.Fraction`` (exact arithmetic).

Pins (tests/test_oracle_splines.py): partition of unity, derivative sum zero,
cardinal values printed in Section 2 (quadratic 1/8, 1/2, 3/4; cubic 1/48,
1/6, 23/48, 2/3), finite differences, mirror symmetry, the support/overlap
index sets against brute force, and the 1D nnz count of Section 3.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence, Tuple


def n_basis(knots: Sequence, p: int) -> int:
    return len(knots) - p - 1


def distinct_knots(knots: Sequence) -> list:
    out = []
    for k in knots:
        if not out or k != out[-1]:
            out.append(k)
    return out


def find_span(knots: Sequence, x) -> int:
    """Index k of the half-open span [xi_k, xi_{k+1}) holding x; the last
    non-empty span is closed on the right (x equal to the domain end)."""
    m = len(knots) - 1
    last = max(k for k in range(m) if knots[k] < knots[k + 1])
    for k in range(m):
        if knots[k] <= x < knots[k + 1]:
            return k
    if x == knots[last + 1]:
        return last
    raise ValueError("point outside the knot vector")


def cox_de_boor(knots: Sequence, p: int, span: int, x) -> Tuple[list, list]:
    """Values and first derivatives at x of the polynomial pieces that the
    degree-p B-splines have on the span [xi_span, xi_{span+1}] (textbook
    Cox-de Boor recursion started from the indicator of that span, 0/0 := 0).
    For x inside the span these are B_i(x), B_i'(x); for x outside it they
    are the extrapolated pieces.  Returns two full-length lists (n entries,
    zero outside span-p..span)."""
    m = len(knots) - 1
    zero = x - x  # 0 in the number type of x
    N = [zero] * m
    N[span] = zero + 1
    prev = N[:]
    for d in range(1, p + 1):
        prev = N[:]
        for i in range(max(0, span - d), min(span, m - d - 1) + 1):
            left = zero
            right = zero
            den_l = knots[i + d] - knots[i]
            den_r = knots[i + d + 1] - knots[i + 1]
            if den_l != 0:
                left = (x - knots[i]) / den_l * prev[i]
            if den_r != 0:
                right = (knots[i + d + 1] - x) / den_r * prev[i + 1]
            N[i] = left + right
    n = m - p
    vals = N[:n]
    ders = [zero] * n
    if p > 0:
        for i in range(max(0, span - p), min(span, n - 1) + 1):
            t = zero
            den_l = knots[i + p] - knots[i]
            den_r = knots[i + p + 1] - knots[i + 1]
            if den_l != 0:
                t = t + p / den_l * prev[i]
            if den_r != 0:
                t = t - p / den_r * prev[i + 1]
            ders[i] = t
    return vals, ders


def basis_and_derivs(knots: Sequence, p: int, x) -> Tuple[list, list]:
    """Values B_i(x) and derivatives B_i'(x), i = 0..n-1, of the degree-p
    B-splines on ``knots`` at x (one-sided from the right at interior knots,
    which is immaterial for the C^{p-1}, p >= 2 splines used here)."""
    return cox_de_boor(knots, p, find_span(knots, x), x)


def support(knots: Sequence, p: int, i: int):
    """Closed hull [xi_i, xi_{i+p+1}] of supp B_i."""
    return knots[i], knots[i + p + 1]


def overlap_set(knots: Sequence, p: int, i: int) -> List[int]:
    """The set I_i of Section 3: indices j with B_i * B_j not identically
    zero, i.e. supports overlapping on an interval of positive length."""
    a_i, b_i = support(knots, p, i)
    out = []
    for j in range(n_basis(knots, p)):
        a_j, b_j = support(knots, p, j)
        if max(a_i, a_j) < min(b_i, b_j):
            out.append(j)
    return out


def exact_knots(knots: Sequence) -> List[Fraction]:
    """The knot values as exact rationals (every float is a dyadic rational)."""
    return [Fraction(k) if not isinstance(k, Fraction) else k for k in knots]
