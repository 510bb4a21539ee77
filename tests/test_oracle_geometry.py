"""Pins for oracle/geometry.py (CPU only)."""
import numpy as np
import pytest

from oracle.geometry import coefficients_from_jacobian, map_and_jacobian
from workloads import control_net, open_uniform_knots, random_open_knots


def grid(seed, n=5):
    rng = np.random.default_rng(seed)
    return [np.sort(rng.uniform(0.02, 0.98, n)) for _ in range(3)]


@pytest.mark.parametrize("p", [2, 4])
def test_identity_map(p):
    kn = [open_uniform_knots(p, 5), random_open_knots(p, 4, seed=1), open_uniform_knots(p, 3)]
    ctrl = control_net(kn, p, None)
    X = grid(p)
    F, J = (t.astype(np.float64) for t in map_and_jacobian(kn, p, ctrl, *X))
    G = np.stack(np.meshgrid(*X, indexing="ij"), -1)
    assert np.abs(F - G).max() < 1e-14
    assert np.abs(J - np.eye(3)).max() < 1e-13
    det, K = coefficients_from_jacobian(J)
    assert np.abs(det - 1).max() < 1e-13 and np.abs(K - np.eye(3)).max() < 1e-13


def test_affine_map():
    p = 3
    kn = [open_uniform_knots(p, 4)] * 3
    A = np.array([[1.1, 0.4, -0.2], [0.1, 0.8, 0.3], [-0.3, 0.2, 1.3]])
    s = np.array([0.5, -1.0, 2.0])
    ctrl = control_net(kn, p, None, affine=A, shift=s)
    X = grid(7)
    F, J = (t.astype(np.float64) for t in map_and_jacobian(kn, p, ctrl, *X))
    G = np.stack(np.meshgrid(*X, indexing="ij"), -1)
    assert np.abs(F - (G @ A.T + s)).max() < 1e-13
    assert np.abs(J - A).max() < 1e-13
    det, K = coefficients_from_jacobian(J, a=np.full(J.shape[:3], 2.5))
    Ai = np.linalg.inv(A)
    assert np.abs(det - np.linalg.det(A)).max() < 1e-13
    assert np.abs(K - 2.5 * np.linalg.det(A) * Ai @ Ai.T).max() < 1e-12


@pytest.mark.parametrize("twist", [0.0, 30.0])
def test_perturbed_map_fd_and_inverse(twist):
    p = 3
    kn = [open_uniform_knots(p, 6)] * 3
    ctrl = control_net(kn, p, seed=5, twist_deg=twist)
    X = grid(11, 4)
    F, J = (t.astype(np.float64) for t in map_and_jacobian(kn, p, ctrl, *X))
    eps = 1e-6
    for b in range(3):
        Xp = [x.copy() for x in X]
        Xm = [x.copy() for x in X]
        Xp[b] = Xp[b] + eps
        Xm[b] = Xm[b] - eps
        Fp = map_and_jacobian(kn, p, ctrl, *Xp)[0].astype(np.float64)
        Fm = map_and_jacobian(kn, p, ctrl, *Xm)[0].astype(np.float64)
        assert np.abs((Fp - Fm) / (2 * eps) - J[..., :, b]).max() < 1e-6
    det, K = coefficients_from_jacobian(J)
    assert det.min() > 0
    Ji = np.linalg.inv(J)
    ref = np.linalg.det(J)[..., None, None] * Ji @ np.swapaxes(Ji, -1, -2)
    assert np.abs(K - ref).max() < 1e-12 * np.abs(ref).max()


def test_extended_precision_jacobian_is_exact_to_fp64():
    """At rational points the oracle's Jacobian (exact 1D tables, extended
    precision sums) agrees with the exact rational Jacobian to < 1 ulp."""
    from fractions import Fraction as Fr
    from oracle.splines import basis_and_derivs, exact_knots
    p = 4
    kn = [open_uniform_knots(p, 8), random_open_knots(p, 7, seed=4), open_uniform_knots(p, 6)]
    ctrl = control_net(kn, p, seed=8, twist_deg=30.0)
    pts = [[Fr(1, 7), Fr(1, 2), Fr(33, 40)], [Fr(3, 11)], [Fr(5, 9), Fr(1, 64)]]
    _, J = map_and_jacobian(kn, p, ctrl, *pts)
    ek = [exact_knots(list(k)) for k in kn]
    for a1, x1 in enumerate(pts[0]):
        for a2, x2 in enumerate(pts[1]):
            for a3, x3 in enumerate(pts[2]):
                t = [basis_and_derivs(ek[k], p, x) for k, x in enumerate((x1, x2, x3))]
                for b in range(3):
                    for c in range(3):
                        s = Fr(0)
                        for i3 in range(len(t[2][0])):
                            f3 = t[2][1 if b == 2 else 0][i3]
                            if f3 == 0:
                                continue
                            for i2 in range(len(t[1][0])):
                                f2 = t[1][1 if b == 1 else 0][i2]
                                if f2 == 0:
                                    continue
                                for i1 in range(len(t[0][0])):
                                    f1 = t[0][1 if b == 0 else 0][i1]
                                    if f1:
                                        s += Fr(float(ctrl[i3, i2, i1, c])) * f1 * f2 * f3
                        got = float(J[a1, a2, a3, c, b])
                        assert abs(got - float(s)) <= 1.0 * np.spacing(abs(float(s))) + 1e-300
