"""Pins of the oracle's element routines against closed forms and invariants.

P1: textbook reference-element matrices (tests/golden/reference_elements.txt), affine
scaling laws, rotation invariance.  P2 elasticity: rigid-body null space and the strain
energy of quadratic displacement fields integrated directly from their analytic
gradients (no basis functions on the test side).
"""

import math

import numpy as np
import pytest

import oracle
from tests._util import duffy_rule, read_reference_elements

REF = read_reference_elements()
TRI = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
TET = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])


def _rand_simplex(d, rng):
    while True:
        x = rng.uniform(-1, 1, size=(d + 1, d))
        J = (x[1:] - x[0]).T
        if abs(np.linalg.det(J)) > 0.2:
            return x


def test_reference_triangle():
    np.testing.assert_allclose(oracle.element_p1(TRI, 1.0, 0.0), REF["tri_K"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.element_p1(TRI, 0.0, 1.0), REF["tri_M"], rtol=0, atol=1e-16)


def test_reference_tet():
    np.testing.assert_allclose(oracle.element_p1(TET, 1.0, 0.0), REF["tet_K"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.element_p1(TET, 0.0, 1.0), REF["tet_M"], rtol=0, atol=1e-17)


def test_orientation_does_not_matter():
    # swapping two vertices flips det J; |det J| keeps the matrix (permuted) the same
    A = oracle.element_p1(TET, 1.3, 0.7)
    B = oracle.element_p1(TET[[1, 0, 2, 3]], 1.3, 0.7)
    P = np.eye(4)[[1, 0, 2, 3]]
    np.testing.assert_allclose(P @ A @ P.T, B, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_p1_scaling_and_rotation(d):
    rng = np.random.default_rng(7)
    x = _rand_simplex(d, rng)
    K = oracle.element_p1(x, 1.0, 0.0)
    M = oracle.element_p1(x, 0.0, 1.0)
    s = 0.37
    np.testing.assert_allclose(oracle.element_p1(s * x + 3.0, 1.0, 0.0), s ** (d - 2) * K, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(oracle.element_p1(s * x - 1.0, 0.0, 1.0), s ** d * M, rtol=1e-12, atol=1e-16)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    np.testing.assert_allclose(oracle.element_p1(x @ Q.T, 1.0, 0.0), K, rtol=1e-12, atol=1e-13)
    # K annihilates constants and is symmetric positive semidefinite of rank d
    np.testing.assert_allclose(K.sum(1), 0.0, atol=1e-13)
    np.testing.assert_allclose(K, K.T, atol=0)
    ev = np.linalg.eigvalsh(K)
    assert ev[0] == pytest.approx(0.0, abs=1e-12) and ev[1] > 0
    # mass: total = volume
    vol = abs(np.linalg.det((x[1:] - x[0]).T)) / math.factorial(d)
    assert M.sum() == pytest.approx(vol, rel=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_p1_energy_of_affine_field(d):
    """u^T K u = |grad u|^2 |T| for affine u (kappa = 1)."""
    rng = np.random.default_rng(11)
    x = _rand_simplex(d, rng)
    a = rng.standard_normal(d)
    u = x @ a + 0.3
    K = oracle.element_p1(x, 1.0, 0.0)
    vol = abs(np.linalg.det((x[1:] - x[0]).T)) / math.factorial(d)
    assert u @ K @ u == pytest.approx(a @ a * vol, rel=1e-12)


# --------------------------------------------------------------------------- P2 elasticity
P2_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _p2_nodes(xv):
    return np.concatenate([xv, np.array([(xv[a] + xv[b]) / 2 for a, b in P2_EDGES])])


def _quadratic_field(rng):
    """u(x) = c + L x + [x^T H_a x]_a; returns (u(x) for x [m][3], grad u [m][3][3])."""
    c = rng.standard_normal(3)
    L = rng.standard_normal((3, 3))
    H = rng.standard_normal((3, 3, 3))
    H = 0.5 * (H + H.transpose(0, 2, 1))

    def u(x):
        return c + x @ L.T + np.einsum("mi,aij,mj->ma", x, H, x)

    def grad(x):  # grad[m][a][i] = d u_a / d x_i
        return L[None] + 2 * np.einsum("aij,mj->mai", H, x)

    return u, grad


def _energy(xv, lam, mu, grad):
    """int_T lam (div u)^2 + 2 mu eps:eps by collapsed Gauss-Legendre on the element."""
    pts, w = duffy_rule(3, 6)
    J = (xv[1:] - xv[0]).T
    X = xv[0] + pts @ J.T
    g = grad(X)
    eps = 0.5 * (g + g.transpose(0, 2, 1))
    div = np.trace(g, axis1=1, axis2=2)
    dens = lam * div ** 2 + 2 * mu * np.einsum("mij,mij->m", eps, eps)
    return float(np.sum(w * dens)) * abs(np.linalg.det(J))


def test_p2_elasticity_energy_of_quadratic_fields():
    rng = np.random.default_rng(3)
    for _ in range(5):
        xv = _rand_simplex(3, rng)
        lam, mu = rng.uniform(0.5, 2), rng.uniform(0.3, 1)
        K = oracle.element_p2_elasticity(xv, lam, mu)
        u, grad = _quadratic_field(rng)
        U = u(_p2_nodes(xv)).ravel()  # dof 3*i + a
        assert U @ K @ U == pytest.approx(_energy(xv, lam, mu, grad), rel=1e-11)


def test_p2_elasticity_polarisation():
    """Bilinear form check: U^T K V against the polarised energy of two fields."""
    rng = np.random.default_rng(5)
    xv = _rand_simplex(3, rng)
    lam, mu = 1.1, 0.6
    K = oracle.element_p2_elasticity(xv, lam, mu)
    u1, g1 = _quadratic_field(rng)
    u2, g2 = _quadratic_field(rng)
    nodes = _p2_nodes(xv)
    U, V = u1(nodes).ravel(), u2(nodes).ravel()

    def gsum(x):
        return g1(x) + g2(x)

    def gdiff(x):
        return g1(x) - g2(x)

    ref = 0.25 * (_energy(xv, lam, mu, gsum) - _energy(xv, lam, mu, gdiff))
    assert U @ K @ V == pytest.approx(ref, rel=1e-11)
    np.testing.assert_allclose(K, K.T, atol=1e-13 * np.abs(K).max())


def test_p2_rigid_body_modes():
    rng = np.random.default_rng(9)
    xv = _rand_simplex(3, rng)
    K = oracle.element_p2_elasticity(xv, 1.7, 0.4)
    nodes = _p2_nodes(xv)
    modes = []
    for a in range(3):
        t = np.zeros((10, 3))
        t[:, a] = 1
        modes.append(t.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w, nodes).ravel())
    for m in modes:
        np.testing.assert_allclose(K @ m, 0.0, atol=1e-12 * np.abs(K).max())
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6


def test_p2_lambda_mu_linear():
    rng = np.random.default_rng(1)
    xv = _rand_simplex(3, rng)
    K1 = oracle.element_p2_elasticity(xv, 1.0, 0.0)
    K2 = oracle.element_p2_elasticity(xv, 0.0, 1.0)
    np.testing.assert_allclose(oracle.element_p2_elasticity(xv, 0.7, 0.2), 0.7 * K1 + 0.2 * K2,
                               rtol=1e-13, atol=1e-14)


def test_p2_basis_means():
    """(1/|T|) int phi: -1/20 at vertices, 1/5 at edge nodes (textbook P2 values)."""
    np.testing.assert_allclose(oracle.p2_phi_mean(), [-0.05] * 4 + [0.2] * 6, rtol=1e-14)
