"""Pins of the oracle's matrix-coefficient form and quadratic load (Sec. 4.1 Eq. (1)-(2)
with the worked example of Sec. 4.2: sigma(x, y) = [[1, -x-y], [x+y, 1]], lambda = 1,
f = -2(x^2 + y^2) + 36), against closed forms that hold on any mesh of the unit square
or cube: for functions u, v that P1 represents exactly (1, x, y, z),
    v^T A u = int grad v . sigma grad u + c int v u     and    v^T b = int v f,
where row i of A is the test function and column j the trial function.  Also the
reduction sigma = I to the Helmholtz form, a hand-computed reference element, the
vanishing row and column sums of the stiffness part, and the adjoint against central
finite differences of the oracle's own forward assembly."""

import numpy as np
import pytest

import meshgen
import oracle

# the worked example's sigma = S0 + x S_x + y S_y
PAPER_SIGMA = [np.eye(2), [[0.0, -1.0], [1.0, 0.0]], [[0.0, -1.0], [1.0, 0.0]]]
# f = 36 - 2 x^2 - 2 y^2 over (1, x, y, z, x^2, xy, xz, y^2, yz, z^2)
PAPER_F = [36.0, 0, 0, 0, -2.0, 0, 0, -2.0, 0, 0]
POLY_EXP = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1),
            (0, 2, 0), (0, 1, 1), (0, 0, 2)]


def _dense(rowptr, colind, vals, n):
    A = np.zeros((n, n))
    for r in range(n):
        for k in range(rowptr[r], rowptr[r + 1]):
            A[r, colind[k]] += vals[k]
    return A


def _box_moment(e):
    """int over [0,1]^3 of x^e0 y^e1 z^e2."""
    return float(np.prod([1.0 / (k + 1) for k in e]))


def _assemble(m, sigma, c, load="none", poly=None, kappa=None):
    rp, ci = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    if kappa is None:
        kappa = np.ones(m.n_elems)
    v, b, _, _ = oracle.assemble_p1(m, kappa, c, load, None, rp, ci, sigma=sigma, poly=poly)
    return _dense(rp, ci, v, m.n_nodes), b


@pytest.mark.parametrize("n,seed", [(3, 1), (6, 2)])
def test_paper_form_on_linear_functions(n, seed):
    m = meshgen.square_tri(n, seed=seed)
    A, _ = _assemble(m, PAPER_SIGMA, 1.0)
    x, y, one = m.coords[0], m.coords[1], np.ones(m.n_nodes)
    # int sigma_11 = int sigma_22 = 1, int sigma_21 = int (x + y) = 1, int sigma_12 = -1;
    # int x^2 = 1/3, int xy = 1/4, int x = 1/2, |Omega| = 1
    assert x @ A @ x == pytest.approx(1.0 + 1.0 / 3.0, rel=1e-13)
    assert y @ A @ y == pytest.approx(1.0 + 1.0 / 3.0, rel=1e-13)
    assert y @ A @ x == pytest.approx(1.0 + 0.25, rel=1e-13)
    assert x @ A @ y == pytest.approx(-1.0 + 0.25, rel=1e-13)
    assert one @ A @ one == pytest.approx(1.0, rel=1e-13)
    assert one @ A @ x == pytest.approx(0.5, rel=1e-13)
    assert x @ A @ one == pytest.approx(0.5, rel=1e-13)


def test_paper_load_moments():
    m = meshgen.square_tri(5, seed=3)
    _, b = _assemble(m, PAPER_SIGMA, 1.0, "poly2", PAPER_F)
    x, y = m.coords[0], m.coords[1]
    # int f = 36 - 2/3 - 2/3;  int x f = 18 - 2/4 - 2/6;  int y f likewise
    assert b.sum() == pytest.approx(36.0 - 4.0 / 3.0, rel=1e-13)
    assert x @ b == pytest.approx(18.0 - 0.5 - 1.0 / 3.0, rel=1e-13)
    assert y @ b == pytest.approx(18.0 - 0.5 - 1.0 / 3.0, rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_general_affine_sigma_and_quadratic_load(dim):
    rng = np.random.default_rng(10 + dim)
    sig = rng.normal(size=(4, 3, 3))
    if dim == 2:
        sig[3] = 0.0
    poly = rng.normal(size=10)
    if dim == 2:
        poly[[3, 6, 8, 9]] = 0.0
    c = 0.7
    m = meshgen.square_tri(4, seed=5) if dim == 2 else meshgen.cube_tet(2, seed=5)
    A, b = _assemble(m, sig, c, "poly2", poly)
    X = [m.coords[a] for a in range(dim)]
    for a in range(dim):
        for q in range(dim):
            # int sigma_aq over the unit box: S0 + sum_k S_k / 2
            isig = sig[0, a, q] + 0.5 * sum(sig[1 + k, a, q] for k in range(dim))
            e = [0, 0, 0]
            e[a] += 1
            e[q] += 1
            assert X[a] @ A @ X[q] == pytest.approx(isig + c * _box_moment(e), rel=1e-12)
    moments = lambda shift: sum(poly[k] * _box_moment(np.add(POLY_EXP[k], shift))
                                for k in range(10))
    assert b.sum() == pytest.approx(moments((0, 0, 0)), rel=1e-12)
    for a in range(dim):
        sh = [0, 0, 0]
        sh[a] = 1
        assert X[a] @ b == pytest.approx(moments(sh), rel=1e-12)
    # stiffness rows and columns sum to zero: A 1 = A^T 1 = c (int l_i)
    _, bl = _assemble(m, sig, c, "poly2", [c])
    np.testing.assert_allclose(A.sum(1), bl, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(A.sum(0), bl, rtol=1e-12, atol=1e-14)


def test_reference_triangle_by_hand():
    """Constant sigma on (0,0), (1,0), (0,1): grad l = (-1,-1), (1,0), (0,1), |T| = 1/2,
    so A_ij = (1/2) grad l_i . sigma grad l_j."""
    s = np.array([[2.0, 3.0], [5.0, 7.0]])
    A = oracle.element_p1_sigma([[0, 0], [1, 0], [0, 1]], [s], kappa=1.0)
    assert A[1, 2] == 0.5 * 3.0 and A[2, 1] == 0.5 * 5.0
    assert A[1, 1] == 0.5 * 2.0 and A[2, 2] == 0.5 * 7.0
    assert A[0, 0] == 0.5 * (2.0 + 3.0 + 5.0 + 7.0)
    assert A[0, 1] == -0.5 * (2.0 + 5.0) and A[1, 0] == -0.5 * (2.0 + 3.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_identity_sigma_is_helmholtz(dim):
    m = meshgen.square_tri(4, seed=7) if dim == 2 else meshgen.cube_tet(2, seed=7)
    kappa = meshgen.coefficients(m.n_elems, "helmholtz", seed=7)[0]
    rp, ci = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    eye = [np.eye(3)]
    v1, b1, _, _ = oracle.assemble_p1(m, kappa, 1.3, "const", [2.5], rp, ci)
    v2, b2, _, _ = oracle.assemble_p1(m, kappa, 1.3, "poly2", None, rp, ci, sigma=eye,
                                      poly=[2.5])
    np.testing.assert_allclose(v2, v1, rtol=1e-14, atol=1e-15 * np.abs(v1).max())
    np.testing.assert_allclose(b2, b1, rtol=1e-14)


def _L(m, kappa, c, sig, poly, rp, ci, G, g):
    v, b, _, _ = oracle.assemble_p1(m, kappa, c, "poly2", None, rp, ci, sigma=sig, poly=poly)
    return float(G @ v + g @ b)


@pytest.mark.parametrize("dim", [2, 3])
def test_sigma_gradients_vs_fd(dim):
    rng = np.random.default_rng(20 + dim)
    sig = rng.normal(size=(4, 3, 3))
    poly = rng.normal(size=10)
    m = meshgen.square_tri(3, seed=8) if dim == 2 else meshgen.cube_tet(2, seed=8)
    kappa = meshgen.coefficients(m.n_elems, "helmholtz", seed=8)[0]
    rp, ci = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    G, g = meshgen.upstream_grads(int(rp[-1]), m.n_nodes, seed=8)
    c = 0.9
    dk, _, dx, _ = oracle.backward_p1(m, kappa, c, "poly2", None, rp, ci, G, g, sigma=sig,
                                      poly=poly)
    for e in range(0, m.n_elems, max(1, m.n_elems // 7)):
        kp, km = kappa.copy(), kappa.copy()
        kp[e] += 0.5
        km[e] -= 0.5
        fd = _L(m, kp, c, sig, poly, rp, ci, G, g) - _L(m, km, c, sig, poly, rp, ci, G, g)
        assert dk[e] == pytest.approx(fd, rel=1e-10, abs=1e-13)
    h = 1e-6
    for _ in range(12):
        n = int(rng.integers(m.n_nodes))
        a = int(rng.integers(dim))
        mp = meshgen.Mesh(m.dim, m.order, m.n, m.coords.copy(), m.conn)
        mm = meshgen.Mesh(m.dim, m.order, m.n, m.coords.copy(), m.conn)
        mp.coords[a, n] += h
        mm.coords[a, n] -= h
        fd = (_L(mp, kappa, c, sig, poly, rp, ci, G, g)
              - _L(mm, kappa, c, sig, poly, rp, ci, G, g)) / (2 * h)
        assert dx[a, n] == pytest.approx(fd, rel=1e-6, abs=1e-8)
