"""Pins of the oracle's gradients (dL/dcoef exact linear identities; dL/dx by complex
step) against central finite differences of the oracle's own forward assembly, and
against translation invariance and Euler homogeneity of the assembled operators."""

import numpy as np
import pytest

import meshgen
import oracle


def _L_p1(m, kappa, c, load, rowptr, colind, G, g):
    vals, rhs, _, _ = oracle.assemble_p1(m, kappa, c, load, None, rowptr, colind)
    return float(G @ vals + g @ rhs)


@pytest.mark.parametrize("kind,load", [("tri", "sinprod"), ("tet", "sinprod"), ("tet", "none")])
def test_p1_gradients_vs_fd(kind, load):
    m = meshgen.square_tri(3, seed=4) if kind == "tri" else meshgen.cube_tet(2, seed=4)
    kappa = meshgen.coefficients(m.n_elems, "helmholtz", seed=4)[0]
    rowptr, colind = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    G, g = meshgen.upstream_grads(int(rowptr[-1]), m.n_nodes, seed=4)
    if load == "none":
        g = np.zeros_like(g)
    c = 1.0
    dk, _, dx, _ = oracle.backward_p1(m, kappa, c, load, None, rowptr, colind, G, g)
    # kappa: L is affine in kappa -> central difference has no truncation error
    for e in range(0, m.n_elems, max(1, m.n_elems // 7)):
        kp, km = kappa.copy(), kappa.copy()
        kp[e] += 0.5
        km[e] -= 0.5
        fd = _L_p1(m, kp, c, load, rowptr, colind, G, g) - _L_p1(m, km, c, load, rowptr, colind, G, g)
        assert dk[e] == pytest.approx(fd, rel=1e-10, abs=1e-13)
    # coordinates: central FD, step 1e-6
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(12):
        n = int(rng.integers(m.n_nodes))
        a = int(rng.integers(m.dim))
        mp = meshgen.Mesh(m.dim, m.order, m.n, m.coords.copy(), m.conn)
        mm = meshgen.Mesh(m.dim, m.order, m.n, m.coords.copy(), m.conn)
        mp.coords[a, n] += h
        mm.coords[a, n] -= h
        fd = (_L_p1(mp, kappa, c, load, rowptr, colind, G, g)
              - _L_p1(mm, kappa, c, load, rowptr, colind, G, g)) / (2 * h)
        assert dx[a, n] == pytest.approx(fd, rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("kind", ["tri", "tet"])
def test_p1_translation_and_homogeneity(kind):
    """With g = 0: sum_n dL/dx_n = 0 (translation), and sum_n x_n . dL/dx_n =
    (d-2) L_K + d L_M (stiffness scales as h^(d-2), mass as h^d)."""
    m = meshgen.square_tri(4, seed=6) if kind == "tri" else meshgen.cube_tet(3, seed=6)
    kappa = meshgen.coefficients(m.n_elems, "helmholtz", seed=6)[0]
    rowptr, colind = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    G, _ = meshgen.upstream_grads(int(rowptr[-1]), m.n_nodes, seed=6)
    g0 = np.zeros(m.n_nodes)
    _, _, dx, _ = oracle.backward_p1(m, kappa, 1.0, "none", None, rowptr, colind, G, g0)
    np.testing.assert_allclose(dx.sum(1), 0.0, atol=1e-12 * np.abs(dx).max())
    LK = _L_p1(m, kappa, 0.0, "none", rowptr, colind, G, g0)
    LM = _L_p1(m, np.zeros_like(kappa), 1.0, "none", rowptr, colind, G, g0)
    d = m.dim
    assert float(np.sum(m.coords * dx)) == pytest.approx((d - 2) * LK + d * LM, rel=1e-11, abs=1e-13)


def test_p2_gradients_vs_fd():
    m = meshgen.cube_tet(1, 2, seed=8)
    coef = meshgen.coefficients(m.n_elems, "elasticity", seed=8)
    rowptr, colind = oracle.pattern(10, 3, m.n_nodes, m.conn)
    G, g = meshgen.upstream_grads(int(rowptr[-1]), 3 * m.n_nodes, seed=8)
    bf = [0.2, -0.1, -1.0]

    def L(mesh, lam, mu):
        v, r, _, _ = oracle.assemble_p2_elasticity(mesh, lam, mu, "const", bf, rowptr, colind)
        return float(G @ v + g @ r)

    dl, _, dm, _, dx, _ = oracle.backward_p2_elasticity(m, coef[0], coef[1], "const", bf,
                                                         rowptr, colind, G, g)
    for e in range(m.n_elems):
        lp, lm_ = coef[0].copy(), coef[0].copy()
        lp[e] += 0.5
        lm_[e] -= 0.5
        assert dl[e] == pytest.approx(L(m, lp, coef[1]) - L(m, lm_, coef[1]), rel=1e-10)
        mp, mm = coef[1].copy(), coef[1].copy()
        mp[e] += 0.5
        mm[e] -= 0.5
        assert dm[e] == pytest.approx(L(m, coef[0], mp) - L(m, coef[0], mm), rel=1e-10)
    # vertex coordinates (the geometry is affine: it depends on the 4 vertices only;
    # moving a vertex moves nothing else in this test, so FD perturbs vertex nodes)
    h = 1e-6
    vertex_nodes = np.unique(m.conn[:4])
    for n in vertex_nodes[:6]:
        for a in range(3):
            mp = meshgen.Mesh(3, 2, m.n, m.coords.copy(), m.conn)
            mm = meshgen.Mesh(3, 2, m.n, m.coords.copy(), m.conn)
            mp.coords[a, n] += h
            mm.coords[a, n] -= h
            fd = (L(mp, coef[0], coef[1]) - L(mm, coef[0], coef[1])) / (2 * h)
            assert dx[a, n] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # translation invariance with g = 0
    _, _, _, _, dx0, _ = oracle.backward_p2_elasticity(m, coef[0], coef[1], "none", None,
                                                       rowptr, colind, G, None)
    np.testing.assert_allclose(dx0.sum(1), 0.0, atol=1e-12 * np.abs(dx0).max())
    # Euler homogeneity: elasticity stiffness scales as h^(d-2) = h in 3D
    v0, _, _, _ = oracle.assemble_p2_elasticity(m, coef[0], coef[1], "none", None, rowptr, colind)
    assert float(np.sum(m.coords * dx0)) == pytest.approx(float(G @ v0), rel=1e-11)
