"""GPU tests of the paper's own assembly design (Sec. 5: Alg. 1 with Fig. 2's thread
mapping; the sparse N x MAX_NZ row layout with neighbour lists, and the dense N x N
output), kept as a baseline: the neighbour lists against the oracle's CSR rows; MAX_NZ = 7
on the 2D triangle meshes; the assembled values, in either layout, against the oracle
under the same 1e-12 scaled rule as every other path."""

import numpy as np
import pytest

import meshgen
import oracle
from tests._util import scaled_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12
PAPER_SIGMA = [np.eye(2), [[0.0, -1.0], [1.0, 0.0]], [[0.0, -1.0], [1.0, 0.0]]]
PAPER_F = [36.0, 0, 0, 0, -2.0, 0, 0, -2.0, 0, 0]


def fem():
    import paper_1802_03433_amd as F

    return F


def _dev(m):
    F = fem()
    dev = torch.device("cuda:0")
    return F.Mesh(torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.conn).to(dev), m.order)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _close(got, ref, scale, what=""):
    ok, worst = scaled_close(got, ref, scale, RTOL)
    assert ok, (what, worst)


@pytest.mark.parametrize("kind", ["tri", "tet"])
def test_neighbour_lists(kind):
    m = meshgen.square_tri(9, seed=1) if kind == "tri" else meshgen.cube_tet(4, seed=1)
    F = fem()
    pat = F.Pattern(_dev(m))
    if kind == "tri":
        assert pat.max_row == 7  # the paper's MAX_NZ for the 2D triangle example
    ln, idx = (_np(t) for t in F.paper_ell(pat, pat.max_row + 2))
    rp, ci = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    assert np.array_equal(ln, np.diff(rp))
    for r in range(m.n_nodes):
        assert np.array_equal(idx[r, : ln[r]], ci[rp[r]: rp[r + 1]])
        assert (idx[r, ln[r]:] == -1).all()
    with pytest.raises(F.FemError) as e:
        F.paper_ell(pat, pat.max_row - 1)
    assert e.value.code == -1


CASES = {
    "tri_sin": lambda F: (meshgen.square_tri(20, seed=2), F.Form("helmholtz", "sinprod"), None, None),
    "tet_sin": lambda F: (meshgen.cube_tet(6, seed=3), F.Form("helmholtz", "sinprod"), None, None),
    "tri_paper": lambda F: (meshgen.square_tri(20, seed=4), F.Form.paper_example(), PAPER_SIGMA, PAPER_F),
    "tet_const": lambda F: (meshgen.cube_tet(5, seed=5), F.Form("helmholtz", "const", load_const=(0.7,)),
                            None, None),
}


def _oracle(m, form, sig, poly, kappa):
    rp, ci = oracle.pattern(m.npe, 1, m.n_nodes, m.conn)
    lc = [0.7] if form.load == "const" else None
    return (rp, ci) + oracle.assemble_p1(m, kappa, form.reaction, form.load, lc, rp, ci,
                                         sigma=sig, poly=poly)


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_layout_parity(name):
    F = fem()
    m, form, sig, poly = CASES[name](F)
    d = _dev(m)
    pat = F.Pattern(d)
    kappa = np.ones(m.n_elems) if sig is not None else meshgen.coefficients(m.n_elems, "helmholtz", seed=9)[0]
    kap = torch.from_numpy(kappa[None]).cuda()
    ell = F.paper_ell(pat)
    v, r = F.assemble_paper(pat, d, form, kap, ell=ell)
    rp, ci, ov, orhs, oav, oar = _oracle(m, form, sig, poly, kappa)
    ln = _np(ell[0])
    vals = _np(v)
    csr = np.concatenate([vals[row, : ln[row]] for row in range(m.n_nodes)])
    _close(csr, ov, oav, "values")
    _close(_np(r), orhs, oar, "rhs")
    # accumulate adds a second assembly
    F.assemble_paper(pat, d, form, kap, ell=ell, values=v, rhs=r, accumulate=True)
    vals2 = _np(v)
    csr2 = np.concatenate([vals2[row, : ln[row]] for row in range(m.n_nodes)])
    _close(csr2, 2 * ov, 2 * oav, "accumulated values")


@pytest.mark.parametrize("name", ["tri_paper", "tet_sin"])
def test_dense_layout_parity(name):
    F = fem()
    m, form, sig, poly = CASES[name](F)
    if m.n_nodes > 2000:
        m = meshgen.square_tri(12, seed=6) if m.dim == 2 else meshgen.cube_tet(4, seed=6)
    d = _dev(m)
    pat = F.Pattern(d)
    kappa = np.ones(m.n_elems) if sig is not None else meshgen.coefficients(m.n_elems, "helmholtz", seed=9)[0]
    v, r = F.assemble_paper(pat, d, form, torch.from_numpy(kappa[None]).cuda())
    rp, ci, ov, orhs, oav, oar = _oracle(m, form, sig, poly, kappa)
    dense = _np(v)
    rows = np.repeat(np.arange(m.n_nodes), np.diff(rp))
    _close(dense[rows, ci], ov, oav, "values")
    mask = np.ones_like(dense, dtype=bool)
    mask[rows, ci] = False
    assert (dense[mask] == 0.0).all()  # nothing outside the pattern
    _close(_np(r), orhs, oar, "rhs")


def test_paper_layout_rejects():
    F = fem()
    m = meshgen.cube_tet(1, 2, seed=1)
    d = _dev(m)
    pat = F.Pattern(d, ncomp=3)
    with pytest.raises(F.FemError) as e:
        F.paper_ell(pat, 200)
    assert e.value.code == -2
    m1 = meshgen.square_tri(3, seed=1)
    d1 = _dev(m1)
    p1 = F.Pattern(d1)
    ln = torch.zeros(m1.n_nodes, dtype=torch.int32, device="cuda")
    idx = torch.zeros((m1.n_nodes, 3), dtype=torch.int32, device="cuda")
    kap = torch.ones((1, m1.n_elems), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FemError) as e:  # max_nz below the longest row
        F.assemble_paper(p1, d1, F.Form("helmholtz", "none"), kap, ell=(ln, idx))
    assert e.value.code == -1


def test_sparse_layout_full_size():
    """The paper's design at the benchmark's size (64^3 x 6 tets, sin load, N x MAX_NZ):
    every stored entry against the oracle."""
    F = fem()
    m = meshgen.cube_tet(64, seed=0)
    d = _dev(m)
    pat = F.Pattern(d)
    kappa = meshgen.coefficients(m.n_elems, "helmholtz", seed=0)
    ell = F.paper_ell(pat)
    v, r = F.assemble_paper(pat, d, F.Form("helmholtz", "sinprod"),
                            torch.from_numpy(kappa).cuda(), ell=ell)
    rp, ci = oracle.pattern(4, 1, m.n_nodes, m.conn)
    ov, orhs, oav, oar = oracle.assemble_p1(m, kappa[0], 1.0, "sinprod", None, rp, ci)
    ln = _np(ell[0])
    vals = _np(v)
    mask = np.arange(vals.shape[1])[None, :] < ln[:, None]
    _close(vals[mask], ov, oav, "values")
    _close(_np(r), orhs, oar, "rhs")
