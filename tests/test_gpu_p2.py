"""GPU parity of the P2 elasticity path (3-component pattern, MFMA element matrices,
tile scatter) against the CPU oracle, through the C ABI.  FP64: |gpu - oracle| <=
1e-12 * max(|oracle|, sum |element contributions|) per entry plus the normwise rule.
The FP32 matrix-core variant is compared against the FP64 result with its measured
relative error reported, not pinned to 1e-12."""

import numpy as np
import pytest

import meshgen
import oracle
from tests._util import scaled_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12
BF = (0.0, 0.0, -1.0)


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


_cache = {}


def c2():
    """40^3 x 6 P2 tetrahedra (384,000 elements, 531,441 nodes) and the oracle result."""
    if "c2" not in _cache:
        m = meshgen.cube_tet(40, 2, seed=0)
        coef = meshgen.coefficients(m.n_elems, "elasticity", seed=0)
        rp, ci = oracle.pattern(10, 3, m.n_nodes, m.conn)
        ov = oracle.assemble_p2_elasticity(m, coef[0], coef[1], "const", BF, rp, ci)
        _cache["c2"] = (m, coef, rp, ci, ov)
    return _cache["c2"]


@pytest.mark.parametrize("n", [1, 2, 5])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_p2_pattern_bit_exact(n, ncomp):
    m = meshgen.cube_tet(n, 2, seed=n)
    pat = fem().Pattern(_dev(m), ncomp=ncomp)
    rp, ci = oracle.pattern(10, ncomp, m.n_nodes, m.conn)
    grp, gci = (_np(t) for t in pat.export())
    assert pat.nnz == int(rp[-1])
    np.testing.assert_array_equal(grp, rp.astype(np.int32))
    np.testing.assert_array_equal(gci, ci)


@pytest.mark.parametrize("scatter", ["atomic", "coloured"])
@pytest.mark.parametrize("load", ["none", "const"])
@pytest.mark.parametrize("n", [1, 2, 5])
def test_p2_forward_parity(n, load, scatter):
    m = meshgen.cube_tet(n, 2, seed=20 + n)
    F = fem()
    d = _dev(m)
    pat = F.Pattern(d, ncomp=3)
    coef = meshgen.coefficients(m.n_elems, "elasticity", seed=n)
    form = F.Form("elasticity", load, load_const=BF)
    v, r = F.assemble(pat, d, form, torch.from_numpy(coef).cuda(), scatter=scatter)
    rp, ci = oracle.pattern(10, 3, m.n_nodes, m.conn)
    ov, orhs, oav, oar = oracle.assemble_p2_elasticity(m, coef[0], coef[1], load, BF, rp, ci)
    ok, worst = scaled_close(_np(v), ov, oav, RTOL)
    assert ok, worst
    if load == "const":
        ok, worst = scaled_close(_np(r), orhs, oar, RTOL)
        assert ok, worst


@pytest.mark.parametrize("tile", [1, 2, 4, 16])
def test_p2_tile_sizes(tile):
    m = meshgen.cube_tet(3, 2, seed=31)
    F = fem()
    d = _dev(m)
    pat = F.Pattern(d, ncomp=3, tile=tile)
    coef = meshgen.coefficients(m.n_elems, "elasticity", seed=31)
    form = F.Form("elasticity", "const", load_const=BF)
    rp, ci = oracle.pattern(10, 3, m.n_nodes, m.conn)
    ov, orhs, oav, oar = oracle.assemble_p2_elasticity(m, coef[0], coef[1], "const", BF, rp, ci)
    for scatter in ("atomic", "coloured"):
        v, r = F.assemble(pat, d, form, torch.from_numpy(coef).cuda(), scatter=scatter)
        assert scaled_close(_np(v), ov, oav, RTOL)[0]
        assert scaled_close(_np(r), orhs, oar, RTOL)[0]


@pytest.mark.parametrize("scatter", ["atomic", "coloured"])
def test_p2_forward_parity_full_size(scatter):
    m, coef, rp, ci, (ov, orhs, oav, oar) = c2()
    F = fem()
    d = _dev(m)
    pat = F.Pattern(d, ncomp=3)
    assert pat.nnz == 134475849
    form = F.Form("elasticity", "const", load_const=BF)
    v, r = F.assemble(pat, d, form, torch.from_numpy(coef).cuda(), scatter=scatter)
    ok, worst = scaled_close(_np(v), ov, oav, RTOL)
    assert ok, worst
    ok, worst = scaled_close(_np(r), orhs, oar, RTOL)
    assert ok, worst


def test_p2_coloured_bitwise_reproducible():
    m = meshgen.cube_tet(6, 2, seed=5)
    F = fem()
    d = _dev(m)
    coef = torch.from_numpy(meshgen.coefficients(m.n_elems, "elasticity", seed=5)).cuda()
    form = F.Form("elasticity", "const", load_const=BF)
    outs = []
    for _ in range(2):
        pat = F.Pattern(d, ncomp=3)
        for _ in range(2):
            v, r = F.assemble(pat, d, form, coef, scatter="coloured")
            outs.append((_np(v).tobytes(), _np(r).tobytes()))
    assert all(o == outs[0] for o in outs)


def test_p2_rigid_modes_and_symmetry_on_gpu_output():
    """Properties that hold at any size: K annihilates the 6 rigid-body modes (Neumann,
    every row) and is symmetric."""
    import scipy.sparse as sp

    m = meshgen.cube_tet(12, 2, seed=7)
    F = fem()
    d = _dev(m)
    pat = F.Pattern(d, ncomp=3)
    coef = meshgen.coefficients(m.n_elems, "elasticity", seed=7)
    v, _ = F.assemble(pat, d, F.Form("elasticity"), torch.from_numpy(coef).cuda())
    rp, ci = (_np(t) for t in pat.export())
    K = sp.csr_matrix((_np(v), ci, rp), shape=(pat.n_rows, pat.n_rows))
    scale = np.abs(K).max()
    assert abs(K - K.T).max() <= 1e-14 * scale
    X = m.coords.T
    for a in range(3):
        t = np.zeros((m.n_nodes, 3))
        t[:, a] = 1.0
        assert np.abs(K @ t.ravel()).max() <= 1e-12 * scale
    for w in np.eye(3):
        assert np.abs(K @ np.cross(w, X).ravel()).max() <= 1e-12 * scale


def test_p2_fp32_matrix_cores_error():
    """FP32 matrix-core variant: inputs of the contraction rounded to FP32 and FP32
    accumulation; its error against the FP64 result is reported (expected ~1e-7)."""
    m = meshgen.cube_tet(8, 2, seed=9)
    F = fem()
    d = _dev(m)
    pat = F.Pattern(d, ncomp=3)
    coef = torch.from_numpy(meshgen.coefficients(m.n_elems, "elasticity", seed=9)).cuda()
    form = F.Form("elasticity", "const", load_const=BF)
    v64, r64 = F.assemble(pat, d, form, coef)
    v32, r32 = F.assemble(pat, d, form, coef, fp32=True)
    a, b = _np(v64), _np(v32)
    rel = np.linalg.norm(b - a) / np.linalg.norm(a)
    print(f"FP32 matrix cores: ||K32 - K64||_F / ||K64||_F = {rel:.3e}, "
          f"max |dK| / max |K| = {np.abs(b - a).max() / np.abs(a).max():.3e}")
    assert 0 < rel < 1e-5
    # the load is not a contraction: same FP64 arithmetic, up to the atomic summation order
    np.testing.assert_allclose(_np(r32), _np(r64), rtol=1e-13, atol=1e-15)
