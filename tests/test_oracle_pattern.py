"""Pins of the oracle's sparsity pattern: nnz closed forms of the structured meshes, a
brute-force dense incidence on tiny meshes, and the paper's MAX_NZ = 7 (Sec. 5)."""

import numpy as np
import pytest

import meshgen
import oracle
from tests._util import read_paper_values


def _brute_dense(n_nodes, conn, ncomp):
    nd = n_nodes * ncomp
    D = np.zeros((nd, nd), dtype=bool)
    for e in range(conn.shape[1]):
        v = conn[:, e]
        for i in v:
            for j in v:
                for a in range(ncomp):
                    for b in range(ncomp):
                        D[ncomp * i + a, ncomp * j + b] = True
    return D


def _csr_to_dense(rowptr, colind, nd):
    D = np.zeros((nd, nd), dtype=bool)
    for r in range(nd):
        cols = colind[rowptr[r]:rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0), "columns must be strictly ascending"
        D[r, cols] = True
    return D


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("kind", ["tri", "tet1", "tet2", "tet2vec"])
def test_pattern_brute_force(kind, n):
    if kind == "tri":
        m, ncomp = meshgen.square_tri(n, seed=n), 1
    elif kind == "tet1":
        m, ncomp = meshgen.cube_tet(n, 1, seed=n), 1
    elif kind == "tet2":
        m, ncomp = meshgen.cube_tet(n, 2, seed=n), 1
    else:
        m, ncomp = meshgen.cube_tet(n, 2, seed=n), 3
    rowptr, colind = oracle.pattern(m.npe, ncomp, m.n_nodes, m.conn)
    nd = m.n_nodes * ncomp
    np.testing.assert_array_equal(_csr_to_dense(rowptr, colind, nd), _brute_dense(m.n_nodes, m.conn, ncomp))


@pytest.mark.parametrize("n", [1, 2, 5, 32])
def test_nnz_closed_form_2d(n):
    m = meshgen.square_tri(n)
    rowptr, _ = oracle.pattern(3, 1, m.n_nodes, m.conn)
    assert rowptr[-1] == 7 * n * n + 6 * n + 1


@pytest.mark.parametrize("n", [1, 2, 3, 8])
def test_nnz_closed_form_3d(n):
    m = meshgen.cube_tet(n, 1)
    rowptr, _ = oracle.pattern(4, 1, m.n_nodes, m.conn)
    assert rowptr[-1] == 15 * n ** 3 + 21 * n ** 2 + 9 * n + 1
    m2 = meshgen.cube_tet(n, 2)
    rp2, _ = oracle.pattern(10, 1, m2.n_nodes, m2.conn)
    assert rp2[-1] == 230 * n ** 3 + 138 * n ** 2 + 24 * n + 1
    rp3, _ = oracle.pattern(10, 3, m2.n_nodes, m2.conn)
    assert rp3[-1] == 9 * rp2[-1]


def test_max_nz_matches_paper():
    """Sec. 5: MAX_NZ = 7 on the 2D P1 example (a node has at most 6 neighbours)."""
    m = meshgen.square_tri(32)
    rowptr, colind = oracle.pattern(3, 1, m.n_nodes, m.conn)
    assert int(np.diff(rowptr).max()) == read_paper_values()["max_nz_2d_p1"]
    # diagonal present in every row
    for r in range(m.n_nodes):
        assert r in colind[rowptr[r]:rowptr[r + 1]]


def test_config_sizes():
    m = meshgen.square_tri(32)
    assert (m.n_nodes, m.n_elems) == (1089, 2048)
    rowptr, _ = oracle.pattern(3, 1, m.n_nodes, m.conn)
    assert rowptr[-1] == 7361
