"""Pins of the oracle's hopping matrices and ELL export (Sec. 2.1, Fig. 2)."""

import math

import numpy as np
import pytest

from oracle.basis import basis_states
from oracle.fock import sector_block
from oracle.hamiltonian import Model
from oracle.hopping import ell_flatten, hopping_matrix, to_ell
from synth import ring_bonds, torus_bonds, two_site_bonds
from tests.golden.load import ell_fig2


def test_ell_fig2_worked_example():
    g = ell_fig2()
    data, ind, width = to_ell(g["A"])
    assert width == 3
    assert np.array_equal(data, g["data"])
    assert np.array_equal(ind, g["indices"])
    assert np.array_equal(ell_flatten(data, "col"), g["data_colmajor"])
    assert np.array_equal(ell_flatten(ind, "col"), g["indices_colmajor"])
    assert np.array_equal(ell_flatten(data, "row"), g["data"].ravel())


CASES = [
    ("ring8", 8, ring_bonds(8), 4, 8, 320),
    ("torus4x4_n5", 16, torus_bonds(4, 4), 5, 20, 64064),
    ("torus4x4_n3", 16, torus_bonds(4, 4), 3, 12, None),
    ("torus6x6_n3", 36, torus_bonds(6, 6), 3, 12, 80784),
]


@pytest.mark.parametrize("name,ns,bonds,n,width,nnz", CASES)
def test_nnz_width_symmetry(name, ns, bonds, n, width, nnz):
    st = basis_states(ns, n)
    h = hopping_matrix(ns, bonds, st)
    # every bond with exactly one end occupied gives one entry per direction
    assert h.nnz == len(bonds) * 2 * math.comb(ns - 2, n - 1)
    if nnz is not None:
        assert h.nnz == nnz
    assert abs(h - h.T).max() == 0.0
    assert np.all(np.abs(h.data) == 1.0)
    _, _, w = to_ell(h)
    assert w == width


def test_bond_counts():
    assert len(ring_bonds(8)) == 8
    assert len(torus_bonds(4, 4)) == 32
    assert len(torus_bonds(6, 6)) == 72
    assert len(ring_bonds(2)) == 1 and two_site_bonds() == [(0, 1)]


@pytest.mark.parametrize("ns,bonds,n", [(8, ring_bonds(8), 1), (8, ring_bonds(8), 4),
                                        (8, ring_bonds(8), 3), (16, torus_bonds(4, 4), 3),
                                        (16, torus_bonds(4, 4), 5), (12, ring_bonds(12), 6)])
def test_single_species_band_sum(ns, bonds, n):
    """With one species the ground energy is the sum of the lowest n single-particle levels."""
    st = basis_states(ns, n)
    h = hopping_matrix(ns, bonds, st).toarray()
    e0 = np.linalg.eigvalsh(h)[0]
    t1 = np.zeros((ns, ns))
    for i, j in bonds:
        t1[i, j] = t1[j, i] = -1.0
    eps = np.linalg.eigvalsh(t1)
    assert abs(e0 - eps[:n].sum()) < 1e-10


def test_ring8_half_band_value():
    # periodic 8-ring, 4 fermions: -2 - 2*sqrt(2); a table without fermion signs
    # would give the antiperiodic value instead
    st = basis_states(8, 4)
    h = hopping_matrix(8, ring_bonds(8), st).toarray()
    assert abs(np.linalg.eigvalsh(h)[0] - (-2.0 - 2.0 * np.sqrt(2.0))) < 1e-12


@pytest.mark.parametrize("ns,bonds,nu,nd,U", [
    (2, two_site_bonds(), 1, 1, 4.0),
    (4, ring_bonds(4), 2, 1, 3.0),
    (4, ring_bonds(4), 2, 2, 2.5),
    (5, ring_bonds(5), 2, 3, 1.5),
    (6, ring_bonds(6), 3, 2, 4.0),
    (6, torus_bonds(3, 2), 2, 2, 5.0),
])
def test_matrix_equals_fock_brute_force(ns, bonds, nu, nd, U):
    """Whole sector matrix from Jordan-Wigner Kronecker products equals the oracle's H."""
    ref = sector_block(ns, bonds, nu, nd, 1.0, U)
    mine = Model(ns, bonds, nu, nd, 1.0, U).dense()
    assert np.max(np.abs(ref - mine)) < 1e-12
