"""Pins of the element-by-element H x (oracle.elements) and of single-species sectors."""

import numpy as np
import pytest

from oracle.elements import hv_elements, rank_in, sector_states
from oracle.fock import sector_block
from oracle.hamiltonian import Model
from synth import complete_bonds, ring_bonds, start_vector, torus_bonds, two_site_bonds


@pytest.mark.parametrize("ns,bonds,nu,nd,t,U", [
    (2, two_site_bonds(), 1, 1, 1.0, 4.0),
    (6, ring_bonds(6), 2, 3, 0.7, 2.5),
    (6, ring_bonds(6), 3, 3, 1.0, 4.0),
    (6, torus_bonds(3, 2), 3, 2, 1.0, 1.5),
    (5, complete_bonds(5), 2, 2, 1.3, 3.0),
    (6, ring_bonds(6), 0, 3, 1.0, 7.0),    # one species: the U term vanishes
    (6, ring_bonds(6), 4, 0, 1.0, 7.0),
])
def test_elements_match_fock_brute_force(ns, bonds, nu, nd, t, U):
    """Every element of H x against the Jordan-Wigner Fock-space Hamiltonian restricted to the sector."""
    su, sd = sector_states(ns, nu, nd)
    h = sector_block(ns, bonds, nu, nd, t, U)
    x = start_vector(71, h.shape[0])
    got = hv_elements(ns, bonds, su, sd, t, U, x, range(h.shape[0]))
    assert np.max(np.abs(got - h @ x)) < 1e-12


def test_elements_agree_with_the_matrix_oracle_on_a_larger_sector():
    """4x4 torus 3+4 (D = 1,019,200): sampled elements against the Kronecker-product matrices."""
    m = Model(16, torus_bonds(4, 4), 3, 4, 1.0, 2.0)
    x = start_vector(72, m.dim)
    picks = [0, 1, 12345, 560 * 1820 - 1, m.dim // 2, m.dim - 1]
    y = m.hv(x)
    got = hv_elements(16, torus_bonds(4, 4), m.st_up, m.st_dn, 1.0, 2.0, x, picks)
    assert np.max(np.abs(got - y[picks])) < 1e-12


def test_rank_rejects_states_outside_the_basis():
    su, _ = sector_states(6, 3, 3)
    assert rank_in(su, 0b000111) == 0 and rank_in(su, 0b111000) == len(su) - 1
    with pytest.raises(KeyError):
        rank_in(su, 0b1111)


def _free_fermion_e0(n_sites, bonds, n, t=1.0):
    """Sum of the n lowest eigenvalues of the single-particle hopping matrix -t A (A: adjacency)."""
    a = np.zeros((n_sites, n_sites))
    for i, j in bonds:
        a[i, j] -= t
        a[j, i] -= t
    return float(np.sort(np.linalg.eigvalsh(a))[:n].sum())


@pytest.mark.parametrize("ns,bonds,n", [(10, ring_bonds(10), 3), (10, ring_bonds(10), 4), (10, ring_bonds(10), 5),
                                        (12, torus_bonds(4, 3), 5), (12, torus_bonds(3, 4), 6),
                                        (9, complete_bonds(9), 4)])
def test_single_species_ground_energy_is_the_free_fermion_sum(ns, bonds, n):
    """One species, hopping only: free fermions, so the many-body E0 is the sum of the n lowest one-particle
    levels, whatever the parity of n (the fermion signs of the wrapping bonds make the ring periodic)."""
    m = Model(ns, bonds, 0, n, 1.0, 5.0)
    e0 = np.linalg.eigvalsh(m.dense())[0]
    assert abs(e0 - _free_fermion_e0(ns, bonds, n)) < 1e-10
