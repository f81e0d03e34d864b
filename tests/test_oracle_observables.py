"""Pins of the oracle's diagonal observables (occupation moments of a state vector)."""

import math

import numpy as np
import pytest

from oracle.fock import annihilator
from oracle.basis import basis_states
from oracle.hamiltonian import Model
from oracle.observables import correlations, occupation_moments
from synth import ring_bonds, start_vector, torus_bonds, two_site_bonds


def _ground(m):
    w, v = np.linalg.eigh(m.dense())
    return w[0], v[:, 0]


@pytest.mark.parametrize("U", [0.5, 4.0, 10.0])
def test_two_site_hellmann_feynman_closed_form(U):
    # dE0/dU = <sum_i n_i,up n_i,dn>; with E0 = (U - sqrt(U^2 + 16 t^2)) / 2 this is (1 - U / sqrt(U^2 + 16)) / 2
    m = Model(2, two_site_bonds(), 1, 1, 1.0, U)
    _, v = _ground(m)
    c = correlations(occupation_moments(v, m.st_up, m.st_dn, 2), 2)
    assert abs(c["docc"].sum() - (1.0 - U / math.sqrt(U * U + 16.0)) / 2.0) < 1e-12


def test_hellmann_feynman_finite_difference_ring8():
    bonds, h = ring_bonds(8), 1e-4
    e_p = np.linalg.eigvalsh(Model(8, bonds, 3, 3, 1.0, 4.0 + h).dense())[0]
    e_m = np.linalg.eigvalsh(Model(8, bonds, 3, 3, 1.0, 4.0 - h).dense())[0]
    m = Model(8, bonds, 3, 3, 1.0, 4.0)
    _, v = _ground(m)
    c = correlations(occupation_moments(v, m.st_up, m.st_dn, 8), 8)
    assert abs(c["docc"].sum() - (e_p - e_m) / (2 * h)) < 1e-7
    # translation invariance of the ring: every site has the same double occupancy
    assert np.ptp(c["docc"]) < 1e-10


def test_moments_match_fock_number_operators():
    """G against <psi| n_a n_b |psi> with n_a = c+_a c_a from the Jordan-Wigner Fock-space operators."""
    ns, nu, nd = 5, 2, 3
    su, sd = basis_states(ns, nu), basis_states(ns, nd)
    psi = start_vector(41, len(su) * len(sd))
    psi /= np.linalg.norm(psi)
    g = occupation_moments(psi, su, sd, ns)
    n_modes = 2 * ns
    fock_idx = np.array([int(a) | (int(b) << ns) for a in su for b in sd])
    full = np.zeros(2 ** n_modes)
    full[fock_idx] = psi
    num = []
    for a in range(n_modes):
        c = annihilator(a, n_modes)
        num.append((c.T @ c).tocsr())
    for a in range(n_modes):
        na_psi = num[a] @ full
        for b in range(n_modes):
            assert abs(full @ (num[b] @ na_psi) - g[a, b]) < 1e-12


def test_sum_rules_random_vector():
    ns, nu, nd = 16, 3, 2
    su, sd = basis_states(ns, nu), basis_states(ns, nd)
    psi = start_vector(42, len(su) * len(sd))
    psi /= np.linalg.norm(psi)
    c = correlations(occupation_moments(psi, su, sd, ns), ns)
    n_i = c["n_up"] + c["n_dn"]
    sz_i = (c["n_up"] - c["n_dn"]) / 2.0
    assert abs(c["n_up"].sum() - nu) < 1e-12 and abs(c["n_dn"].sum() - nd) < 1e-12
    # sum_j n_j = N and sum_j S^z_j = (N_up - N_dn)/2 are fixed in the sector
    assert np.max(np.abs(c["nn"].sum(axis=1) - (nu + nd) * n_i)) < 1e-12
    assert np.max(np.abs(c["szsz"].sum(axis=1) - 0.5 * (nu - nd) * sz_i)) < 1e-12
    # n^2 = n on the diagonal of the spin blocks; symmetry
    assert np.allclose(np.diag(c["nn"]), n_i + 2 * c["docc"], atol=1e-12)
    assert np.allclose(c["nn"], c["nn"].T, atol=1e-14) and np.allclose(c["szsz"], c["szsz"].T, atol=1e-14)


def test_u0_double_occupancy_factorises_ring6():
    """At U = 0 a closed shell (3 per species on the 6-ring) has a non-degenerate ground state that is a product
    of up and down Slater determinants, so <n_i,up n_i,dn> = <n_i,up><n_i,dn> = (N/N_s)^2 per site."""
    m = Model(6, ring_bonds(6), 3, 3, 1.0, 0.0)
    w, v = np.linalg.eigh(m.dense())
    assert w[1] - w[0] > 1e-6          # non-degenerate: N = 3 is a closed shell on the 6-ring
    c = correlations(occupation_moments(v[:, 0], m.st_up, m.st_dn, 6), 6)
    assert np.max(np.abs(c["docc"] - 0.25)) < 1e-10


def _fock_spin_flip(psi, su, sd, ns):
    """<psi| S+_i S-_j |psi> with S+- built from the Fock-space Jordan-Wigner annihilators."""
    n_modes = 2 * ns
    fock_idx = np.array([int(a) | (int(b) << ns) for a in su for b in sd])
    full = np.zeros(2 ** n_modes)
    full[fock_idx] = psi
    c_ = [annihilator(m, n_modes) for m in range(n_modes)]
    out = np.zeros((ns, ns))
    for i in range(ns):
        sp = (c_[i].T @ c_[ns + i]).tocsr()            # c+_i,up c_i,dn
        for j in range(ns):
            sm = (c_[ns + j].T @ c_[j]).tocsr()        # c+_j,dn c_j,up
            out[i, j] = full @ (sp @ (sm @ full))
    return out


@pytest.mark.parametrize("ns,nu,nd", [(4, 2, 2), (5, 2, 3), (4, 1, 3)])
def test_spin_flip_moments_match_fock_operators(ns, nu, nd):
    from oracle.observables import spin_flip_moments
    su, sd = basis_states(ns, nu), basis_states(ns, nd)
    psi = start_vector(43 + ns, len(su) * len(sd))
    assert np.max(np.abs(spin_flip_moments(psi, su, sd, ns) - _fock_spin_flip(psi, su, sd, ns))) < 1e-12


@pytest.mark.parametrize("ns,bonds", [(8, ring_bonds(8)), (6, ring_bonds(6)), (4, torus_bonds(2, 2))])
def test_singlet_ground_state_su2(ns, bonds):
    """On a bipartite lattice at half filling the ground state is a spin singlet (Lieb): <S+_i S-_j> =
    2 <S^z_i S^z_j> off the diagonal, and sum_ij <S_i . S_j> = S(S+1) = 0."""
    from oracle.observables import spin_correlations, spin_flip_moments
    m = Model(ns, bonds, ns // 2, ns // 2, 1.0, 4.0)
    _, v = _ground(m)
    g = occupation_moments(v, m.st_up, m.st_dn, ns)
    c = spin_flip_moments(v, m.st_up, m.st_dn, ns)
    zz = correlations(g, ns)["szsz"]
    off = ~np.eye(ns, dtype=bool)
    assert np.max(np.abs(c[off] - 2.0 * zz[off])) < 1e-10
    ss = spin_correlations(g, c, ns)
    assert abs(ss.sum()) < 1e-10
    # the diagonal of C is <n_up (1 - n_dn)>
    assert np.max(np.abs(np.diag(c) - (np.diag(g)[:ns] - np.diag(g[:ns, ns:])))) < 1e-12


def test_two_site_singlet_spin_correlation():
    """Two-site Hubbard ground state (a singlet): <S_0 . S_1> = -(3/4) * (1 - 2 d) with d = <n_up n_dn> per site
    (each site is singly occupied with probability 1 - 2d and the two spins then form the singlet)."""
    from oracle.observables import spin_correlations, spin_flip_moments
    U = 3.0
    m = Model(2, two_site_bonds(), 1, 1, 1.0, U)
    _, v = _ground(m)
    g = occupation_moments(v, m.st_up, m.st_dn, 2)
    ss = spin_correlations(g, spin_flip_moments(v, m.st_up, m.st_dn, 2), 2)
    d = g[0, 2]
    assert abs(ss[0, 1] - (-0.75 * (1.0 - 2.0 * d))) < 1e-12
    assert 0.0 < d < 0.25


@pytest.mark.parametrize("ns,bonds,nu,nd,U", [(8, ring_bonds(8), 3, 2, 2.0), (6, torus_bonds(3, 2), 3, 3, 4.0),
                                              (6, ring_bonds(6), 0, 3, 1.0)])
def test_energy_is_kinetic_plus_double_occupancy(ns, bonds, nu, nd, U):
    """For any state: <H> = -t sum_{b, sigma} K[b, sigma] + U sum_i <n_i,up n_i,dn>."""
    from oracle.observables import bond_moments
    t = 0.8
    m = Model(ns, bonds, nu, nd, t, U)
    psi = start_vector(44 + ns, m.dim)
    k = bond_moments(psi, m.st_up, m.st_dn, ns, bonds)
    g = occupation_moments(psi, m.st_up, m.st_dn, ns)
    assert abs(psi @ m.hv(psi) - (-t * k.sum() + U * np.trace(g[:ns, ns:]))) < 1e-10 * max(1.0, abs(psi @ m.hv(psi)))


def test_bond_moments_match_fock_operators():
    from oracle.observables import bond_moments
    ns, nu, nd = 5, 2, 3
    bonds = ring_bonds(5) + [(0, 2)]
    su, sd = basis_states(ns, nu), basis_states(ns, nd)
    psi = start_vector(45, len(su) * len(sd))
    fock_idx = np.array([int(a) | (int(b) << ns) for a in su for b in sd])
    full = np.zeros(2 ** (2 * ns))
    full[fock_idx] = psi
    c_ = [annihilator(m_, 2 * ns) for m_ in range(2 * ns)]
    k = bond_moments(psi, su, sd, ns, bonds)
    for b, (i, j) in enumerate(bonds):
        for s_ in range(2):
            a, bb = s_ * ns + i, s_ * ns + j
            op = (c_[a].T @ c_[bb] + c_[bb].T @ c_[a]).tocsr()
            assert abs(full @ (op @ full) - k[b, s_]) < 1e-12
