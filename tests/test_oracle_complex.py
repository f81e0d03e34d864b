"""Pins of the oracle with complex hopping amplitudes (the checkerboard workload's kind of Hamiltonian)."""

import numpy as np
import pytest

from oracle.elements import hv_elements
from oracle.fock import sector_block
from oracle.hamiltonian import Model
from oracle.lanczos import ground_energy, lanczos
from synth import (checkerboard_terms, complete_bonds, ring_bonds, start_vector, start_vector_complex)


def _random_amps(seed, n):
    r = np.random.default_rng(seed)
    return list(r.uniform(-1.0, 1.0, n) + 1j * r.uniform(-1.0, 1.0, n))


SMALL = [
    (6, ring_bonds(6), 2, 3, 0.8, 2.5),
    (5, complete_bonds(5), 2, 2, 1.0, 3.0),
    (6, ring_bonds(6), 3, 3, 1.0, 4.0),
    (6, ring_bonds(6), 0, 3, 1.0, 1.0),
]


@pytest.mark.parametrize("ns,bonds,nu,nd,t,U", SMALL)
def test_complex_matrices_match_fock_brute_force(ns, bonds, nu, nd, t, U):
    amps = _random_amps(ns * 10 + nu, len(bonds))
    m = Model(ns, bonds, nu, nd, t, U, amps)
    h = m.dense()
    ref = sector_block(ns, bonds, nu, nd, t, U, amps)
    assert np.max(np.abs(h - ref)) < 1e-13
    assert np.max(np.abs(h - h.conj().T)) == 0.0


@pytest.mark.parametrize("ns,bonds,nu,nd,t,U", SMALL)
def test_complex_elements_match_fock_brute_force(ns, bonds, nu, nd, t, U):
    amps = _random_amps(ns * 10 + nu + 1, len(bonds))
    ref = sector_block(ns, bonds, nu, nd, t, U, amps)
    m = Model(ns, bonds, nu, nd, t, U, amps)
    x = start_vector_complex(91, ref.shape[0])
    got = hv_elements(ns, bonds, m.st_up, m.st_dn, t, U, x, range(ref.shape[0]), amps)
    assert np.max(np.abs(got - ref @ x)) < 1e-12
    assert np.max(np.abs(m.hv(x) - ref @ x)) < 1e-12


def test_pure_gauge_phases_leave_the_spectrum_unchanged():
    """a_ij = -|t_ij| exp(i(theta_i - theta_j)) is the real model after c_i -> exp(i theta_i) c_i."""
    ns, bonds = 6, ring_bonds(6) + [(0, 3)]
    mags = np.random.default_rng(3).uniform(0.5, 1.5, len(bonds))
    theta = np.random.default_rng(4).uniform(0, 2 * np.pi, ns)
    amps = [-m * np.exp(1j * (theta[i] - theta[j])) for m, (i, j) in zip(mags, bonds)]
    real = Model(ns, bonds, 2, 3, 1.0, 3.0, [-m for m in mags])
    cplx = Model(ns, bonds, 2, 3, 1.0, 3.0, amps)
    assert np.max(np.abs(np.linalg.eigvalsh(real.dense()) - np.linalg.eigvalsh(cplx.dense()))) < 1e-12
    # and the plain real model (every a = -t) is the same as amplitudes -t
    plain = Model(6, ring_bonds(6), 2, 3, 1.0, 3.0)
    viaamps = Model(6, ring_bonds(6), 2, 3, 1.0, 3.0, [-1.0] * 6)
    assert np.max(np.abs(plain.dense() - viaamps.dense())) == 0.0


def test_conjugated_amplitudes_give_the_same_spectrum():
    """Complex conjugation (time reversal) maps H to its conjugate, which has the same spectrum."""
    amps = _random_amps(5, 10)
    a = Model(5, complete_bonds(5), 2, 2, 1.0, 2.0, amps)
    b = Model(5, complete_bonds(5), 2, 2, 1.0, 2.0, [complex(z).conjugate() for z in amps])
    assert np.max(np.abs(np.linalg.eigvalsh(a.dense()) - np.linalg.eigvalsh(b.dense()))) < 1e-12


def _one_particle(ns, terms, t=1.0):
    h = np.zeros((ns, ns), dtype=np.complex128)
    for (i, j), a in terms:
        h[i, j] += t * a
        h[j, i] += t * np.conj(a)
    return np.linalg.eigvalsh(h)


@pytest.mark.parametrize("nu,nd", [(2, 1), (1, 1), (0, 3)])
def test_checkerboard_u0_band_sum(nu, nd):
    """18-site checkerboard at U = 0: E0 = sum of the lowest N_up plus the lowest N_dn one-particle levels
    of the Hermitian hopping matrix (free fermions; complex nearest-neighbour amplitudes)."""
    terms = checkerboard_terms(3, 3, 1.0, np.pi / 4, 0.3, 0.2)
    bonds, amps = [b for b, _ in terms], [a for _, a in terms]
    m = Model(18, bonds, nu, nd, 1.0, 0.0, amps)
    lv = _one_particle(18, terms)
    assert abs(np.linalg.eigvalsh(m.dense())[0] - (lv[:nu].sum() + lv[:nd].sum())) < 1e-10


def test_complex_lanczos_reaches_the_dense_ground_energy():
    terms = checkerboard_terms(3, 3, 1.0, np.pi / 4, 0.3, 0.2)
    m = Model(18, [b for b, _ in terms], 2, 1, 1.0, 4.0, [a for _, a in terms])
    e_dense = np.linalg.eigvalsh(m.dense())[0]
    x = start_vector_complex(92, m.dim)
    assert abs(ground_energy(m.hv, x, 120) - e_dense) < 1e-9
    r = lanczos(m.hv, x, 10)
    assert np.all(np.isfinite(r["a"])) and np.all(r["b"][1:] > 0)
    # a real start vector gives the real-path coefficients when the amplitudes are real
    mr = Model(8, ring_bonds(8), 2, 2, 1.0, 3.0, [-1.0] * 8)
    xr = start_vector(93, mr.dim)
    r1, r2 = lanczos(mr.hv, xr, 10), lanczos(Model(8, ring_bonds(8), 2, 2, 1.0, 3.0).hv, xr, 10)
    assert np.max(np.abs(r1["a"] - r2["a"])) < 1e-13
