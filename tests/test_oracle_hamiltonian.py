"""Pins of the oracle's H and H.v (Eq. 1, 3-5) against closed forms and symmetries."""

import math

import numpy as np
import pytest

from oracle.hamiltonian import Model
from synth import complete_bonds, ring_bonds, start_vector, torus_bonds, two_site_bonds


def _e0_dense(m):
    return np.linalg.eigvalsh(m.dense())[0]


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 8.0, 13.7])
def test_two_site_closed_form(U):
    m = Model(2, two_site_bonds(), 1, 1, 1.0, U)
    assert m.dim == 4
    assert abs(_e0_dense(m) - (U - math.sqrt(U * U + 16.0)) / 2.0) < 1e-12


def test_two_site_t_scaling():
    t, U = 0.7, 2.0
    m = Model(2, two_site_bonds(), 1, 1, t, U)
    assert abs(_e0_dense(m) - (U - math.sqrt(U * U + 16.0 * t * t)) / 2.0) < 1e-12


def test_hv_matches_kron_definition():
    for (ns, bonds, nu, nd, U) in [(8, ring_bonds(8), 4, 4, 4.0), (8, ring_bonds(8), 3, 2, 2.0),
                                   (16, torus_bonds(4, 4), 2, 3, 1.0)]:
        m = Model(ns, bonds, nu, nd, 1.0, U)
        x = start_vector(11, m.dim)
        assert np.max(np.abs(m.hv(x) - m.full_sparse() @ x)) < 1e-12


def test_hv_rows_subset():
    m = Model(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0)
    x = start_vector(5, m.dim)
    rows = [0, 7, 559]
    full = m.hv(x).reshape(m.dim_up, m.dim_dn)
    assert np.max(np.abs(m.hv_rows(x, rows) - full[rows])) < 1e-12


def test_trace_identity():
    # tr H = U * D * N_up * N_dn / N_s  (each site is doubly occupied in that fraction of states)
    for (ns, bonds, nu, nd, U) in [(8, ring_bonds(8), 4, 4, 4.0), (16, torus_bonds(4, 4), 3, 2, 2.5)]:
        m = Model(ns, bonds, nu, nd, 1.0, U)
        assert abs(m.docc.sum() * U - U * m.dim * nu * nd / ns) < 1e-6
        assert abs(m.full_sparse().diagonal().sum() - U * m.dim * nu * nd / ns) < 1e-6


def test_u0_band_sum_ring8():
    m = Model(8, ring_bonds(8), 4, 4, 1.0, 0.0)
    assert abs(_e0_dense(m) - 2.0 * (-2.0 - 2.0 * math.sqrt(2.0))) < 1e-10


def test_u0_band_sum_torus_closed_form():
    # eps(k) = -2t (cos kx + cos ky) on the 4x4 torus; lowest 3 levels: -4, -2, -2
    m = Model(16, torus_bonds(4, 4), 3, 3, 1.0, 0.0)
    from scipy.sparse.linalg import eigsh
    e0 = eigsh(m.full_sparse(), k=1, which="SA", tol=1e-12)[0][0]
    assert abs(e0 - (-16.0)) < 1e-9


@pytest.mark.parametrize("nu,nd", [(1, 2), (2, 1), (2, 2), (3, 1)])
def test_particle_hole_symmetry(nu, nd):
    # bipartite 6-ring: E0(Ns-Nu, Ns-Nd) = E0(Nu, Nd) + U (Ns - Nu - Nd)
    ns, U = 6, 3.0
    a = _e0_dense(Model(ns, ring_bonds(ns), nu, nd, 1.0, U))
    b = _e0_dense(Model(ns, ring_bonds(ns), ns - nu, ns - nd, 1.0, U))
    assert abs(b - (a + U * (ns - nu - nd))) < 1e-10


def test_spin_flip_symmetry():
    a = _e0_dense(Model(8, ring_bonds(8), 3, 2, 1.0, 4.0))
    b = _e0_dense(Model(8, ring_bonds(8), 2, 3, 1.0, 4.0))
    assert abs(a - b) < 1e-10


def test_unit_vector_columns():
    m = Model(6, ring_bonds(6), 2, 2, 1.0, 2.0)
    h = m.dense()
    for k in [0, 5, 100, m.dim - 1]:
        e = np.zeros(m.dim)
        e[k] = 1.0
        assert np.array_equal(m.hv(e), h[:, k])


@pytest.mark.parametrize("n,nu,nd", [(6, 3, 3), (7, 2, 3), (7, 4, 1), (5, 2, 0)])
def test_u0_band_sum_complete_graph(n, nu, nd):
    # all-to-all hopping -t sum_{i<j} (c+_i c_j + h.c.): one-particle levels -t(n-1) once and +t (n-1 times),
    # so N fermions of one species have E = -t(n-1) + (N-1) t.  Most bonds join non-adjacent indices,
    # so every fermion sign of the tables enters; a table without them gives other levels.
    t = 0.9
    m = Model(n, complete_bonds(n), nu, nd, t, 0.0)
    band = lambda N: 0.0 if N == 0 else -t * (n - 1) + (N - 1) * t
    assert abs(_e0_dense(m) - (band(nu) + band(nd))) < 1e-10


def test_popcount_matches_bit_by_bit_count():
    from oracle.hamiltonian import popcount_u64
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2 ** 63, 2000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 2000, dtype=np.uint64)
    a = np.concatenate([a, np.array([0, 1, 2 ** 64 - 1, 2 ** 63, 0xFFFF0000FFFF0000], dtype=np.uint64)])
    ref = np.array([bin(int(v)).count("1") for v in a])
    assert np.array_equal(popcount_u64(a), ref)
