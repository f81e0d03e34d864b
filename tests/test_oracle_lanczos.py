"""Pins of the oracle's Lanczos iteration (Alg. 1) and tridiagonal solve (Sec. 2.2)."""

import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.hamiltonian import Model
from oracle.lanczos import (fix_gauge, ground_energy, ground_state_two_pass, lanczos,
                            lowest_eigvec_T, ritz_lowest, tridiag_lowest)
from synth import ring_bonds, start_vector, torus_bonds, two_site_bonds


@pytest.fixture(scope="module")
def ring8():
    return Model(8, ring_bonds(8), 4, 4, 1.0, 4.0)


def test_tridiag_small_closed_forms():
    assert tridiag_lowest([3.5], []) == 3.5
    a1, a2, b = 1.3, -0.4, 0.9
    ref = ((a1 + a2) - math.sqrt((a1 - a2) ** 2 + 4 * b * b)) / 2
    assert abs(tridiag_lowest([a1, a2], [b]) - ref) < 1e-14


def test_tridiag_vs_dense_random():
    rng = np.random.default_rng(7)
    for m in (3, 50, 300):
        a, b = rng.normal(size=m), rng.uniform(0.1, 2.0, m - 1)
        t = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        assert abs(tridiag_lowest(a, b) - np.linalg.eigvalsh(t)[0]) < 1e-12


def test_c1_e0_matches_dense(ring8):
    e_dense = np.linalg.eigvalsh(ring8.dense())[0]
    e_lz = ground_energy(ring8.hv, start_vector(1, ring8.dim), 100)
    assert abs(e_lz - e_dense) <= 1e-10 * abs(e_dense)


def test_lanczos_relation_and_orthogonality(ring8):
    """H F_k = F_k T_k + b_{k+1} f_{k+1} e_k^T and F_k^T F_k = I in the early steps."""
    k = 12
    r = lanczos(ring8.hv, start_vector(1, ring8.dim), k + 1, vectors=True)
    F = np.stack(r["f"][:k], axis=1)
    a, b = r["a"], r["b"]
    T = np.diag(a[:k]) + np.diag(b[1:k], 1) + np.diag(b[1:k], -1)
    H = ring8.full_sparse()
    resid = H @ F - F @ T
    resid[:, -1] -= b[k] * r["f"][k]
    assert np.max(np.abs(resid)) < 1e-12
    assert np.max(np.abs(F.T @ F - np.eye(k))) < 1e-10


def test_first_coefficients_by_definition(ring8):
    # a_1 = f1.H f1 and b_2 = |H f1 - a_1 f1| straight from the definition
    f = start_vector(1, ring8.dim)
    f = f / np.linalg.norm(f)
    H = ring8.dense()
    a1 = f @ H @ f
    b2 = np.linalg.norm(H @ f - a1 * f)
    r = lanczos(ring8.hv, f, 2)
    assert abs(r["a"][0] - a1) < 1e-12 and abs(r["b"][1] - b2) < 1e-12 and r["b"][0] == 0.0


def test_ritz_monotone_and_variational(ring8):
    e_dense = np.linalg.eigvalsh(ring8.dense())[0]
    r = lanczos(ring8.hv, start_vector(1, ring8.dim), 60)
    e = ritz_lowest(r["a"], r["b"])
    assert np.all(np.diff(e) <= 1e-12)
    assert np.all(e >= e_dense - 1e-12)


def test_full_krylov_reproduces_spectrum():
    m = Model(2, two_site_bonds(), 1, 1, 1.0, 4.0)
    r = lanczos(m.hv, np.array([0.3, -0.5, 0.7, 0.2]), 10)
    a, b = r["a"], r["b"]
    k = len(a)
    T = np.diag(a) + np.diag(b[1:k], 1) + np.diag(b[1:k], -1)
    spec = np.linalg.eigvalsh(m.dense())
    # the start vector has no weight on the antisymmetric (spin-singlet-odd) states,
    # so the Krylov space has dimension < 4; every Ritz value is an eigenvalue
    for w in np.linalg.eigvalsh(T):
        assert np.min(np.abs(spec - w)) < 1e-10
    assert abs(np.linalg.eigvalsh(T)[0] - spec[0]) < 1e-12


def test_breakdown_on_exact_eigenvector():
    m = Model(2, two_site_bonds(), 1, 1, 1.0, 4.0)
    w, v = np.linalg.eigh(m.dense())
    r = lanczos(m.hv, v[:, 0], 5)
    assert r["breakdown"] and len(r["a"]) == 1
    assert abs(r["a"][0] - (4.0 - math.sqrt(32.0)) / 2.0) < 1e-12


def test_zero_start_vector_rejected(ring8):
    with pytest.raises(ValueError):
        lanczos(ring8.hv, np.zeros(ring8.dim), 3)


def test_against_arpack_midsize():
    from scipy.sparse.linalg import LinearOperator, eigsh
    m = Model(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0)
    op = LinearOperator((m.dim, m.dim), matvec=m.hv, dtype=np.float64)
    e_arpack = eigsh(op, k=1, which="SA", tol=1e-13, v0=np.ones(m.dim))[0][0]
    e_lz = ground_energy(m.hv, start_vector(4, m.dim), 200)
    assert abs(e_lz - e_arpack) <= 1e-10 * abs(e_arpack)


def test_two_pass_ground_state(ring8):
    e, v = ground_state_two_pass(ring8.hv, start_vector(1, ring8.dim), 120)
    w, vecs = np.linalg.eigh(ring8.dense())
    assert abs(e - w[0]) < 1e-10 * abs(w[0])
    assert abs(abs(v @ vecs[:, 0]) - 1.0) < 1e-9
    assert np.linalg.norm(ring8.hv(v) - e * v) < 1e-7
    g = fix_gauge(v, 0)
    assert g[0] > 0 or abs(g[0]) < 1e-3 * np.max(np.abs(g))


def test_lowest_eigvec_T():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=40), rng.uniform(0.2, 1.0, 39)
    y = lowest_eigvec_T(a, b)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.linalg.norm(T @ y - tridiag_lowest(a, b) * y) < 1e-12


def test_fix_gauge_follows_the_stated_reading():
    """The eigenvector gauge: the reference amplitude is made positive; below 1e-3 of the largest magnitude
    the largest-magnitude entry decides instead, the lowest index among equal magnitudes."""
    g = fix_gauge(np.array([-0.5, 0.3, 0.8]), 0)
    assert g.tolist() == [0.5, -0.3, -0.8]                       # negative reference: flipped
    assert fix_gauge(np.array([0.5, -0.3]), 0).tolist() == [0.5, -0.3]   # positive reference: kept
    g = fix_gauge(np.array([1e-4, 0.2, -0.9]), 0)                # reference too small: entry 2 decides
    assert g.tolist() == [-1e-4, -0.2, 0.9]
    g = fix_gauge(np.array([-1e-3, 1.0]), 0)                     # exactly 1e-3 of the largest: the reference decides
    assert g.tolist() == [1e-3, -1.0]
    g = fix_gauge(np.array([0.0, -0.7, 0.7]), 0)                 # tie in magnitude: the lower index decides
    assert g.tolist() == [-0.0, 0.7, -0.7]
    g = fix_gauge(np.array([0.25, -0.5, 0.75]), 2)               # any reference index
    assert g.tolist() == [0.25, -0.5, 0.75]
