"""Parity of the HIP Lanczos iteration (Alg. 1) and ground-state runs with the oracle."""

import math

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.hamiltonian import Model
from oracle.lanczos import lanczos, ritz_lowest
from synth import ring_bonds, start_vector, torus_bonds, two_site_bonds
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring8():
    return Model(8, ring_bonds(8), 4, 4, 1.0, 4.0)


@pytest.fixture(scope="module")
def ring8_e0(ring8):
    return float(np.linalg.eigvalsh(ring8.dense())[0])


def test_c1_f64_e0_and_coefficients(ring8, ring8_e0):
    """8-site ring 4+4, U=4, 100 steps from the seed-1 start: E0 within 1e-10 of dense LAPACK."""
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, "f64")
    x_host, x = seeded_start(1, h.dim, "f64")
    announce("lanczos C1 f64")
    r = h.ground_energy(x, 100, tol=0.0)
    assert r["status"] == ed.ED_OK and r["steps"] == 100
    assert abs(r["e0"] - ring8_e0) <= 1e-10 * abs(ring8_e0)
    ref = lanczos(ring8.hv, x_host, 20)
    amax = np.max(np.abs(ref["a"]))
    assert np.max(np.abs(r["a"][:20] - ref["a"])) <= 1e-12 * amax
    assert np.max(np.abs(r["b"][:21] - ref["b"])) <= 1e-12 * amax
    assert r["b"][0] == 0.0


def test_c1_mixed_e0(ring8, ring8_e0):
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, "f32")
    _, x = seeded_start(1, h.dim, "f32")
    announce("lanczos C1 f32 mixed")
    r = h.ground_energy(x, 100, tol=0.0)
    assert abs(r["e0"] - ring8_e0) <= 1e-6 * abs(ring8_e0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("U", [0.0, 4.0, 10.0])
def test_two_site_closed_form(dtype, U):
    h = ham(2, two_site_bonds(), 1, 1, 1.0, U, dtype)
    _, x = seeded_start(3, 4, dtype)
    announce("lanczos two-site %s U=%g" % (dtype, U))
    r = h.ground_energy(x, 10, tol=0.0)
    exact = (U - math.sqrt(U * U + 16.0)) / 2.0
    assert r["status"] == ed.ED_BREAKDOWN and r["steps"] <= 4
    assert abs(r["e0"] - exact) <= (1e-12 if dtype == "f64" else 1e-6) * abs(exact)


def test_breakdown_on_eigenvector():
    m = Model(2, two_site_bonds(), 1, 1, 1.0, 4.0)
    w, v = np.linalg.eigh(m.dense())
    h = ham(2, two_site_bonds(), 1, 1, 1.0, 4.0, "f64")
    announce("lanczos breakdown two-site")
    r = h.ground_energy(torch.from_numpy(v[:, 0].copy()).cuda(), 10)
    assert r["status"] == ed.ED_BREAKDOWN and r["steps"] == 1
    assert abs(r["e0"] - w[0]) < 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_zero_and_nan_start_rejected(dtype):
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, dtype)
    announce("lanczos bad start %s" % dtype)
    with pytest.raises(ed.EdError) as e:
        h.ground_energy(torch.zeros(h.dim, dtype=h.torch_dtype, device="cuda:0"), 10)
    assert e.value.code == ed._ffi.ED_EINVAL
    bad = torch.ones(h.dim, dtype=h.torch_dtype, device="cuda:0")
    bad[5] = float("nan")
    with pytest.raises(ed.EdError):
        h.ground_energy(bad, 10)


def test_step_by_step_matches_oracle_t44_3x3():
    """ed_lanczos_step one call at a time: a_j, b_j for 20 steps within 1e-12 |a|."""
    bonds = torus_bonds(4, 4)
    m = Model(16, bonds, 3, 3, 1.0, 4.0)
    h = ham(16, bonds, 3, 3, 1.0, 4.0, "f64")
    x_host, x = seeded_start(4, m.dim, "f64")
    run = h.lanczos(40)
    announce("lanczos steps t44 3+3")
    run.init(x)
    for _ in range(20):
        run.step()
    got = run.read()
    ref = lanczos(m.hv, x_host, 20)
    amax = np.max(np.abs(ref["a"]))
    assert got["steps"] == 20 and got["status"] == ed.ED_OK
    assert np.max(np.abs(got["a"] - ref["a"])) <= 1e-12 * amax
    assert np.max(np.abs(got["b"] - ref["b"])) <= 1e-12 * amax
    # the newest stored vector is b_21 f_21 (normalisation is deferred)
    full = lanczos(m.hv, x_host, 21, vectors=True)
    f21 = full["f"][20]
    stored = run.f_cur.cpu().numpy()
    assert abs(np.linalg.norm(stored) - got["b"][20]) <= 1e-12 * got["b"][20]
    assert float(np.max(np.abs(stored / got["b"][20] - f21))) <= 1e-9


def test_max_steps_freezes_state():
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, "f64")
    _, x = seeded_start(1, h.dim, "f64")
    run = h.lanczos(5)
    announce("lanczos freeze at max_steps")
    run.init(x)
    for _ in range(9):
        run.step()
    got = run.read()
    assert got["steps"] == 5 and got["status"] == ed.ED_NOT_CONVERGED


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bitwise_reproducible(dtype):
    bonds = torus_bonds(4, 4)
    h = ham(16, bonds, 4, 4, 1.0, 3.0, dtype)
    _, x = seeded_start(9, h.dim, dtype)
    announce("lanczos reproducible %s" % dtype)
    r1 = h.ground_energy(x, 40)
    r2 = h.ground_energy(x, 40)
    assert np.array_equal(r1["a"], r2["a"]) and np.array_equal(r1["b"], r2["b"])


def test_c3_u0_closed_form():
    """6x6 torus, 3+3, U=0: E0 = -20 (sum of the lowest band levels -4, -3, -3 per species)."""
    bonds = torus_bonds(6, 6)
    for dtype, tol in (("f64", 1e-10), ("f32", 1e-6)):
        h = ham(36, bonds, 3, 3, 1.0, 0.0, dtype)
        _, x = seeded_start(3, h.dim, dtype)
        announce("lanczos C3 6x6 3+3 %s" % dtype)
        r = h.ground_energy(x, 300, tol=1e-12 if dtype == "f64" else 1e-7, check_every=12)
        assert abs(r["e0"] - (-20.0)) <= tol * 20.0, (dtype, r["e0"], r["steps"])
        del h, x


def test_c5_ritz_values_monotone_and_variational():
    """4x4 half filling, 30 f64 steps: E0(j) non-increasing, above the U=0 bound shifted by
    the smallest diagonal (E0 >= band sum at U=0 since U >= 0)."""
    bonds = torus_bonds(4, 4)
    h = ham(16, bonds, 8, 8, 1.0, 4.0, "f64")
    _, x = seeded_start(5, h.dim, "f64")
    announce("lanczos C5 f64 30 steps")
    r = h.ground_energy(x, 30)
    e = ritz_lowest(r["a"], r["b"])
    assert np.all(np.diff(e) <= 1e-10)
    assert e[-1] >= -24.0 - 1e-9


def test_two_pass_ground_state_c1(ring8, ring8_e0):
    w, vecs = np.linalg.eigh(ring8.dense())
    for dtype, tol in (("f64", 1e-9), ("f32", 1e-5)):
        h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, dtype)
        _, x = seeded_start(1, h.dim, dtype)
        announce("ground state C1 %s" % dtype)
        e0, steps, v = h.ground_state(x, 80)
        v = v.double().cpu().numpy()
        assert abs(e0 - w[0]) <= 1e-10 * abs(w[0]) if dtype == "f64" else abs(e0 - w[0]) <= 1e-6 * abs(w[0])
        assert abs(np.linalg.norm(v) - 1.0) < (1e-12 if dtype == "f64" else 1e-6)
        assert abs(abs(v @ vecs[:, 0]) - 1.0) <= tol


def test_ground_energy_newest_vector_after_partial_chunk():
    """ed_ground_energy with max_steps not a multiple of its step chunk (steps launched past max_steps are
    no-ops): afterwards f_cur holds b_{m+1} f_{m+1}, the same vector m single steps leave there."""
    h = ham(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0, "f64")
    _, x = seeded_start(23, h.dim, "f64")
    ra, rb = h.lanczos(100), h.lanczos(100)
    announce("ground_energy f_cur after 100 steps in chunks of 12")
    ra.ground_energy(x, tol=0.0, check_every=12)
    rb.init(x)
    for _ in range(100):
        rb.step()
    ga, gb = ra.read(), rb.read()
    assert ga["steps"] == gb["steps"] == 100
    assert np.array_equal(ga["a"], gb["a"]) and np.array_equal(ga["b"], gb["b"])
    assert torch.equal(ra.f_cur, rb.f_cur) and torch.equal(ra.f_prev, rb.f_prev)
    fa = ra.f_cur.cpu().numpy()
    assert abs(np.linalg.norm(fa) - ga["b"][100]) <= 1e-12 * ga["b"][100]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ground_state_gauge_follows_the_oracle_rule(dtype):
    """The device's gauge against oracle.lanczos.fix_gauge on the device's own ungauged vector: at a reference
    element of normal size, and at one below 1e-3 of the largest magnitude (the 8-ring's ground state has
    symmetry zeros), where the largest-magnitude element decides."""
    from oracle.lanczos import fix_gauge
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, dtype)
    _, x = seeded_start(1, h.dim, dtype)
    announce("ground state gauge ring8 4+4 %s" % dtype)
    _, _, v0 = h.ground_state(x, 80, gauge_index=-1)
    v0 = v0.double().cpu().numpy()
    r = np.abs(v0) / np.abs(v0).max()
    small = int(np.nonzero(r < 1e-4)[0][0])
    big = int(np.argmax(r > 0.5))
    for k in (big, small):
        _, _, v = h.ground_state(x, 80, gauge_index=k)
        assert np.array_equal(v.double().cpu().numpy(), fix_gauge(v0, k)), k


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ground_state_to_a_tolerance_is_the_fixed_step_run(dtype):
    """ed_ground_state with tol > 0 (pass 1 until E0 settles, then `extra` more steps) gives the same E0, step
    count and vector bits as the fixed-m call with m = (ed_ground_energy's stopping step) + extra."""
    h = ham(16, torus_bonds(4, 4), 4, 4, 1.0, 3.0, dtype)
    _, x = seeded_start(31, h.dim, dtype)
    tol, extra = (1e-10 if dtype == "f64" else 1e-7), 12
    announce("ground state to a tolerance 4x4 4+4 %s" % dtype)
    r = h.ground_energy(x, 400, tol=tol, check_every=15)
    assert r["status"] == ed.ED_OK
    m = r["steps"] + extra
    e_a, k_a, v_a = h.ground_state(x, m, gauge_index=0)
    e_b, k_b, v_b = h.ground_state(x, 400, gauge_index=0, tol=tol, extra=extra)
    assert (k_a, k_b) == (m, m)
    assert e_a == e_b
    assert torch.equal(v_a, v_b)
