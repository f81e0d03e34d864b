"""Parity of the fused two-pass Lanczos step (ed_lanczos_steps) with the oracle's Alg. 1 and with the
reference step (ed_lanczos_step), through the C ABI."""

import numpy as np
import pytest

import paper_1511_00863_amd as ed
from oracle.hamiltonian import Model
from oracle.lanczos import lanczos, tridiag_lowest
from synth import ring_bonds, torus_bonds, two_site_bonds
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu

# (label, n_sites, bonds, n_up, n_dn, U): rows of several lengths (odd, ragged against the 16- and
# 32-column stripes, several rows per down-pass workgroup), tables of 1 to 4 chunks, species that
# cannot hop
CASES = [
    ("ring8 4+4", 8, ring_bonds(8), 4, 4, 4.0),
    ("t44 3+3", 16, torus_bonds(4, 4), 3, 3, 4.0),
    ("t44 3+4", 16, torus_bonds(4, 4), 3, 4, 2.5),
    ("ring9 4+3", 9, ring_bonds(9), 4, 3, 3.0),
    ("ring10 0+5", 10, ring_bonds(10), 0, 5, 0.0),
    ("ring10 5+0", 10, ring_bonds(10), 5, 0, 0.0),
    ("t33 4+5", 9, torus_bonds(3, 3), 4, 5, 6.0),
]


@pytest.mark.parametrize("label,n_sites,bonds,n_up,n_dn,U", CASES, ids=[c[0] for c in CASES])
def test_fused_coefficients_match_oracle(label, n_sites, bonds, n_up, n_dn, U):
    """20 fused float64 steps: a_j, b_j equal the oracle's Alg. 1 to 1e-12 max|a|, and the stored vector
    after the run is b_21 f_21 (the contract of ed_lanczos_step)."""
    m = Model(n_sites, bonds, n_up, n_dn, 1.0, U)
    steps = min(20, m.dim - 1)
    h = ham(n_sites, bonds, n_up, n_dn, 1.0, U, "f64")
    x_host, x = seeded_start(11, h.dim, "f64")
    run = h.lanczos(steps + 2)
    announce("fused f64 %s, %d steps" % (label, steps))
    run.init(x)
    run.steps(steps)
    got = run.read()
    ref = lanczos(m.hv, x_host, steps + 1, vectors=True)
    amax = np.max(np.abs(ref["a"]))
    assert got["steps"] == steps and got["status"] == ed.ED_OK
    assert np.max(np.abs(got["a"] - ref["a"][:steps])) <= 1e-12 * amax
    assert np.max(np.abs(got["b"] - ref["b"][:steps + 1])) <= 1e-12 * amax
    stored = run.f_cur.cpu().numpy()
    bn = got["b"][steps]
    assert abs(np.linalg.norm(stored) - bn) <= 1e-12 * bn
    assert float(np.max(np.abs(stored / bn - ref["f"][steps]))) <= 1e-9


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_equals_reference_step(dtype):
    """The fused run and the reference step follow the same Alg. 1 order: a_j, b_j agree to rounding."""
    bonds = torus_bonds(4, 4)
    h = ham(16, bonds, 4, 4, 1.0, 4.0, dtype)
    _, x = seeded_start(13, h.dim, dtype)
    r1, r2 = h.lanczos(30), h.lanczos(30)
    announce("fused vs reference step %s t44 4+4" % dtype)
    r1.init(x)
    r1.steps(25)
    r2.init(x)
    for _ in range(25):
        r2.step()
    g1, g2 = r1.read(), r2.read()
    tol = 1e-11 if dtype == "f64" else 1e-5
    amax = np.max(np.abs(g2["a"]))
    assert g1["steps"] == g2["steps"] == 25
    assert np.max(np.abs(g1["a"] - g2["a"])) <= tol * amax
    assert np.max(np.abs(g1["b"] - g2["b"])) <= tol * amax


def test_fused_runs_chain_and_mix_with_reference_steps():
    """Runs of fused steps, single reference steps and fused runs again continue one Alg. 1 iteration."""
    m = Model(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0)
    h = ham(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0, "f64")
    x_host, x = seeded_start(17, h.dim, "f64")
    run = h.lanczos(40)
    announce("fused runs chained t44 3+3")
    run.init(x)
    run.steps(5)
    run.step()
    run.steps(1)
    run.steps(7)
    run.step()
    got = run.read()
    ref = lanczos(m.hv, x_host, 15)
    amax = np.max(np.abs(ref["a"]))
    assert got["steps"] == 15
    assert np.max(np.abs(got["a"] - ref["a"])) <= 1e-12 * amax
    assert np.max(np.abs(got["b"] - ref["b"])) <= 1e-12 * amax


def test_fused_mixed_e0_and_local_orthogonality():
    """Mixed form (float32 vectors, float64 scalars, local re-orthogonalisation): E0 of the 8-ring within
    1e-6 of dense LAPACK after 100 fused steps."""
    m = Model(8, ring_bonds(8), 4, 4, 1.0, 4.0)
    e_exact = float(np.linalg.eigvalsh(m.dense())[0])
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, "f32")
    _, x = seeded_start(1, h.dim, "f32")
    run = h.lanczos(100)
    announce("fused mixed ring8 100 steps")
    run.init(x)
    run.steps(100)
    got = run.read()
    e0 = tridiag_lowest(got["a"], got["b"][1:100])
    assert got["steps"] == 100
    assert abs(e0 - e_exact) <= 1e-6 * abs(e_exact)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_freezes_at_max_steps(dtype):
    """Steps launched past max_steps are no-ops; the closing update still gives b_{m+1} and F_{m+1}."""
    m = Model(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0)
    h = ham(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0, dtype)
    x_host, x = seeded_start(19, h.dim, dtype)
    run = h.lanczos(7)
    announce("fused freeze %s" % dtype)
    run.init(x)
    run.steps(10)
    got = run.read()
    assert got["steps"] == 7 and got["status"] == ed.ED_NOT_CONVERGED
    ref = lanczos(m.hv, x_host, 7)
    tol = 1e-12 if dtype == "f64" else 1e-5
    amax = np.max(np.abs(ref["a"]))
    assert np.max(np.abs(got["b"] - ref["b"])) <= tol * amax


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_breakdown_on_invariant_subspace(dtype):
    """Two-site model (dim 4): the Krylov space closes after at most 4 steps; the run reports a breakdown
    and T gives the closed-form E0 = (U - sqrt(U^2 + 16 t^2)) / 2."""
    U = 4.0
    h = ham(2, two_site_bonds(), 1, 1, 1.0, U, dtype)
    _, x = seeded_start(3, 4, dtype)
    run = h.lanczos(10)
    announce("fused breakdown two-site %s" % dtype)
    run.init(x)
    run.steps(10)
    got = run.read()
    assert got["status"] == ed.ED_BREAKDOWN and got["steps"] <= 4
    e0 = tridiag_lowest(got["a"], got["b"][1:got["steps"]])
    exact = (U - np.sqrt(U * U + 16.0)) / 2.0
    assert abs(e0 - exact) <= (1e-12 if dtype == "f64" else 1e-6) * abs(exact)


def test_ground_energy_newest_vector_after_partial_chunk():
    """ed_ground_energy with max_steps not a multiple of its step chunk: afterwards f_cur holds the newest
    vector b_{m+1} f_{m+1}, as after m single steps."""
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
    amax = np.max(np.abs(gb["a"]))
    assert np.max(np.abs(ga["a"][:20] - gb["a"][:20])) <= 1e-11 * amax
    fa, fb = ra.f_cur.cpu().numpy(), rb.f_cur.cpu().numpy()
    # both are b_101 f_101 of their own (rounding-wise different) runs: compare what rounding leaves alone
    assert abs(np.linalg.norm(fa) - ga["b"][100]) <= 1e-12 * ga["b"][100]
    assert abs(np.linalg.norm(fb) - gb["b"][100]) <= 1e-12 * gb["b"][100]
    # f_101 is orthogonal to f_100 (the vector before it) in both runs
    assert abs(float(fa @ ra.f_prev.cpu().numpy())) <= 1e-8 * np.linalg.norm(fa) * np.linalg.norm(ra.f_prev.cpu().numpy())
