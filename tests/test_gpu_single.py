"""One spin species: every particle has the same spin, so H is the full single-species hopping matrix.

The library runs this as the sector (N_up = 0, N_dn = N): one row of length D, which the down-part kernel
splits into column blocks (the rows are far longer than LDS), with no up part to add.  Parity with the
oracle on mid-size sectors (every launch tile, bit-identical across tiles), oracle-recomputed elements
at the paper's 26-site size, and the free-fermion ground energy (sum of the N lowest one-particle
levels) at full size.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.elements import hv_elements
from oracle.basis import basis_states
from oracle.hamiltonian import Model
from synth import ring_bonds, torus_bonds, workload
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu

# (name, n_sites, bonds, n_up, n_dn): long rows (no LDS staging), split into column blocks
MID = [
    ("ring19_0x6_16bit", 19, ring_bonds(19), 0, 6),       # D = 27,132: 16-bit tables, a float64 row above LDS
    ("ring20_0x7_32bit", 20, ring_bonds(20), 0, 7),       # D = 77,520: 32-bit tables
    ("t45_0x6_32bit", 20, torus_bonds(4, 5), 0, 6),       # D = 38,760
    ("ring18_1x7_rows", 18, ring_bonds(18), 1, 7),        # 18 rows of 31,824: column blocks of several rows
]


def _tol(dtype):
    return 1e-12 if dtype == "f64" else 2e-5


def _tile_count():
    nu, nd = ctypes.c_int32(0), ctypes.c_int32(0)
    ed.lib().ed_tile_count(ctypes.byref(nu), ctypes.byref(nd))
    return nu.value, nd.value


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", MID, ids=[c[0] for c in MID])
def test_long_rows_match_oracle_on_every_tile(case, dtype):
    name, ns, bonds, nu, nd = case
    m = Model(ns, bonds, nu, nd, 1.0, 2.0)
    h = ham(ns, bonds, nu, nd, 1.0, 2.0, dtype)
    x_host, x = seeded_start(81, m.dim, dtype)
    announce("long rows %s %s dim=%d" % (name, dtype, m.dim))
    ref = h.hv(x).clone()
    want = m.hv(x_host)
    got = ref.double().cpu().numpy()
    assert float(np.max(np.abs(got - want))) <= _tol(dtype) * max(1.0, float(np.max(np.abs(want))))
    _, n_dn = _tile_count()
    for di in range(1, n_dn):
        h.tile = di << 8
        assert torch.equal(h.hv(x), ref), (di, h.tile_params())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_wavefront_chunk_counts_give_the_same_bits(dtype):
    """With ed_ham.wch_dn the down part of a species alone reads only the table chunks of each wavefront's
    widest column; H x and 30 Lanczos steps are the same bits as reading every chunk (16- and 32-bit
    tables, every launch tile)."""
    for name, ns, bonds, n in (("ring19_0x6", 19, ring_bonds(19), 6), ("ring20_0x7", 20, ring_bonds(20), 7),
                               ("t45_0x6", 20, torus_bonds(4, 5), 6)):
        h = ham(ns, bonds, 0, n, 1.0, 2.0, dtype)
        assert h.dn.dev_wch is not None
        _, x = seeded_start(85, h.dim, dtype)
        announce("wavefront chunk counts %s %s dim=%d" % (name, dtype, h.dim))
        wch = h.dn.dev_wch
        _, n_dn = _tile_count()
        for di in range(n_dn):
            h.tile = di << 8
            h.dn.dev_wch = wch
            y1 = h.hv(x).clone()
            r1 = h.ground_energy(x, 30, tol=0.0)
            h.dn.dev_wch = None
            y0 = h.hv(x).clone()
            r0 = h.ground_energy(x, 30, tol=0.0)
            assert torch.equal(y0, y1), (name, di)
            assert np.array_equal(r0["a"], r1["a"]) and np.array_equal(r0["b"], r1["b"]), (name, di)
        h.dn.dev_wch = wch


def test_single_species_lanczos_matches_oracle():
    """Alg. 1 coefficients of a one-species float64 run against the oracle's Lanczos on the same start."""
    from oracle.lanczos import lanczos
    ns, bonds, n = 20, ring_bonds(20), 7
    m = Model(ns, bonds, 0, n, 1.0, 0.0)
    h = ham(ns, bonds, 0, n, 1.0, 0.0, "f64")
    x_host, x = seeded_start(82, m.dim, "f64")
    announce("one-species lanczos ring20 7 f64")
    r = h.ground_energy(x, 40, tol=0.0)
    ref = lanczos(m.hv, x_host, 20)
    amax = np.max(np.abs(ref["a"]))
    assert np.max(np.abs(r["a"][:20] - ref["a"])) <= 1e-12 * amax
    assert np.max(np.abs(r["b"][:21] - ref["b"])) <= 1e-12 * amax


def test_single_species_mixed_e0():
    ns, bonds, n = 20, ring_bonds(20), 7
    h = ham(ns, bonds, 0, n, 1.0, 0.0, "f32")
    _, x = seeded_start(84, h.dim, "f32")
    announce("one-species lanczos ring20 7 mixed")
    r = h.ground_energy(x, 150, tol=0.0)
    exact = _free_fermion_e0(ns, bonds, n)
    assert abs(r["e0"] - exact) <= 1e-6 * abs(exact)


def _free_fermion_e0(n_sites, bonds, n):
    adj = np.zeros((n_sites, n_sites))
    for i, j in bonds:
        adj[i, j] -= 1.0
        adj[j, i] -= 1.0
    return float(np.sort(np.linalg.eigvalsh(adj))[:n].sum())


@pytest.mark.parametrize("name", ["ring26_0x13", "torus5x6_0x9"])
def test_full_size_single_species_free_fermion_energy(name):
    """The paper's one-species sizes (26-site chain; a 30-site lattice): E0 = sum of the N lowest levels."""
    wl = workload(name)
    h = ed.Hamiltonian.from_lattice(wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, wl.t, wl.U, "f64", "cuda:0")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    _, x = seeded_start(wl.seed, h.dim, "f64")
    announce("ground energy %s f64 dim=%d" % (name, h.dim))
    r = h.ground_energy(x, 300, tol=1e-12, check_every=15)
    exact = _free_fermion_e0(wl.n_sites, wl.bonds, wl.n_dn)
    assert r["status"] == 0, (r["status"], r["steps"])
    assert abs(r["e0"] - exact) <= 1e-9 * abs(exact), (r["e0"], exact)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_ring26_sampled_elements(dtype):
    """26 sites, 13 particles (D = 10,400,600): elements of H x recomputed one by one from the operators."""
    wl = workload("ring26_0x13")
    h = ed.Hamiltonian.from_lattice(wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, wl.t, wl.U, dtype, "cuda:0")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    x_host, x = seeded_start(wl.seed, h.dim, dtype)
    announce("hv full ring26 13 %s dim=%d" % (dtype, h.dim))
    y = h.hv(x).double().cpu().numpy()
    rng = np.random.default_rng(83)
    picks = sorted(set([0, 1, h.dim // 2, h.dim - 2, h.dim - 1] + rng.integers(0, h.dim, 400).tolist()))
    st_dn = basis_states(wl.n_sites, wl.n_dn)
    ref = hv_elements(wl.n_sites, wl.bonds, np.zeros(1, dtype=np.uint64), st_dn, wl.t, wl.U, x_host, picks)
    got = y[picks]
    assert float(np.max(np.abs(got - ref))) <= _tol(dtype) * max(1.0, float(np.max(np.abs(ref))))
