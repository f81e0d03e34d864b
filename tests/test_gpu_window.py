"""Rows too long for LDS, by column blocks with their neighbour windows staged in LDS (k_down_win over
ed_row_windows): the same H x bits as the kernel that gathers such rows from global memory, and the
oracle's H x and Alg. 1 coefficients in the ascending basis.

Case: 18-site chain, 1 up and 9 down particles (18 x 48,620 = 875,160 states).  The down species is in
band order (ed_band_order), where a block of 8192 states and all its neighbours span at most about
15,000 states; its rows (389 KB in FP64, 194 KB in FP32) do not fit LDS, and it takes 32-bit tables.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.hamiltonian import Model
from oracle.lanczos import lanczos
from synth import ring_bonds
from tests.gpu_util import announce, seeded_start

pytestmark = pytest.mark.gpu

NS, NU, ND = 18, 1, 9


@pytest.fixture(scope="module")
def species():
    bonds = ring_bonds(NS)
    up = ed.SpinTables(NS, bonds, NU, "cuda:0")
    dn = ed.SpinTables(NS, bonds, ND, "cuda:0", order="band")
    return bonds, up, dn


def _window_tiles(h):
    nu_, nd_ = ctypes.c_int32(0), ctypes.c_int32(0)
    ed.lib().ed_tile_count(ctypes.byref(nu_), ctypes.byref(nd_))
    return [di for di in range(nd_.value) if h.tile_params(di << 8)["dn_kind"] == 2]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_window_tiles_match_global_rows_and_oracle(species, dtype):
    bonds, up, dn = species
    assert dn.entry_bytes == 4 and dn.win_cols > 0 and (dn.win_max + 1) * (8 if dtype == "f64" else 4) <= 152 * 1024
    h = ed.Hamiltonian(up, dn, 1.0, 2.5, dtype)
    wins = _window_tiles(h)
    assert wins, "no windowed tile applies"
    x_host, x = seeded_start(97, h.dim, dtype)
    xo = h.to_basis_order(x)
    announce("windowed down rows 18-site 1+9 %s, tiles %s" % (dtype, wins))
    h.tile = 0
    ref = h.hv(xo).clone()
    for di in wins:
        h.tile = di << 8
        assert torch.equal(h.hv(xo), ref), (di, h.tile_params())
    m = Model(NS, bonds, NU, ND, 1.0, 2.5)
    got = h.to_ascending(ref).double().cpu().numpy()
    want = m.hv(x_host)
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert float(np.max(np.abs(got - want))) <= tol * max(1.0, float(np.max(np.abs(want))))


def test_window_tile_lanczos_matches_oracle(species):
    """Alg. 1 on the windowed tile from P f_1: the oracle's a_j, b_j (float64, 20 steps)."""
    bonds, up, dn = species
    h = ed.Hamiltonian(up, dn, 1.0, 2.5, "f64")
    wins = _window_tiles(h)
    h.tile = wins[0] << 8
    x_host, x = seeded_start(98, h.dim, "f64")
    announce("windowed down rows, lanczos 18-site 1+9 f64, tile %d" % h.tile)
    r = h.ground_energy(h.to_basis_order(x), 30, tol=0.0)
    ref = lanczos(Model(NS, bonds, NU, ND, 1.0, 2.5).hv, x_host, 20)
    amax = np.max(np.abs(ref["a"]))
    assert np.max(np.abs(r["a"][:20] - ref["a"])) <= 1e-12 * amax
    assert np.max(np.abs(r["b"][:21] - ref["b"])) <= 1e-12 * amax


def test_window_tile_mixed_form_energy(species):
    """The mixed form (float32 vectors, float64 partial sums) on a windowed tile: E0 after 60 steps within
    1e-6 of the float64 run on the global-gather tile."""
    bonds, up, dn = species
    _, x64 = seeded_start(99, up.dim * dn.dim, "f64")
    h64 = ed.Hamiltonian(up, dn, 1.0, 2.5, "f64")
    announce("windowed down rows, mixed form 18-site 1+9")
    r64 = h64.ground_energy(h64.to_basis_order(x64), 60, tol=0.0)
    h = ed.Hamiltonian(up, dn, 1.0, 2.5, "f32")
    h.tile = _window_tiles(h)[0] << 8
    r = h.ground_energy(h.to_basis_order(x64.float()), 60, tol=0.0)
    assert r["steps"] == 60
    assert abs(r["e0"] - r64["e0"]) <= 1e-6 * abs(r64["e0"]), (r["e0"], r64["e0"])


def test_window_wider_than_its_room_falls_back_to_global_rows(species):
    """A window pair wider than win_max (here block 0 given the whole row) is not staged: that block is
    gathered from global memory, and H x keeps the global-gather kernel's bits."""
    bonds, up, dn = species
    h = ed.Hamiltonian(up, dn, 1.0, 2.5, "f64")
    di = _window_tiles(h)[0]
    _, x = seeded_start(100, h.dim, "f64")
    xo = h.to_basis_order(x)
    h.tile = 0
    ref = h.hv(xo).clone()
    saved = dn.dev_win
    try:
        bad = saved.clone()
        bad[0], bad[1] = 0, dn.dim
        assert dn.dim > dn.win_max
        dn.dev_win = bad
        h.tile = di << 8
        announce("windowed down rows, an over-wide window for block 0")
        assert torch.equal(h.hv(xo), ref)
    finally:
        dn.dev_win = saved
