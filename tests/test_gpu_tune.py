"""The launch-configuration autotuner: every candidate tile computes the same H x bit for bit."""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from synth import complete_bonds, ring_bonds, torus_bonds
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ns,bonds,nu,nd", [(16, torus_bonds(4, 4), 4, 4), (16, torus_bonds(4, 4), 3, 5),
                                            (8, ring_bonds(8), 4, 4), (12, complete_bonds(12), 6, 6),
                                            # up tables of 3 chunks (width 20) and of 4 chunks (width 32,
                                            # the benchmark's shape)
                                            (16, torus_bonds(4, 4), 5, 5), (16, torus_bonds(4, 4), 8, 8),
                                            # odd row counts (the two-row down kernel's last block has one row)
                                            (11, ring_bonds(11), 3, 3), (15, ring_bonds(15), 7, 7)])
def test_every_tile_gives_identical_hv(ns, bonds, nu, nd, dtype):
    h = ham(ns, bonds, nu, nd, 1.0, 3.0, dtype)
    _, x = seeded_start(21, h.dim, dtype)
    announce("tune all tiles %d+%d %s" % (nu, nd, dtype))
    ref = h.hv(x).clone()
    import ctypes
    nu_, nd_ = ctypes.c_int32(0), ctypes.c_int32(0)
    ed.lib().ed_tile_count(ctypes.byref(nu_), ctypes.byref(nd_))
    for ui in range(nu_.value):
        for di in ([0] if ui else range(nd_.value)):
            h.tile = ui | (di << 8)
            y = h.hv(x)
            assert torch.equal(y, ref), (ui, di, h.tile_params())
    h.tile = 0
    r = h.tune(x, reps=1)
    assert r["tile"] & 0xFF < nu_.value and (r["tile"] >> 8) < nd_.value
    assert torch.equal(h.hv(x), ref)
    assert (r["up_ms"][1:] != 0).all()


def test_tuned_lanczos_matches_default():
    """A tile changes the number of partial-sum slots, hence the order of the float64
    reductions: coefficients agree to roundoff across tiles and bit for bit for one tile."""
    h = ham(16, torus_bonds(4, 4), 4, 4, 1.0, 2.0, "f64")
    _, x = seeded_start(22, h.dim, "f64")
    announce("tuned lanczos")
    r0 = h.ground_energy(x, 30)
    h.tune(x, reps=1)
    r1 = h.ground_energy(x, 30)
    r2 = h.ground_energy(x, 30)
    scale = np.max(np.abs(r0["a"]))
    assert np.max(np.abs(r0["a"][:20] - r1["a"][:20])) <= 1e-12 * scale
    assert np.array_equal(r1["a"], r2["a"]) and np.array_equal(r1["b"], r2["b"])
    assert abs(r0["e0"] - r1["e0"]) <= 1e-12 * abs(r0["e0"])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ns,bonds,nu,nd", [(16, torus_bonds(4, 4), 4, 4), (11, ring_bonds(11), 3, 3),
                                            (15, ring_bonds(15), 7, 7)])
def test_two_row_down_kernel_in_lanczos(ns, bonds, nu, nd, dtype):
    """The two-row down kernel (down tiles 10-12) in Lanczos runs, odd and even row counts: the same H x
    bits as the one-row kernel, so a run differs from the default tile's only through the order of the
    float64 partial sums (float64: coefficients to 1e-12; mixed form: E0 to 1e-6)."""
    import ctypes
    h = ham(ns, bonds, nu, nd, 1.0, 3.0, dtype)
    _, x = seeded_start(23, h.dim, dtype)
    nu_, nd_ = ctypes.c_int32(0), ctypes.c_int32(0)
    ed.lib().ed_tile_count(ctypes.byref(nu_), ctypes.byref(nd_))
    pairs = [di for di in range(nd_.value) if h.tile_params(di << 8)["dn_kind"] == 1]
    assert pairs, "no two-row tile applies"
    announce("two-row down kernel, lanczos %d+%d on %d sites %s, tiles %s" % (nu, nd, ns, dtype, pairs))
    h.tile = 0
    r0 = h.ground_energy(x, 40, tol=0.0)
    scale = np.max(np.abs(r0["a"]))
    for di in pairs:
        h.tile = di << 8
        r1 = h.ground_energy(x, 40, tol=0.0)
        assert r1["steps"] == r0["steps"]
        if dtype == "f64":
            assert np.max(np.abs(r0["a"][:20] - r1["a"][:20])) <= 1e-12 * scale, di
            assert abs(r0["e0"] - r1["e0"]) <= 1e-12 * abs(r0["e0"]), di
        else:
            assert abs(r0["e0"] - r1["e0"]) <= 1e-6 * abs(r0["e0"]), di
