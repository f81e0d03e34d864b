"""ed_ground_energy_noalloc (the run on the library's device scratch) against ed_ground_energy (the run
on a caller's workspace): the same step kernels, so the same coefficients and E0 bit for bit, on two
calls in a row, the second on a smaller instance; and the capacity checks."""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from synth import ring_bonds, start_vector, torus_bonds
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _both(h, seed, max_steps, tol, check_every):
    x = torch.from_numpy(start_vector(seed, h.dim)).to("cuda:0", h.torch_dtype)
    r_ws = h.lanczos(max_steps).ground_energy(x, tol=tol, check_every=check_every)
    run = h.lanczos(max_steps)
    r_na = run.ground_energy_noalloc(x, tol=tol, check_every=check_every)
    return r_ws, r_na, run


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_equals_workspace_run_twice(dtype):
    bonds = torus_bonds(4, 4)
    big = ed.Hamiltonian(ed.SpinTables(16, bonds, 4, "cuda:0"), ed.SpinTables(16, bonds, 4, "cuda:0"), 1.0, 4.0,
                         dtype)
    small = ed.Hamiltonian(ed.SpinTables(8, ring_bonds(8), 4, "cuda:0"), ed.SpinTables(8, ring_bonds(8), 4, "cuda:0"),
                           1.0, 4.0, dtype)
    for h, seed, label in ((big, 31, "4x4 4+4"), (small, 1, "8-ring 4+4")):
        announce("noalloc run %s %s" % (label, dtype))
        r_ws, r_na, run = _both(h, seed, 200, 1e-10 if dtype == "f64" else 1e-7, 12)
        assert r_na["status"] == r_ws["status"]
        assert r_na["steps"] == r_ws["steps"] and r_na["e0"] == r_ws["e0"], (label, r_na["e0"], r_ws["e0"])
        assert np.array_equal(r_na["a"], r_ws["a"]) and np.array_equal(r_na["b"], r_ws["b"])
        st = run.read()
        assert st["steps"] >= r_na["steps"]


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    h = ed.Hamiltonian(ed.SpinTables(8, ring_bonds(8), 4, "cuda:0"), ed.SpinTables(8, ring_bonds(8), 4, "cuda:0"),
                       1.0, 4.0, "f64")
    x = torch.from_numpy(start_vector(1, h.dim)).to("cuda:0", torch.float64)
    announce("noalloc capacity checks")
    with pytest.raises(ed.EdError) as err:
        h.lanczos(5000).ground_energy_noalloc(x)
    assert err.value.code == ed._ffi.ED_ECAPACITY
