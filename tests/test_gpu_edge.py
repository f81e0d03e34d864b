"""Edge cases of the device path: the widest hopping tables, species without hopping,
and the limits the batched launch enforces."""

import math

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from paper_1511_00863_amd import EdError
from synth import complete_bonds, ring_bonds
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_widest_tables_u0_closed_form(dtype):
    """All-to-all hopping on 12 sites, 6+6, U = 0: 36 hops per state (table stride 40).
    One-particle levels -t(n-1) once and +t (n-1 times): E0 = 2 (-(n-1) + (N-1)) t = -12 t."""
    h = ham(12, complete_bonds(12), 6, 6, 1.0, 0.0, dtype)
    assert h.up.width == 36 and h.dn.width == 36
    _, x = seeded_start(31, h.dim, dtype)
    announce("complete12 6+6 U=0 %s" % dtype)
    r = h.ground_energy(x, 60, tol=1e-12 if dtype == "f64" else 1e-7, check_every=5)
    assert abs(r["e0"] - (-12.0)) <= (1e-10 if dtype == "f64" else 1e-6) * 12.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nu,nd", [(3, 0), (0, 3)])
def test_single_species_band_sum(nu, nd, dtype):
    """One species on the 8-ring (the other empty, so its table is empty): E0 is the band
    sum of the three lowest levels -2 cos(2 pi k / 8), i.e. -2 - 2 sqrt(2), whatever U."""
    h = ham(8, ring_bonds(8), nu, nd, 1.0, 5.0, dtype)
    assert h.dim == 56
    _, x = seeded_start(32, h.dim, dtype)
    announce("ring8 %d+%d single species %s" % (nu, nd, dtype))
    r = h.ground_energy(x, 56, tol=1e-12 if dtype == "f64" else 1e-7, check_every=4)
    exact = -2.0 - 2.0 * math.sqrt(2.0)
    assert abs(r["e0"] - exact) <= (1e-10 if dtype == "f64" else 1e-6) * abs(exact)


def test_batch_rejects_unsupported_shapes():
    """The batched launch handles tables up to stride 32 and both species hopping;
    anything else is refused on the host with a clear code, before any launch."""
    wide = ham(12, complete_bonds(12), 6, 6, 1.0, 1.0, "f32")
    _, x = seeded_start(33, wide.dim, "f32")
    announce("batch rejects stride 40")
    with pytest.raises(EdError) as e:
        ed.ground_energy_batch([wide], [x], 50, tol=1e-6)
    assert e.value.code == -3
    wide_up = ham(16, complete_bonds(16), 8, 1, 1.0, 1.0, "f32")   # up stride 64, down stride 16
    _, z = seeded_start(35, wide_up.dim, "f32")
    with pytest.raises(EdError) as e:
        ed.ground_energy_batch([wide_up], [z], 50, tol=1e-6)
    assert e.value.code == -3
    no_up = ham(8, ring_bonds(8), 0, 3, 1.0, 1.0, "f32")
    _, y = seeded_start(34, no_up.dim, "f32")
    with pytest.raises(EdError) as e:
        ed.ground_energy_batch([no_up], [y], 50, tol=1e-6)
    assert e.value.code == -1
