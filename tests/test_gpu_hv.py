"""Parity of the HIP H.v (Eq. 3-5 plus the U term) with the oracle, element by element."""

import numpy as np
import pytest
import torch

from oracle.hamiltonian import Model
from synth import complete_bonds, ring_bonds, torus_bonds, two_site_bonds
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu

# (name, n_sites, bonds, n_up, n_dn, t, U)
SMALL = [
    ("two_site", 2, two_site_bonds(), 1, 1, 1.0, 4.0),
    ("ring8_4x4_U4", 8, ring_bonds(8), 4, 4, 1.0, 4.0),
    ("ring8_3x2_U2", 8, ring_bonds(8), 3, 2, 0.7, 2.0),
    ("ring6_0x3", 6, ring_bonds(6), 0, 3, 1.0, 3.0),
    ("ring6_3x0", 6, ring_bonds(6), 3, 0, 1.0, 3.0),
    ("ring6_6x2_full", 6, ring_bonds(6), 6, 2, 1.0, 1.5),
    ("t44_3x3_U4", 16, torus_bonds(4, 4), 3, 3, 1.0, 4.0),
    ("t44_2x4_U1.5", 16, torus_bonds(4, 4), 2, 4, 1.0, 1.5),
    ("t44_4x1_U8", 16, torus_bonds(4, 4), 4, 1, 1.0, 8.0),
    ("ring12_6x5", 12, ring_bonds(12), 6, 5, 1.0, 2.0),
    # all-to-all hopping: the widest tables (36 hops -> stride 40; 64 hops = the largest stride accepted)
    ("complete12_6x6", 12, complete_bonds(12), 6, 6, 1.0, 2.5),
    ("complete16_8x1_maxwidth_up", 16, complete_bonds(16), 8, 1, 1.0, 3.0),
    ("complete16_1x8_maxwidth_dn", 16, complete_bonds(16), 1, 8, 0.6, 3.0),
]


def _tol_check(y, ref, dtype):
    scale = max(1.0, float(np.max(np.abs(ref))))
    err = np.abs(y - ref)
    if dtype == "f64":
        assert float(err.max()) <= 1e-12 * scale
    else:
        assert np.linalg.norm(y - ref) <= 2e-6 * np.linalg.norm(ref) + 1e-30
        assert float(err.max()) <= 2e-5 * scale


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
def test_hv_small_exact(case, dtype):
    name, ns, bonds, nu, nd, t, U = case
    m = Model(ns, bonds, nu, nd, t, U)
    h = ham(ns, bonds, nu, nd, t, U, dtype)
    x_host, x = seeded_start(7, m.dim, dtype)
    announce("hv %s %s dim=%d" % (name, dtype, m.dim))
    y = h.hv(x)
    torch.cuda.synchronize()
    _tol_check(y.double().cpu().numpy(), m.hv(x_host), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hv_unit_vectors_give_columns(dtype):
    m = Model(6, ring_bonds(6), 2, 3, 1.0, 2.5)
    h = ham(6, ring_bonds(6), 2, 3, 1.0, 2.5, dtype)
    H = m.dense()
    for k in (0, 17, m.dim - 1):
        e = np.zeros(m.dim)
        e[k] = 1.0
        announce("hv unit column %d %s" % (k, dtype))
        y = h.hv(torch.from_numpy(e).to("cuda:0", h.torch_dtype))
        assert np.array_equal(y.double().cpu().numpy(), H[:, k])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name,nu,rows", [("t44_5x5", 5, [0, 1, 2047, 4366, 4367]),
                                          ("t44_8x8", 8, [0, 1, 6434, 12869])])
def test_hv_full_size_sampled_rows(name, nu, rows, dtype):
    """At the benchmark sizes: rows of H x recomputed one by one by the oracle."""
    bonds = torus_bonds(4, 4)
    m = Model(16, bonds, nu, nu, 1.0, 4.0)
    h = ham(16, bonds, nu, nu, 1.0, 4.0, dtype)
    x_host, x = seeded_start(5, m.dim, dtype)
    announce("hv full %s %s dim=%d" % (name, dtype, m.dim))
    y = h.hv(x)
    torch.cuda.synchronize()
    Y = y.view(m.dim_up, m.dim_dn)
    ref = m.hv_rows(x_host, rows)
    got = Y[rows].double().cpu().numpy()
    del y, Y, x
    _tol_check(got, ref, dtype)


def test_hv_linearity_and_symmetry_f64():
    """<u, H v> = <H u, v> and H(a u + v) = a H u + H v, at the 4x4 5+5 size."""
    bonds = torus_bonds(4, 4)
    h = ham(16, bonds, 5, 5, 1.0, 4.0, "f64")
    _, u = seeded_start(11, h.dim, "f64")
    _, v = seeded_start(12, h.dim, "f64")
    announce("hv symmetry 4x4 5+5")
    hu, hv_ = h.hv(u), h.hv(v)
    lhs, rhs = float(torch.dot(u, hv_)), float(torch.dot(hu, v))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    w = h.hv(2.5 * u + v)
    assert float((w - (2.5 * hu + hv_)).abs().max()) <= 1e-11 * float(w.abs().max())


def test_hv_rejects_aliasing():
    import paper_1511_00863_amd as ed
    h = ham(8, ring_bonds(8), 4, 4, 1.0, 4.0, "f64")
    _, x = seeded_start(1, h.dim, "f64")
    with pytest.raises(ed.EdError):
        h.hv(x, x)
