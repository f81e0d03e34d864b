"""32-bit device tables: the format for per-spin dimensions above 15-bit ranks.

Small sectors are run with the 32-bit format forced, against the 16-bit format
(same arithmetic, so the same bits, for every launch tile) and the oracle.  At
full size, the 18-site chain at 9 + 9 (D = 48620^2 = 2,363,904,400; 18.9 GB per
float64 vector) is checked on rows the oracle recomputes one by one, and at
U = 0 against the closed-form ground energy.
"""

import ctypes
import math

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.hamiltonian import Model
from synth import complete_bonds, ring_bonds, start_vector, torus_bonds
from tests.gpu_util import announce, seeded_start

pytestmark = pytest.mark.gpu

SMALL = [
    ("ring8_3x2", 8, ring_bonds(8), 3, 2),
    ("t44_3x3", 16, torus_bonds(4, 4), 3, 3),
    ("t44_5x2", 16, torus_bonds(4, 4), 5, 2),
    ("ring6_0x3", 6, ring_bonds(6), 0, 3),
    ("complete12_6x5", 12, complete_bonds(12), 6, 5),   # strides 40 and 40: eight-chunk variants
]


def _pair(ns, bonds, nu, nd, U, dtype, eb_up, eb_dn):
    up = ed.SpinTables(ns, bonds, nu, "cuda:0", eb_up)
    dn = ed.SpinTables(ns, bonds, nd, "cuda:0", eb_dn)
    return ed.Hamiltonian(up, dn, 1.0, U, dtype)


def _tile_count():
    nu, nd = ctypes.c_int32(0), ctypes.c_int32(0)
    ed.lib().ed_tile_count(ctypes.byref(nu), ctypes.byref(nd))
    return nu.value, nd.value


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
def test_wide_tables_give_the_narrow_bits_for_every_tile(case, dtype):
    name, ns, bonds, nu, nd = case
    narrow = _pair(ns, bonds, nu, nd, 2.5, dtype, 2, 2)
    wide = _pair(ns, bonds, nu, nd, 2.5, dtype, 4, 4)
    assert wide.up.entry_bytes == 4 and wide.dn.entry_bytes == 4
    x_host, x = seeded_start(61, narrow.dim, dtype)
    announce("wide tables %s %s" % (name, dtype))
    ref = narrow.hv(x).clone()
    m = Model(ns, bonds, nu, nd, 1.0, 2.5)
    want = m.hv(x_host)
    got = wide.hv(x).double().cpu().numpy()
    scale = max(1.0, float(np.max(np.abs(want))))
    assert float(np.max(np.abs(got - want))) <= (1e-12 if dtype == "f64" else 2e-5) * scale
    n_up, n_dn = _tile_count()
    for ui in range(n_up):
        for di in ([0] if ui else range(n_dn)):
            narrow.tile = wide.tile = ui | (di << 8)
            assert torch.equal(wide.hv(x), ref), (ui, di, wide.tile_params())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mixed_formats_per_species(dtype):
    """Up spin with 32-bit tables, down spin with 16-bit ones, and the reverse."""
    ns, bonds, nu, nd = 16, torus_bonds(4, 4), 4, 3
    m = Model(ns, bonds, nu, nd, 1.0, 3.0)
    x_host, x = seeded_start(62, m.dim, dtype)
    want = m.hv(x_host)
    for eb in ((4, 2), (2, 4)):
        h = _pair(ns, bonds, nu, nd, 3.0, dtype, *eb)
        announce("mixed formats %s %s" % (eb, dtype))
        got = h.hv(x).double().cpu().numpy()
        scale = max(1.0, float(np.max(np.abs(want))))
        assert float(np.max(np.abs(got - want))) <= (1e-12 if dtype == "f64" else 2e-5) * scale


def test_wide_lanczos_is_the_narrow_run():
    """A Lanczos run over 32-bit tables repeats the 16-bit run exactly (same launch shape: the
    rows are shorter than 1024, so both formats take 256-thread down-part workgroups)."""
    narrow = _pair(16, torus_bonds(4, 4), 3, 3, 4.0, "f64", 2, 2)
    wide = _pair(16, torus_bonds(4, 4), 3, 3, 4.0, "f64", 4, 4)
    assert narrow.tile_params() == wide.tile_params()
    _, x = seeded_start(63, narrow.dim, "f64")
    announce("wide lanczos 4x4 3+3")
    r0 = narrow.ground_energy(x, 60, tol=0.0)
    r1 = wide.ground_energy(x, 60, tol=0.0)
    assert np.array_equal(r0["a"], r1["a"]) and np.array_equal(r0["b"], r1["b"]) and r0["e0"] == r1["e0"]


# ---------------------------------------------------------------------------
# full size: the 18-site chain at 9 + 9

RING18 = (18, ring_bonds(18), 9)
RING18_ROWS = [0, 1, 24310, 48618, 48619]


@pytest.fixture(scope="module")
def ring18_tables():
    ns, bonds, n = RING18
    announce("ring18 9+9 tables")
    tab = ed.SpinTables(ns, bonds, n, "cuda:0")
    assert tab.dim == 48620 and tab.entry_bytes == 4
    yield tab
    del tab
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_ring18_9x9_sampled_rows(ring18_tables, dtype):
    ns, bonds, n = RING18
    h = ed.Hamiltonian(ring18_tables, ring18_tables, 1.0, 4.0, dtype)
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    assert h.dim == 2363904400
    x_host = start_vector(8, h.dim)
    if dtype == "f32":
        x32 = x_host.astype(np.float32)
        del x_host
        x = torch.from_numpy(x32).to("cuda:0")
        x_host = x32.astype(np.float64)
        del x32
    else:
        x = torch.from_numpy(x_host).to("cuda:0")
    announce("hv full ring18 9+9 %s dim=%d" % (dtype, h.dim))
    y = h.hv(x)
    torch.cuda.synchronize()
    got = y.view(h.dim_up, h.dim_dn)[RING18_ROWS].double().cpu().numpy()
    del x, y
    torch.cuda.empty_cache()
    ref = Model(ns, bonds, n, n, 1.0, 4.0).hv_rows(x_host, RING18_ROWS)
    del x_host
    scale = max(1.0, float(np.max(np.abs(ref))))
    if dtype == "f64":
        assert float(np.max(np.abs(got - ref))) <= 1e-12 * scale
    else:
        assert np.linalg.norm(got - ref) <= 2e-6 * np.linalg.norm(ref)
        assert float(np.max(np.abs(got - ref))) <= 2e-5 * scale


def test_full_size_ring18_9x9_u0_closed_form(ring18_tables):
    """At U = 0 the ground state fills the 9 lowest levels -2t cos(2 pi k / 18) of each species;
    with an odd particle number the Jordan-Wigner string leaves the ring periodic, k = 0, +-1..+-4."""
    h = ed.Hamiltonian(ring18_tables, ring18_tables, 1.0, 0.0, "f64")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    exact = 2.0 * sum(-2.0 * math.cos(2.0 * math.pi * k / 18.0) for k in range(-4, 5))
    g = torch.Generator(device="cuda:0")
    g.manual_seed(9)
    x = torch.rand(h.dim, dtype=torch.float64, device="cuda:0", generator=g) - 0.5
    announce("ground energy ring18 9+9 U=0 f64 dim=%d" % h.dim)
    r = h.ground_energy(x, 200, tol=1e-11, check_every=15)
    del x
    torch.cuda.empty_cache()
    assert r["status"] == 0, (r["status"], r["steps"])
    assert abs(r["e0"] - exact) <= 1e-9 * abs(exact), (r["e0"], exact)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_ring18_9x9_band_order_windowed_rows(dtype):
    """The bench's scale run: both species in band order, the cached tile, which stages each 8192-state
    column block of a row with its neighbour window in LDS (k_down_win).  Five full rows of H x, carried
    back to the ascending order, against the oracle."""
    ns, bonds, n = RING18
    announce("ring18 9+9 band-order tables")
    tab = ed.SpinTables(ns, bonds, n, "cuda:0", order="band")
    h = ed.Hamiltonian(tab, tab, 1.0, 4.0, dtype)
    src = ed.api.apply_tuned_tile(h, tune_if_missing=False)
    assert src == "cache" and h.tile_params()["dn_kind"] == 2, (src, h.tile_params())
    x_host = start_vector(8, h.dim)
    if dtype == "f32":
        x32 = x_host.astype(np.float32)
        del x_host
        x = torch.from_numpy(x32).to("cuda:0")
        x_host = x32.astype(np.float64)
        del x32
    else:
        x = torch.from_numpy(x_host).to("cuda:0")
    announce("hv full ring18 9+9 band order %s dim=%d, tile %d" % (dtype, h.dim, h.tile))
    xo = h.to_basis_order(x)
    del x
    y = h.hv(xo)
    del xo
    ya = h.to_ascending(y)
    del y
    torch.cuda.synchronize()
    got = ya.view(h.dim_up, h.dim_dn)[RING18_ROWS].double().cpu().numpy()
    del ya, h, tab
    torch.cuda.empty_cache()
    ref = Model(ns, bonds, n, n, 1.0, 4.0).hv_rows(x_host, RING18_ROWS)
    del x_host
    scale = max(1.0, float(np.max(np.abs(ref))))
    if dtype == "f64":
        assert float(np.max(np.abs(got - ref))) <= 1e-12 * scale
    else:
        assert np.linalg.norm(got - ref) <= 2e-6 * np.linalg.norm(ref)
        assert float(np.max(np.abs(got - ref))) <= 2e-5 * scale
