"""Complex hopping amplitudes (the paper's checkerboard lattice has complex nearest-neighbour hoppings).

The device keeps complex vectors as (re, im) pairs: H x uses the complex up- and down-part kernels, the rest
of the Lanczos step runs on the pairs as real values.  Parity with the oracle's complex matrices and
element-by-element H x, the oracle's Hermitian Lanczos, U = 0 band sums of the one-particle Hermitian
matrix, and the two-pass ground state's residual.
"""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.elements import hv_elements
from oracle.hamiltonian import Model
from oracle.lanczos import lanczos
from synth import checkerboard_terms, ring_bonds, start_vector_complex, workload
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

CB = checkerboard_terms(3, 3, 1.0, np.pi / 4, 0.3, 0.2)
CB_BONDS, CB_AMPS = [b for b, _ in CB], [a for _, a in CB]
_R = np.random.default_rng(7)
RING_AMPS = list(_R.uniform(-1, 1, 6) + 1j * _R.uniform(-1, 1, 6))

# (name, n_sites, bonds, amps, n_up, n_dn)
CASES = [
    ("checker18_2x1", 18, CB_BONDS, CB_AMPS, 2, 1),
    ("checker18_2x2", 18, CB_BONDS, CB_AMPS, 2, 2),
    ("ring6_2x3_random", 6, ring_bonds(6), RING_AMPS, 2, 3),
    ("checker18_0x3", 18, CB_BONDS, CB_AMPS, 0, 3),
    ("checker18_0x6_long", 18, CB_BONDS, CB_AMPS, 0, 6),     # a 297 KB complex row: column blocks (FP64)
    ("checker18_1x6_long", 18, CB_BONDS, CB_AMPS, 1, 6),     # 18 such rows
]


def _ham(ns, bonds, amps, nu, nd, U, dtype):
    return ed.Hamiltonian.from_lattice(ns, bonds, nu, nd, 1.0, U, dtype, "cuda:0", amps=amps)


def _start(seed, dim, dtype):
    """(host complex128 copy as the device sees it, device tensor)."""
    x = start_vector_complex(seed, dim)
    if dtype == "f32":
        x = x.astype(np.complex64).astype(np.complex128)
    td = torch.complex128 if dtype == "f64" else torch.complex64
    return x, torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", td)


def _close(got, want, dtype):
    scale = max(1.0, float(np.max(np.abs(want))))
    assert float(np.max(np.abs(got - want))) <= (1e-12 if dtype == "f64" else 2e-5) * scale


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_complex_hv_matches_oracle(case, dtype):
    name, ns, bonds, amps, nu, nd = case
    m = Model(ns, bonds, nu, nd, 1.0, 2.5, amps)
    h = _ham(ns, bonds, amps, nu, nd, 2.5, dtype)
    assert h.cplx and h.torch_dtype in (torch.complex128, torch.complex64)
    x_host, x = _start(101, m.dim, dtype)
    announce("complex hv %s %s dim=%d" % (name, dtype, m.dim))
    y = h.hv(x)
    _close(y.to(torch.complex128).cpu().numpy(), m.hv(x_host), dtype)
    assert torch.equal(h.hv(x), y)   # reproducible


def test_complex_lanczos_matches_oracle():
    m = Model(18, CB_BONDS, 2, 2, 1.0, 4.0, CB_AMPS)
    h = _ham(18, CB_BONDS, CB_AMPS, 2, 2, 4.0, "f64")
    x_host, x = _start(102, m.dim, "f64")
    announce("complex lanczos checker18 2+2")
    r = h.ground_energy(x, 40, tol=0.0)
    ref = lanczos(m.hv, x_host, 20)
    amax = np.max(np.abs(ref["a"]))
    assert np.max(np.abs(r["a"][:20] - ref["a"])) <= 1e-12 * amax
    assert np.max(np.abs(r["b"][:21] - ref["b"])) <= 1e-12 * amax


def _levels(ns, bonds, amps):
    h = np.zeros((ns, ns), dtype=np.complex128)
    for (i, j), a in zip(bonds, amps):
        h[i, j] += a
        h[j, i] += np.conj(a)
    return np.linalg.eigvalsh(h)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_complex_u0_band_sum_checker18_3x3(dtype):
    """D = 665,856 complex: E0 at U = 0 is twice the sum of the 3 lowest one-particle levels."""
    h = _ham(18, CB_BONDS, CB_AMPS, 3, 3, 0.0, dtype)
    _, x = _start(103, h.dim, dtype)
    announce("complex u0 checker18 3+3 %s" % dtype)
    r = h.ground_energy(x, 300, tol=1e-11 if dtype == "f64" else 1e-7, check_every=15)
    exact = 2.0 * _levels(18, CB_BONDS, CB_AMPS)[:3].sum()
    assert abs(r["e0"] - exact) <= (1e-9 if dtype == "f64" else 1e-6) * abs(exact), (r["e0"], exact)


def test_complex_two_pass_ground_state_residual():
    """|H v - E0 v| of the two-pass vector, with H applied by the oracle, and |v| = 1."""
    m = Model(18, CB_BONDS, 2, 2, 1.0, 4.0, CB_AMPS)
    h = _ham(18, CB_BONDS, CB_AMPS, 2, 2, 4.0, "f64")
    _, x = _start(104, m.dim, "f64")
    announce("complex ground state checker18 2+2")
    r = h.ground_energy(x, 300, tol=1e-13, check_every=10)
    e0, steps, v = h.ground_state(x, r["steps"] + 10)
    vh = v.cpu().numpy()
    assert abs(np.vdot(vh, vh).real - 1.0) < 1e-12
    assert np.linalg.norm(m.hv(vh) - e0 * vh) < 1e-6
    from scipy.sparse.linalg import eigsh   # ARPACK on the oracle's sparse matrix (a dense eigh would take minutes)
    e_ref = float(eigsh(m.full_sparse(), k=1, which="SA", tol=1e-13)[0][0])
    assert abs(e0 - e_ref) < 1e-9
    with pytest.raises(ed.EdError):
        h.ground_state(x, 10, gauge_index=0)


def test_real_only_calls_reject_complex_instances():
    h = _ham(18, CB_BONDS, CB_AMPS, 2, 1, 4.0, "f64")
    _, x = _start(105, h.dim, "f64")
    announce("complex rejections")
    with pytest.raises(ed.EdError):
        h.occupation_moments(x, 18)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_complex_tiles_give_the_same_bits_and_tune(dtype):
    """Every tile the autotuner times on a complex instance (rows per up tile, down workgroup size) gives
    the same H x bits as the default tile, and the tuner returns one of them."""
    h = _ham(18, CB_BONDS, CB_AMPS, 3, 2, 4.0, dtype)
    _, x = _start(106, h.dim, dtype)
    announce("complex tiles checker18 3+2 %s" % dtype)
    h.tile = 0
    ref = h.hv(x).clone()
    r = h.tune(x, reps=1, apply=False)
    ups = [i for i, m in enumerate(r["up_ms"]) if m > 0]
    dns = [i for i, m in enumerate(r["dn_ms"]) if m > 0]
    assert ups and dns
    rcs = [h.tile_params(ui)["up_rows"] for ui in ups]
    assert len(set(rcs)) == len(rcs)                  # one candidate per distinct rows-per-tile
    for ui in ups:
        for di in dns:
            h.tile = ui | (di << 8)
            assert torch.equal(h.hv(x), ref), (ui, di, h.tile_params())
    assert (r["tile"] & 0xFF) in ups and (r["tile"] >> 8) in dns
    h.tile = 0
    assert ed.api.tune_key(h).endswith("c128" if dtype == "f64" else "c64")


# ---------------------------------------------------------------------------
# full size: the 18-site checkerboard at 5 + 5 (D = 73,410,624 complex)

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_checker18_5x5_sampled_elements(dtype):
    wl = workload("checker18_5x5")
    h = ed.Hamiltonian.from_lattice(wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, wl.t, wl.U, dtype, "cuda:0",
                                    amps=list(wl.amps))
    assert h.dim == 73410624
    x_host, x = _start(wl.seed, h.dim, dtype)
    announce("complex hv full checker18 5+5 %s dim=%d" % (dtype, h.dim))
    y = h.hv(x).to(torch.complex128).cpu().numpy()
    del x
    torch.cuda.empty_cache()
    rng = np.random.default_rng(106)
    picks = sorted(set([0, 1, h.dim // 2, h.dim - 1] + rng.integers(0, h.dim, 300).tolist()))
    ref = hv_elements(wl.n_sites, wl.bonds, h.up.states, h.dn.states, wl.t, wl.U, x_host, picks, list(wl.amps))
    _close(y[picks], ref, dtype)


def test_full_size_checker18_5x5_u0_band_sum():
    wl = workload("checker18_5x5")
    h = ed.Hamiltonian.from_lattice(wl.n_sites, wl.bonds, wl.n_up, wl.n_dn, wl.t, 0.0, "f64", "cuda:0",
                                    amps=list(wl.amps))
    _, x = _start(wl.seed, h.dim, "f64")
    announce("complex u0 full checker18 5+5 f64 dim=%d" % h.dim)
    r = h.ground_energy(x, 300, tol=1e-11, check_every=15)
    exact = 2.0 * _levels(18, wl.bonds, wl.amps)[:5].sum()
    assert r["status"] == 0, (r["status"], r["steps"])
    assert abs(r["e0"] - exact) <= 1e-9 * abs(exact), (r["e0"], exact)
