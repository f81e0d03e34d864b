"""The whole H x at the benchmark's size against the oracle's Eq. 4-5, element by element.

4x4 periodic Hubbard at half filling, 8 + 8 (dim 165,636,900), U = 4, in the configuration the
benchmark times: the up species in band order, the down species in hop-count order and the tile from the
tuning cache.  The device
result is mapped back to the ascending basis and compared with oracle.Model.hv over every element,
float64 to 1e-12 and the float32 H.v to 2e-6 of max |H x| (float32 accumulation over up to 65 terms).
"""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.hamiltonian import Model
from synth import start_vector, workload
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    w = workload("torus4x4_8x8")
    m = Model(w.n_sites, w.bonds, w.n_up, w.n_dn, w.t, w.U)
    _ = m.docc
    return w, m


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_c5_full_vector_tuned_tile_hop_order(c5, dtype, tol):
    w, m = c5
    up = ed.SpinTables(w.n_sites, w.bonds, w.n_up, "cuda:0", order="band")
    dn = ed.SpinTables(w.n_sites, w.bonds, w.n_dn, "cuda:0", order="hops")
    h = ed.Hamiltonian(up, dn, w.t, w.U, dtype)
    src = ed.api.apply_tuned_tile(h, tune_if_missing=False)
    x = start_vector(w.seed, h.dim)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    announce("full-size H.v 4x4 8+8 %s, tile %d (%s), params %s" % (dtype, h.tile, src, h.tile_params()))
    xd = h.to_basis_order(torch.from_numpy(x).to("cuda:0", h.torch_dtype))
    y = h.to_ascending(h.hv(xd)).double().cpu().numpy()
    del xd
    torch.cuda.empty_cache()
    ref = m.hv(x)
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(y - ref)))
    assert err <= tol * scale, (err / scale)
    assert np.linalg.norm(y - ref) <= tol * np.linalg.norm(ref)
