"""Helpers shared by the GPU tests (no arithmetic of the method)."""

import sys

import numpy as np
import torch

import paper_1511_00863_amd as ed
from synth import start_vector


def announce(msg: str):
    """Name the case before a GPU step, flushed, so a crash log says which case ran."""
    sys.stdout.write("[gpu] %s\n" % msg)
    sys.stdout.flush()


def device_vec(x: np.ndarray, dtype: str) -> torch.Tensor:
    td = torch.float64 if dtype == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda:0", dtype=td)


def seeded_start(seed: int, dim: int, dtype: str):
    """(host float64 copy as the device sees it, device tensor)."""
    x = start_vector(seed, dim)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    return x, device_vec(x, dtype)


def ham(n_sites, bonds, n_up, n_dn, t, U, dtype, tile=0):
    return ed.Hamiltonian.from_lattice(n_sites, bonds, n_up, n_dn, t, U, dtype, "cuda:0", tile)
