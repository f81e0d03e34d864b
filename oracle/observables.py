"""Diagonal observables of a state vector in the occupation basis.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The ground-state vector of the two-pass Lanczos run gives expectation values.
Those that are diagonal in the occupation basis (Sec. 2.1: a basis state
fixes every n_i,sigma) are weighted sums over the basis with weights
|psi_x|^2.  All of them follow from one matrix over the 2*N_s occupation
bits b(x) = (n_0,up .. n_{Ns-1},up, n_0,dn .. n_{Ns-1},dn):

    G = sum_x |psi_x|^2 b(x) b(x)^T          (2 N_s x 2 N_s, symmetric)

from which (with G_ab = <n_a n_b>):
    double occupancy of site i   <n_i,up n_i,dn>   = G[i, N_s + i]
    density correlation           <n_i n_j>         = sum over the four spin blocks
    spin correlation              <S^z_i S^z_j>     = (G_uu - G_ud - G_du + G_dd)[i, j] / 4
    densities                     <n_i,sigma>       = the diagonal (n^2 = n)

This module computes G straight from that definition with one dense bit
matrix per basis state, with no use of the product structure of the basis
(the device computes it through row and column sums instead).
"""

import numpy as np


def occupation_bits(states: np.ndarray, n_sites: int) -> np.ndarray:
    """Row x = the n_sites occupation numbers of basis state x (bit i = site i)."""
    s = np.asarray(states, dtype=np.uint64)
    return ((s[:, None] >> np.arange(n_sites, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.float64)


def occupation_moments(psi: np.ndarray, st_up: np.ndarray, st_dn: np.ndarray, n_sites: int) -> np.ndarray:
    """G = sum_x |psi_x|^2 b(x) b(x)^T over the basis x = (i_up, i_dn), index i_up * D_dn + i_dn."""
    bu = occupation_bits(st_up, n_sites)
    bd = occupation_bits(st_dn, n_sites)
    du, dd = len(st_up), len(st_dn)
    w = np.abs(np.asarray(psi, dtype=np.float64)) ** 2
    g = np.zeros((2 * n_sites, 2 * n_sites))
    for iu in range(du):
        # b(x) for the D_dn states sharing this up state, stacked as rows
        b = np.concatenate([np.broadcast_to(bu[iu], (dd, n_sites)), bd], axis=1)
        g += b.T @ (w[iu * dd:(iu + 1) * dd, None] * b)
    return g


def correlations(g: np.ndarray, n_sites: int) -> dict:
    """Named observables from G (see the module docstring)."""
    ns = n_sites
    uu, ud, du, dd = g[:ns, :ns], g[:ns, ns:], g[ns:, :ns], g[ns:, ns:]
    return {
        "docc": np.diag(ud).copy(),                         # <n_i,up n_i,dn>
        "n_up": np.diag(uu).copy(),
        "n_dn": np.diag(dd).copy(),
        "nn": uu + ud + du + dd,                            # <n_i n_j>
        "szsz": (uu - ud - du + dd) / 4.0,                  # <S^z_i S^z_j>
    }
