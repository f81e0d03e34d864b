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

from .basis import occupations


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


def spin_flip_moments(psi: np.ndarray, st_up: np.ndarray, st_dn: np.ndarray, n_sites: int) -> np.ndarray:
    """C[i, j] = sum_x psi_x * <x'| S+_i S-_j |x> psi_x' over the basis (real psi; raw, not normalised),
    with S+_i = c+_i,up c_i,dn and S-_j = c+_j,dn c_j,up.

    The operator string c+_i,up c_i,dn c+_j,dn c_j,up is applied right to left to the occupation list of
    all 2 N_s modes (mode = sigma * N_s + site, every up mode before every down mode, the same order as
    the basis), one operator at a time, counting occupied modes below each operator for its sign."""
    from .hopping import annihilate, create
    ns = n_sites
    d_dn = len(st_dn)
    index_up = {int(s): k for k, s in enumerate(st_up)}
    index_dn = {int(s): k for k, s in enumerate(st_dn)}
    psi = np.asarray(psi, dtype=np.float64)
    c = np.zeros((ns, ns))
    for iu, su in enumerate(st_up):
        for idn, sd in enumerate(st_dn):
            amp = psi[iu * d_dn + idn]
            if amp == 0.0:
                continue
            occ = [(int(su) >> k) & 1 for k in range(ns)] + [(int(sd) >> k) & 1 for k in range(ns)]
            for i in range(ns):
                for j in range(ns):
                    state, sign = occ, 1
                    for op, mode in ((annihilate, j), (create, ns + j), (annihilate, ns + i), (create, i)):
                        r = op(state, mode)
                        if r is None:
                            state = None
                            break
                        s_, state = r
                        sign *= s_
                    if state is None:
                        continue
                    m_up = sum(1 << k for k in range(ns) if state[k])
                    m_dn = sum(1 << k for k in range(ns) if state[ns + k])
                    c[i, j] += sign * amp * psi[index_up[m_up] * d_dn + index_dn[m_dn]]
    return c


def spin_correlations(g: np.ndarray, c: np.ndarray, n_sites: int) -> np.ndarray:
    """<S_i . S_j> from the occupation moments G and the spin-flip moments C (both normalised):
    <S^z_i S^z_j> + (C[i, j] + C[j, i]) / 2 off the diagonal, and <S_i^2> = 3/4 <(n_up - n_dn)^2> on it."""
    ns = n_sites
    zz = correlations(g, ns)["szsz"]
    out = zz + 0.5 * (c + c.T)
    for i in range(ns):
        nu, nd, nud = g[i, i], g[ns + i, ns + i], g[i, ns + i]
        out[i, i] = 0.75 * (nu + nd - 2.0 * nud)
    return out


def bond_moments(psi: np.ndarray, st_up: np.ndarray, st_dn: np.ndarray, n_sites: int, bonds) -> np.ndarray:
    """K[b, sigma] = sum_x psi_x <x'| c+_i,sigma c_j,sigma + c+_j,sigma c_i,sigma |x> psi_x' for bond b = (i, j)
    (real psi, raw sums).  The hops are applied with ``hopping.hop`` to the species' occupation list; a hop of
    either species moves a pair of operators, so the other species adds no sign."""
    from .hopping import hop, mask_of
    d_dn = len(st_dn)
    index_up = {int(s): k for k, s in enumerate(st_up)}
    index_dn = {int(s): k for k, s in enumerate(st_dn)}
    psi = np.asarray(psi, dtype=np.float64)
    k_out = np.zeros((len(bonds), 2))
    for iu, su in enumerate(st_up):
        occ_u = occupations(int(su), n_sites)
        for idn, sd in enumerate(st_dn):
            amp = psi[iu * d_dn + idn]
            occ_d = occupations(int(sd), n_sites)
            for b, (i, j) in enumerate(bonds):
                for (p, q) in ((i, j), (j, i)):
                    r = hop(occ_u, p, q)
                    if r is not None:
                        k_out[b, 0] += r[0] * amp * psi[index_up[mask_of(r[1])] * d_dn + idn]
                    r = hop(occ_d, p, q)
                    if r is not None:
                        k_out[b, 1] += r[0] * amp * psi[iu * d_dn + index_dn[mask_of(r[1])]]
    return k_out
