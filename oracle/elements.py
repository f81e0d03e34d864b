"""(H x) at selected basis states, straight from the operator form of the
Hamiltonian (Eq. 1 and the on-site U term), one element at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a basis state p = (s_up, s_dn) with flat index i_up * D_dn + i_dn:

    (H x)[p] = sum over species sigma, bonds (i, j) and both directions (a, b):
                   -t * <p| c+_a,sigma c_b,sigma |q> x[q]
               + U * (number of sites occupied by both species) * x[p]

H is real symmetric, so the states q with <p|c+_a c_b|q> != 0 are those
reached from p by c+_b c_a, with the same sign.  The operators act on an
explicit occupation list (``hopping.hop``); the target state's index is found
by binary search in the explicitly enumerated basis.  Nothing here builds a
matrix, so it serves sectors far larger than the oracle's matrices reach
(tens of millions of states), at a few microseconds per term.

Reading of the species order: all up operators stand left of all down
operators, so a down-species hop moves a pair of operators past the up ones
and the up occupation adds no sign (the same reading as ``hopping``).
"""

import numpy as np

from .basis import basis_states, occupations
from .hopping import hop, mask_of


def rank_in(states: np.ndarray, mask: int) -> int:
    """Position of ``mask`` in the ascending basis ``states`` (binary search)."""
    k = int(np.searchsorted(states, np.uint64(mask)))
    if k >= len(states) or int(states[k]) != mask:
        raise KeyError("state %#x is not in the basis" % mask)
    return k


def species_terms(occ: list, bonds, states: np.ndarray, amps=None):
    """(matrix element / t, index q) of every nonzero <p| H_sigma |q> for the row state p = occ.

    For the term a c+_i c_j, <p| c+_i c_j |q> is nonzero for q = c+_j c_i p, with the sign of that
    application (real); the Hermitian partner conj(a) c+_j c_i gives q = c+_i c_j p.  Without
    amplitudes every a is -1."""
    out = []
    for k, (i, j) in enumerate(bonds):
        a = -1.0 if amps is None else complex(amps[k])
        ac = a if amps is None else a.conjugate()
        for (p_, q_, amp) in ((j, i, a), (i, j, ac)):
            r = hop(occ, p_, q_)
            if r is not None:
                sign, new = r
                out.append((amp * sign, rank_in(states, mask_of(new))))
    return out


def hv_elements(n_sites: int, bonds, st_up: np.ndarray, st_dn: np.ndarray, t: float, U: float,
                x: np.ndarray, picks, amps=None) -> np.ndarray:
    """(H x)[p] for each flat index p in ``picks`` (float64, or complex128 with amplitudes or a
    complex x).  amps: optional complex amplitude per bond, as in ``hamiltonian.Model``."""
    d_dn = len(st_dn)
    bonds = [tuple(int(v) for v in b) for b in bonds]
    cplx = amps is not None or np.iscomplexobj(x)
    out = np.zeros(len(picks), dtype=np.complex128 if cplx else np.float64)
    val = complex if cplx else float
    for n, p in enumerate(picks):
        iu, idn = divmod(int(p), d_dn)
        su, sd = int(st_up[iu]), int(st_dn[idn])
        acc = val(0)
        for h, k in species_terms(occupations(su, n_sites), bonds, st_up, amps):
            acc += t * h * val(x[k * d_dn + idn])
        for h, k in species_terms(occupations(sd, n_sites), bonds, st_dn, amps):
            acc += t * h * val(x[iu * d_dn + k])
        acc += U * bin(su & sd).count("1") * val(x[p])
        out[n] = acc
    return out


def sector_states(n_sites: int, n_up: int, n_dn: int):
    """The two per-species bases (ascending), as the flat index expects."""
    su = basis_states(n_sites, n_up)
    sd = su if n_dn == n_up else basis_states(n_sites, n_dn)
    return su, sd
