"""Per-spin occupation basis (Sec. 2.1, Eq. 2 and the integer representation of
single-species states).

Reading (the paper defers the details to its companion paper): bit i of a basis
integer is site i; the states of one species are all integers with exactly N
set bits below 2**N_s, in ascending order; the index of a two-species state is
``i_up * D_dn + i_dn`` (the vector is D_up subvectors of length D_dn, Sec. 4).
"""

import itertools
import math

import numpy as np


def basis_states(n_sites: int, n_part: int) -> np.ndarray:
    """All n_part-subsets of the n_sites sites as bitmasks, ascending (uint64)."""
    masks = [sum(1 << p for p in combo)
             for combo in itertools.combinations(range(n_sites), n_part)]
    return np.array(sorted(masks), dtype=np.uint64)


def index_of(states: np.ndarray) -> dict:
    """Map bitmask -> position in ``states`` (a plain dictionary)."""
    return {int(s): k for k, s in enumerate(states)}


def sector_dim(n_sites: int, n_up: int, n_dn: int) -> int:
    """Eq. 2: dim H = C(N_s, N_up) * C(N_s, N_dn)."""
    return math.comb(n_sites, n_up) * math.comb(n_sites, n_dn)


def occupations(mask: int, n_sites: int) -> list:
    """Occupation numbers n_0 .. n_{N_s - 1} of a bitmask."""
    return [(int(mask) >> i) & 1 for i in range(n_sites)]
