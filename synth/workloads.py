"""Named workloads: lattice, fillings, couplings, precision, step budget, seed.

The synthetic configurations the benchmarks and parity tests use.
Nothing here computes anything of the method.
"""

from dataclasses import dataclass, field
from typing import List, Tuple

from .lattice import checkerboard_terms, ring_bonds, torus_bonds

# synthetic checkerboard amplitudes: t1 = 1, phase pi/4, next-nearest 0.3, third-nearest 0.2
CHECKER_PARAMS = (1.0, 0.7853981633974483, 0.3, 0.2)
_CHECKER18 = checkerboard_terms(3, 3, *CHECKER_PARAMS)


@dataclass(frozen=True)
class Workload:
    name: str
    n_sites: int
    bonds: Tuple[Tuple[int, int], ...]
    n_up: int
    n_dn: int
    t: float
    U: float
    steps: int
    seed: int
    note: str = ""
    amps: Tuple[complex, ...] = ()     # a complex amplitude per bond (empty: -t on every bond)


def _wl(name, n_sites, bonds, n, t, U, steps, seed, note=""):
    return Workload(name, n_sites, tuple(bonds), n, n, t, U, steps, seed, note)


WORKLOADS = {
    "ring8_4x4": _wl("ring8_4x4", 8, ring_bonds(8), 4, 1.0, 4.0, 100, 1,
                     "1-D periodic 8-site Hubbard chain, 4 up + 4 down, dim 4900"),
    "torus4x4_5x5": _wl("torus4x4_5x5", 16, torus_bonds(4, 4), 5, 1.0, 4.0, 200, 2,
                        "4x4 periodic Hubbard, 5 up + 5 down, dim 19,079,424"),
    "torus6x6_3x3": _wl("torus6x6_3x3", 36, torus_bonds(6, 6), 3, 1.0, 0.0, 300, 3,
                        "6x6 periodic tight binding (U=0), 3 up + 3 down, dim 50,979,600"),
    # the other fillings of the 64-instance batch (tuned like the others)
    "torus4x4_3x3": _wl("torus4x4_3x3", 16, torus_bonds(4, 4), 3, 1.0, 4.0, 200, 12,
                        "4x4 periodic Hubbard, 3 up + 3 down, dim 313,600"),
    "torus4x4_4x4": _wl("torus4x4_4x4", 16, torus_bonds(4, 4), 4, 1.0, 4.0, 200, 13,
                        "4x4 periodic Hubbard, 4 up + 4 down, dim 3,312,400"),
    "torus4x4_6x6": _wl("torus4x4_6x6", 16, torus_bonds(4, 4), 6, 1.0, 4.0, 200, 14,
                        "4x4 periodic Hubbard, 6 up + 6 down, dim 64,128,064"),
    "torus4x4_8x8": _wl("torus4x4_8x8", 16, torus_bonds(4, 4), 8, 1.0, 4.0, 300, 5,
                        "4x4 periodic Hubbard at half filling, 8 up + 8 down, dim 165,636,900"),
    # one species: every particle has the same spin (N_up = 0); the hopping alone, no on-site term
    "ring26_0x13": Workload("ring26_0x13", 26, tuple(ring_bonds(26)), 0, 13, 1.0, 0.0, 100, 7,
                            "26-site periodic chain, 13 particles of one species, dim 10,400,600"),
    "torus5x6_0x9": Workload("torus5x6_0x9", 30, tuple(torus_bonds(5, 6)), 0, 9, 1.0, 0.0, 100, 8,
                             "30-site 5x6 periodic square lattice, 9 particles of one species, dim 14,307,150"),
    # complex amplitudes: the paper's largest two-species checkerboard case
    "checker18_5x5": Workload("checker18_5x5", 18, tuple(b for b, _ in _CHECKER18), 5, 5, 1.0, 4.0, 100, 9,
                              "18-site checkerboard (3x3 two-site cells, 12 bonds per site, synthetic complex "
                              "amplitudes), 5 up + 5 down, dim 73,410,624 complex",
                              tuple(a for _, a in _CHECKER18)),
    "ring18_9x9": _wl("ring18_9x9", 18, ring_bonds(18), 9, 1.0, 4.0, 100, 6,
                      "18-site periodic Hubbard chain at half filling, 9 up + 9 down, dim 2,363,904,400 "
                      "(18.9 GB per float64 vector; 48620 states per species need 32-bit tables)"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
