"""Lattice geometries as bond lists (the <ij> of the hopping sum, Eq. 1).

A bond is an unordered pair of distinct sites, stored as (min, max).  Periodic
boundaries are always used (Sec. 2.1).  Site numbering on a 2-D lattice is
``x + Lx*y``; bit ``i`` of a basis integer is site ``i``.  Duplicate pairs,
which periodic wrapping produces when a side has length 2, are kept once.
"""

from typing import List, Tuple

Bond = Tuple[int, int]


def _dedup(pairs) -> List[Bond]:
    seen = set()
    out: List[Bond] = []
    for i, j in pairs:
        if i == j:
            continue
        key = (min(i, j), max(i, j))
        if key not in seen:
            seen.add(key)
            out.append(key)
    return out


def site_index(x: int, y: int, lx: int) -> int:
    return x + lx * y


def ring_bonds(n_sites: int) -> List[Bond]:
    """1-D periodic chain with nearest-neighbour bonds (i, i+1 mod n)."""
    return _dedup((i, (i + 1) % n_sites) for i in range(n_sites))


def torus_bonds(lx: int, ly: int) -> List[Bond]:
    """Periodic lx-by-ly square lattice, nearest-neighbour bonds."""
    pairs = []
    for y in range(ly):
        for x in range(lx):
            s = site_index(x, y, lx)
            pairs.append((s, site_index((x + 1) % lx, y, lx)))
            pairs.append((s, site_index(x, (y + 1) % ly, lx)))
    return _dedup(pairs)


def two_site_bonds() -> List[Bond]:
    """The two-site system with its single bond (0, 1)."""
    return [(0, 1)]


def complete_bonds(n_sites: int) -> List[Bond]:
    """Every pair of sites bonded (all-to-all hopping).  Not a lattice of the
    paper: it gives the widest hopping tables at a small dimension (a state
    with N particles has N * (n_sites - N) hops), for edge-case tests."""
    return [(i, j) for i in range(n_sites) for j in range(i + 1, n_sites)]
