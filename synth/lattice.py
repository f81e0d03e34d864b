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


def checkerboard_bonds(l1: int, l2: int) -> List[Bond]:
    """Checkerboard lattice: l1 x l2 periodic unit cells of two sites, A = 2k and B = 2k + 1 for cell
    k = c1 + l1*c2 (B sits at the cell centre).  Each site has 12 bonds: 4 nearest neighbours on the other
    sublattice, 4 next-nearest along the cell axes a1, a2 and 4 third-nearest along a1 +- a2.  Needs
    l1, l2 >= 3, so that no two of these land on the same pair of sites."""
    return [b for b, _ in checkerboard_terms(l1, l2, 1.0, 0.0, 1.0, 1.0)]


def checkerboard_terms(l1: int, l2: int, t1: float, phi: float, t2: float, t3: float):
    """Bonds of ``checkerboard_bonds`` with a complex amplitude each: the term a * c+_i c_j + h.c. for bond
    (i, j), i < j.  These are synthetic stand-ins for a flat-band checkerboard model:
      nearest neighbours   -t1 exp(+-i phi): +phi for A -> B hops along the (+,+) and (-,-) diagonals,
                           -phi along (+,-) and (-,+);
      next-nearest         -t2 along a1 and +t2 along a2 from A sites, the opposite signs from B sites;
      third-nearest        -t3.
    Returns a list of ((i, j), complex amplitude) in a fixed order."""
    import cmath
    if l1 < 3 or l2 < 3:
        raise ValueError("checkerboard cells need l1, l2 >= 3")

    def cell(c1, c2):
        return (c1 % l1) + l1 * (c2 % l2)

    terms = {}

    def add(i, j, amp):   # term amp * c+_i c_j (+ h.c.), stored on the ordered pair
        if i == j:
            raise ValueError("self bond")
        key, a = ((i, j), amp) if i < j else ((j, i), amp.conjugate())
        if key in terms:
            raise ValueError("two terms on the pair %r: the cell grid is too small" % (key,))
        terms[key] = a

    nn = -t1 * cmath.exp(1j * phi)
    for c2 in range(l2):
        for c1 in range(l1):
            a = 2 * cell(c1, c2)
            # the four B neighbours of A: B(c) at (+1/2,+1/2), B(c-a1) at (-,+), B(c-a2) at (+,-), B(c-a1-a2) at (-,-)
            add(a, 2 * cell(c1, c2) + 1, nn)
            add(a, 2 * cell(c1 - 1, c2) + 1, nn.conjugate())
            add(a, 2 * cell(c1, c2 - 1) + 1, nn.conjugate())
            add(a, 2 * cell(c1 - 1, c2 - 1) + 1, nn)
            for s, sign in ((0, 1.0), (1, -1.0)):      # sublattice A, B
                i = 2 * cell(c1, c2) + s
                add(i, 2 * cell(c1 + 1, c2) + s, complex(-t2 * sign))
                add(i, 2 * cell(c1, c2 + 1) + s, complex(t2 * sign))
                add(i, 2 * cell(c1 + 1, c2 + 1) + s, complex(-t3))
                add(i, 2 * cell(c1 + 1, c2 - 1) + s, complex(-t3))
    return sorted(terms.items())
