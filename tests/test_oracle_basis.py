"""Pins of the oracle's basis (Sec. 2.1, Eq. 2) against printed sizes and brute enumeration."""

import math

import numpy as np
import pytest

from oracle.basis import basis_states, index_of, sector_dim
from tests.golden.load import paper_sizes


@pytest.mark.parametrize("row", paper_sizes())
def test_printed_sizes(row):
    kind, ns, nu, nd, val, tol = row
    d = sector_dim(ns, nu, nd)
    got = d if kind == "dim" else 16 * d          # complex double = 16 bytes per entry
    assert abs(got - val) <= tol


@pytest.mark.parametrize("ns,n", [(1, 0), (1, 1), (4, 2), (8, 4), (10, 3), (12, 6)])
def test_basis_equals_popcount_filter(ns, n):
    st = basis_states(ns, n)
    brute = [s for s in range(1 << ns) if bin(s).count("1") == n]   # ascending by construction
    assert st.tolist() == brute
    assert len(st) == math.comb(ns, n)


def test_colex_rank_closed_form():
    # ascending integers of fixed popcount are in colex order, whose rank is
    # sum_k C(p_k, k+1) over the set bits p_0 < p_1 < ...
    st = basis_states(16, 8)
    for k in list(range(0, len(st), 97)) + [len(st) - 1]:
        s = int(st[k])
        pos = [i for i in range(16) if (s >> i) & 1]
        assert sum(math.comb(p, j + 1) for j, p in enumerate(pos)) == k


def test_index_map_is_bijection():
    st = basis_states(10, 5)
    idx = index_of(st)
    assert all(idx[int(s)] == k for k, s in enumerate(st))
    assert len(idx) == len(st)


@pytest.mark.parametrize("ns,n,d", [(8, 4, 70), (16, 5, 4368), (36, 3, 7140), (16, 8, 12870),
                                    (16, 3, 560), (16, 4, 1820), (16, 6, 8008)])
def test_workload_dims(ns, n, d):
    assert sector_dim(ns, n, n) == d * d
