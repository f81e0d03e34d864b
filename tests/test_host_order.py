"""Reordered bases on the host: the hop-count order (ed_hop_order) and the permuted basis and ELL table
(ed_permute_basis), checked against the oracle's basis and hopping matrix.  Reordering a species by a
permutation P turns its hopping matrix into P H P^T, so the permuted table must hold exactly the oracle's
matrix with rows and columns taken in the order perm."""

import ctypes

import numpy as np
import pytest

import paper_1511_00863_amd as ed
from paper_1511_00863_amd import _ffi
from oracle.basis import basis_states
from oracle.hopping import hopping_matrix, hopping_matrix_complex
from synth import checkerboard_terms, ring_bonds, torus_bonds

CASES = [
    ("torus4x4_3", 16, torus_bonds(4, 4), 3),
    ("ring12_5", 12, ring_bonds(12), 5),
    ("torus3x4_6", 12, torus_bonds(3, 4), 6),
    ("ring9_1", 9, ring_bonds(9), 1),
]


def _dense(table, dim):
    """The exported ELL table (either layout) as a dense matrix."""
    w = table["width"]
    vals = np.asarray(table["vals"])
    out = np.zeros((dim, dim), dtype=vals.dtype)
    for r in range(dim):
        for k in range(table["nnz"][r]):
            at = r * w + k if table["layout"] == ed.ED_ROW_MAJOR else k * dim + r
            out[r, table["cols"][at]] += vals[at]
    return out


def _oracle_hops(h):
    return np.asarray((h != 0).sum(axis=1)).ravel()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_hop_order_is_the_stable_sort_by_oracle_hop_count(case):
    _, ns, bonds, n = case
    st = basis_states(ns, n)
    hops = _oracle_hops(hopping_matrix(ns, bonds, st))
    tab = ed.build_hopping(ns, bonds, st)
    perm = ed.hop_order(tab["nnz"])
    want = sorted(range(st.size), key=lambda r: (-hops[r], r))
    assert perm.tolist() == want


@pytest.mark.parametrize("layout", [ed.ED_ROW_MAJOR, ed.ED_COL_MAJOR])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_permuted_table_is_the_oracle_matrix_reordered(case, layout):
    _, ns, bonds, n = case
    st = basis_states(ns, n)
    h = hopping_matrix(ns, bonds, st).toarray()
    tab = ed.build_hopping(ns, bonds, st, layout)
    perm = ed.hop_order(tab["nnz"])
    st2, tab2 = ed.permute_basis(st, tab, perm)
    assert np.array_equal(st2, st[perm])
    assert np.array_equal(_dense(tab2, st.size), h[np.ix_(perm, perm)])
    # rows stay in ascending column order with the padding at the end: the packers accept them
    ed.pack_tables(tab2, st.size, 2)
    ed.pack_tables(tab2, st.size, 4)
    # padding of the exported format
    for r in range(st.size):
        for k in range(tab2["nnz"][r], tab2["width"]):
            at = r * tab2["width"] + k if layout == ed.ED_ROW_MAJOR else k * st.size + r
            assert tab2["cols"][at] == 0 and tab2["vals"][at] == 0.0


def test_hop_order_puts_equal_hop_counts_together_on_the_paper_lattice():
    """4x4 torus, 8 per species: after the sort a 64-column wavefront holds at most two hop counts except
    where the count changes, and the chunks of 8 table entries it needs drop from 3.19 to 2.48 on average."""
    st = basis_states(16, 8)
    tab = ed.build_hopping(16, torus_bonds(4, 4), st)
    nnz = tab["nnz"]
    perm = ed.hop_order(nnz)

    def chunks_per_wave(counts):
        pad = (-counts.size) % 64
        w = np.concatenate([counts, np.zeros(pad, dtype=counts.dtype)]).reshape(-1, 64)
        return float(((w.max(axis=1) + 7) // 8).mean())

    before, after = chunks_per_wave(nnz), chunks_per_wave(nnz[perm])
    assert after < before
    assert abs(before - 3.193) < 1e-3 and abs(after - 2.480) < 1e-3
    assert np.all(np.diff(nnz[perm]) <= 0)


def test_permuted_complex_table_is_the_oracle_matrix_reordered():
    terms = checkerboard_terms(3, 3, 1.0, np.pi / 4, 0.3, 0.2)
    bonds = [b for b, _ in terms]
    amps = [a for _, a in terms]
    st = basis_states(18, 3)
    h = hopping_matrix_complex(18, bonds, amps, st).toarray()
    tab = ed.api.build_hopping_complex(18, bonds, amps, st, ed.ED_COL_MAJOR)
    perm = ed.hop_order(tab["nnz"])
    st2, tab2 = ed.permute_basis(st, tab, perm)
    assert np.array_equal(st2, st[perm])
    assert np.array_equal(_dense(tab2, st.size), h[np.ix_(perm, perm)])
    ed.api.pack_tables_complex(tab2, st.size)


def test_species_that_cannot_hop_and_single_state_bases():
    for ns, n in ((6, 0), (6, 6)):
        st = basis_states(ns, n)
        tab = ed.build_hopping(ns, ring_bonds(ns), st)
        assert tab["width"] == 0
        perm = ed.hop_order(tab["nnz"])
        assert perm.tolist() == [0]
        st2, tab2 = ed.permute_basis(st, tab, perm)
        assert np.array_equal(st2, st) and tab2["width"] == 0
    # a species with no hop anywhere is left in its order
    assert ed.hop_order(np.zeros(5, dtype=np.int32)).tolist() == [0, 1, 2, 3, 4]


def test_order_errors():
    st = basis_states(8, 3)
    tab = ed.build_hopping(8, ring_bonds(8), st)
    bad = np.arange(st.size)
    bad[3] = bad[4]                                  # repeated entry
    with pytest.raises(ed.EdError) as e:
        ed.permute_basis(st, tab, bad)
    assert e.value.code == _ffi.ED_EINVAL
    bad = np.arange(st.size)
    bad[0] = st.size                                 # out of range
    with pytest.raises(ed.EdError):
        ed.permute_basis(st, tab, bad)
    with pytest.raises(ed.EdError):
        ed.hop_order(np.array([1, -1, 2], dtype=np.int32))
    lib = ed.lib()
    perm = np.arange(st.size, dtype=np.int64)
    out = np.zeros(st.size, dtype=np.uint64)
    nz = np.zeros(st.size, dtype=np.int32)
    cols = np.zeros(tab["cols"].size, dtype=np.int32)
    vals = np.zeros(tab["vals"].size)
    p = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    for nv in (0, 3):
        assert lib.ed_permute_basis(p(st, ctypes.c_uint64), p(tab["cols"], ctypes.c_int32), p(tab["vals"], ctypes.c_double),
                                    p(tab["nnz"], ctypes.c_int32), st.size, tab["width"], ed.ED_COL_MAJOR, nv,
                                    p(perm, ctypes.c_int64), p(out, ctypes.c_uint64), p(cols, ctypes.c_int32),
                                    p(vals, ctypes.c_double), p(nz, ctypes.c_int32)) == _ffi.ED_EINVAL


def test_order_field_and_rank_based_calls_validated_on_the_host():
    """ed_ham.order: 0..3; the spin-flip and bond moments (colex-rank lookups) need 0; vector permutation
    argument errors return before any device work."""
    lib = ed.lib()
    dummy = ctypes.c_void_p(4096)   # never dereferenced

    def ham(**kw):
        f = dict(dim_up=70, dim_dn=70, w_up=8, w_dn=8, tab_up=dummy, tab_dn=dummy, st_up=dummy, st_dn=dummy,
                 t=1.0, U=4.0, dtype=0, tile=0, eb_up=0, eb_dn=0, cplx=0, order=0, amp_up=None, amp_dn=None)
        f.update(kw)
        return _ffi.EdHam(**f)

    n = ctypes.c_int64(0)
    for order in (1, 2, 3):
        h = ham(order=order)
        assert lib.ed_workspace_size(ctypes.byref(h), 4, ctypes.byref(n)) == 0
        assert lib.ed_occupation_moments_ws(ctypes.byref(h), 8, ctypes.byref(n)) == 0
        assert lib.ed_spin_flip_moments_ws(ctypes.byref(h), 8, ctypes.byref(n)) == _ffi.ED_EINVAL
        assert b"ascending" in lib.ed_last_error()
        assert lib.ed_bond_moments_ws(ctypes.byref(h), 8, 4, ctypes.byref(n)) == _ffi.ED_EINVAL
    assert lib.ed_spin_flip_moments_ws(ctypes.byref(ham()), 8, ctypes.byref(n)) == 0
    for order in (-1, 4):
        assert lib.ed_workspace_size(ctypes.byref(ham(order=order)), 4, ctypes.byref(n)) == _ffi.ED_EINVAL
    h = ham()
    buf = ctypes.c_void_p(1 << 20)
    assert lib.ed_permute_vector(ctypes.byref(h), None, None, None, buf, None) == _ffi.ED_EINVAL
    assert lib.ed_permute_vector(ctypes.byref(h), None, None, buf, buf, None) == _ffi.ED_EINVAL
    near = ctypes.c_void_p((1 << 20) + 8 * 70 * 70 - 8)        # overlaps the last element
    assert lib.ed_permute_vector(ctypes.byref(h), None, None, buf, near, None) == _ffi.ED_EINVAL
    assert b"overlap" in lib.ed_last_error()


def test_spin_tables_order_option():
    t = ed.SpinTables(16, torus_bonds(4, 4), 3, "cpu", order="hops")
    st = basis_states(16, 3)
    assert np.array_equal(t.states, st[t.perm])
    assert np.all(np.diff(t.table["nnz"]) <= 0)
    h = ed.Hamiltonian.from_lattice(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0, "f64", "cpu", order=("ascending", "hops"))
    assert h.order_bits == 2 and h.up is not h.dn and h.up.perm is None
    h = ed.Hamiltonian.from_lattice(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0, "f64", "cpu", order="hops")
    assert h.order_bits == 3 and h.up is h.dn
    with pytest.raises(ValueError):
        ed.SpinTables(8, ring_bonds(8), 3, "cpu", order="random")


def _cm_checks(adj, deg, perm):
    """The order perm[::-1] is a Cuthill-McKee order of the graph adj: every connected part is contiguous
    and starts at one vertex; every other vertex has an earlier neighbour, its parent (the earliest one);
    parents never move back along the order (a breadth-first sweep); and the children of one parent come
    fewest-neighbours first, then lowest index."""
    n = len(adj)
    order = perm[::-1]
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    last_parent = -1
    for i, v in enumerate(order):
        earlier = [pos[u] for u in adj[v] if pos[u] < i]
        if not earlier:                      # the start of a connected part: nothing before it reaches it
            assert all(pos[u] > i for u in adj[v])
            last_parent = -1
            continue
        par = min(earlier)
        assert par >= last_parent, (i, par, last_parent)
        if par == last_parent:
            prev = order[i - 1]
            assert (deg[prev], prev) < (deg[v], v)
        last_parent = par


def _adjacency(h):
    h = h.tocsr() if hasattr(h, "tocsr") else h
    return [sorted(set(np.nonzero(np.asarray(h[r].todense() if hasattr(h[r], "todense") else h[r]).ravel())[0])
                   - {r}) for r in range(h.shape[0])]


def _bandwidth(adj, perm):
    pos = np.empty(len(adj), dtype=np.int64)
    pos[perm] = np.arange(len(adj))
    return max((abs(int(pos[r]) - int(pos[c])) for r in range(len(adj)) for c in adj[r]), default=0)


@pytest.mark.parametrize("layout", [ed.ED_ROW_MAJOR, ed.ED_COL_MAJOR])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_band_order_is_reverse_cuthill_mckee_of_the_oracle_graph(case, layout):
    """ed_band_order against the oracle's hopping matrix: a permutation, a Cuthill-McKee order reversed,
    and no wider than the ascending order."""
    _, ns, bonds, n = case
    st = basis_states(ns, n)
    adj = _adjacency(hopping_matrix(ns, bonds, st))
    deg = np.array([len(a) for a in adj])
    perm = ed.band_order(ed.build_hopping(ns, bonds, st, layout))
    assert np.array_equal(np.sort(perm), np.arange(st.size))
    _cm_checks(adj, deg, perm)
    assert _bandwidth(adj, perm) <= _bandwidth(adj, np.arange(st.size))
    # both layouts give the same order
    other = ed.ED_COL_MAJOR if layout == ed.ED_ROW_MAJOR else ed.ED_ROW_MAJOR
    assert np.array_equal(perm, ed.band_order(ed.build_hopping(ns, bonds, st, other)))


def test_band_order_with_disconnected_parts():
    """Two separate 4-site rings with two particles: three connected parts (2+0, 1+1, 0+2 particles), each
    contiguous in the order."""
    bonds = ring_bonds(4) + [(a + 4, b + 4) for a, b in ring_bonds(4)]
    st = basis_states(8, 2)
    adj = _adjacency(hopping_matrix(8, bonds, st))
    deg = np.array([len(a) for a in adj])
    perm = ed.band_order(ed.build_hopping(8, bonds, st))
    assert np.array_equal(np.sort(perm), np.arange(st.size))
    _cm_checks(adj, deg, perm)
    left = np.array([bin(int(s) & 0xF).count("1") for s in st])   # particles on the first ring
    runs = left[perm]
    assert np.count_nonzero(np.diff(runs)) == 2                    # three contiguous parts


def test_band_order_narrows_the_half_filled_4x4_up_graph():
    """4x4 torus, 8 particles (12,870 states): the reordered graph's bandwidth is well below the
    ascending order's."""
    st = basis_states(16, 8)
    tab = ed.build_hopping(16, torus_bonds(4, 4), st, ed.ED_ROW_MAJOR)
    perm = ed.band_order(tab)
    assert np.array_equal(np.sort(perm), np.arange(st.size))
    cols = tab["cols"].reshape(st.size, tab["width"])
    adj = [cols[r, :tab["nnz"][r]].tolist() for r in range(st.size)]
    wa, wb = _bandwidth(adj, np.arange(st.size)), _bandwidth(adj, perm)
    assert wb < 0.7 * wa, (wa, wb)


def test_band_order_rejects_bad_tables():
    lib = ed.lib()
    p = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))  # noqa: E731
    cols = np.array([1, 0], dtype=np.int32)
    perm = np.zeros(2, dtype=np.int64)
    assert lib.ed_band_order(p(cols, ctypes.c_int32), p(np.array([1, 2], dtype=np.int32), ctypes.c_int32), 2, 1,
                             ed.ED_ROW_MAJOR, p(perm, ctypes.c_int64)) == _ffi.ED_EINVAL      # nnz above width
    bad = np.array([1, 5], dtype=np.int32)
    assert lib.ed_band_order(p(bad, ctypes.c_int32), p(np.array([1, 1], dtype=np.int32), ctypes.c_int32), 2, 1,
                             ed.ED_ROW_MAJOR, p(perm, ctypes.c_int64)) == _ffi.ED_EINVAL      # column out of range
    assert lib.ed_band_order(p(cols, ctypes.c_int32), p(np.array([1, 1], dtype=np.int32), ctypes.c_int32), 2, 1,
                             ed.ED_ROW_MAJOR, p(perm, ctypes.c_int64)) == 0
    assert sorted(perm.tolist()) == [0, 1]


def test_spin_tables_band_order():
    t = ed.SpinTables(16, torus_bonds(4, 4), 3, "cpu", order="band")
    st = basis_states(16, 3)
    assert np.array_equal(t.states, st[t.perm])
    assert np.array_equal(t.perm, ed.band_order(ed.build_hopping(16, torus_bonds(4, 4), st)))
    h = ed.Hamiltonian.from_lattice(16, torus_bonds(4, 4), 3, 3, 1.0, 4.0, "f64", "cpu", order=("band", "hops"))
    assert h.order_bits == 3 and h.up is not h.dn


def test_row_windows_hold_each_block_and_its_neighbours():
    """ed_row_windows against a brute-force scan: every state of a block and every table column of those
    states lies in [lo, hi); lo and hi are multiples of 4 (hi capped at dim) and as tight as that allows;
    max_window is the widest.  Both layouts, ascending and band order, a block size that leaves a ragged
    last block."""
    from paper_1511_00863_amd import api
    from synth import ring_bonds, torus_bonds
    for ns, bonds, n in ((16, torus_bonds(4, 4), 5), (12, ring_bonds(12), 6)):
        st = api.build_basis(ns, n)
        for layout in (api.ED_ROW_MAJOR, api.ED_COL_MAJOR):
            tab = api.build_hopping(ns, bonds, st, layout=layout)
            for order in ("ascending", "band"):
                t = tab
                if order == "band":
                    _, t = api.permute_basis(st, tab, api.band_order(tab))
                D, W = st.size, t["width"]
                cols = t["cols"].reshape(D, W) if layout == api.ED_ROW_MAJOR else t["cols"].reshape(W, D).T
                for bc in (64, 192):
                    lo_hi, widest = api.row_windows(t, bc)
                    nblk = (D + bc - 1) // bc
                    assert lo_hi.size == 2 * nblk
                    want_w = 0
                    for b in range(nblk):
                        c0, c1 = b * bc, min(D, (b + 1) * bc)
                        nb = [int(c) for r in range(c0, c1) for c in cols[r, :t["nnz"][r]]]
                        lo = min([c0] + nb) // 4 * 4
                        hi = min(D, (max([c1 - 1] + nb) + 1 + 3) // 4 * 4)
                        assert (lo_hi[2 * b], lo_hi[2 * b + 1]) == (lo, hi), (ns, n, layout, order, bc, b)
                        want_w = max(want_w, hi - lo)
                    assert widest == want_w
    with pytest.raises(Exception):
        api.row_windows(tab, 100)   # not a multiple of 64


def test_windowed_table_holds_window_relative_columns():
    """ed_pack_tables_windowed against a decode by hand: in the 8-interleaved part, entry k of row r is
    ((col - lo_b) << 1) | (value < 0) with b = r // block_cols, padding 0xFFFF after the row's nonzeros; the
    row-major part is all padding.  Band order, both layouts; a window that leaves a column out is refused."""
    from paper_1511_00863_amd import api
    from synth import torus_bonds
    st = api.build_basis(16, 5)
    for layout in (api.ED_ROW_MAJOR, api.ED_COL_MAJOR):
        tab = api.build_hopping(16, torus_bonds(4, 4), st, layout=layout)
        _, t = api.permute_basis(st, tab, api.band_order(tab))
        D, W = st.size, t["width"]
        stride = api.table_stride(W)
        bc = 512
        lo_hi, _ = api.row_windows(t, bc)
        packed = api.pack_tables_windowed(t, D, bc, lo_hi)
        assert np.all(packed[:D * stride] == 0xFFFF)
        inter = packed[D * stride:].reshape(stride // 8, D, 8)
        if layout == api.ED_ROW_MAJOR:
            cols, vals = t["cols"].reshape(D, W), t["vals"].reshape(D, W)
        else:
            cols, vals = t["cols"].reshape(W, D).T, t["vals"].reshape(W, D).T
        for r in range(0, D, 37):
            lo = lo_hi[2 * (r // bc)]
            for k in range(stride):
                e = int(inter[k // 8, r, k % 8])
                if k < t["nnz"][r]:
                    assert e == ((int(cols[r, k]) - lo) << 1) | (1 if vals[r, k] < 0 else 0), (r, k)
                else:
                    assert e == 0xFFFF
    bad = lo_hi.copy()
    bad[1] = bad[0] + 8   # block 0's window no longer holds its rows
    with pytest.raises(Exception):
        api.pack_tables_windowed(t, D, bc, bad)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_wave_chunks_are_the_widest_row_of_each_64(case):
    """ed_wave_chunks: per 64 consecutive rows (the last group ragged), the 8-entry chunks of the row with the
    most hops, the hop counts taken from the oracle's matrix; ascending and hop-count order."""
    _, ns, bonds, n = case
    st = basis_states(ns, n)
    hops = _oracle_hops(hopping_matrix(ns, bonds, st))
    tab = ed.build_hopping(ns, bonds, st)
    for order in ("ascending", "hops"):
        perm = np.arange(st.size) if order == "ascending" else ed.hop_order(tab["nnz"])
        t = tab if order == "ascending" else ed.permute_basis(st, tab, perm)[1]
        got = ed.wave_chunks(t["nnz"])
        h = hops[perm]
        want = [max((int(v) + 7) // 8 for v in h[g:g + 64]) for g in range(0, st.size, 64)]
        assert got.tolist() == want, (order,)


def test_wave_chunks_errors():
    with pytest.raises(ed.EdError):
        ed.wave_chunks(np.array([3, -1, 2], dtype=np.int32))
    with pytest.raises(ed.EdError):
        ed.wave_chunks(np.zeros(0, dtype=np.int32))
