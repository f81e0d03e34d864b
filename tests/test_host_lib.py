"""Host-side library calls (no GPU): basis, ranks, ELL export, packer, tridiagonal
solver, error paths, and the exported symbol set of include/ed.h."""

import os
import re
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla

import paper_1511_00863_amd as ed
from paper_1511_00863_amd import _ffi
from oracle.basis import basis_states
from oracle.hopping import hopping_matrix, to_ell
from synth import complete_bonds, ring_bonds, torus_bonds, two_site_bonds

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ed.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ed_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    decl = _declared()
    assert len(decl) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", _ffi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ed_[a-z0-9_]+)", out))
    missing = [d for d in decl if d not in exported]
    assert not missing, missing
    lib = ed.lib()
    for d in decl:
        assert hasattr(lib, d)
    assert set(decl) == set(_ffi.exported_names())


@pytest.mark.parametrize("ns,n", [(1, 0), (1, 1), (2, 1), (8, 4), (16, 5), (16, 8), (36, 3), (20, 10)])
def test_basis_matches_oracle(ns, n):
    st = ed.build_basis(ns, n)
    if ns <= 20:
        assert np.array_equal(st, basis_states(ns, n))
    assert np.all(np.diff(st.astype(np.float64)) > 0) if st.size > 1 else True
    assert np.array_equal(ed.state_rank(ns, n, st), np.arange(st.size))


def test_basis_errors():
    with pytest.raises(ed.EdError) as e:
        ed.build_basis(65, 3)
    assert e.value.code == _ffi.ED_EOVERFLOW
    with pytest.raises(ed.EdError) as e:
        ed.build_basis(8, 9)
    assert e.value.code == _ffi.ED_EINVAL
    with pytest.raises(ed.EdError) as e:
        ed.build_basis(40, 20)          # C(40,20) > 2^31
    assert e.value.code == _ffi.ED_EOVERFLOW
    import ctypes
    d = ctypes.c_int64(0)
    buf = np.zeros(3, dtype=np.uint64)
    rc = ed.lib().ed_build_basis(8, 4, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 3, ctypes.byref(d))
    assert rc == _ffi.ED_ECAPACITY and d.value == 70


def test_rank_rejects_foreign_state():
    with pytest.raises(ed.EdError):
        ed.state_rank(8, 4, np.array([0b111], dtype=np.uint64))


CASES = [("two_site", 2, two_site_bonds(), 1), ("ring8_n4", 8, ring_bonds(8), 4), ("ring8_n3", 8, ring_bonds(8), 3),
         ("t44_n3", 16, torus_bonds(4, 4), 3), ("t44_n5", 16, torus_bonds(4, 4), 5),
         ("t66_n3", 36, torus_bonds(6, 6), 3), ("ring6_n0", 6, ring_bonds(6), 0), ("ring6_n6", 6, ring_bonds(6), 6)]


@pytest.mark.parametrize("name,ns,bonds,n", CASES)
def test_hopping_ell_bit_exact_vs_oracle(name, ns, bonds, n):
    st = basis_states(ns, n)
    data, ind, width = to_ell(hopping_matrix(ns, bonds, st))
    for layout, order in ((ed.ED_ROW_MAJOR, "C"), (ed.ED_COL_MAJOR, "F")):
        t = ed.build_hopping(ns, bonds, st, layout)
        assert t["width"] == width
        if width:
            assert np.array_equal(t["cols"], ind.flatten(order=order).astype(np.int32))
            assert np.array_equal(t["vals"], data.flatten(order=order))
        assert np.array_equal(t["nnz"], (data != 0).sum(axis=1)) if width else True


def test_hopping_half_filling_4x4_vs_oracle():
    st = basis_states(16, 8)
    data, ind, width = to_ell(hopping_matrix(16, torus_bonds(4, 4), st))
    t = ed.build_hopping(16, torus_bonds(4, 4), st, ed.ED_ROW_MAJOR)
    assert width == 32 and t["width"] == 32
    assert np.array_equal(t["cols"], ind.ravel().astype(np.int32))
    assert np.array_equal(t["vals"], data.ravel())
    assert int(t["nnz"].sum()) == 219648


def test_pack_tables_roundtrip():
    st = ed.build_basis(16, 5)
    t = ed.build_hopping(16, torus_bonds(4, 4), st, ed.ED_ROW_MAJOR)
    w8 = ed.api.table_stride(t["width"])
    assert w8 % 8 == 0 and w8 >= t["width"]
    packed = ed.pack_tables(t, st.size)
    assert packed.size == 2 * st.size * w8
    p = packed[:st.size * w8].reshape(st.size, w8)      # [r, k]
    il = packed[st.size * w8:].reshape(w8 // 8, st.size, 8)
    assert np.array_equal(il.transpose(1, 0, 2).reshape(st.size, w8), p)
    cols = t["cols"].reshape(st.size, t["width"])
    vals = t["vals"].reshape(st.size, t["width"])
    for r in range(0, st.size, 37):
        for k in range(w8):
            e = int(p[r, k])
            if k < t["nnz"][r]:
                assert e >> 1 == cols[r, k] and ((e & 1) == 1) == (vals[r, k] < 0)
            else:
                assert e == 0xFFFF
    # the column-major export packs to the same device table
    tc = ed.build_hopping(16, torus_bonds(4, 4), st, ed.ED_COL_MAJOR)
    assert np.array_equal(ed.pack_tables(tc, st.size), packed)


def test_pack_tables32_widens_the_16bit_table():
    """The 32-bit format holds the same entries (padding all ones) in the same two layouts."""
    st = ed.build_basis(16, 5)
    t = ed.build_hopping(16, torus_bonds(4, 4), st, ed.ED_COL_MAJOR)
    p16 = ed.pack_tables(t, st.size)
    p32 = ed.pack_tables(t, st.size, entry_bytes=4)
    assert p32.dtype == np.uint32 and p32.size == p16.size
    want = np.where(p16 == 0xFFFF, np.uint32(0xFFFFFFFF), p16.astype(np.uint32))
    assert np.array_equal(p32, want)


def test_pack_tables32_beyond_15bit_ranks_matches_oracle():
    """18-site chain, 9 particles: 48620 states, more than 15-bit ranks hold.  The 16-bit packer
    refuses; the 32-bit table decodes to the oracle's hopping matrix (columns and signs), row by row."""
    n_sites, n = 18, 9
    st = ed.build_basis(n_sites, n)
    assert st.size == 48620
    t = ed.build_hopping(n_sites, ring_bonds(n_sites), st, ed.ED_COL_MAJOR)
    with pytest.raises(ed.EdError) as ei:
        ed.pack_tables(t, st.size)
    assert ei.value.code == -3          # ED_EOVERFLOW
    p = ed.pack_tables(t, st.size, entry_bytes=4)
    w8 = ed.api.table_stride(t["width"])
    rm = p[:st.size * w8].reshape(st.size, w8)
    il = p[st.size * w8:].reshape(w8 // 8, st.size, 8)
    assert np.array_equal(il.transpose(1, 0, 2).reshape(st.size, w8), rm)
    h = hopping_matrix(n_sites, ring_bonds(n_sites), basis_states(n_sites, n), 1.0).tocsr()
    for r in list(range(0, st.size, 997)) + [st.size - 1]:
        row = h.getrow(r)
        order = np.argsort(row.indices)
        cols, vals = row.indices[order], row.data[order]
        e = rm[r]
        live = e != 0xFFFFFFFF
        assert live.sum() == cols.size and np.all(~live[cols.size:])
        assert np.array_equal((e[live] >> 1).astype(np.int64), cols)
        # the sign bit: the entry is the matrix element at t = 1
        assert np.array_equal(np.where(e[live] & 1, -1.0, 1.0), vals)


def test_complex_tables_decode_to_the_oracle_matrix():
    """18-site checkerboard (complex nearest-neighbour amplitudes): the exported rows and the packed
    complex table (column, amplitude index) reproduce the oracle's complex hopping matrix."""
    from oracle.hopping import hopping_matrix_complex
    from synth import checkerboard_terms
    terms = checkerboard_terms(3, 3, 1.0, np.pi / 4, 0.3, 0.2)
    bonds, amps = [b for b, _ in terms], [a for _, a in terms]
    st = ed.build_basis(18, 3)
    t = ed.api.build_hopping_complex(18, bonds, amps, st, ed.ED_ROW_MAJOR)
    ref = hopping_matrix_complex(18, bonds, amps, basis_states(18, 3)).toarray()
    w = t["width"]
    assert w == int(np.max(np.count_nonzero(ref, axis=1)))
    cols, vals = t["cols"].reshape(st.size, w), t["vals"].reshape(st.size, w)
    got = np.zeros_like(ref)
    for r in range(st.size):
        for k in range(t["nnz"][r]):
            got[r, cols[r, k]] = vals[r, k]
    assert np.max(np.abs(got - ref)) < 1e-15
    packed, table, n = ed.api.pack_tables_complex(t, st.size)
    amp = table[0::2] + 1j * table[1::2]
    assert 1 <= n <= 64 and np.all(amp[n:] == 0)
    w8 = ed.api.table_stride(w)
    rm = packed[:st.size * w8].reshape(st.size, w8)
    il = packed[st.size * w8:].reshape(w8 // 8, st.size, 8)
    assert np.array_equal(il.transpose(1, 0, 2).reshape(st.size, w8), rm)
    dec = np.zeros_like(ref)
    for r in range(st.size):
        for e in rm[r]:
            if e != 0xFFFFFFFF:
                dec[r, int(e) >> 6] = amp[int(e) & 63]
    assert np.array_equal(dec, got)
    # every amplitude -1 is the real table
    tr = ed.build_hopping(18, bonds, st, ed.ED_ROW_MAJOR)
    tc = ed.api.build_hopping_complex(18, bonds, [-1.0] * len(bonds), st, ed.ED_ROW_MAJOR)
    assert np.array_equal(tc["cols"], tr["cols"]) and np.array_equal(tc["vals"].real, tr["vals"])
    assert np.all(tc["vals"].imag == 0)


def test_hopping_errors():
    st = ed.build_basis(4, 2)
    with pytest.raises(ed.EdError):
        ed.build_hopping(4, [(0, 1), (1, 0)], st)       # duplicate unordered bond
    with pytest.raises(ed.EdError):
        ed.build_hopping(4, [(0, 4)], st)               # site out of range
    with pytest.raises(ed.EdError):
        ed.build_hopping(4, [(2, 2)], st)


def test_pack_rejects_non_unit_values():
    t = {"cols": np.array([0, 1], dtype=np.int32), "vals": np.array([2.0, 1.0]),
         "nnz": np.array([1, 1], dtype=np.int32), "width": 1, "layout": ed.ED_ROW_MAJOR}
    with pytest.raises(ed.EdError):
        ed.pack_tables(t, 2)


def test_tridiag_closed_forms():
    assert ed.tridiag_lowest([2.5], []) == 2.5
    a1, a2, b = 1.3, -0.4, 0.9
    ref = ((a1 + a2) - np.sqrt((a1 - a2) ** 2 + 4 * b * b)) / 2
    assert abs(ed.tridiag_lowest([a1, a2], [b]) - ref) < 1e-15 * 4


@pytest.mark.parametrize("m", [3, 17, 100, 300])
def test_tridiag_vs_lapack(m):
    rng = np.random.default_rng(m)
    for _ in range(5):
        a, b = rng.normal(size=m) * 10, rng.uniform(0.01, 3.0, m - 1)
        ref = sla.eigh_tridiagonal(a, b, eigvals_only=True)[0]
        nrm = np.abs(a).max() + 2 * b.max()
        assert abs(ed.tridiag_lowest(a, b) - ref) <= 1e-13 * nrm
        e, y = ed.tridiag_lowest_vector(a, b)
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        assert abs(np.linalg.norm(y) - 1) < 1e-12
        assert np.linalg.norm(T @ y - e * y) < 1e-10 * nrm


def test_tridiag_near_degenerate_vector():
    # tiny off-diagonal coupling between two blocks: eigenvector still accurate
    a = np.array([1.0, 1.0, -3.0, 0.5])
    b = np.array([0.5, 1e-9, 0.2])
    e, y = ed.tridiag_lowest_vector(a, b)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    w, v = np.linalg.eigh(T)
    assert abs(e - w[0]) < 1e-14 and abs(abs(y @ v[:, 0]) - 1) < 1e-12


def test_tridiag_rejects_nan():
    with pytest.raises(ed.EdError):
        ed.tridiag_lowest([1.0, np.nan], [0.5])


def test_device_calls_validate_before_touching_the_device():
    """Bad descriptors are rejected on the host with the documented codes (no GPU needed)."""
    import ctypes
    lib = ed.lib()
    dummy = ctypes.c_void_p(4096)   # never dereferenced: every case fails validation first

    def ham(**kw):
        f = dict(dim_up=70, dim_dn=70, w_up=8, w_dn=8, tab_up=dummy, tab_dn=dummy, st_up=dummy, st_dn=dummy,
                 t=1.0, U=4.0, dtype=0, tile=0)
        f.update(kw)
        return _ffi.EdHam(**f)

    nbytes = ctypes.c_int64(0)
    assert lib.ed_workspace_size(ctypes.byref(ham()), 10, ctypes.byref(nbytes)) == 0 and nbytes.value > 0
    cases = [
        (dict(dim_up=40000), -3),            # per-spin dimension above 15-bit ranks
        (dict(dim_dn=0), -1),
        (dict(w_up=12), -1),                 # stride not a multiple of 8
        (dict(w_dn=72), -3),                 # stride above 64
        (dict(w_up=8, tab_up=None), -1),     # hopping without a table
        (dict(st_dn=None), -1),
        (dict(dtype=7), -1),
        (dict(tile=0x7FFF0000), -1),
        (dict(U=float("nan")), -1),
        (dict(t=float("inf")), -1),
    ]
    for kw, code in cases:
        h = ham(**kw)
        assert lib.ed_workspace_size(ctypes.byref(h), 10, ctypes.byref(nbytes)) == code, kw
        assert lib.ed_hv(ctypes.byref(h), dummy, ctypes.c_void_p(8192), dummy, None) == code, kw
        assert lib.ed_last_error().decode()
    for kw, code in [(dict(eb_up=3), -1), (dict(eb_dn=1), -1),
                     (dict(eb_up=4, dim_up=(1 << 30) + 1), -3), (dict(eb_dn=2, dim_dn=40000), -3)]:
        h = ham(**kw)
        assert lib.ed_workspace_size(ctypes.byref(h), 10, ctypes.byref(nbytes)) == code, kw
    # 32-bit tables lift the 15-bit rank limit of a species (validation only: nothing is launched)
    assert lib.ed_workspace_size(ctypes.byref(ham(eb_up=4, dim_up=48620)), 10, ctypes.byref(nbytes)) == 0
    # a species without hopping may pass no table
    h = ham(w_dn=0, tab_dn=None)
    assert lib.ed_workspace_size(ctypes.byref(h), 10, ctypes.byref(nbytes)) == 0


def test_spin_correlations_match_oracle_formula():
    from oracle.observables import spin_correlations
    r = np.random.default_rng(9)
    ns = 5
    g = r.uniform(0, 1, (2 * ns, 2 * ns))
    g = (g + g.T) / 2
    c = r.uniform(-0.5, 0.5, (ns, ns))
    assert np.max(np.abs(ed.spin_correlations(g, c, ns) - spin_correlations(g, c, ns))) < 1e-15


def test_complex_tables_reject_bad_inputs():
    st = ed.build_basis(6, 2)
    bonds = ring_bonds(6)
    with pytest.raises(ed.EdError) as e:
        ed.api.build_hopping_complex(6, bonds, [1.0] * 5 + [complex(float("nan"), 0.0)], st)
    assert e.value.code == -1
    # more than 64 distinct values cannot be indexed with 6 bits
    many = ed.build_basis(12, 2)
    cb = complete_bonds(12)
    amps = [complex(1.0 + 0.01 * k, 0.0) for k in range(len(cb))]   # 66 distinct amplitudes
    t = ed.api.build_hopping_complex(12, cb, amps, many)
    with pytest.raises(ed.EdError) as e:
        ed.api.pack_tables_complex(t, many.size)
    assert e.value.code == -3


def test_observable_and_complex_descriptors_validated_on_the_host():
    """Argument errors of the observables and of complex descriptors are returned before any device work."""
    import ctypes
    lib = ed.lib()
    dummy = ctypes.c_void_p(4096)   # never dereferenced

    def ham(**kw):
        f = dict(dim_up=70, dim_dn=70, w_up=8, w_dn=8, tab_up=dummy, tab_dn=dummy, st_up=dummy, st_dn=dummy,
                 t=1.0, U=4.0, dtype=0, tile=0, eb_up=0, eb_dn=0, cplx=0, order=0, amp_up=None, amp_dn=None)
        f.update(kw)
        return _ffi.EdHam(**f)

    n = ctypes.c_int64(0)
    assert lib.ed_workspace_size(ctypes.byref(ham(cplx=2)), 4, ctypes.byref(n)) == -1
    # complex amplitudes need 32-bit complex tables and amplitude arrays
    assert lib.ed_workspace_size(ctypes.byref(ham(cplx=1)), 4, ctypes.byref(n)) == -1
    ok = ham(cplx=1, eb_up=4, eb_dn=4, amp_up=dummy, amp_dn=dummy)
    assert lib.ed_workspace_size(ctypes.byref(ok), 4, ctypes.byref(n)) == 0
    # real-only calls refuse complex instances
    assert lib.ed_occupation_moments_ws(ctypes.byref(ok), 8, ctypes.byref(n)) == -1
    assert lib.ed_spin_flip_moments_ws(ctypes.byref(ok), 8, ctypes.byref(n)) == -1
    # observables: site count and bonds
    real = ham()
    assert lib.ed_spin_flip_moments_ws(ctypes.byref(real), 33, ctypes.byref(n)) == -1
    assert lib.ed_bond_moments_ws(ctypes.byref(real), 8, 0, ctypes.byref(n)) == -1
    bad = (ctypes.c_int32 * 2)(3, 3)
    c = (ctypes.c_double * 2)()
    assert lib.ed_bond_moments(ctypes.byref(real), 8, bad, 1, dummy, dummy, 1 << 20, None, c) == -1
    out_of_range = (ctypes.c_int32 * 2)(0, 8)
    assert lib.ed_bond_moments(ctypes.byref(real), 8, out_of_range, 1, dummy, dummy, 1 << 20, None, c) == -1
    assert lib.ed_last_error().decode()
