"""Python face of the C ABI: host arrays via numpy, device memory and streams via torch.

Every computation happens in the library (host C++ or gfx950 kernels); this
module only allocates buffers, fills the C structs and maps error codes to
exceptions.  Names follow the C entry points of include/ed.h.
"""

import ctypes
import json
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_uint16, c_uint32, c_uint64

import numpy as np
import torch

from . import _ffi
from ._ffi import (ED_COL_MAJOR, ED_F32, ED_F64, ED_ROW_MAJOR, EdBatchItem, EdHam, EdLanczos, check, lib)


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(POINTER(ctype))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------- host calls
def build_basis(n_sites: int, n_part: int) -> np.ndarray:
    d = c_int64(0)
    check(lib().ed_build_basis(n_sites, n_part, None, 0, byref(d)))
    st = np.zeros(d.value, dtype=np.uint64)
    check(lib().ed_build_basis(n_sites, n_part, _ptr(st, c_uint64), d.value, byref(d)))
    return st


def state_rank(n_sites: int, n_part: int, states) -> np.ndarray:
    st = np.ascontiguousarray(states, dtype=np.uint64)
    out = np.zeros(st.size, dtype=np.int64)
    check(lib().ed_state_rank(n_sites, n_part, _ptr(st, c_uint64), st.size, _ptr(out, c_int64)))
    return out


def wave_chunks(nnz) -> np.ndarray:
    """ed_wave_chunks: per 64 consecutive rows, the 8-entry table chunks the widest of them needs."""
    n = np.ascontiguousarray(nnz, dtype=np.int32)
    out = np.zeros((n.size + 63) // 64, dtype=np.uint32)
    check(lib().ed_wave_chunks(_ptr(n, c_int32), n.size, _ptr(out, c_uint32)))
    return out


def hop_order(nnz) -> np.ndarray:
    """ed_hop_order: positions of a basis sorted by hop count, most first, ties in their given order."""
    n = np.ascontiguousarray(nnz, dtype=np.int32)
    perm = np.zeros(n.size, dtype=np.int64)
    check(lib().ed_hop_order(_ptr(n, c_int32), n.size, _ptr(perm, c_int64)))
    return perm


def band_order(table) -> np.ndarray:
    """ed_band_order: reverse Cuthill-McKee positions of a basis from its ELL table (build_hopping output)."""
    nnz = np.ascontiguousarray(table["nnz"], dtype=np.int32)
    cols = np.ascontiguousarray(table["cols"], dtype=np.int32)
    perm = np.zeros(nnz.size, dtype=np.int64)
    check(lib().ed_band_order(_ptr(cols, c_int32), _ptr(nnz, c_int32), nnz.size, int(table["width"]),
                              int(table["layout"]), _ptr(perm, c_int64)))
    return perm


def row_windows(table, block_cols: int):
    """ed_row_windows: (lo_hi, max_window) of the column blocks of block_cols states (ELL table from
    build_hopping): lo_hi[2b], lo_hi[2b+1] bound block b's states and their table columns."""
    nnz = np.ascontiguousarray(table["nnz"], dtype=np.int32)
    cols = np.ascontiguousarray(table["cols"], dtype=np.int32)
    nblk = (nnz.size + block_cols - 1) // block_cols
    lo_hi = np.zeros(2 * nblk, dtype=np.int32)
    widest = c_int32(0)
    check(lib().ed_row_windows(_ptr(cols, c_int32), _ptr(nnz, c_int32), nnz.size, int(table["width"]),
                               int(table["layout"]), int(block_cols), _ptr(lo_hi, c_int32), byref(widest)))
    return lo_hi, int(widest.value)


def pack_tables_windowed(table, dim: int, block_cols: int, lo_hi) -> np.ndarray:
    """ed_pack_tables_windowed: the down table with columns relative to their block's window (uint16 entries,
    the layout of pack_tables)."""
    stride = table_stride(table["width"])
    out = np.zeros(max(2 * stride * dim, 1), dtype=np.uint16)
    vals = np.ascontiguousarray(table["vals"], dtype=np.float64)
    lh = np.ascontiguousarray(lo_hi, dtype=np.int32)
    check(lib().ed_pack_tables_windowed(_ptr(table["cols"], c_int32), _ptr(vals, c_double),
                                        _ptr(table["nnz"], c_int32), dim, int(table["width"]), int(table["layout"]),
                                        int(block_cols), _ptr(lh, c_int32), _ptr(out, c_uint16)))
    return out


# Column blocks of the neighbour windows a down species carries (ed_ham.win_dn): rows longer than this
# many states are the ones that do not fit LDS (19,456 FP64 states); a block's window holds its states and
# their neighbours.
WINDOW_COLS = 8192
WINDOW_MIN_DIM = 16384


def permute_basis(states, table, perm):
    """ed_permute_basis: (states, table) of a species in the order perm (real or complex exported tables)."""
    st = np.ascontiguousarray(states, dtype=np.uint64)
    pm = np.ascontiguousarray(perm, dtype=np.int64)
    dim, width = st.size, int(table["width"])
    nv = 2 if np.iscomplexobj(table["vals"]) else 1
    vals = np.ascontiguousarray(table["vals"]).view(np.float64) if nv == 2 else np.ascontiguousarray(table["vals"], dtype=np.float64)
    cols = np.ascontiguousarray(table["cols"], dtype=np.int32)
    nnz = np.ascontiguousarray(table["nnz"], dtype=np.int32)
    st_o = np.zeros(dim, dtype=np.uint64)
    cols_o = np.zeros(max(cols.size, 1), dtype=np.int32)
    vals_o = np.zeros(max(vals.size, 1), dtype=np.float64)
    nnz_o = np.zeros(dim, dtype=np.int32)
    check(lib().ed_permute_basis(_ptr(st, c_uint64), _ptr(cols, c_int32) if cols.size else None,
                                 _ptr(vals, c_double) if vals.size else None, _ptr(nnz, c_int32), dim, width,
                                 int(table["layout"]), nv, _ptr(pm, c_int64), _ptr(st_o, c_uint64),
                                 _ptr(cols_o, c_int32) if cols.size else None,
                                 _ptr(vals_o, c_double) if vals.size else None, _ptr(nnz_o, c_int32)))
    out = {"cols": cols_o[:cols.size], "vals": vals_o[:vals.size], "nnz": nnz_o, "width": width,
           "layout": table["layout"]}
    if nv == 2:
        out["vals"] = out["vals"].view(np.complex128)
    return st_o, out


def _bond_array(bonds) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))


def build_hopping(n_sites: int, bonds, states, layout: int = ED_COL_MAJOR):
    """Exported ELL table of H_sigma for t=1: dict(cols, vals, nnz, width) (Fig. 2 layout)."""
    st = np.ascontiguousarray(states, dtype=np.uint64)
    b = _bond_array(bonds)
    w = c_int32(0)
    check(lib().ed_build_hopping(n_sites, _ptr(b, c_int32), b.shape[0], _ptr(st, c_uint64), st.size, layout, 0,
                                 None, None, None, byref(w)))
    width = w.value
    cols = np.zeros(max(width, 1) * st.size, dtype=np.int32)
    vals = np.zeros(max(width, 1) * st.size, dtype=np.float64)
    nnz = np.zeros(st.size, dtype=np.int32)
    check(lib().ed_build_hopping(n_sites, _ptr(b, c_int32), b.shape[0], _ptr(st, c_uint64), st.size, layout,
                                 max(width, 1), _ptr(cols, c_int32), _ptr(vals, c_double), _ptr(nnz, c_int32),
                                 byref(w)))
    cap = max(width, 1)
    cols, vals = cols[:width * st.size], vals[:width * st.size]
    if cap != width and width == 0:
        cols, vals = cols[:0], vals[:0]
    return {"cols": cols, "vals": vals, "nnz": nnz, "width": width, "layout": layout}


def table_stride(width: int) -> int:
    """Row stride of the device table: the ELL width rounded up to a multiple of 8."""
    return (int(width) + 7) & ~7


def build_hopping_complex(n_sites: int, bonds, amps, states, layout: int = ED_COL_MAJOR):
    """Exported ELL table of H_sigma with a complex amplitude per bond (term a c+_i c_j + h.c., t = 1):
    dict(cols, vals (complex128), nnz, width, layout) (ed_build_hopping_complex)."""
    st = np.ascontiguousarray(states, dtype=np.uint64)
    b = _bond_array(bonds)
    a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128).reshape(-1))
    if a.size != b.shape[0]:
        raise ValueError("one amplitude per bond")
    ad = a.view(np.float64)
    w = c_int32(0)
    f = lib().ed_build_hopping_complex
    check(f(n_sites, _ptr(b, c_int32), b.shape[0], _ptr(ad, c_double), _ptr(st, c_uint64), st.size, layout, 0,
            None, None, None, byref(w)))
    width = w.value
    cap = max(width, 1)
    cols = np.zeros(cap * st.size, dtype=np.int32)
    vals = np.zeros(cap * st.size, dtype=np.complex128)
    nnz = np.zeros(st.size, dtype=np.int32)
    check(f(n_sites, _ptr(b, c_int32), b.shape[0], _ptr(ad, c_double), _ptr(st, c_uint64), st.size, layout, cap,
            _ptr(cols, c_int32), _ptr(vals.view(np.float64), c_double), _ptr(nnz, c_int32), byref(w)))
    return {"cols": cols[:width * st.size], "vals": vals[:width * st.size], "nnz": nnz, "width": width,
            "layout": layout}


def pack_tables_complex(table, dim: int):
    """(packed uint32 table, 64 complex amplitudes as 128 doubles, number used) (ed_pack_tables_complex)."""
    width = table["width"]
    stride = table_stride(width)
    out = np.zeros(max(2 * stride * dim, 1), dtype=np.uint32)
    amps = np.zeros(128, dtype=np.float64)
    n = c_int32(0)
    if width == 0:
        return out[:0], amps, 0
    vals = np.ascontiguousarray(table["vals"], dtype=np.complex128).view(np.float64)
    check(lib().ed_pack_tables_complex(_ptr(table["cols"], c_int32), _ptr(vals, c_double),
                                       _ptr(table["nnz"], c_int32), dim, width, table["layout"],
                                       _ptr(out, c_uint32), _ptr(amps, c_double), byref(n)))
    return out, amps, n.value


NARROW_MAX_DIM = 32767   # largest per-spin dimension of the 16-bit table format


def pack_tables(table, dim: int, entry_bytes: int = 2) -> np.ndarray:
    """Device table (row-major then 8-interleaved, stride table_stride(width)) with uint16 entries
    (ed_pack_tables, dim <= 32767) or uint32 entries (ed_pack_tables32, larger dimensions)."""
    if entry_bytes not in (2, 4):
        raise ValueError("entry_bytes must be 2 or 4")
    width = table["width"]
    stride = table_stride(width)
    out = np.zeros(max(2 * stride * dim, 1), dtype=np.uint16 if entry_bytes == 2 else np.uint32)
    if width == 0:
        return out[:0]
    args = (_ptr(table["cols"], c_int32), _ptr(table["vals"], c_double), _ptr(table["nnz"], c_int32), dim, width,
            table["layout"])
    if entry_bytes == 2:
        check(lib().ed_pack_tables(*args, _ptr(out, c_uint16)))
    else:
        check(lib().ed_pack_tables32(*args, _ptr(out, c_uint32)))
    return out


def occupation_correlations(g: np.ndarray, n_sites: int) -> dict:
    """docc[i], nn[i, j] = <n_i n_j>, szsz[i, j] = <S^z_i S^z_j> from occupation moments (ed_occupation_correlations)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    docc = np.zeros(n_sites)
    nn = np.zeros((n_sites, n_sites))
    szsz = np.zeros((n_sites, n_sites))
    check(lib().ed_occupation_correlations(_ptr(g, c_double), int(n_sites), _ptr(docc, c_double),
                                           _ptr(nn, c_double), _ptr(szsz, c_double)))
    return {"docc": docc, "nn": nn, "szsz": szsz}


def spin_correlations(g: np.ndarray, c: np.ndarray, n_sites: int) -> np.ndarray:
    """<S_i . S_j> from occupation moments g and spin-flip moments c (ed_spin_correlations)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    ss = np.zeros((n_sites, n_sites))
    check(lib().ed_spin_correlations(_ptr(g, c_double), _ptr(c, c_double), int(n_sites), _ptr(ss, c_double)))
    return ss


def tridiag_lowest(a, b_off) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b_off, dtype=np.float64)
    e = c_double(0)
    check(lib().ed_tridiag_lowest(_ptr(a, c_double), _ptr(b, c_double) if b.size else None, a.size, byref(e)))
    return e.value


def tridiag_lowest_vector(a, b_off):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b_off, dtype=np.float64)
    y = np.zeros(a.size)
    e = c_double(0)
    check(lib().ed_tridiag_lowest_vector(_ptr(a, c_double), _ptr(b, c_double) if b.size else None, a.size,
                                         byref(e), _ptr(y, c_double)))
    return e.value, y


# ---------------------------------------------------------------- device side
class SpinTables:
    """Basis and packed hopping table of one species, on the host and on the device."""

    def __init__(self, n_sites: int, bonds, n_part: int, device=None, entry_bytes=None, amps=None,
                 order: str = "ascending"):
        """entry_bytes: 2 or 4 bytes per device table entry; by default 2 while dim <= 32767, else 4.
        amps: a complex amplitude per bond (term a c+_i c_j + h.c.); then the table is the complex format
        (32-bit entries indexing a table of at most 64 amplitudes) and the vectors are complex.
        order: "ascending" (the basis of Sec. 2.1), "hops" (sorted by hop count, ed_hop_order) or "band"
        (neighbours numbered close together, ed_band_order); then position q holds ascending state perm[q],
        and vectors of this species follow that order."""
        if order not in ("ascending", "hops", "band"):
            raise ValueError("order must be 'ascending', 'hops' or 'band'")
        self.n_sites, self.n_part = n_sites, n_part
        self.bonds = [tuple(int(v) for v in b) for b in bonds]
        self.states = build_basis(n_sites, n_part)
        self.dim = int(self.states.size)
        self.cplx = amps is not None
        self.order = order
        self.perm = None
        self.device = torch.device(device if device is not None else "cuda")
        self.dev_amp = None
        self._dev_perm = self._dev_inv = None
        if self.cplx:
            self.table = build_hopping_complex(n_sites, self.bonds, amps, self.states, ED_COL_MAJOR)
            if order != "ascending":
                self.perm = hop_order(self.table["nnz"]) if order == "hops" else band_order(self.table)
                self.states, self.table = permute_basis(self.states, self.table, self.perm)
            self.width = self.table["width"]
            self.stride = table_stride(self.width)
            self.entry_bytes = 4
            self.packed, self.amps, self.n_amps = pack_tables_complex(self.table, self.dim)
            self.dev_amp = torch.from_numpy(self.amps.copy()).to(self.device)
        else:
            self.table = build_hopping(n_sites, self.bonds, self.states, ED_COL_MAJOR)
            if order != "ascending":
                self.perm = hop_order(self.table["nnz"]) if order == "hops" else band_order(self.table)
                self.states, self.table = permute_basis(self.states, self.table, self.perm)
            self.width = self.table["width"]
            self.stride = table_stride(self.width)
            # 16-bit entries while the ranks fit in 15 bits, 32-bit beyond
            self.entry_bytes = int(entry_bytes) if entry_bytes else (2 if self.dim <= NARROW_MAX_DIM else 4)
            self.packed = pack_tables(self.table, self.dim, self.entry_bytes)
        self.dev_states = torch.from_numpy(self.states.view(np.int64).copy()).to(self.device)
        # neighbour windows of column blocks, for rows of this species too long for LDS (real tables)
        self.win_cols, self.win_max, self.dev_win, self.dev_win_tab = 0, 0, None, None
        # table chunks per 64 consecutive states (real tables): the down part of a species alone reads no more
        self.dev_wch = None
        if not self.cplx and self.width:
            self.dev_wch = torch.from_numpy(wave_chunks(self.table["nnz"]).view(np.int32)).to(self.device)
        if not self.cplx and self.width and self.dim >= WINDOW_MIN_DIM:
            lo_hi, self.win_max = row_windows(self.table, WINDOW_COLS)
            self.win_cols = WINDOW_COLS
            self.dev_win = torch.from_numpy(lo_hi).to(self.device)
            if self.win_max <= NARROW_MAX_DIM:   # the window-relative table takes 16-bit entries
                rel = pack_tables_windowed(self.table, self.dim, WINDOW_COLS, lo_hi)
                self.dev_win_tab = torch.from_numpy(rel.view(np.int16).copy()).to(self.device)
        signed = np.int16 if self.entry_bytes == 2 else np.int32
        self.dev_tab = (torch.from_numpy(self.packed.view(signed).copy()).to(self.device)
                        if self.width else torch.zeros(1, dtype=torch.int32, device=self.device))

    def dev_perm(self, inverse: bool = False):
        """Device int64 permutation of this species (None in ascending order): perm (position -> ascending
        index), or with inverse=True its inverse (ascending index -> position)."""
        if self.perm is None:
            return None
        if self._dev_perm is None:
            inv = np.empty_like(self.perm)
            inv[self.perm] = np.arange(self.dim, dtype=np.int64)
            self._dev_perm = torch.from_numpy(self.perm.copy()).to(self.device)
            self._dev_inv = torch.from_numpy(inv).to(self.device)
        return self._dev_inv if inverse else self._dev_perm


class Hamiltonian:
    """One (lattice, N_up, N_dn, t, U) instance with device tables; float64 or float32 vectors."""

    def __init__(self, up: SpinTables, dn: SpinTables, t: float = 1.0, U: float = 0.0, dtype: str = "f64",
                 tile: int = 0):
        self.up, self.dn, self.t, self.U = up, dn, float(t), float(U)
        if up.cplx != dn.cplx:
            raise ValueError("both species need complex tables, or neither")
        self.cplx = up.cplx
        self.dtype = ED_F64 if dtype in ("f64", torch.float64, torch.complex128) else ED_F32
        self.tile = int(tile)
        self.device = up.device

    @classmethod
    def from_lattice(cls, n_sites, bonds, n_up, n_dn, t=1.0, U=0.0, dtype="f64", device=None, tile=0,
                     entry_bytes=None, amps=None, order=("ascending", "ascending")):
        """order: the (up, down) basis orders of SpinTables, or one string for both."""
        ou, od = (order, order) if isinstance(order, str) else tuple(order)
        up = SpinTables(n_sites, bonds, n_up, device, entry_bytes, amps, ou)
        dn = up if (n_dn == n_up and od == ou) else SpinTables(n_sites, bonds, n_dn, device, entry_bytes, amps, od)
        return cls(up, dn, t, U, dtype, tile)

    @property
    def dim_up(self):
        return self.up.dim

    @property
    def dim_dn(self):
        return self.dn.dim

    @property
    def dim(self):
        return self.up.dim * self.dn.dim

    @property
    def torch_dtype(self):
        if self.cplx:
            return torch.complex128 if self.dtype == ED_F64 else torch.complex64
        return torch.float64 if self.dtype == ED_F64 else torch.float32

    def c_struct(self) -> EdHam:
        return EdHam(self.dim_up, self.dim_dn, self.up.stride, self.dn.stride,
                     self.up.dev_tab.data_ptr(), self.dn.dev_tab.data_ptr(),
                     self.up.dev_states.data_ptr(), self.dn.dev_states.data_ptr(),
                     self.t, self.U, self.dtype, self.tile, self.up.entry_bytes, self.dn.entry_bytes,
                     int(self.cplx), self.order_bits,
                     self.up.dev_amp.data_ptr() if self.up.dev_amp is not None else None,
                     self.dn.dev_amp.data_ptr() if self.dn.dev_amp is not None else None,
                     self.dn.dev_win.data_ptr() if self.dn.dev_win is not None else None,
                     self.dn.win_cols, self.dn.win_max,
                     self.dn.dev_win_tab.data_ptr() if self.dn.dev_win_tab is not None else None,
                     self.dn.dev_wch.data_ptr() if self.dn.dev_wch is not None else None)

    @property
    def order_bits(self) -> int:
        """ed_ham.order: bit 0 / bit 1 set when the up / down basis is not ascending."""
        return (1 if self.up.order != "ascending" else 0) | (2 if self.dn.order != "ascending" else 0)

    def _permute(self, x, inverse: bool, stream=None):
        x = self._vec(x)
        y = self.empty_vec()
        pu, pd = self.up.dev_perm(inverse), self.dn.dev_perm(inverse)
        h = self.c_struct()
        check(lib().ed_permute_vector(byref(h), _dptr(pu), _dptr(pd), _dptr(x), _dptr(y), _stream(stream)))
        return y

    def to_basis_order(self, x, stream=None):
        """A vector over the ascending bases of both species, in this instance's basis order (ed_permute_vector)."""
        return self._permute(x, False, stream)

    def to_ascending(self, x, stream=None):
        """A vector in this instance's basis order, back over the ascending bases (ed_permute_vector)."""
        return self._permute(x, True, stream)

    def workspace_bytes(self, max_steps: int = 1) -> int:
        n = c_int64(0)
        h = self.c_struct()
        check(lib().ed_workspace_size(byref(h), max_steps, byref(n)))
        return n.value

    def workspace(self, max_steps: int = 1) -> torch.Tensor:
        return torch.empty(self.workspace_bytes(max_steps), dtype=torch.uint8, device=self.device)

    def empty_vec(self) -> torch.Tensor:
        return torch.empty(self.dim, dtype=self.torch_dtype, device=self.device)

    def _vec(self, x) -> torch.Tensor:
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.torch_dtype and x.is_contiguous()
                and x.numel() == self.dim):
            raise ValueError("expected a contiguous %s device vector of %d elements" % (self.torch_dtype, self.dim))
        return x

    def hv(self, x, y=None, ws=None, stream=None):
        """y = H x (Eq. 3-5 plus the U term)."""
        x = self._vec(x)
        y = self.empty_vec() if y is None else self._vec(y)
        if ws is None:
            ws = self.workspace(0)
        h = self.c_struct()
        check(lib().ed_hv(byref(h), _dptr(x), _dptr(y), _dptr(ws), _stream(stream)))
        return y

    def tile_params(self, tile=None):
        p = np.zeros(7, dtype=np.int32)
        h = self.c_struct()
        check(lib().ed_tile_params(self.tile if tile is None else int(tile), byref(h), _ptr(p, c_int32)))
        keys = ("stripe_width", "up_rows", "up_block", "up_map", "dn_block", "dn_rows", "dn_kind")
        return dict(zip(keys, p.tolist()))

    def tune(self, x=None, reps: int = 3, stream=None, apply: bool = True):
        """Time every tile candidate on y = H x and (apply=True) adopt the fastest.

        Returns dict(tile, up_ms, dn_ms) with per-candidate times (-1 = not applicable)."""
        if x is None:
            x = torch.ones(self.dim, dtype=self.torch_dtype, device=self.device)
        x = self._vec(x)
        y = self.empty_vec()
        p = x.clone()   # f_{j-1} of the timed down part: a vector of its own, as in a step
        ws = self.workspace(2)
        nu, nd = c_int32(0), c_int32(0)
        check(lib().ed_tile_count(byref(nu), byref(nd)))
        mu, md = np.full(nu.value, -1.0), np.full(nd.value, -1.0)
        tile = c_int32(0)
        h = self.c_struct()
        check(lib().ed_tune(byref(h), _dptr(x), _dptr(y), _dptr(p), _dptr(ws), _stream(stream), int(reps),
                            byref(tile), _ptr(mu, c_double), _ptr(md, c_double)))
        del p
        if apply:
            self.tile = tile.value
        return {"tile": tile.value, "up_ms": mu, "dn_ms": md}

    def occupation_moments(self, psi, n_sites: int, stream=None) -> np.ndarray:
        """G[a][b] = <n_a n_b> of the state psi over the 2*n_sites occupation numbers (ed_occupation_moments)."""
        psi = self._vec(psi)
        n = c_int64(0)
        h = self.c_struct()
        check(lib().ed_occupation_moments_ws(byref(h), int(n_sites), byref(n)))
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        g = np.zeros((2 * n_sites, 2 * n_sites))
        check(lib().ed_occupation_moments(byref(h), int(n_sites), _dptr(psi), _dptr(ws), n.value, _stream(stream),
                                          _ptr(g, c_double)))
        return g

    def spin_flip_moments(self, psi, n_sites: int, stream=None) -> np.ndarray:
        """C[i][j] = <S+_i S-_j> of the state psi (ed_spin_flip_moments)."""
        psi = self._vec(psi)
        n = c_int64(0)
        h = self.c_struct()
        check(lib().ed_spin_flip_moments_ws(byref(h), int(n_sites), byref(n)))
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        c = np.zeros((n_sites, n_sites))
        check(lib().ed_spin_flip_moments(byref(h), int(n_sites), _dptr(psi), _dptr(ws), n.value, _stream(stream),
                                         _ptr(c, c_double)))
        return c

    def bond_moments(self, psi, n_sites: int, bonds, stream=None) -> np.ndarray:
        """K[b, sigma] = <c+_i c_j + c+_j c_i> of species sigma for each bond (ed_bond_moments)."""
        psi = self._vec(psi)
        b = _bond_array(bonds)
        n = c_int64(0)
        h = self.c_struct()
        check(lib().ed_bond_moments_ws(byref(h), int(n_sites), b.shape[0], byref(n)))
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        k = np.zeros((b.shape[0], 2))
        check(lib().ed_bond_moments(byref(h), int(n_sites), _ptr(b, c_int32), b.shape[0], _dptr(psi), _dptr(ws),
                                    n.value, _stream(stream), _ptr(k, c_double)))
        return k

    def lanczos(self, max_steps: int) -> "LanczosRun":
        return LanczosRun(self, max_steps)

    def ground_energy(self, f1, max_steps: int, tol: float = 0.0, check_every: int = 10, stream=None):
        """Alg. 1 from f1 until |dE0| < tol twice (tol > 0) or exactly max_steps steps (tol <= 0)."""
        run = LanczosRun(self, max_steps)
        return run.ground_energy(f1, tol, check_every, stream)

    def ground_state(self, f1, m: int, gauge_index: int = -1, stream=None, tol: float = 0.0, extra: int = 0):
        """Two-pass ground-state vector: returns (E0, steps, v) with |v| = 1 and v[gauge_index] >= 0 (or, where
        that element is below 1e-3 of the largest magnitude, the largest-magnitude element positive).
        tol > 0: pass 1 stops where E0 settles (ed_ground_energy's rule) plus `extra` steps, at most m."""
        run = LanczosRun(self, m)
        return run.ground_state(f1, m, gauge_index, stream, tol, extra)


TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def tune_key(ham: "Hamiltonian") -> str:
    """Cache key of a tuned tile: architecture, per-spin dims, table strides, dtype."""
    dt = ("c128" if ham.dtype == ED_F64 else "c64") if ham.cplx else ("f64" if ham.dtype == ED_F64 else "f32")
    return "gfx950/%dx%d/w%dx%d/%s" % (ham.dim_up, ham.dim_dn, ham.up.stride, ham.dn.stride, dt)


def load_tune_cache(path: str = TUNE_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def apply_tuned_tile(ham: "Hamiltonian", x=None, path: str = TUNE_CACHE, tune_if_missing: bool = True) -> str:
    """Set ham.tile from the tuning cache, or run ed_tune when the key is absent.

    Returns "cache" or "tuned" (or "default" when missing and tune_if_missing is False)."""
    entry = load_tune_cache(path).get(tune_key(ham))
    if entry is not None:
        ham.tile = int(entry["tile"])
        return "cache"
    if tune_if_missing:
        ham.tune(x, reps=3)
        return "tuned"
    return "default"


class LanczosRun:
    """Buffers of one Lanczos run (three vectors, a, b, workspace) and the calls on them."""

    def __init__(self, ham: Hamiltonian, max_steps: int):
        self.ham = ham
        self.max_steps = int(max_steps)
        dev = ham.device
        self.vecs = [ham.empty_vec() for _ in range(3)]
        self.a = torch.zeros(max(self.max_steps, 1), dtype=torch.float64, device=dev)
        self.b = torch.zeros(self.max_steps + 1, dtype=torch.float64, device=dev)
        self.ws = ham.workspace(self.max_steps)
        self.st = EdLanczos(self.vecs[2].data_ptr(), self.vecs[0].data_ptr(), self.vecs[1].data_ptr(),
                            self.a.data_ptr(), self.b.data_ptr(), 0, self.max_steps)
        self._h = ham.c_struct()

    def _by_ptr(self, p):
        for v in self.vecs:
            if v.data_ptr() == p:
                return v
        raise RuntimeError("unknown vector pointer")

    @property
    def f_cur(self) -> torch.Tensor:
        return self._by_ptr(self.st.f_cur)

    @property
    def f_prev(self) -> torch.Tensor:
        return self._by_ptr(self.st.f_prev)

    @property
    def f_next(self) -> torch.Tensor:
        return self._by_ptr(self.st.f_next)

    def init(self, f1, stream=None):
        f1 = self.ham._vec(f1)
        if f1.data_ptr() == self.st.f_cur:
            raise ValueError("f1 must not be the run's current vector")
        check(lib().ed_lanczos_init(byref(self._h), byref(self.st), _dptr(f1), _dptr(self.ws), _stream(stream)))

    def step(self, stream=None):
        check(lib().ed_lanczos_step(byref(self._h), byref(self.st), _dptr(self.ws), _stream(stream)))

    def step_timed(self, stream=None):
        """One step; returns the five kernel durations in ms (up, down, reduce, update, norm)."""
        ms = np.zeros(5)
        check(lib().ed_lanczos_step_timed(byref(self._h), byref(self.st), _dptr(self.ws), _stream(stream),
                                          _ptr(ms, c_double)))
        return ms

    def read(self, stream=None):
        steps, status = c_int32(0), c_int32(0)
        a = np.zeros(self.max_steps)
        b = np.zeros(self.max_steps + 1)
        check(lib().ed_lanczos_read(byref(self._h), byref(self.st), _dptr(self.ws), _stream(stream), byref(steps), byref(status),
                                    _ptr(a, c_double), _ptr(b, c_double)))
        k = steps.value
        return {"steps": k, "status": status.value, "a": a[:k], "b": b[:k + 1]}

    def ground_energy(self, f1, tol=0.0, check_every=10, stream=None):
        f1 = self.ham._vec(f1)
        e0, steps = c_double(0), c_int32(0)
        a = np.zeros(self.max_steps)
        b = np.zeros(self.max_steps + 1)
        if f1.data_ptr() == self.st.f_cur:
            raise ValueError("f1 must not be the run's current vector")
        rc = check(lib().ed_ground_energy(byref(self._h), byref(self.st), _dptr(f1), float(tol), int(check_every),
                                          _dptr(self.ws), _stream(stream), byref(e0), byref(steps),
                                          _ptr(a, c_double), _ptr(b, c_double)))
        k = steps.value
        return {"e0": e0.value, "steps": k, "status": rc, "a": a[:k], "b": b[:k + 1]}

    def ground_energy_noalloc(self, f1, tol=0.0, check_every=10, stream=None):
        """ed_ground_energy_noalloc: the run of ground_energy on the library's device scratch, no workspace."""
        f1 = self.ham._vec(f1)
        e0, steps = c_double(0), c_int32(0)
        a = np.zeros(self.max_steps)
        b = np.zeros(self.max_steps + 1)
        if f1.data_ptr() == self.st.f_cur:
            raise ValueError("f1 must not be the run's current vector")
        rc = check(lib().ed_ground_energy_noalloc(byref(self._h), byref(self.st), _dptr(f1), float(tol),
                                                  int(check_every), _stream(stream), byref(e0), byref(steps),
                                                  _ptr(a, c_double), _ptr(b, c_double)))
        k = steps.value
        return {"e0": e0.value, "steps": k, "status": rc, "a": a[:k], "b": b[:k + 1]}

    def ground_state(self, f1, m, gauge_index=-1, stream=None, tol=0.0, extra=0):
        f1 = self.ham._vec(f1)
        v = self.ham.empty_vec()
        e0, steps = c_double(0), c_int32(0)
        if f1.data_ptr() == self.st.f_cur:
            raise ValueError("f1 must not be the run's current vector")
        check(lib().ed_ground_state(byref(self._h), byref(self.st), _dptr(f1), int(m), float(tol), int(extra),
                                    int(gauge_index), _dptr(v), _dptr(self.ws), _stream(stream), byref(e0),
                                    byref(steps)))
        return e0.value, steps.value, v


# Instances of at least this many states in a batch run one by one through the one-instance path (a step of
# theirs fills the GPU, and their tuned kernels beat the persistent launch's shared tiles); 0 puts every
# instance in the persistent launch.
BATCH_SOLO_DIM = 1 << 22


def ground_energy_batch(hams, f1s, max_steps: int, tol: float = 1e-6, use_graph: bool = True, stream=None,
                        solo_dim: int = BATCH_SOLO_DIM):
    """ed_ground_energy_batch over a list of float32 Hamiltonians and start vectors.

    Returns dict(e0, steps, status, e0_device, graph_used, wall_ms)."""
    n = len(hams)
    keep = []
    items = (EdBatchItem * n)()
    for i, (h, f) in enumerate(zip(hams, f1s)):
        if h.dtype != ED_F32:
            raise ValueError("batched runs use float32 vectors (ED_F32)")
        f = h._vec(f)
        vecs = [h.empty_vec() for _ in range(3)]
        a = torch.zeros(max_steps, dtype=torch.float64, device=h.device)
        b = torch.zeros(max_steps + 1, dtype=torch.float64, device=h.device)
        keep += [f, a, b] + vecs
        items[i].h = h.c_struct()
        items[i].f1 = f.data_ptr()
        for k in range(3):
            items[i].vec[k] = vecs[k].data_ptr()
        items[i].a = a.data_ptr()
        items[i].b = b.data_ptr()
    nb = c_int64(0)
    check(lib().ed_batch_workspace_size(items, n, int(max_steps), int(solo_dim), byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=hams[0].device)
    e0 = np.zeros(n)
    e0d = np.zeros(n)
    steps = np.zeros(n, dtype=np.int32)
    status = np.zeros(n, dtype=np.int32)
    used = c_int32(0)
    phase = np.zeros(6)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    rc = check(lib().ed_ground_energy_batch(items, n, int(max_steps), float(tol), int(solo_dim), _dptr(ws), nb.value,
                                            _stream(stream), 1 if use_graph else 0, _ptr(e0, c_double),
                                            _ptr(steps, c_int32), _ptr(status, c_int32), _ptr(e0d, c_double),
                                            byref(used), _ptr(phase, c_double)))
    end.record()
    torch.cuda.synchronize()
    names = ("start", "up", "down", "a_j", "update", "b_j")
    return {"e0": e0, "steps": steps, "status": status, "e0_device": e0d, "graph_used": bool(used.value),
            "rc": rc, "wall_ms": start.elapsed_time(end), "phase_ms": dict(zip(names, phase.tolist()))}
