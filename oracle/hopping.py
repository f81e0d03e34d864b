"""Per-spin hopping matrices H_sigma and their ELL form (Sec. 2.1, Eq. 1, Fig. 2).

H_sigma = -t * sum over bonds (i, j) of (c+_i c_j + c+_j c_i) for one species.

Fermion signs (the paper defers them to its companion paper).  Reading:
operators are ordered by site index within a species, all up operators before
all down operators.  A state is the product of its creation operators in
ascending site order acting on the vacuum, so applying c_k or c+_k picks up
(-1)**(number of occupied sites below k).  The operators are applied here one
at a time to an explicit occupation list, which is a different formulation
from any closed-form "sites between i and j" rule.

ELL (Fig. 2): two dense arrays, data and indices, of width = the largest
number of nonzeros in a row; within a row the entries are in ascending column
order and the padding at the end is 0 in both arrays.  Flattening is
column-major for the GPU and row-major for the CPU in the paper.
"""

import numpy as np
import scipy.sparse as sp

from .basis import index_of, occupations


def annihilate(occ: list, k: int):
    """c_k on an occupation list: (sign, new list) or None if site k is empty."""
    if not occ[k]:
        return None
    sign = -1 if sum(occ[:k]) % 2 else 1
    new = list(occ)
    new[k] = 0
    return sign, new


def create(occ: list, k: int):
    """c+_k on an occupation list: (sign, new list) or None if site k is full."""
    if occ[k]:
        return None
    sign = -1 if sum(occ[:k]) % 2 else 1
    new = list(occ)
    new[k] = 1
    return sign, new


def hop(occ: list, i: int, j: int):
    """c+_i c_j |occ>: apply c_j first, then c+_i.  (sign, new list) or None."""
    r = annihilate(occ, j)
    if r is None:
        return None
    s1, mid = r
    r = create(mid, i)
    if r is None:
        return None
    s2, new = r
    return s1 * s2, new


def mask_of(occ: list) -> int:
    return sum(1 << k for k, n in enumerate(occ) if n)


def hopping_matrix(n_sites: int, bonds, states: np.ndarray, t: float = 1.0) -> sp.csr_matrix:
    """H_sigma in the given basis, element [row, col] = <row| H_sigma |col>."""
    idx = index_of(states)
    rows, cols, vals = [], [], []
    for col, s in enumerate(states):
        occ = occupations(int(s), n_sites)
        for (i, j) in bonds:
            for (a, b) in ((i, j), (j, i)):
                r = hop(occ, a, b)
                if r is None:
                    continue
                sign, new = r
                rows.append(idx[mask_of(new)])
                cols.append(col)
                vals.append(-t * sign)
    d = len(states)
    m = sp.coo_matrix((vals, (rows, cols)), shape=(d, d)).tocsr()
    m.sum_duplicates()
    return m


def to_ell(a):
    """ELL form of a matrix (dense array or scipy sparse), Fig. 2.

    Returns (data, indices, width) with data/indices of shape (rows, width):
    nonzeros in ascending column order, padding 0 at the end of each row.
    """
    a = sp.csr_matrix(a)
    a.sort_indices()
    nnz = np.diff(a.indptr)
    width = int(nnz.max()) if len(nnz) else 0
    data = np.zeros((a.shape[0], width))
    ind = np.zeros((a.shape[0], width), dtype=np.int64)
    for r in range(a.shape[0]):
        lo, hi = a.indptr[r], a.indptr[r + 1]
        order = np.argsort(a.indices[lo:hi], kind="stable")
        data[r, :hi - lo] = a.data[lo:hi][order]
        ind[r, :hi - lo] = a.indices[lo:hi][order]
    return data, ind, width


def ell_flatten(mat: np.ndarray, layout: str) -> np.ndarray:
    """Flatten an ELL array: 'col' = column-major (GPU), 'row' = row-major (CPU)."""
    return mat.flatten(order="F" if layout == "col" else "C")


def hopping_matrix_complex(n_sites: int, bonds, amps, states: np.ndarray) -> sp.csr_matrix:
    """One species' hopping with a complex amplitude per bond: sum over bonds (i, j) of
    a_ij c+_i c_j + conj(a_ij) c+_j c_i (Hermitian by construction).  With every a_ij = -t this is
    ``hopping_matrix``.  Element [row, col] = <row| H_sigma |col>, complex128."""
    idx = index_of(states)
    rows, cols, vals = [], [], []
    for col, s in enumerate(states):
        occ = occupations(int(s), n_sites)
        for (i, j), a in zip(bonds, amps):
            a = complex(a)
            for (p, q, amp) in ((i, j, a), (j, i, a.conjugate())):
                r = hop(occ, p, q)            # c+_p c_q |col>
                if r is None:
                    continue
                sign, new = r
                rows.append(idx[mask_of(new)])
                cols.append(col)
                vals.append(amp * sign)
    d = len(states)
    m = sp.coo_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(d, d)).tocsr()
    m.sum_duplicates()
    return m
