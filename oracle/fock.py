"""Brute force in the full Fock space (tiny lattices only, N_s <= 6).

Independent of ``hopping``: fermion operators are Jordan-Wigner matrices built
from Kronecker products.  Mode m = sigma * N_s + i (all up modes first, then
all down modes); the Fock index has bit m = occupation of mode m, so the
Kronecker factor of the highest mode is leftmost.  c_m carries a Z string on
every mode below m.  The Hamiltonian is Eq. 1 plus the on-site U term, built
operator by operator, then restricted to the (N_up, N_dn) sector and reindexed
to i_up * D_dn + i_dn.
"""

import numpy as np
import scipy.sparse as sp

from .basis import basis_states, index_of

_A = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))   # a|1> = |0>
_Z = sp.csr_matrix(np.diag([1.0, -1.0]))
_I = sp.identity(2, format="csr")


def annihilator(m: int, n_modes: int) -> sp.csr_matrix:
    op = sp.identity(1, format="csr")
    for k in reversed(range(n_modes)):       # leftmost factor = highest mode
        f = _A if k == m else (_Z if k < m else _I)
        op = sp.kron(op, f, format="csr")
    return op


def fock_hamiltonian(n_sites: int, bonds, t: float, U: float, amps=None) -> sp.csr_matrix:
    """amps: optional complex amplitude per bond, term t * (a c+_i c_j + conj(a) c+_j c_i); default -1."""
    n_modes = 2 * n_sites
    c = [annihilator(m, n_modes) for m in range(n_modes)]
    cd = [op.T.tocsr() for op in c]
    dim = 2 ** n_modes
    h = sp.csr_matrix((dim, dim), dtype=np.complex128 if amps is not None else np.float64)
    for sigma in range(2):
        for k, (i, j) in enumerate(bonds):
            a, b = sigma * n_sites + i, sigma * n_sites + j
            if amps is None:
                h = h - t * (cd[a] @ c[b] + cd[b] @ c[a])
            else:
                amp = complex(amps[k])
                h = h + t * (amp * (cd[a] @ c[b]) + amp.conjugate() * (cd[b] @ c[a]))
    for i in range(n_sites):
        nu = cd[i] @ c[i]
        nd = cd[n_sites + i] @ c[n_sites + i]
        h = h + U * (nu @ nd)
    return h.tocsr()


def sector_block(n_sites: int, bonds, n_up: int, n_dn: int, t: float, U: float, amps=None) -> np.ndarray:
    """Dense sector Hamiltonian in the ordering index = i_up * D_dn + i_dn."""
    h = fock_hamiltonian(n_sites, bonds, t, U, amps)
    su, sd = basis_states(n_sites, n_up), basis_states(n_sites, n_dn)
    fock_idx = [int(a) | (int(b) << n_sites) for a in su for b in sd]
    return h[fock_idx][:, fock_idx].toarray()


def fock_spectrum_sector(n_sites, bonds, n_up, n_dn, t, U) -> np.ndarray:
    return np.linalg.eigvalsh(sector_block(n_sites, bonds, n_up, n_dn, t, U))
