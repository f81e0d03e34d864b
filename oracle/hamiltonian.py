"""The two-species Hamiltonian and its action on a vector (Eq. 1, 3, 4, 5).

H = H_up x I_dn + I_up x H_dn + U * sum_i n_i,up n_i,dn  (Eq. 3; the on-site
term is diagonal in the occupation basis, Sec. 1).  No chemical potential and
no U/2 shift (reading).  With X the D_up-by-D_dn view of a vector (row i_up,
column i_dn):

    H x  <->  H_up X  +  X H_dn^T  +  U * Docc o X              (Eq. 4 and 5)

where Docc[r, c] = number of doubly occupied sites = popcount(s_up[r] & s_dn[c]).
``full_sparse`` assembles the plain Kronecker-product definition instead.
"""

import numpy as np
import scipy.sparse as sp

from .basis import basis_states
from .hopping import hopping_matrix, hopping_matrix_complex


# number of set bits of every 16-bit value, counted one by one
_POP16 = np.array([bin(i).count("1") for i in range(1 << 16)], dtype=np.int64)


def popcount_u64(a: np.ndarray) -> np.ndarray:
    """Set bits of each 64-bit word: the sum over its four 16-bit quarters."""
    a = np.asarray(a, dtype=np.uint64)
    out = np.zeros(a.shape, dtype=np.int64)
    for k in range(4):
        out += _POP16[((a >> np.uint64(16 * k)) & np.uint64(0xFFFF)).astype(np.int64)]
    return out


def double_occupancy(states_up: np.ndarray, states_dn: np.ndarray) -> np.ndarray:
    """Docc[r, c] = popcount(s_up[r] & s_dn[c]), shape (D_up, D_dn)."""
    return popcount_u64(states_up[:, None] & states_dn[None, :]).astype(np.float64)


class Model:
    """Everything the oracle needs for one (lattice, N_up, N_dn, t, U) instance."""

    def __init__(self, n_sites, bonds, n_up, n_dn, t=1.0, U=0.0, amps=None):
        """amps: optional complex amplitude a_ij per bond (term t * (a_ij c+_i c_j + h.c.) for both
        species); without it every bond carries -t (Eq. 1)."""
        self.n_sites, self.bonds = n_sites, list(bonds)
        self.n_up, self.n_dn, self.t, self.U = n_up, n_dn, float(t), float(U)
        self.amps = None if amps is None else [complex(a) for a in amps]
        self.st_up = basis_states(n_sites, n_up)
        self.st_dn = basis_states(n_sites, n_dn)

        def hop_matrix(states):
            if self.amps is None:
                return hopping_matrix(n_sites, self.bonds, states, self.t)
            return self.t * hopping_matrix_complex(n_sites, self.bonds, self.amps, states)

        self.h_up = hop_matrix(self.st_up)
        self.h_dn = self.h_up if (n_dn == n_up) else hop_matrix(self.st_dn)
        self._docc = None

    @property
    def docc(self) -> np.ndarray:
        if self._docc is None:
            self._docc = double_occupancy(self.st_up, self.st_dn)
        return self._docc

    @property
    def dim_up(self):
        return len(self.st_up)

    @property
    def dim_dn(self):
        return len(self.st_dn)

    @property
    def dim(self):
        return self.dim_up * self.dim_dn

    def hv(self, x: np.ndarray) -> np.ndarray:
        """y = H x by Eq. 4 (up part on whole subvectors) and Eq. 5 (down part per subvector)."""
        X = self._view(x).reshape(self.dim_up, self.dim_dn)
        up = self.h_up @ X
        dn = (self.h_dn @ X.T).T
        return (up + dn + self.U * self.docc * X).ravel()

    def _view(self, x):
        x = np.asarray(x)
        return x.astype(np.complex128) if (np.iscomplexobj(x) or self.amps is not None) else x.astype(np.float64)

    def hv_rows(self, x: np.ndarray, rows) -> np.ndarray:
        """(H x)[r, :] for selected up-rows r only, shape (len(rows), D_dn)."""
        X = self._view(x).reshape(self.dim_up, self.dim_dn)
        rows = np.asarray(rows)
        up = self.h_up[rows] @ X
        dn = (self.h_dn @ X[rows].T).T
        docc = double_occupancy(self.st_up[rows], self.st_dn)
        return up + dn + self.U * docc * X[rows]

    def full_sparse(self) -> sp.csr_matrix:
        """The plain definition: kron(H_up, I) + kron(I, H_dn) + diag(U * Docc)."""
        iu = sp.identity(self.dim_up, format="csr")
        idn = sp.identity(self.dim_dn, format="csr")
        h = sp.kron(self.h_up, idn) + sp.kron(iu, self.h_dn)
        return (h + sp.diags(self.U * self.docc.ravel())).tocsr()

    def dense(self) -> np.ndarray:
        return self.full_sparse().toarray()
