"""MI355X (gfx950) exact diagonalisation of two-species lattice models.

The Lanczos ground-state method of Siro and Harju (Alg. 1) with a matrix-free
H.v over the fixed-(N_up, N_dn) occupation basis (Eq. 3-5), as a C-ABI library
of hand-written HIP kernels (include/ed.h).  This package is its thin Python
binding; torch supplies device memory and streams.
"""

from ._ffi import (ED_BREAKDOWN, ED_COL_MAJOR, ED_F32, ED_F64, ED_NOT_CONVERGED, ED_OK, ED_ROW_MAJOR, EdError,
                   lib)
from .api import (Hamiltonian, LanczosRun, SpinTables, band_order, build_basis, build_hopping, ground_energy_batch,
                  hop_order, occupation_correlations, pack_tables, permute_basis, row_windows, spin_correlations,
                  state_rank, tridiag_lowest, tridiag_lowest_vector, wave_chunks)

__all__ = ["Hamiltonian", "LanczosRun", "SpinTables", "build_basis", "build_hopping", "ground_energy_batch",
           "hop_order", "band_order", "row_windows", "wave_chunks", "pack_tables", "permute_basis",
           "occupation_correlations", "spin_correlations",
           "state_rank", "tridiag_lowest", "tridiag_lowest_vector", "EdError", "lib",
           "ED_OK", "ED_BREAKDOWN", "ED_NOT_CONVERGED", "ED_F64", "ED_F32", "ED_ROW_MAJOR", "ED_COL_MAJOR"]
