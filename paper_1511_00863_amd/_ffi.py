"""ctypes view of the C ABI in include/ed.h (argument marshalling only).

Loading fails loudly when the built library is missing: there is no fallback.
"""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_uint16, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libed_mi355x.so")

ED_OK, ED_BREAKDOWN, ED_NOT_CONVERGED = 0, 1, 2
ED_EINVAL, ED_ECAPACITY, ED_EOVERFLOW, ED_EDEVICE = -1, -2, -3, -4
ED_F64, ED_F32 = 0, 1
ED_ROW_MAJOR, ED_COL_MAJOR = 0, 1
ED_MLP_NPARAM = 37377


class EdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ed error %d: %s" % (code, msg))
        self.code = code


class EdHam(ctypes.Structure):
    _fields_ = [("dim_up", c_int64), ("dim_dn", c_int64), ("w_up", c_int32), ("w_dn", c_int32),
                ("tab_up", c_void_p), ("tab_dn", c_void_p), ("st_up", c_void_p), ("st_dn", c_void_p),
                ("t", c_double), ("U", c_double), ("dtype", c_int32), ("tile", c_int32),
                ("eb_up", c_int32), ("eb_dn", c_int32), ("cplx", c_int32), ("order", c_int32),
                ("amp_up", c_void_p), ("amp_dn", c_void_p), ("win_dn", c_void_p), ("win_cols", c_int32),
                ("win_max", c_int32), ("win_tab", c_void_p), ("wch_dn", c_void_p)]


class EdBatchItem(ctypes.Structure):
    _fields_ = [("h", EdHam), ("f1", c_void_p), ("vec", c_void_p * 3), ("a", c_void_p), ("b", c_void_p)]


class EdLanczos(ctypes.Structure):
    _fields_ = [("f_prev", c_void_p), ("f_cur", c_void_p), ("f_next", c_void_p),
                ("a", c_void_p), ("b", c_void_p), ("j", c_int32), ("max_steps", c_int32)]


_PROTOS = {
    "ed_batch_workspace_size": (c_int, [POINTER(EdBatchItem), c_int32, c_int32, c_int64, POINTER(c_int64)]),
    "ed_ground_energy_batch": (c_int, [POINTER(EdBatchItem), c_int32, c_int32, c_double, c_int64, c_void_p, c_int64,
                                       c_void_p, c_int32, POINTER(c_double), POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_double), POINTER(c_int32), POINTER(c_double)]),
    "ed_last_error": (c_char_p, []),
    "ed_version": (c_char_p, []),
    "ed_build_basis": (c_int, [c_int, c_int, POINTER(c_uint64), c_int64, POINTER(c_int64)]),
    "ed_state_rank": (c_int, [c_int, c_int, POINTER(c_uint64), c_int64, POINTER(c_int64)]),
    "ed_build_hopping": (c_int, [c_int, POINTER(c_int32), c_int, POINTER(c_uint64), c_int64, c_int, c_int32,
                                 POINTER(c_int32), POINTER(c_double), POINTER(c_int32), POINTER(c_int32)]),
    "ed_pack_tables": (c_int, [POINTER(c_int32), POINTER(c_double), POINTER(c_int32), c_int64, c_int32, c_int,
                               POINTER(c_uint16)]),
    "ed_pack_tables32": (c_int, [POINTER(c_int32), POINTER(c_double), POINTER(c_int32), c_int64, c_int32, c_int,
                                 POINTER(c_uint32)]),
    "ed_build_hopping_complex": (c_int, [c_int, POINTER(c_int32), c_int, POINTER(c_double), POINTER(c_uint64),
                                         c_int64, c_int, c_int32, POINTER(c_int32), POINTER(c_double),
                                         POINTER(c_int32), POINTER(c_int32)]),
    "ed_pack_tables_complex": (c_int, [POINTER(c_int32), POINTER(c_double), POINTER(c_int32), c_int64, c_int32,
                                       c_int, POINTER(c_uint32), POINTER(c_double), POINTER(c_int32)]),
    "ed_tridiag_lowest": (c_int, [POINTER(c_double), POINTER(c_double), c_int, POINTER(c_double)]),
    "ed_hop_order": (c_int, [POINTER(c_int32), c_int64, POINTER(c_int64)]),
    "ed_wave_chunks": (c_int, [POINTER(c_int32), c_int64, POINTER(c_uint32)]),
    "ed_band_order": (c_int, [POINTER(c_int32), POINTER(c_int32), c_int64, c_int32, c_int, POINTER(c_int64)]),
    "ed_row_windows": (c_int, [POINTER(c_int32), POINTER(c_int32), c_int64, c_int32, c_int, c_int32,
                               POINTER(c_int32), POINTER(c_int32)]),
    "ed_pack_tables_windowed": (c_int, [POINTER(c_int32), POINTER(c_double), POINTER(c_int32), c_int64, c_int32,
                                        c_int, c_int32, POINTER(c_int32), POINTER(c_uint16)]),
    "ed_permute_basis": (c_int, [POINTER(c_uint64), POINTER(c_int32), POINTER(c_double), POINTER(c_int32), c_int64,
                                 c_int32, c_int, c_int32, POINTER(c_int64), POINTER(c_uint64), POINTER(c_int32),
                                 POINTER(c_double), POINTER(c_int32)]),
    "ed_permute_vector": (c_int, [POINTER(EdHam), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ed_occupation_moments_ws": (c_int, [POINTER(EdHam), c_int32, POINTER(c_int64)]),
    "ed_occupation_moments": (c_int, [POINTER(EdHam), c_int32, c_void_p, c_void_p, c_int64, c_void_p,
                                      POINTER(c_double)]),
    "ed_occupation_correlations": (c_int, [POINTER(c_double), c_int32, POINTER(c_double), POINTER(c_double),
                                           POINTER(c_double)]),
    "ed_spin_flip_moments_ws": (c_int, [POINTER(EdHam), c_int32, POINTER(c_int64)]),
    "ed_spin_flip_moments": (c_int, [POINTER(EdHam), c_int32, c_void_p, c_void_p, c_int64, c_void_p,
                                     POINTER(c_double)]),
    "ed_spin_correlations": (c_int, [POINTER(c_double), POINTER(c_double), c_int32, POINTER(c_double)]),
    "ed_bond_moments_ws": (c_int, [POINTER(EdHam), c_int32, c_int32, POINTER(c_int64)]),
    "ed_bond_moments": (c_int, [POINTER(EdHam), c_int32, POINTER(c_int32), c_int32, c_void_p, c_void_p, c_int64,
                                c_void_p, POINTER(c_double)]),
    "ed_tridiag_lowest_vector": (c_int, [POINTER(c_double), POINTER(c_double), c_int, POINTER(c_double),
                                         POINTER(c_double)]),
    "ed_workspace_size": (c_int, [POINTER(EdHam), c_int32, POINTER(c_int64)]),
    "ed_hv": (c_int, [POINTER(EdHam), c_void_p, c_void_p, c_void_p, c_void_p]),
    "ed_tune": (c_int, [POINTER(EdHam), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                        POINTER(c_int32), POINTER(c_double), POINTER(c_double)]),
    "ed_tile_count": (c_int, [POINTER(c_int32), POINTER(c_int32)]),
    "ed_tile_params": (c_int, [c_int32, POINTER(EdHam), POINTER(c_int32)]),
    "ed_lanczos_init": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_void_p, c_void_p]),
    "ed_lanczos_step": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_void_p]),
    "ed_lanczos_step_timed": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_void_p, POINTER(c_double)]),
    "ed_lanczos_read": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_void_p, POINTER(c_int32), POINTER(c_int32),
                                POINTER(c_double), POINTER(c_double)]),
    "ed_ground_energy": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_double, c_int32, c_void_p,
                                 c_void_p, POINTER(c_double), POINTER(c_int32), POINTER(c_double),
                                 POINTER(c_double)]),
    "ed_ground_energy_noalloc": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_double, c_int32,
                                         c_void_p, POINTER(c_double), POINTER(c_int32), POINTER(c_double),
                                         POINTER(c_double)]),
    "ed_ground_state": (c_int, [POINTER(EdHam), POINTER(EdLanczos), c_void_p, c_int32, c_double, c_int32, c_int64,
                                c_void_p, c_void_p, c_void_p, POINTER(c_double), POINTER(c_int32)]),
    "ed_mlp_workspace_size": (c_int, [c_int64, POINTER(c_int64)]),
    "ed_mlp_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "ed_mlp_backward": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ed_mlp_adam": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_float, c_float, c_float, c_float,
                            c_void_p]),
    "ed_mlp_start_vector": (c_int, [c_void_p, POINTER(EdHam), c_void_p, c_void_p]),
    "ed_mlp_row_cdf": (c_int, [c_void_p, POINTER(EdHam), c_void_p, c_void_p]),
    "ed_mlp_sample": (c_int, [c_void_p, POINTER(EdHam), c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
}

_lib = None


def lib():
    """The loaded library (ctypes.CDLL) with prototypes set.  Raises if not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libed_mi355x.so is not built (run __graft_entry__.build()); "
                              "there is no fallback path")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def exported_names():
    return list(_PROTOS)


def last_error() -> str:
    return lib().ed_last_error().decode()


def check(rc: int, allow=(ED_OK,)) -> int:
    """Raise EdError for negative codes; return informational codes unchanged."""
    if rc < 0 or (rc > 0 and rc not in allow and rc not in (ED_BREAKDOWN, ED_NOT_CONVERGED)):
        raise EdError(rc, last_error())
    return rc
