"""ctypes loader for libmbefci.so (built in place by ``build.py``).

The HIP library is the only compute path: if it is missing this module raises,
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbefci.so")

c_int32, c_int64, c_double, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                  ctypes.c_void_p, ctypes.c_size_t)


class Options(ctypes.Structure):
    _fields_ = [("a", c_double), ("max_order", c_int32), ("e_tol", c_double), ("r_tol", c_double),
                ("max_iter", c_int32), ("max_space", c_int32), ("batched", c_int32),
                ("gradient", c_int32), ("profile", c_int32), ("sigma_variant", c_int32),
                ("pspace", c_int32), ("linked_rows", c_int32), ("stream_last", c_int32),
                ("graph", c_int32), ("autotune", c_int32), ("restart_keep", c_int32),
                ("spin_shift", c_double), ("whole_dim", c_int32), ("base_model", c_int32),
                ("sym_shift", c_double), ("irrep", c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("ntuples", c_int64), ("sigma_calls", c_int64), ("sigma_launches", c_int64),
                ("sigma_flops", c_double), ("sigma_bytes", c_double), ("sigma_ms", c_double),
                ("sigma_total_ms", c_double), ("iterations_total", c_int64),
                ("iterations_max", c_int64), ("solve_ms", c_double),
                ("gs_second_pass", c_int64), ("second_pass", c_int64), ("gather_ms", c_double),
                ("graph_batches", c_int64), ("tuned_classes", c_int64),
                ("whole_batches", c_int64)]


class ClassStats(ctypes.Structure):
    _fields_ = [("n_active", c_int32), ("n_alpha", c_int32), ("n_beta", c_int32), ("kernel", c_int32),
                ("dim", c_int64), ("tuples", c_int64), ("iterations", c_int64), ("sigma_calls", c_int64),
                ("sigma_launches", c_int64), ("sigma_flops", c_double), ("sigma_ms", c_double),
                ("gather_ms", c_double), ("sigma_total_ms", c_double), ("wall_ms", c_double)]


ENERGY_FN = ctypes.CFUNCTYPE(c_int32, c_void_p, c_int32, c_int64, ctypes.POINTER(ctypes.c_int16),
                             ctypes.POINTER(c_double))

# (name, restype, argtypes) of every exported symbol declared in include/mbefci.h
SIGNATURES = [
    ("mbefci_version", ctypes.c_char_p, []),
    ("mbefci_default_options", None, [ctypes.POINTER(Options)]),
    ("mbefci_create", c_int32, [ctypes.POINTER(c_void_p), c_int32, c_void_p]),
    ("mbefci_destroy", None, [c_void_p]),
    ("mbefci_last_error", ctypes.c_char_p, [c_void_p]),
    ("mbefci_set_hamiltonian", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_double]),
    ("mbefci_set_spaces", c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int32]),
    ("mbefci_set_options", c_int32, [c_void_p, ctypes.POINTER(Options)]),
    ("mbefci_set_pi_pairs", c_int32, [c_void_p, c_void_p, c_int32]),
    ("mbefci_workspace_query", c_int32, [c_void_p, c_int32, c_int64, c_void_p,
                                         ctypes.POINTER(c_size_t), ctypes.POINTER(c_size_t)]),
    ("mbefci_solve_tuples", c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_size_t,
                                      c_void_p, c_void_p]),
    ("mbefci_solve_tuples_noalloc", c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_void_p]),
    ("mbefci_run", c_int32, [c_void_p, c_void_p, c_size_t, ctypes.POINTER(c_void_p)]),
    ("mbefci_run_host", c_int32, [c_void_p, ENERGY_FN, c_void_p, ctypes.POINTER(c_void_p)]),
    ("mbefci_result_norders", c_int32, [c_void_p]),
    ("mbefci_result_order", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                      ctypes.POINTER(c_void_p), ctypes.POINTER(c_double),
                                      ctypes.POINTER(c_double)]),
    ("mbefci_result_total", c_double, [c_void_p]),
    ("mbefci_order_solve", c_int32, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_size_t]),
    ("mbefci_order_close", c_int32, [c_void_p, c_void_p]),
    ("mbefci_result_free", None, [c_void_p]),
    ("mbefci_tuple_sigma", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p,
                                     c_int32]),
    ("mbefci_tuple_hdiag", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("mbefci_tuple_shape", c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(c_int64),
                                     ctypes.POINTER(c_int64), ctypes.POINTER(c_int32),
                                     ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    ("mbefci_string_tables", c_int32, [c_int32, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_int32),
                                       c_void_p, c_void_p]),
    ("mbefci_get_stats", c_int32, [c_void_p, ctypes.POINTER(Stats)]),
    ("mbefci_get_class_stats", c_int32, [c_void_p, ctypes.POINTER(c_int32), c_void_p]),
    ("mbefci_backward", c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_size_t, c_void_p, c_void_p]),
    ("mbefci_tuple_base", c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("mbefci_result_base", c_double, [c_void_p]),
    ("mbefci_casscf", c_int32, [c_void_p, c_void_p, c_size_t, c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    ("mbefci_set_orbital_irreps", c_int32, [c_void_p, c_void_p]),
    ("mbefci_hf", c_int32, [c_void_p, c_void_p, c_size_t, c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    ("mbefci_get_hamiltonian", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("mbefci_tuple_rdm", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p,
                                   c_void_p]),
]

_lib = None


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmbefci.so not built ({LIB_PATH}); run __graft_entry__.build() or "
                              "python paper_1905_02786_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
