"""ctypes declarations of libmembed.so (include/membed.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MEMBED_LIBRARY names another build of the library (the tuner's variants);
# by default the in-tree build is loaded
LIB_PATH = os.environ.get("MEMBED_LIBRARY") or os.path.join(_HERE, "libmembed.so")

c_int, c_int64, c_double, c_void_p, c_size_t, c_uint64 = (
    ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t,
    ctypes.c_uint64)

ME_OK = 0
ME_WARN_NOT_CONVERGED = 1
ME_WARN_EPS_ZERO = 2
ME_FP64, ME_MIXED = 0, 1
ME_PRECOND_NONE, ME_PRECOND_JACOBI, ME_PRECOND_CHEBYSHEV = 0, 1, 2
ME_CHEB_LAPLACIAN, ME_CHEB_FULL = 0, 1
ME_ADDR_AUTO, ME_ADDR_GLOBAL = 0, 1
ME_ITER_FP32, ME_ITER_FP16 = 0, 1
ME_LAUNCH_AUTO, ME_LAUNCH_STREAM, ME_LAUNCH_GRAPH = 0, 1, 2
ME_PRODUCT_FP64, ME_PRODUCT_FP32 = 0, 1

STATUS_NAMES = {
    0: "ME_OK", 1: "ME_WARN_NOT_CONVERGED", 2: "ME_WARN_EPS_ZERO", -1: "ME_ERR_INVALID_ARG",
    -2: "ME_ERR_NOT_SYMMETRIC", -3: "ME_ERR_SELF_LOOP", -4: "ME_ERR_BAD_WEIGHT",
    -5: "ME_ERR_ISOLATED_NODE", -6: "ME_ERR_K_RANGE", -7: "ME_ERR_WORKSPACE", -8: "ME_ERR_HIP",
    -9: "ME_ERR_BREAKDOWN", -10: "ME_ERR_TOO_LARGE",
}


class MeCsr(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("rowptr", c_void_p), ("col", c_void_p),
                ("val", c_void_p)]


class MeOpts(ctypes.Structure):
    _fields_ = [("precision", c_int), ("precond", c_int), ("max_iter", c_int),
                ("eps_max_iter", c_int), ("eps_tol", c_double), ("check_every", c_int),
                ("seed", c_uint64), ("cheb_degree", c_int), ("cheb_op", c_int),
                ("addressing", c_int), ("cheb_iterates", c_int), ("launch", c_int),
                ("cholqr_passes", c_int), ("product", c_int)]


class MeInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("eps_iterations", c_int),
                ("block", c_int), ("eps", c_double), ("mu", c_double),
                ("max_residual", c_double), ("orth_error", c_double),
                ("ms_build", c_double), ("ms_solve", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MeServerOpts(ctypes.Structure):
    _fields_ = [("mem_budget", c_size_t), ("max_active", c_int), ("opts", MeOpts),
                ("workspace", c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "me_opts_default": (None, [ctypes.POINTER(MeOpts)]),
    "me_status_string": (ctypes.c_char_p, [c_int]),
    "me_build_workspace_bytes": (c_int, [ctypes.POINTER(MeCsr), ctypes.POINTER(MeOpts),
                                         c_void_p, ctypes.POINTER(c_size_t)]),
    "me_build_graph_ops": (c_int, [ctypes.POINTER(MeCsr), ctypes.POINTER(MeOpts), c_void_p,
                                   c_size_t, c_void_p, ctypes.POINTER(c_void_p),
                                   ctypes.POINTER(MeInfo)]),
    "me_graph_ops_query": (c_int, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64),
                                   ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                   ctypes.POINTER(c_int)]),
    "me_graph_ops_bytes": (c_size_t, [c_void_p]),
    "me_graph_ops_export": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
    "me_graph_ops_order": (c_int, [c_void_p, c_void_p, c_void_p]),
    "me_apply": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "me_embed_workspace_bytes": (c_size_t, [c_void_p, c_int, ctypes.POINTER(MeOpts)]),
    "me_embed": (c_int, [c_void_p, c_int, c_double, ctypes.POINTER(MeOpts), c_void_p, c_void_p,
                         c_size_t, c_void_p, c_void_p, ctypes.POINTER(MeInfo), c_void_p]),
    "me_embed_batch_workspace_bytes": (c_int, [c_int, ctypes.POINTER(MeCsr),
                                               ctypes.POINTER(c_int), ctypes.POINTER(MeOpts),
                                               c_void_p, ctypes.POINTER(c_size_t)]),
    "me_embed_batch": (c_int, [c_int, ctypes.POINTER(MeCsr), ctypes.POINTER(c_int), c_double,
                               ctypes.POINTER(MeOpts), c_void_p, c_size_t,
                               ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                               ctypes.POINTER(MeInfo), c_void_p]),
    "me_knn_workspace_bytes": (c_size_t, [c_int64, c_int, c_int]),
    "me_knn_graph": (c_int, [c_void_p, c_int64, c_int, c_int, c_void_p, c_size_t, c_void_p,
                             c_void_p, c_void_p, ctypes.POINTER(c_int64),
                             ctypes.POINTER(c_double), c_void_p]),
    "me_cluster_workspace_bytes": (c_size_t, [c_int64, c_int, c_int]),
    "me_kmeans": (c_int, [c_void_p, c_int64, c_int, c_int, ctypes.POINTER(c_double), c_int,
                          c_void_p, c_size_t, c_void_p, c_void_p, ctypes.POINTER(c_int),
                          c_void_p]),
    "me_gmm": (c_int, [c_void_p, c_int64, c_int, c_int, c_void_p, c_int, c_double, c_void_p,
                       c_size_t, c_void_p, c_void_p, c_void_p, c_void_p,
                       ctypes.POINTER(c_double), ctypes.POINTER(c_int), c_void_p]),
    "me_cluster_scores": (c_int, [c_void_p, c_void_p, c_int64, c_int, c_int, c_void_p, c_size_t,
                                  ctypes.POINTER(c_double), c_void_p]),
    "me_betweenness_workspace_bytes": (c_size_t, [c_int64]),
    "me_betweenness": (c_int, [ctypes.POINTER(MeCsr), c_void_p, c_size_t, c_void_p,
                               ctypes.POINTER(c_double), c_void_p]),
    "me_embed_noalloc_max_bytes": (c_size_t, []),
    "me_embed_noalloc": (c_int, [c_void_p, c_int, c_double, ctypes.POINTER(MeOpts), c_void_p,
                                 c_void_p, c_void_p, ctypes.POINTER(MeInfo), c_void_p]),
    "me_graph_ops_destroy": (None, [c_void_p]),
    "me_server_opts_default": (None, [ctypes.POINTER(MeServerOpts)]),
    "me_server_create": (c_int, [ctypes.POINTER(MeServerOpts), c_void_p,
                                 ctypes.POINTER(c_void_p)]),
    "me_server_request_bytes": (c_int, [ctypes.POINTER(MeCsr), c_int, c_void_p,
                                        ctypes.POINTER(c_size_t)]),
    "me_server_submit": (c_int, [c_void_p, ctypes.POINTER(MeCsr), c_int, c_double, c_void_p,
                                 c_void_p, ctypes.POINTER(c_int64)]),
    "me_server_step": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "me_server_poll": (c_int, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(MeInfo), c_int,
                               ctypes.POINTER(c_int)]),
    "me_server_destroy": (None, [c_void_p]),
    "me_kernel_timing": (c_int, [c_int]),
    "me_kernel_timing_read": (c_int, [ctypes.POINTER(c_int64), ctypes.POINTER(c_double),
                                      ctypes.POINTER(c_double)]),
    "me_step_form": (c_int, [c_int, c_int, c_int64]),
    "me_step_form_reset": (None, []),
}

KT_OFF, KT_SPMM_A, KT_GRAM_RR, KT_COMBINE, KT_CHEB = 0, 1, 2, 3, 4

_lib = None


def load():
    """Loads the built library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} not found: build it with `python -m paper_2112_07862_amd.build` "
            "(the HIP library is required; there is no CPU path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
