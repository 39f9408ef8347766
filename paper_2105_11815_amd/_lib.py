"""ctypes declarations of the C interface in include/ski.h (libski.so).

Argument marshalling only: every step of the solver runs in the HIP library.
Loading fails loudly when the library has not been built.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libski.so")

SKI_OK, SKI_WNOCONV, SKI_WEARLY = 0, 1, 2
SKI_EINVAL, SKI_ENOMEM, SKI_EDEVICE, SKI_ERANK, SKI_ESTATE = -1, -2, -3, -4, -5
SKI_DENSE, SKI_DENSE_COLMAJOR, SKI_CSR = 0, 1, 2
SKI_FP64, SKI_FP32, SKI_BF16 = 0, 1, 2
SKI_OP_LLS, SKI_OP_NORMAL = 0, 1
SKI_QR_AUTO, SKI_QR_HOUSEHOLDER, SKI_QR_PIVOTED, SKI_QR_PIVOTED_HOUSEHOLDER, SKI_QR_PIVOTED_COD = 0, 1, 2, 3, 4
SKI_QR_SPARSE = 5
SKI_HASH, SKI_HASH_VARIANT, SKI_SAMPLE_ROWS = 0, 1, 2

STATUS_NAMES = {0: "OK", 1: "WNOCONV", 2: "WEARLY", -1: "EINVAL", -2: "ENOMEM",
                -3: "EDEVICE", -4: "ERANK", -5: "ESTATE"}

EXPORTED = ["ski_create", "ski_destroy", "ski_params_default", "ski_sketch", "ski_factor",
            "ski_solve", "ski_gradients", "ski_last_error", "ski_get_dims", "ski_get_hash",
            "ski_get_dsign", "ski_get_SA", "ski_get_R", "ski_set_profiling",
            "ski_set_profiling_mask", "ski_get_profile", "ski_get_pivots",
            "ski_get_factor_stats", "ski_sketch_noalloc"]
PROF_CLASSES = 16
PROF_NAMES = ["lsqr_pass", "pass_reduce", "tri_gemv", "spmv_csr", "spmv_csrT", "lsqr_step",
              "hash", "wht_gather", "gather", "qr", "trtri", "qr_householder", "qr_pivoted",
              "sparse_sketch", "sparse_fronts", "sparse_root"]


class SkiMatrix(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int64), ("kind", C.c_int32),
                ("a", C.c_void_p), ("lda", C.c_int64),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("nnz", C.c_int64)]


class SkiParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("m", C.c_int64), ("s", C.c_int32),
                ("hadamard", C.c_int32), ("seed", C.c_uint64), ("sketch_prec", C.c_int32),
                ("qr_prec", C.c_int32), ("tau_a", C.c_double), ("tau_r", C.c_double),
                ("it_max", C.c_int64), ("rcond", C.c_double), ("rcond_thres", C.c_double),
                ("perturb", C.c_double), ("qr_panel", C.c_int32), ("hash_kind", C.c_int32)]


class SkiInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("status", C.c_int32), ("early_exit", C.c_int32),
                ("rnorm", C.c_double), ("arnorm", C.c_double), ("wnorm_est", C.c_double),
                ("tc", C.c_double), ("cond_est", C.c_double), ("ms_sketch", C.c_float),
                ("ms_factor", C.c_float), ("ms_solve", C.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libski.so (built by paper_2105_11815_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build the HIP library first "
                           "(python -m paper_2105_11815_amd.build)")
    lib = C.CDLL(LIB_PATH)
    H = C.c_void_p
    P = C.c_void_p
    i64, i32 = C.c_int64, C.c_int32
    lib.ski_create.argtypes = [C.POINTER(H)]
    lib.ski_destroy.argtypes = [H]
    lib.ski_params_default.argtypes = [i32, C.POINTER(SkiParams)]
    lib.ski_params_default.restype = None
    lib.ski_sketch.argtypes = [H, C.POINTER(SkiMatrix), P, i32, i64, C.POINTER(SkiParams), P]
    lib.ski_factor.argtypes = [H, P]
    lib.ski_solve.argtypes = [H, i32, P, i32, i64, P, i64, C.POINTER(SkiInfo), P]
    lib.ski_gradients.argtypes = [H, P, i64, P, i64, P, i64, i32, P, i64, P, i64, P]
    lib.ski_last_error.argtypes = [H]
    lib.ski_last_error.restype = C.c_char_p
    lib.ski_get_dims.argtypes = [H, P]
    lib.ski_get_hash.argtypes = [H, P, P, P, P, P]
    lib.ski_get_dsign.argtypes = [H, P]
    lib.ski_get_SA.argtypes = [H, P]
    lib.ski_get_R.argtypes = [H, P, P, P]
    lib.ski_set_profiling.argtypes = [H, i32]
    lib.ski_set_profiling_mask.argtypes = [H, C.c_uint32]
    lib.ski_get_profile.argtypes = [H, P, P]
    lib.ski_get_pivots.argtypes = [H, P, P]
    lib.ski_get_factor_stats.argtypes = [H, P]
    lib.ski_sketch_noalloc.argtypes = [C.POINTER(SkiMatrix), P, i32, i64, C.POINTER(SkiParams),
                                       P, P]
    for name in EXPORTED:
        if name not in ("ski_params_default", "ski_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
