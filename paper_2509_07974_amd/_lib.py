"""ctypes view of the C ABI declared in include/fpcf4.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpcf4.so")

OK, E_INVALID_ARG, E_UNSUPPORTED, E_OUT_OF_MEMORY, E_DEVICE, E_BUDGET, E_CANCELLED = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
FP64, MIXED_FP16, MIXED_BF16 = 0, 1, 2
NMAX_SUPPORTED = 16
NMAX3_SUPPORTED = 32
NBINS_SUPPORTED = 128
NOALLOC_SCRATCH_BYTES = 64 << 20

STATUS_NAMES = {
    OK: "OK", E_INVALID_ARG: "E_INVALID_ARG", E_UNSUPPORTED: "E_UNSUPPORTED",
    E_OUT_OF_MEMORY: "E_OUT_OF_MEMORY", E_DEVICE: "E_DEVICE", E_BUDGET: "E_BUDGET",
    E_CANCELLED: "E_CANCELLED",
}


class Catalogue(C.Structure):
    _fields_ = [("n", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p),
                ("g1", C.c_void_p), ("g2", C.c_void_p),
                ("w", C.c_void_p),
                ("mem", C.c_int32)]


class Bins(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("edges", C.c_void_p)]


class Tree(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("reserved", C.c_int32),
                ("delta1", C.c_double), ("rmin", C.c_double)]


class Options(C.Structure):
    _fields_ = [("nmax", C.c_int32), ("precision", C.c_int32),
                ("subtract_degenerate", C.c_int32), ("reserved", C.c_int32),
                ("centers", C.c_void_p), ("ncenters", C.c_int64),
                ("tile_centers", C.c_int64), ("stream", C.c_void_p)]


class Profile(C.Structure):
    _fields_ = [("stage_a_ms", C.c_double), ("relayout_ms", C.c_double),
                ("stage_b_ms", C.c_double), ("corr_ms", C.c_double),
                ("stage_a_launches", C.c_int64), ("stage_b_launches", C.c_int64),
                ("steps", C.c_int64), ("pairs", C.c_int64), ("centres", C.c_int64),
                ("stage_b_mfma_flops", C.c_double), ("stage_b_useful_flops", C.c_double)]


class Fpcf4Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libfpcf4.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run python -m paper_2509_07974_amd.build")
    try:
        # load PyTorch's HIP runtime first so the library binds to the same one
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.estimate_4pcf_multipoles.argtypes = [P(Catalogue), P(Bins), P(Options), C.c_void_p, C.c_int32]
    L.estimate_4pcf_multipoles.restype = C.c_int32
    L.fpcf4_debug_multipoles.argtypes = [P(Catalogue), P(Bins), P(Options), C.c_void_p, C.c_void_p, C.c_void_p]
    L.fpcf4_debug_multipoles.restype = C.c_int32
    L.fpcf4_debug_pair_plan.argtypes = [C.c_int32, C.c_void_p, P(C.c_int64)]
    L.fpcf4_debug_pair_plan.restype = C.c_int32
    L.fpcf4_debug_corr_plan.argtypes = [C.c_int32, C.c_void_p, P(C.c_int64)]
    L.fpcf4_debug_corr_plan.restype = C.c_int32
    L.fpcf4_debug_sort_pairs.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                                         C.c_void_p]
    L.fpcf4_debug_sort_pairs.restype = C.c_int32
    L.fpcf4_to_natural.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.fpcf4_to_natural.restype = C.c_int32
    L.fpcf4_plan.argtypes = [P(Catalogue), P(Bins), P(Options), P(C.c_size_t), P(C.c_int64)]
    L.fpcf4_plan.restype = C.c_int32
    L.fpcf4_request_create.argtypes = [P(Catalogue), P(Bins), P(Options), C.c_void_p, C.c_size_t, P(C.c_void_p)]
    L.fpcf4_request_create.restype = C.c_int32
    L.fpcf4_request_step.argtypes = [C.c_void_p, C.c_int64]
    L.fpcf4_request_step.restype = C.c_int32
    L.fpcf4_request_finalize.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    L.fpcf4_request_finalize.restype = C.c_int32
    L.fpcf4_request_destroy.argtypes = [C.c_void_p]
    L.fpcf4_request_destroy.restype = None
    L.fpcf4_last_error.argtypes = []
    L.fpcf4_last_error.restype = C.c_char_p
    L.fpcf4_version.argtypes = []
    L.fpcf4_version.restype = C.c_char_p
    L.fpcf4_profile_enable.argtypes = [C.c_int32]
    L.fpcf4_profile_enable.restype = C.c_int32
    L.fpcf4_profile_read.argtypes = [P(Profile)]
    L.fpcf4_profile_read.restype = C.c_int32
    L.fpcf4_output_elems.argtypes = [C.c_int32, C.c_int32]
    L.fpcf4_output_elems.restype = C.c_int64
    L.estimate_3pcf_multipoles.argtypes = [P(Catalogue), P(Bins), P(Options), C.c_void_p, C.c_int32]
    L.estimate_3pcf_multipoles.restype = C.c_int32
    L.fpcf4_output3_elems.argtypes = [C.c_int32, C.c_int32]
    L.fpcf4_output3_elems.restype = C.c_int64
    L.fpcf4_to_natural_triplets.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                            C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                                            C.c_void_p]
    L.fpcf4_to_natural_triplets.restype = C.c_int32
    L.estimate_4pcf_multipoles_tree.argtypes = [P(Catalogue), P(Bins), P(Options), P(Tree), C.c_void_p,
                                                C.c_int32]
    L.estimate_4pcf_multipoles_tree.restype = C.c_int32
    L.estimate_4pcf_multipoles_noalloc.argtypes = [P(Catalogue), P(Bins), P(Options), C.c_void_p, C.c_int32]
    L.estimate_4pcf_multipoles_noalloc.restype = C.c_int32
    L.estimate_3pcf_multipoles_doubletree.argtypes = [P(Catalogue), P(Bins), P(Options), P(Tree), P(Tree),
                                                      C.c_void_p, C.c_int32]
    L.estimate_3pcf_multipoles_doubletree.restype = C.c_int32
    _lib = L
    return L


def check(status: int):
    if status != OK:
        raise Fpcf4Error(status, lib().fpcf4_last_error().decode())


EXPORTED = [
    "estimate_4pcf_multipoles", "fpcf4_debug_multipoles", "fpcf4_to_natural", "fpcf4_plan",
    "fpcf4_request_create", "fpcf4_request_step", "fpcf4_request_finalize",
    "fpcf4_request_destroy", "fpcf4_last_error", "fpcf4_version", "fpcf4_output_elems",
    "fpcf4_profile_enable", "fpcf4_profile_read", "estimate_3pcf_multipoles", "fpcf4_output3_elems",
    "fpcf4_to_natural_triplets", "estimate_4pcf_multipoles_tree", "estimate_4pcf_multipoles_noalloc",
    "estimate_3pcf_multipoles_doubletree", "fpcf4_debug_pair_plan", "fpcf4_debug_corr_plan",
    "fpcf4_debug_sort_pairs",
]
