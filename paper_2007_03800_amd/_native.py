"""ctypes view of include/sdl.h (argument marshalling only; all work runs in libsdl.so)."""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsdl.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "sdl.h")

SDL_FP64, SDL_FP32, SDL_BF16, SDL_MIXED_BF16 = 0, 1, 2, 3
STATUS = {0: "SDL_OK", -1: "SDL_E_INVAL", -2: "SDL_E_SHAPE", -3: "SDL_E_DEVICE", -4: "SDL_E_NOMEM",
          -5: "SDL_E_SINGULAR", -6: "SDL_E_NONFINITE", -7: "SDL_E_UNSUPPORTED"}
KERNEL_CLASSES = ["sparse_code", "tmod_sums", "reduce", "solve", "prep", "rmse", "rescale", "spare"]


class Problem(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_int32), ("m2", ctypes.c_int32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("s", ctypes.c_int32), ("reserved", ctypes.c_int32), ("N", ctypes.c_int64),
                ("Y", ctypes.c_void_p), ("D1", ctypes.c_void_p), ("D2", ctypes.c_void_p),
                ("supp", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("res2", ctypes.c_void_p)]


TENSOR_MAX_MODES = 4


class TensorProblem(ctypes.Structure):
    _fields_ = [("nmodes", ctypes.c_int32), ("s", ctypes.c_int32), ("m", ctypes.c_int32 * TENSOR_MAX_MODES),
                ("n", ctypes.c_int32 * TENSOR_MAX_MODES), ("N", ctypes.c_int64), ("Y", ctypes.c_void_p),
                ("D", ctypes.c_void_p * TENSOR_MAX_MODES), ("supp", ctypes.c_void_p), ("coef", ctypes.c_void_p),
                ("res2", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("early_stops", ctypes.c_int64), ("fp64_pivots", ctypes.c_int64), ("unused_atoms", ctypes.c_int64),
                ("singular_updates", ctypes.c_int64), ("kernel_ms", ctypes.c_double * 8),
                ("kernel_launches", ctypes.c_int64 * 8), ("proposals_accepted", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("near_tie_rescores", ctypes.c_int64),
                ("near_tie_overflows", ctypes.c_int64)]

    def as_dict(self):
        return dict(early_stops=self.early_stops, fp64_pivots=self.fp64_pivots, unused_atoms=self.unused_atoms,
                    singular_updates=self.singular_updates, proposals_accepted=self.proposals_accepted,
                    fallbacks=self.fallbacks, near_tie_rescores=self.near_tie_rescores,
                    near_tie_overflows=self.near_tie_overflows,
                    kernel_ms={KERNEL_CLASSES[i]: self.kernel_ms[i] for i in range(8) if self.kernel_launches[i]},
                    kernel_launches={KERNEL_CLASSES[i]: self.kernel_launches[i] for i in range(8)
                                     if self.kernel_launches[i]})


class Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("schedule", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("timing", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("stop_rel", ctypes.c_double), ("dep_eps", ctypes.c_double), ("pivot_fp64", ctypes.c_double),
                ("stats", ctypes.POINTER(Stats)), ("proposer", ctypes.c_void_p), ("tau", ctypes.c_double),
                ("err2", ctypes.c_double), ("tie_band", ctypes.c_double), ("fallback_margin", ctypes.c_double),
                ("deterministic", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("method", ctypes.c_int32), ("reserved1", ctypes.c_int32)]


class SdlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


_lib = None


def lib():
    """Load libsdl.so; raises if the HIP library has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsdl.so is not built; run `python -m paper_2007_03800_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Problem)
        L.sdl_default_options.argtypes = [ctypes.POINTER(Options)]
        L.sdl_default_options.restype = None
        L.sdl_sparse_code.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p]
        L.sdl_tmod_update.argtypes = [P, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(Options), ctypes.c_void_p]
        L.sdl_learn.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(Options),
                                ctypes.c_void_p]
        for f in (L.sdl_sparse_code, L.sdl_tmod_update, L.sdl_learn):
            f.restype = ctypes.c_int
        L.sdl_autotune.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p]
        L.sdl_autotune.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int32)
        L.sdl_tuned_config.argtypes = [ctypes.c_int32] * 5 + [ip, ip, ip, ip, ctypes.POINTER(ctypes.c_double)]
        L.sdl_tuned_config.restype = ctypes.c_int
        L.sdl_kernel_variants.argtypes = [ctypes.c_int32] * 5 + [ip, ctypes.c_int32]
        L.sdl_kernel_variants.restype = ctypes.c_int
        L.sdl_set_kernel_variant.argtypes = [ctypes.c_int32] * 9
        L.sdl_set_kernel_variant.restype = ctypes.c_int
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sdl_proposer_create.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.c_uint64, ctypes.POINTER(vp)]
        L.sdl_proposer_destroy.argtypes = [vp]
        L.sdl_proposer_destroy.restype = None
        L.sdl_proposer_num_params.argtypes = [vp]
        L.sdl_proposer_num_params.restype = i64
        L.sdl_proposer_get_params.argtypes = [vp, vp]
        L.sdl_proposer_set_params.argtypes = [vp, vp]
        L.sdl_proposer_gradient.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp]
        L.sdl_proposer_train.argtypes = [vp, vp, vp, i32, i64, i32, i32, ctypes.c_float, ctypes.c_uint64, vp, vp]
        L.sdl_proposer_logits.argtypes = [vp, vp, i64, vp, vp]
        L.sdl_learned_sparse_code.argtypes = [vp, P, i32, vp, ctypes.POINTER(Options), vp]
        L.sdl_proposer_calibrate.argtypes = [vp, P, ctypes.c_double, ctypes.POINTER(Options),
                                             ctypes.POINTER(ctypes.c_double), vp]
        L.sdl_proposer_save.argtypes = [vp, ctypes.c_char_p]
        L.sdl_proposer_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        L.sdl_sparse_code_sums.argtypes = [P, i32, vp, ctypes.POINTER(Options), vp]
        L.sdl_workspace_bytes.argtypes = [P, i32, i32, i32, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]
        L.sdl_mixed_supported.argtypes = [i32] * 5
        TP = ctypes.POINTER(TensorProblem)
        L.sdl_tensor_sparse_code.argtypes = [TP, ctypes.POINTER(Options), ctypes.c_void_p]
        L.sdl_tensor_update.argtypes = [TP, ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p]
        L.sdl_tensor_learn.argtypes = [TP, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(Options), ctypes.c_void_p]
        for f in (L.sdl_tensor_sparse_code, L.sdl_tensor_update, L.sdl_tensor_learn):
            f.restype = ctypes.c_int
        L.sdl_image_to_patches.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
        L.sdl_image_to_patches.restype = ctypes.c_int
        L.sdl_patches_to_image.argtypes = [P, i32, i32, ctypes.POINTER(Options), vp, vp]
        L.sdl_patches_to_image.restype = ctypes.c_int
        L.sdl_sparse_code_noalloc.argtypes = [P, i32, ctypes.POINTER(Options), vp]
        L.sdl_sparse_code_noalloc.restype = ctypes.c_int
        for f in (L.sdl_proposer_save, L.sdl_proposer_load, L.sdl_sparse_code_sums, L.sdl_workspace_bytes,
                  L.sdl_mixed_supported):
            f.restype = ctypes.c_int
        L.sdl_probe_hbm_copy.argtypes = [vp, vp, ctypes.c_size_t, i32, ctypes.POINTER(ctypes.c_double), vp]
        L.sdl_probe_hbm_copy.restype = ctypes.c_int
        L.sdl_probe_peak.argtypes = [i32, vp, i32, ctypes.POINTER(ctypes.c_double), vp]
        L.sdl_probe_peak.restype = ctypes.c_int
        for f in (L.sdl_proposer_create, L.sdl_proposer_get_params, L.sdl_proposer_set_params,
                  L.sdl_proposer_gradient, L.sdl_proposer_train, L.sdl_proposer_logits, L.sdl_learned_sparse_code,
                  L.sdl_proposer_calibrate):
            f.restype = ctypes.c_int
        L.sdl_last_error.restype = ctypes.c_char_p
        L.sdl_last_error.argtypes = []
        L.sdl_abi_version.restype = ctypes.c_int
        _lib = L
    return _lib


def check(status):
    if status != 0:
        raise SdlError(status, lib().sdl_last_error().decode())


def default_options() -> Options:
    o = Options()
    lib().sdl_default_options(ctypes.byref(o))
    return o


def header_functions():
    """Names of the functions include/sdl.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sdl_[a-z0-9_]+)\s*\(", txt)))
