"""ctypes declarations of the C ABI in include/hts.h (argument marshalling only).

The shared library is built in-tree by paper_2508_10307_amd.build; there is
no other implementation to fall back to: if libhts.so is missing, loading it
raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhts.so")

HTS_OK = 0
HTS_ERR_INVALID = 1
HTS_ERR_UNSUPPORTED = 2
HTS_ERR_WORKSPACE = 3
HTS_ERR_HIP = 4
HTS_MATCH_BF16 = 0
HTS_MATCH_FP32 = 1
HTS_FLAG_WEIGHTED = 1
HTS_FLAG_FOURIER_THRESHOLD = 2
HTS_SHORTLIST_BINS = 130

c_i32 = ctypes.c_int32
c_f32 = ctypes.c_float
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t


class HtsParams(ctypes.Structure):
    _fields_ = [("ps", c_i32), ("stride", c_i32), ("window", c_i32), ("K", c_i32),
                ("tau_mult", c_f32), ("gcp_num", c_i32), ("gcp_den", c_i32),
                ("match_mode", c_i32), ("flags", c_i32), ("tune", c_i32)]


class HtsImage(ctypes.Structure):
    _fields_ = [("noisy", c_vp), ("out", c_vp), ("C", c_i32), ("H", c_i32), ("W", c_i32),
                ("sigma", c_f32)]


class HtsState(ctypes.Structure):
    _fields_ = [("idx", c_vp), ("masks", c_vp), ("U", c_vp), ("V", c_vp), ("cnt", c_vp)]


P = ctypes.POINTER(HtsParams)

# name -> (restype, argtypes); every entry point declared in include/hts.h
SIGNATURES = {
    "hts_default_params": (None, [P]),
    "hts_ref_grid": (c_i32, [c_i32, c_i32, P, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "hts_workspace_size": (c_i32, [P, c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "hts_match": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hts_basis": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                          c_sz, c_vp]),
    "hts_filter": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_f32, c_vp, c_vp, c_vp, c_i32, c_i32,
                           c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hts_aggregate": (c_i32, [P, c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp,
                              c_vp, c_vp]),
    "hts_denoise": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_f32, c_vp, c_vp, c_vp, c_vp, c_vp,
                            c_vp, c_vp, c_sz, c_vp]),
    "hts_denoise_batch_staged": (c_i32, [P, ctypes.POINTER(HtsImage), c_i32, c_vp, c_sz, c_vp,
                                         ctypes.POINTER(c_vp), c_i32]),
    "hts_denoise_noalloc": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_f32, c_vp, c_vp]),
    "hts_match_fallback_count": (c_i32, [P, c_i32, c_i32, c_i32, c_vp, c_sz, c_vp, c_vp]),
    "hts_batch_fallback_counts": (c_i32, [P, ctypes.POINTER(HtsImage), c_i32, c_vp, c_sz, c_vp,
                                          c_vp]),
    "hts_batch_workspace_size": (c_i32, [P, ctypes.POINTER(HtsImage), c_i32,
                                         ctypes.POINTER(c_sz)]),
    "hts_batch_shortlist_histogram": (c_i32, [P, ctypes.POINTER(HtsImage), c_i32, c_vp, c_sz,
                                              c_vp, c_vp]),
    "hts_denoise_batch": (c_i32, [P, ctypes.POINTER(HtsImage), c_i32, c_vp, c_sz, c_vp]),
    "hts_denoise_batch_save": (c_i32, [P, ctypes.POINTER(HtsImage), ctypes.POINTER(HtsState),
                                       c_i32, c_vp, c_sz, c_vp]),
    "hts_denoise_batch_backward": (c_i32, [P, ctypes.POINTER(HtsImage),
                                           ctypes.POINTER(HtsState), c_i32, c_vp, c_sz, c_vp]),
    "hts_denoise_grad_tau": (c_i32, [P, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_i32,
                                     c_f32, c_f32, c_vp, c_vp, c_sz, c_vp]),
    "hts_adapt_sigma": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_i32, c_f32, c_f32,
                                c_i32, c_vp, c_vp, c_vp]),
    "hts_denoise_batch_adaptive": (c_i32, [P, ctypes.POINTER(HtsImage), c_i32, c_vp, c_i32,
                                           c_f32, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hts_denoise_backward": (c_i32, [P, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32,
                                     c_i32, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hts_denoise_backward_basis": (c_i32, [P, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                           c_i32, c_i32, c_i32, c_vp, c_vp, c_sz, c_vp]),
    "hts_video_workspace_size": (c_i32, [P, c_i32, c_i32, c_i32, c_i32, c_i32,
                                         ctypes.POINTER(c_sz)]),
    "hts_denoise_video": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_f32, c_vp, c_vp,
                                  c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hts_denoise_video_backward": (c_i32, [P, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp,
                                           c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hts_autotune": (c_i32, [P, c_i32, c_i32, c_i32, ctypes.c_char_p, ctypes.POINTER(c_i32),
                             c_vp, c_sz, c_vp]),
    "hts_status_string": (ctypes.c_char_p, [c_i32]),
    "hts_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libhts.so (built by paper_2508_10307_amd.build) and declare its
    entry points.  Raises if the library is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2508_10307_amd.build); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class HtsError(RuntimeError):
    def __init__(self, name, status):
        msg = load().hts_status_string(status).decode()
        super().__init__(f"{name} failed: {msg} (status {status})")
        self.status = status


def check(name, status):
    if status != HTS_OK:
        raise HtsError(name, status)
