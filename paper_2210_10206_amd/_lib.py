"""ctypes view of the C ABI declared in include/sarabande_hip.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SB_LIB_PATH names another build of the same sources (the host-sanitizer build of
# build.build(sanitize=True)); the in-tree library is the default.
LIB_PATH = os.environ.get("SB_LIB_PATH") or os.path.join(_HERE, "libsarabande_hip.so")

SB_OK, SB_EINVAL, SB_EUNSUPPORTED, SB_EWORKSPACE, SB_EHIP, SB_ENOMEM, SB_ENONFINITE, SB_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
SB_PREC_FP32, SB_PREC_SPLIT_BF16 = 0, 1
SB_IN_F32, SB_IN_F64 = 0, 1
SB_FLAG_KEEP_COEFFS, SB_FLAG_UNFUSED, SB_FLAG_NO_MFMA, SB_FLAG_ODD_PARITY, SB_FLAG_NO_PACK = 1, 2, 4, 8, 16
SB_FLAG_CHECK_FINITE = 32
SB_FLAG_REGEN_KERNELS = 64
SB_FLAG_HALF_KERNELS = 128
SB_FLAG_KEEP_FOR_ADJOINT = 256
SB_WARN_BOX_TRUNCATED = 1

# Every function the header declares, with its ctypes signature.
c_i32, c_i64, c_u32, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_size_t)


class SbProblem(ctypes.Structure):
    _fields_ = [("ndim", c_i32), ("npcf", c_i32), ("nbins", c_i32),
                ("bin_edges", ctypes.POINTER(c_dbl)), ("lmax", c_i32), ("precision", c_i32),
                ("input_dtype", c_i32), ("flags", c_u32)]


class SbLaunchRecord(ctypes.Structure):
    _fields_ = [("stage", c_i32), ("kernel", c_i32), ("fft_n", c_i32), ("fft_sign", c_i32), ("batch", c_i32),
                ("bytes", c_dbl), ("flops", c_dbl), ("ms", c_dbl)]


P = ctypes.POINTER
SIGNATURES = {
    "sb_plan_create": (c_i32, [P(SbProblem), c_i32, P(c_i64), P(c_vp)]),
    "sb_plan_destroy": (None, [c_vp]),
    "sb_plan_workspace": (c_i32, [c_vp, P(c_sz), P(c_sz)]),
    "sb_plan_set_scratch_limit": (c_i32, [c_vp, ctypes.c_uint64]),
    "sb_plan_set_field_batch": (c_i32, [c_vp, c_i32]),
    "sb_plan_get_field_batch": (c_i32, [c_vp, P(c_i32)]),
    "sb_fft_variants": (c_i32, [c_i32]),
    "sb_plan_set_fft_variant": (c_i32, [c_vp, c_i32, c_i32, c_i32]),
    "sb_plan_get_fft_variant": (c_i32, [c_vp, c_i32, c_i32, P(c_i32)]),
    "sb_plan_set_contract_tile": (c_i32, [c_vp, c_i32]),
    "sb_plan_get_contract_tile": (c_i32, [c_vp, P(c_i32), P(c_i32), P(c_i32)]),
    "sb_plan_bind": (c_i32, [c_vp, c_vp, c_sz, c_vp, c_sz]),
    "sb_prepare": (c_i32, [c_vp, c_vp]),
    "sb_zeta_size": (c_i32, [c_vp, P(c_i64)]),
    "sb_zeta_index": (c_i32, [c_vp, P(c_i32), P(c_i32), P(P(c_i32))]),
    "sb_bin_counts": (c_i32, [c_vp, c_i32, P(c_i64)]),
    "sb_plan_warnings": (c_i32, [c_vp, P(c_u32)]),
    "sb_forward": (c_i32, [c_vp, P(c_vp), c_vp, c_vp]),
    "sb_normalize": (c_i32, [c_vp, P(c_vp), c_vp, c_vp, c_vp]),
    "sb_forward_noalloc": (c_i32, [c_vp, P(c_vp), c_vp, c_vp]),
    "sb_backward": (c_i32, [c_vp, P(c_vp), c_vp, P(c_vp), c_vp]),
    "sb_coeffs": (c_i32, [c_vp, c_i32, P(c_vp)]),
    "sb_autotune": (c_i32, [c_vp, c_vp, ctypes.c_char_p]),
    "sb_forward_graph": (c_i32, [c_vp, P(c_vp), c_vp, c_vp]),
    "sb_profile": (c_i32, [c_vp, c_i32]),
    "sb_stage_times": (c_i32, [c_vp, P(c_dbl), P(c_i32), P(c_dbl), P(c_i32)]),
    "sb_profile_read": (c_i32, [c_vp, c_i32, P(c_i32), P(SbLaunchRecord)]),
    "sb_status_str": (ctypes.c_char_p, [c_i32]),
    "sb_last_error": (ctypes.c_char_p, []),
    "sb_version": (c_i32, []),
}

_LIB = None


class SbError(RuntimeError):
    pass


def load():
    """Load the in-tree library; fail loudly when it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise SbError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_10206_amd.build` "
                      "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(status: int, what: str = ""):
    if status != SB_OK:
        lib = load()
        msg = lib.sb_last_error().decode(errors="replace")
        name = lib.sb_status_str(status).decode()
        raise SbError(f"{what}: {name} ({status}): {msg}")
