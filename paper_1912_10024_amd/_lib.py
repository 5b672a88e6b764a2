"""ctypes view of libsse.so (declared in include/sse.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsse.so")

SSE_OK, SSE_ERR_NULL, SSE_ERR_DIMS, SSE_ERR_WORKSPACE, SSE_ERR_PRECISION, SSE_ERR_HIP, SSE_ERR_NBR = range(7)
# the sse_precision codes of include/sse.h ("bf16x3" is declared there but not built;
# "fp16" and "fp16_unscaled" are the single-term comparison forms, one table only)
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16x3": 3, "fp16x2": 4, "fp16": 5, "fp16_unscaled": 6}
EXPORTS = ("sse_abi_version", "sse_last_error", "sse_workspace_bytes", "sse_effective_flops",
           "sse_forward", "sse_forward_signed", "sse_forward_ex", "sse_backward", "sse_backward_signed",
           "sse_check_nbr", "sse_combine_d", "sse_absorption_d", "sse_phonon_forward", "sse_backward_noalloc",
           "sse_noalloc_scratch_bytes")


class SSEDims(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in ("nkz", "ne", "nqz", "nw", "na", "nb", "norb", "g_slots")]

    @classmethod
    def of(cls, d):
        return cls(*[int(x) for x in d.as_tuple()])


_lib = None


def load():
    """Load the in-tree libsse.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_10024_amd.build`")
    from . import build as _build

    stamp = LIB_PATH + ".sha256"
    recorded = open(stamp).read().strip() if os.path.exists(stamp) else None
    if recorded != _build.source_hash():
        raise RuntimeError(f"{LIB_PATH} was not built from the current sources (recorded source hash {recorded!r}); "
                           "rebuild it with `python -m paper_1912_10024_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I64, SZ = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_size_t
    DP = ctypes.POINTER(SSEDims)
    lib.sse_abi_version.argtypes, lib.sse_abi_version.restype = [], ctypes.c_int
    lib.sse_last_error.argtypes, lib.sse_last_error.restype = [], ctypes.c_char_p
    lib.sse_workspace_bytes.argtypes = [DP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SZ)]
    lib.sse_effective_flops.argtypes = [DP, ctypes.POINTER(D)]
    lib.sse_forward.argtypes = [DP, P, P, P, P, D, D, ctypes.c_int, P, P, SZ, P]
    lib.sse_forward_signed.argtypes = [DP, P, P, P, P, P, D, D, ctypes.c_int, P, P, SZ, P]
    lib.sse_forward_ex.argtypes = [DP, P, P, P, P, P, P, D, D, ctypes.c_int, P, P, SZ, P]
    lib.sse_backward.argtypes = [DP, P, P, P, P, D, D, P, P, P, P, P, SZ, P]
    lib.sse_backward_signed.argtypes = [DP, P, P, P, P, P, D, D, P, P, P, P, P, P, SZ, P]
    lib.sse_backward_noalloc.argtypes = [DP, P, P, P, P, D, D, P, P, P, P, P]
    lib.sse_noalloc_scratch_bytes.argtypes, lib.sse_noalloc_scratch_bytes.restype = [], SZ
    lib.sse_check_nbr.argtypes = [DP, P, P, SZ, P]
    lib.sse_combine_d.argtypes = [DP, P, P, P, P, SZ, P]
    lib.sse_absorption_d.argtypes = [DP, P, P, P]
    lib.sse_phonon_forward.argtypes = [DP, P, P, P, P, D, D, P, P]
    for f in (lib.sse_workspace_bytes, lib.sse_effective_flops, lib.sse_forward, lib.sse_forward_signed,
              lib.sse_forward_ex, lib.sse_backward, lib.sse_backward_signed, lib.sse_check_nbr, lib.sse_combine_d,
              lib.sse_absorption_d, lib.sse_phonon_forward, lib.sse_backward_noalloc):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().sse_last_error().decode()
