"""The C-ABI library loads, exports every declared symbol and rejects bad
calls before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1912_10024_amd import _lib, flops
from paper_1912_10024_amd.inputs import CONFIGS, Dims

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(sse_\w+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert {"sse_forward", "sse_forward_signed", "sse_backward", "sse_workspace_bytes", "sse_check_nbr",
            "sse_effective_flops", "sse_last_error", "sse_abi_version"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTS) <= declared


def test_abi_version(lib):
    txt = open(os.path.join(ROOT, "include", "sse.h")).read()
    v = int(re.search(r"#define SSE_ABI_VERSION (\d+)", txt).group(1))
    assert lib.sse_abi_version() == v


def _call_forward(lib, d, ptrs=(1, 1, 1, 1), out=1, precision=0, ws=None, wsb=0):
    cd = _lib.SSEDims(*d) if isinstance(d, tuple) else _lib.SSEDims.of(d)
    P = ctypes.c_void_p
    G, D, dH, nbr = (P(x) if x else None for x in ptrs)
    return lib.sse_forward(ctypes.byref(cd), G, D, dH, nbr, 0.0, 1.0, precision, P(out) if out else None,
                           P(ws) if ws else None, wsb, None)


@pytest.mark.parametrize("bad", [
    (0, 4, 0, 2, 3, 2, 2, 1), (3, -1, 3, 2, 3, 2, 2, 1), (3, 4, 2, 2, 3, 2, 2, 1),  # nqz != nkz
    (3, 4, 3, 2, 3, 2, 2, 0), (3, 4, 3, 2, 3, 2, 33, 1), (1 << 40, 1 << 40, 1 << 40, 2, 3, 2, 2, 1)])
def test_bad_dims_rejected_before_launch(lib, bad):
    assert _call_forward(lib, bad) == _lib.SSE_ERR_DIMS
    assert lib.sse_last_error()


def test_null_pointers_rejected(lib):
    d = CONFIGS["tiny"]
    for i in range(4):
        ptrs = [1, 1, 1, 1]
        ptrs[i] = 0
        assert _call_forward(lib, d, ptrs=tuple(ptrs)) == _lib.SSE_ERR_NULL
    assert _call_forward(lib, d, out=0) == _lib.SSE_ERR_NULL
    assert lib.sse_forward(None, None, None, None, None, 0.0, 0.0, 0, None, None, 0, None) == _lib.SSE_ERR_NULL


def test_bad_precision_rejected(lib):
    assert _call_forward(lib, CONFIGS["tiny"], precision=7) == _lib.SSE_ERR_PRECISION
    assert "precision" in lib.sse_last_error().decode()


def test_precision_codes_match_the_interface():
    """The header's sse_precision codes are the interface's (FP64 0, FP32 1,
    BF16X2 2, BF16X3 3) plus FP16X2 4 and the single-term comparison forms FP16 5
    and FP16_UNSCALED 6, and the binding uses the same codes."""
    txt = open(os.path.join(ROOT, "include", "sse.h")).read()
    enum = txt[txt.index("enum sse_precision"):txt.index("};", txt.index("enum sse_precision"))]
    enum = re.sub(r"/\*.*?\*/", "", enum, flags=re.S)
    codes = {m.group(1).lower(): int(m.group(2)) for m in re.finditer(r"SSE_(\w+)\s*=\s*(\d+)", enum)}
    assert codes == {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16x3": 3, "fp16x2": 4, "fp16": 5, "fp16_unscaled": 6}
    assert codes == _lib.PRECISIONS


@pytest.mark.parametrize("name", ["fp16", "fp16_unscaled"])
def test_single_term_forms_refuse_two_tables(lib, name):
    """The single-term fp16 forms take one coefficient table: a signed call with
    Dm != Dp is a precision error before any launch (the pointers here are never
    dereferenced), while Dm == Dp passes the precision check and stops at the
    workspace check (no workspace given)."""
    cd = _lib.SSEDims.of(CONFIGS["mid"])
    P = ctypes.c_void_p
    prec = _lib.PRECISIONS[name]
    args = lambda dm: (ctypes.byref(cd), P(8), P(16), P(dm), P(32), P(64), 0.0, 1.0, prec, P(128))
    assert lib.sse_forward_signed(*args(24), None, 0, None) == _lib.SSE_ERR_PRECISION
    assert "one coefficient table" in lib.sse_last_error().decode()
    assert lib.sse_forward_signed(*args(16), None, 0, None) == _lib.SSE_ERR_WORKSPACE


def test_declared_but_unbuilt_precision_is_rejected(lib):
    """SSE_BF16X3 is declared but has no kernel: a precision error before any
    launch (the pointers here are never dereferenced)."""
    assert _call_forward(lib, CONFIGS["tiny"], precision=_lib.PRECISIONS["bf16x3"]) == _lib.SSE_ERR_PRECISION
    assert "not built" in lib.sse_last_error().decode()


def test_workspace_too_small_rejected(lib):
    d = CONFIGS["mid"]
    need = ctypes.c_size_t(0)
    cd = _lib.SSEDims.of(d)
    assert lib.sse_workspace_bytes(ctypes.byref(cd), 0, 0, ctypes.byref(need)) == 0
    if need.value > 0:
        assert _call_forward(lib, d, ws=None, wsb=0) == _lib.SSE_ERR_WORKSPACE


def test_effective_flops_matches_model(lib):
    for d in CONFIGS.values():
        out = ctypes.c_double(0)
        cd = _lib.SSEDims.of(d)
        assert lib.sse_effective_flops(ctypes.byref(cd), ctypes.byref(out)) == 0
        assert out.value == flops.f_eff(d)


def test_backward_and_check_reject_bad_input(lib):
    cd = _lib.SSEDims(3, 4, 2, 2, 3, 2, 2, 1)
    assert lib.sse_backward(ctypes.byref(cd), *([ctypes.c_void_p(1)] * 4), 0.0, 1.0, ctypes.c_void_p(1),
                            None, None, None, None, 0, None) == _lib.SSE_ERR_DIMS
    good = _lib.SSEDims.of(CONFIGS["tiny"])
    assert lib.sse_check_nbr(ctypes.byref(good), None, ctypes.c_void_p(1), 256, None) == _lib.SSE_ERR_NULL
    assert lib.sse_check_nbr(ctypes.byref(good), ctypes.c_void_p(1), None, 0, None) == _lib.SSE_ERR_WORKSPACE


def test_phonon_forward_rejects_bad_input(lib):
    P = ctypes.c_void_p
    bad = _lib.SSEDims(3, 4, 2, 2, 3, 2, 2, 1)  # nqz != nkz
    assert lib.sse_phonon_forward(ctypes.byref(bad), P(1), P(1), P(1), P(1), 0.0, -1.0, P(1), None) == _lib.SSE_ERR_DIMS
    big = _lib.SSEDims(3, 4, 3, 200, 3, 2, 2, 1)  # nqz * nw beyond the vector-ALU kernel, not the matrix-core shape
    assert lib.sse_phonon_forward(ctypes.byref(big), P(1), P(1), P(1), P(1), 0.0, -1.0, P(1), None) == _lib.SSE_ERR_DIMS
    assert b"kernel" in lib.sse_last_error()
    good = _lib.SSEDims.of(CONFIGS["tiny"])
    for i in range(5):
        ptrs = [P(1)] * 5
        ptrs[i] = None
        assert lib.sse_phonon_forward(ctypes.byref(good), *ptrs[:4], 0.0, -1.0, ptrs[4], None) == _lib.SSE_ERR_NULL


def test_signed_forward_rejects_bad_input(lib):
    P = ctypes.c_void_p
    good = _lib.SSEDims.of(CONFIGS["tiny"])
    bad = _lib.SSEDims(3, 4, 2, 2, 3, 2, 2, 1)  # nqz != nkz
    args = lambda: [P(1)] * 6
    assert lib.sse_forward_signed(ctypes.byref(bad), *args()[:5], 0.0, 1.0, 0, P(1), None, 0, None) == _lib.SSE_ERR_DIMS
    for i in range(5):
        ptrs = args()[:5]
        ptrs[i] = None  # G, Dp, Dm, dH, nbr
        assert lib.sse_forward_signed(ctypes.byref(good), *ptrs, 0.0, 1.0, 0, P(1), None, 0, None) == _lib.SSE_ERR_NULL
    assert lib.sse_forward_signed(ctypes.byref(good), *args()[:5], 0.0, 1.0, 0, None, None, 0, None) == _lib.SSE_ERR_NULL
    assert lib.sse_forward_signed(ctypes.byref(good), *args()[:5], 0.0, 1.0, 9, P(1), None, 0, None) == _lib.SSE_ERR_PRECISION


def test_signed_forward_reduced_precision_needs_matrix_core_shape(lib):
    """Shapes without a matrix-core kernel run in fp64 only: a reduced precision
    is rejected before any launch (fake pointers are never dereferenced)."""
    P = ctypes.c_void_p
    generic = _lib.SSEDims(3, 11, 3, 4, 6, 3, 5, 2)
    for prec in (1, 2):
        rc = lib.sse_forward_signed(ctypes.byref(generic), *[P(1)] * 5, 0.0, 1.0, prec, P(1), P(1), 256, None)
        assert rc == _lib.SSE_ERR_PRECISION
        assert b"precision" in lib.sse_last_error()


def _round256(x):
    return (x + 255) // 256 * 256


@pytest.mark.parametrize("dims", [
    Dims(nkz=7, ne=256, nqz=7, nw=10, na=1024, nb=4, norb=10, g_slots=1),   # matrix-core adjoint shape
    Dims(nkz=7, ne=70, nqz=7, nw=10, na=37, nb=3, norb=10, g_slots=2),
    Dims(nkz=3, ne=16, nqz=3, nw=2, na=16, nb=4, norb=4, g_slots=5),        # other kernels
])
def test_backward_workspace_matches_the_documented_layout(lib, dims):
    """sse_workspace_bytes(op = 1) is what include/sse.h documents for the
    adjoint: the reverse adjacency and dispatch order, 4 (4 na + 1 + na nb)
    bytes; the d grad H shares, 16 S na nb 3 norb^2 (S = ceil(ne / 32) on the
    matrix-core shape, nkz otherwise, and nkz for the signed form); the
    atom-major copy of dSigma on the matrix-core phonon shape, 16 na nkz ne
    norb^2 (one-table form); each rounded up to 256, the larger of the two forms."""
    d = dims
    mfma = d.norb == 10 and d.nkz == 7 and d.nqz == 7 and d.nw == 10
    csr = _round256(4 * (4 * d.na + 1 + d.na * d.nb))
    shares = (d.ne + 31) // 32 if mfma else d.nkz
    one_table = csr + _round256(16 * shares * d.na * d.nb * 3 * d.norb ** 2)
    if mfma and d.nb in (3, 4):
        one_table += _round256(16 * d.na * d.nkz * d.ne * d.norb ** 2)
    signed = csr + _round256(16 * d.nkz * d.na * d.nb * 3 * d.norb ** 2)
    need = ctypes.c_size_t(0)
    assert lib.sse_workspace_bytes(ctypes.byref(_lib.SSEDims.of(d)), 0, 1, ctypes.byref(need)) == _lib.SSE_OK
    assert need.value == max(one_table, signed)
