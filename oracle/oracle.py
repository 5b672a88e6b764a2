"""Python access to the CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never does.

``build()`` compiles ``sse_oracle.c`` with gcc into ``liboracle.so`` next to
this file; the functions below wrap its entry points for numpy complex128
arrays.  See ``sse_oracle.c`` for the formula (Eq. 3 of the paper) and the
layouts.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sse_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-ffp-contract=off", src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    with open(out + ".sha256", "w") as fh:
        fh.write(_source_hash(src) + "\n")
    return out


def _source_hash(src: str = SRC) -> str:
    with open(src, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _stale(src: str = SRC, out: str = LIB) -> bool:
    """True if the library is missing or was built from another version of the source."""
    stamp = out + ".sha256"
    if not (os.path.exists(out) and os.path.exists(stamp)):
        return True
    with open(stamp) as fh:
        return fh.read().strip() != _source_hash(src)


def _open(path):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_sse_points.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P]
    lib.oracle_sse_forward.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_sse_backward.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P, P]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_combine_d.argtypes = [P, P, P, P]
    lib.oracle_pse_points.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P]
    lib.oracle_pse_forward.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_sse_points_signed.argtypes = [P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P]
    lib.oracle_sse_forward_signed.argtypes = [P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_sse_points_ex.argtypes = [P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P]
    lib.oracle_sse_forward_ex.argtypes = [P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_sse_backward_signed.argtypes = [P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P, P, P]
    for f in (lib.oracle_sse_points, lib.oracle_sse_forward, lib.oracle_sse_backward, lib.oracle_num_threads,
              lib.oracle_combine_d, lib.oracle_pse_points, lib.oracle_pse_forward, lib.oracle_sse_points_signed,
              lib.oracle_sse_forward_signed, lib.oracle_sse_points_ex, lib.oracle_sse_forward_ex,
              lib.oracle_sse_backward_signed):
        f.restype = ctypes.c_int
    return lib


def current_lib_path() -> str:
    """Path of a liboracle.so built from the current sse_oracle.c (rebuilt if stale)."""
    if _stale():
        build()
    return LIB


def _load():
    global _lib
    if _lib is None:
        if _stale():
            build()
        _lib = _open(LIB)
    return _lib


def _ptr(x):
    return None if x is None else x.ctypes.data_as(ctypes.c_void_p)


def _dims_array(dims) -> np.ndarray:
    return np.asarray(dims.as_tuple(), dtype=np.int64)


def _check(arr, shape, dtype, name):
    if arr.shape != tuple(shape) or arr.dtype != dtype or not arr.flags.c_contiguous:
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, got {arr.dtype} {arr.shape}")


def _check_inputs(dims, G, D, dH, nbr):
    _check(G, dims.g_shape, np.complex128, "G")
    _check(D, dims.d_shape, np.complex128, "D")
    _check(dH, dims.dh_shape, np.complex128, "dH")
    _check(nbr, dims.nbr_shape, np.int32, "nbr")


def num_threads(lib=None) -> int:
    return int((lib or _load()).oracle_num_threads())


def sse_forward(dims, G, D, dH, nbr, alpha=1j, lib=None) -> np.ndarray:
    """Full Sigma[nkz, ne, na, norb, norb] (Eq. 3)."""
    _check_inputs(dims, G, D, dH, nbr)
    out = np.zeros(dims.sigma_shape, dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_forward(_ptr(dd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr),
                                    float(np.real(alpha)), float(np.imag(alpha)), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sse_forward failed with status {rc}")
    return out


def sse_points(dims, G, D, dH, nbr, pts, alpha=1j, lib=None) -> np.ndarray:
    """Sigma blocks at output points pts[p] = (k, e, a); returns [npts, norb, norb]."""
    _check_inputs(dims, G, D, dH, nbr)
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((pts.shape[0], dims.norb, dims.norb), dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_points(_ptr(dd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr),
                                   float(np.real(alpha)), float(np.imag(alpha)), pts.shape[0], _ptr(pts), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sse_points failed with status {rc}")
    return out


def sse_forward_signed(dims, G, Dp, Dm, dH, nbr, alpha=1j, lib=None) -> np.ndarray:
    """Full Sigma of Eq. 3 over signed frequencies: terms with G at E - w read
    Dp (coefficient at +w), terms with G at E + w read Dm (coefficient at -w)."""
    _check_inputs(dims, G, Dp, dH, nbr)
    _check(Dm, dims.d_shape, np.complex128, "Dm")
    out = np.zeros(dims.sigma_shape, dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_forward_signed(_ptr(dd), _ptr(G), _ptr(Dp), _ptr(Dm), _ptr(dH), _ptr(nbr),
                                                    float(np.real(alpha)), float(np.imag(alpha)), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sse_forward_signed failed with status {rc}")
    return out


def sse_points_signed(dims, G, Dp, Dm, dH, nbr, pts, alpha=1j, lib=None) -> np.ndarray:
    """Blocks of sse_forward_signed at output points pts[p] = (k, e, a)."""
    _check_inputs(dims, G, Dp, dH, nbr)
    _check(Dm, dims.d_shape, np.complex128, "Dm")
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((pts.shape[0], dims.norb, dims.norb), dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_points_signed(_ptr(dd), _ptr(G), _ptr(Dp), _ptr(Dm), _ptr(dH), _ptr(nbr),
                                                   float(np.real(alpha)), float(np.imag(alpha)), pts.shape[0],
                                                   _ptr(pts), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sse_points_signed failed with status {rc}")
    return out


def sse_forward_ex(dims, G, Dp, Dm, dH, dHba, nbr, alpha=1j, lib=None) -> np.ndarray:
    """Full Sigma of Eq. 3 with one coefficient table per sign of the frequency
    and the stored right factor dHba[a, n, j] = grad_j H_ba (None: dH[a, n, j]^H)."""
    _check_inputs(dims, G, Dp, dH, nbr)
    _check(Dm, dims.d_shape, np.complex128, "Dm")
    if dHba is not None:
        _check(dHba, dims.dh_shape, np.complex128, "dHba")
    out = np.zeros(dims.sigma_shape, dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_forward_ex(_ptr(dd), _ptr(G), _ptr(Dp), _ptr(Dm), _ptr(dH), _ptr(dHba),
                                                _ptr(nbr), float(np.real(alpha)), float(np.imag(alpha)), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sse_forward_ex failed with status {rc}")
    return out


def sse_points_ex(dims, G, Dp, Dm, dH, dHba, nbr, pts, alpha=1j, lib=None) -> np.ndarray:
    """Blocks of sse_forward_ex at output points pts[p] = (k, e, a)."""
    _check_inputs(dims, G, Dp, dH, nbr)
    _check(Dm, dims.d_shape, np.complex128, "Dm")
    if dHba is not None:
        _check(dHba, dims.dh_shape, np.complex128, "dHba")
    pts = np.ascontiguousarray(np.asarray(pts, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((pts.shape[0], dims.norb, dims.norb), dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_points_ex(_ptr(dd), _ptr(G), _ptr(Dp), _ptr(Dm), _ptr(dH), _ptr(dHba),
                                               _ptr(nbr), float(np.real(alpha)), float(np.imag(alpha)),
                                               pts.shape[0], _ptr(pts), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_sse_points_ex failed with status {rc}")
    return out


def sse_backward_signed(dims, G, Dp, Dm, dH, nbr, dSigma, alpha=1j, need=("G", "D", "dH"), lib=None):
    """Gradients (dG, dDp, dDm, ddH) of a real scalar through sse_forward_signed,
    with dL/dSigma = dSigma (PyTorch convention)."""
    _check_inputs(dims, G, Dp, dH, nbr)
    _check(Dm, dims.d_shape, np.complex128, "Dm")
    _check(dSigma, dims.sigma_shape, np.complex128, "dSigma")
    dG = np.zeros(dims.g_shape, dtype=np.complex128) if "G" in need else None
    dDp = np.zeros(dims.d_shape, dtype=np.complex128) if "D" in need else None
    dDm = np.zeros(dims.d_shape, dtype=np.complex128) if "D" in need else None
    ddH = np.zeros(dims.dh_shape, dtype=np.complex128) if "dH" in need else None
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_backward_signed(_ptr(dd), _ptr(G), _ptr(Dp), _ptr(Dm), _ptr(dH), _ptr(nbr),
                                                     float(np.real(alpha)), float(np.imag(alpha)), _ptr(dSigma),
                                                     _ptr(dG), _ptr(dDp), _ptr(dDm), _ptr(ddH))
    if rc:
        raise RuntimeError(f"oracle_sse_backward_signed failed with status {rc}")
    return dG, dDp, dDm, ddH


def sse_backward(dims, G, D, dH, nbr, dSigma, alpha=1j, need=("G", "D", "dH"), lib=None):
    """Gradients (dG, dD, ddH) of a real scalar with dL/dSigma = dSigma (PyTorch convention)."""
    _check_inputs(dims, G, D, dH, nbr)
    _check(dSigma, dims.sigma_shape, np.complex128, "dSigma")
    dG = np.zeros(dims.g_shape, dtype=np.complex128) if "G" in need else None
    dD = np.zeros(dims.d_shape, dtype=np.complex128) if "D" in need else None
    ddH = np.zeros(dims.dh_shape, dtype=np.complex128) if "dH" in need else None
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_sse_backward(_ptr(dd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr),
                                     float(np.real(alpha)), float(np.imag(alpha)), _ptr(dSigma),
                                     _ptr(dG), _ptr(dD), _ptr(ddH))
    if rc:
        raise RuntimeError(f"oracle_sse_backward failed with status {rc}")
    return dG, dD, ddH


def combine_d(dims, Dfull, nbr, lib=None) -> np.ndarray:
    """The Eq. 3 bracket D_ba - D_bb - D_aa + D_ab per neighbour slot from the
    [nqz, nw, na, nb+1, 3, 3] blocks (slot 0 = D_aa, slot 1+n = D_{a,nbr[a,n]})."""
    _check(Dfull, (dims.nqz, dims.nw, dims.na, dims.nb + 1, 3, 3), np.complex128, "Dfull")
    _check(nbr, dims.nbr_shape, np.int32, "nbr")
    out = np.zeros(dims.d_shape, dtype=np.complex128)
    dd = _dims_array(dims)
    rc = (lib or _load()).oracle_combine_d(_ptr(dd), _ptr(Dfull), _ptr(nbr), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_combine_d failed with status {rc}")
    return out


def absorption_d(dims, Dopp) -> np.ndarray:
    """Coefficients of the absorption branch (frequency -w) of Eq. 3's integral
    over signed frequencies, from the combined table of the opposite component.

    For real displacement fields the lesser and greater phonon Green's functions
    are related by D<_ab(q, -w) = D>_ba(-q, w) (and with < and > exchanged).  The
    bracket D_ba - D_bb - D_aa + D_ab of Eq. 3 is symmetric in a <-> b, so on the
    combined per-neighbour tables the relation reads, with the Cartesian indices
    exchanged:  Dm[q, w, a, n, i, j] = Dopp[(-q) mod Nqz, w, a, n, j, i]."""
    _check(Dopp, dims.d_shape, np.complex128, "Dopp")
    out = np.empty_like(Dopp)
    for q in range(dims.nqz):
        out[q] = np.swapaxes(Dopp[(-q) % dims.nqz], -1, -2)
    return out


def _check_pse_inputs(dims, Gs, Go, dH, nbr):
    _check(Gs, dims.g_shape, np.complex128, "Gs")
    _check(Go, dims.g_shape, np.complex128, "Go")
    _check(dH, dims.dh_shape, np.complex128, "dH")
    _check(nbr, dims.nbr_shape, np.int32, "nbr")


def pse_forward(dims, Gs, Go, dH, nbr, beta=-1j, lib=None) -> np.ndarray:
    """Phonon self-energy Pi [nqz, nw, na, nb, 3, 3] (Eq. 4, off-diagonal blocks):
    Gs of the same component as Pi at the atom, Go of the opposite one at the
    neighbour."""
    _check_pse_inputs(dims, Gs, Go, dH, nbr)
    out = np.zeros(dims.d_shape, dtype=np.complex128)
    dd = _dims_array(dims)
    b = complex(beta)
    rc = (lib or _load()).oracle_pse_forward(_ptr(dd), _ptr(Gs), _ptr(Go), _ptr(dH), _ptr(nbr), b.real, b.imag,
                                             _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_pse_forward failed with status {rc}")
    return out


def pse_points(dims, Gs, Go, dH, nbr, pts, beta=-1j, lib=None) -> np.ndarray:
    """Pi blocks at pts = [(q, w-1, a, n), ...] -> [npts, 3, 3]."""
    _check_pse_inputs(dims, Gs, Go, dH, nbr)
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.int64).reshape(-1, 4))
    out = np.zeros((p.shape[0], 3, 3), dtype=np.complex128)
    dd = _dims_array(dims)
    b = complex(beta)
    rc = (lib or _load()).oracle_pse_points(_ptr(dd), _ptr(Gs), _ptr(Go), _ptr(dH), _ptr(nbr), b.real, b.imag,
                                            p.shape[0], _ptr(p), _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_pse_points failed with status {rc}")
    return out


def sse_status(dims_tuple, G, D, dH, nbr, lib=None) -> int:
    """Raw status of the forward entry point for arbitrary (possibly invalid) dims."""
    dd = np.asarray(dims_tuple, dtype=np.int64)
    out = np.zeros(max(1, G.size), dtype=np.complex128)
    return int((lib or _load()).oracle_sse_forward(_ptr(dd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr), 0.0, 1.0, _ptr(out)))


class Bound:
    """The functions above bound to one loaded oracle library (used to run the
    pins against deliberately broken copies of the oracle)."""

    def __init__(self, path):
        self.lib = _open(path)

    def sse_forward(self, *a, **k):
        return sse_forward(*a, lib=self.lib, **k)

    def sse_points(self, *a, **k):
        return sse_points(*a, lib=self.lib, **k)

    def sse_forward_signed(self, *a, **k):
        return sse_forward_signed(*a, lib=self.lib, **k)

    def sse_points_signed(self, *a, **k):
        return sse_points_signed(*a, lib=self.lib, **k)

    def sse_backward(self, *a, **k):
        return sse_backward(*a, lib=self.lib, **k)

    def sse_forward_ex(self, *a, **k):
        return sse_forward_ex(*a, lib=self.lib, **k)

    def sse_points_ex(self, *a, **k):
        return sse_points_ex(*a, lib=self.lib, **k)

    def sse_backward_signed(self, *a, **k):
        return sse_backward_signed(*a, lib=self.lib, **k)

    def sse_status(self, *a, **k):
        return sse_status(*a, lib=self.lib, **k)

    def combine_d(self, *a, **k):
        return combine_d(*a, lib=self.lib, **k)

    def pse_forward(self, *a, **k):
        return pse_forward(*a, lib=self.lib, **k)

    def pse_points(self, *a, **k):
        return pse_points(*a, lib=self.lib, **k)
