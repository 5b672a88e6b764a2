"""PyTorch binding of libsse: argument marshalling only.

Every step of the computation runs in the HIP kernels behind the C ABI
(include/sse.h); PyTorch supplies device memory and the current stream.
There is no fallback: if libsse.so is missing or the tensors are not on a HIP
device, these functions raise.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .inputs import Dims

PRECISIONS = _lib.PRECISIONS


def dims_of(G: torch.Tensor, D: torch.Tensor, dH: torch.Tensor, nbr: torch.Tensor) -> Dims:
    if G.dim() != 6 or D.dim() != 6 or dH.dim() != 5 or nbr.dim() != 2:
        raise ValueError("expected G[nkz,ne,na,slots,norb,norb], D[nqz,nw,na,nb,3,3], dH[na,nb,3,norb,norb], nbr[na,nb]")
    nkz, ne, na, gs, norb, norb2 = G.shape
    nqz, nw, na2, nb, three, three2 = D.shape
    d = Dims(nkz=nkz, ne=ne, nqz=nqz, nw=nw, na=na, nb=nb, norb=norb, g_slots=gs)
    if norb2 != norb or three != 3 or three2 != 3 or na2 != na:
        raise ValueError(f"inconsistent shapes G{tuple(G.shape)} D{tuple(D.shape)}")
    if tuple(dH.shape) != d.dh_shape:
        raise ValueError(f"dH must be {d.dh_shape}, got {tuple(dH.shape)}")
    if tuple(nbr.shape) != d.nbr_shape:
        raise ValueError(f"nbr must be {d.nbr_shape}, got {tuple(nbr.shape)}")
    return d


def _resolved(t: torch.Tensor) -> torch.Tensor:
    """The tensor with PyTorch's lazy conjugate and negative bits applied, so its
    memory holds the values it stands for (a .conj() view shares its base's
    memory and would otherwise be read unconjugated)."""
    return t.resolve_conj().resolve_neg() if t is not None else None


def _check_tensor(t: torch.Tensor, name: str, dtype=torch.complex128):
    if t.is_conj() or t.is_neg():
        raise ValueError(f"{name} carries a lazy conjugate/negative bit; resolve it first")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _raise(rc: int, what: str):
    if rc != _lib.SSE_OK:
        raise RuntimeError(f"{what} failed (status {rc}): {_lib.last_error()}")


def workspace(d: Dims, precision: str = "fp64", backward: bool = False, device="cuda", op: int = None) -> torch.Tensor:
    """Workspace for sse_forward (op 0), sse_backward (op 1) or sse_combine_d (op 2)."""
    lib = _lib.load()
    nbytes = ctypes.c_size_t(0)
    cd = _lib.SSEDims.of(d)
    op = int(backward) if op is None else op
    _raise(lib.sse_workspace_bytes(ctypes.byref(cd), PRECISIONS.get(precision, -1), op, ctypes.byref(nbytes)),
           "sse_workspace_bytes")
    return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=device)


def effective_flops(d: Dims) -> float:
    lib = _lib.load()
    out = ctypes.c_double(0.0)
    cd = _lib.SSEDims.of(d)
    _raise(lib.sse_effective_flops(ctypes.byref(cd), ctypes.byref(out)), "sse_effective_flops")
    return float(out.value)


def check_nbr(nbr: torch.Tensor, na: int) -> None:
    """Raise if any neighbour entry lies outside [0, na) (synchronous)."""
    _check_tensor(nbr, "nbr", torch.int32)
    lib = _lib.load()
    d = Dims(nkz=1, ne=1, nqz=1, nw=1, na=na, nb=nbr.shape[1], norb=1, g_slots=1)
    ws = workspace(d, device=nbr.device)
    cd = _lib.SSEDims.of(d)
    _raise(lib.sse_check_nbr(ctypes.byref(cd), _ptr(nbr), _ptr(ws), ws.numel(), _stream(nbr.device)), "sse_check_nbr")


def combine_d(Dfull: torch.Tensor, nbr: torch.Tensor) -> torch.Tensor:
    """Eq. 3 bracket D_ba - D_bb - D_aa + D_ab per neighbour slot from the
    [nqz, nw, na, nb+1, 3, 3] phonon blocks; needs a symmetric neighbour table."""
    Dfull = _resolved(Dfull)
    _check_tensor(Dfull, "Dfull")
    _check_tensor(nbr, "nbr", torch.int32)
    if Dfull.dim() != 6 or Dfull.shape[4:] != (3, 3) or Dfull.shape[3] != nbr.shape[1] + 1 or Dfull.shape[2] != nbr.shape[0]:
        raise ValueError(f"Dfull must be [nqz, nw, na, nb+1, 3, 3] for nbr {tuple(nbr.shape)}")
    nqz, nw, na = Dfull.shape[:3]
    d = Dims(nkz=nqz, ne=1, nqz=nqz, nw=nw, na=na, nb=nbr.shape[1], norb=1, g_slots=1)
    out = torch.empty(d.d_shape, dtype=torch.complex128, device=Dfull.device)
    ws = workspace(d, device=Dfull.device, op=2)
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    _raise(lib.sse_combine_d(ctypes.byref(cd), _ptr(Dfull), _ptr(nbr), _ptr(out), _ptr(ws), ws.numel(),
                             _stream(Dfull.device)), "sse_combine_d")
    return out


def absorption_d(Dopp: torch.Tensor) -> torch.Tensor:
    """Coefficients at -w for the signed-frequency form (the Dm argument of
    forward_signed / forward_ex) from the combined [nqz, nw, na, nb, 3, 3] table of
    the opposite component: Dm[q,w,a,n,i,j] = Dopp[(-q) mod nqz, w, a, n, j, i]
    (D<_ab(q, -w) = D>_ba(-q, w) for real displacement fields)."""
    Dopp = _resolved(Dopp)
    _check_tensor(Dopp, "Dopp")
    if Dopp.dim() != 6 or Dopp.shape[4:] != (3, 3):
        raise ValueError("Dopp must be [nqz, nw, na, nb, 3, 3]")
    nqz, nw, na, nb = Dopp.shape[:4]
    d = Dims(nkz=nqz, ne=1, nqz=nqz, nw=nw, na=na, nb=nb, norb=1, g_slots=1)
    out = torch.empty_like(Dopp)
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    _raise(lib.sse_absorption_d(ctypes.byref(cd), _ptr(Dopp), _ptr(out), _stream(Dopp.device)), "sse_absorption_d")
    return out


def forward(G, D, dH, nbr, alpha=1j, precision: str = "fp64", out=None, ws=None) -> torch.Tensor:
    """Sigma[nkz, ne, na, norb, norb] = Eq. 3 (one of lesser/greater).  precision
    is a key of PRECISIONS (the sse_precision codes: fp64, fp32, bf16x2, fp16x2,
    and the single-term comparison forms fp16 and fp16_unscaled)."""
    return _forward(G, D, D, dH, None, nbr, alpha, precision, out, ws)


def forward_signed(G, Dp, Dm, dH, nbr, alpha=1j, precision: str = "fp64", out=None, ws=None) -> torch.Tensor:
    """Sigma of Eq. 3 over both signs of the frequency: the terms with G at
    E - w read Dp (coefficients at +w), those with G at E + w read Dm (at -w);
    both in D's layout.  Dm is Dp gives forward()."""
    return forward_ex(G, Dp, dH, nbr, Dm=Dm, alpha=alpha, precision=precision, out=out, ws=ws)


def forward_ex(G, Dp, dH, nbr, Dm=None, dHba=None, alpha=1j, precision: str = "fp64", out=None, ws=None) -> torch.Tensor:
    """Sigma of Eq. 3 with its full input contract: Dm (coefficients at -w, for
    the terms with G at E + w; None or Dp itself: the one-table form) and dHba,
    the stored right factor grad_j H_ba[a, n, j] in dH's layout (None: the
    Hermitian reading dH^H)."""
    if Dm is None or Dm is Dp:
        Dm = Dp
    else:
        Dp, Dm = _resolved(Dp), _resolved(Dm)
        _check_tensor(Dm, "Dm")
        if Dm.shape != Dp.shape:
            raise ValueError(f"Dm must have Dp's shape {tuple(Dp.shape)}")
    if dHba is not None:
        dHba = _resolved(dHba)
        _check_tensor(dHba, "dHba")
        if dHba.shape != dH.shape:
            raise ValueError(f"dHba must have dH's shape {tuple(dH.shape)}")
    return _forward(G, Dp, Dm, dH, dHba, nbr, alpha, precision, out, ws)


def _forward(G, D, Dm, dH, dHba, nbr, alpha, precision, out, ws) -> torch.Tensor:
    same = Dm is D
    G, D, dH = _resolved(G), _resolved(D), _resolved(dH)
    Dm = D if same else Dm
    d = dims_of(G, D, dH, nbr)
    for t, n in ((G, "G"), (D, "D"), (dH, "dH")):
        _check_tensor(t, n)
    _check_tensor(nbr, "nbr", torch.int32)
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    if out is None:
        out = torch.empty(d.sigma_shape, dtype=torch.complex128, device=G.device)
    else:
        _check_tensor(out, "out")
        if tuple(out.shape) != d.sigma_shape:
            raise ValueError(f"out must be {d.sigma_shape}")
    if ws is None:
        ws = workspace(d, precision, device=G.device)
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    a = complex(alpha)
    if dHba is not None:
        rc = lib.sse_forward_ex(ctypes.byref(cd), _ptr(G), _ptr(D), _ptr(Dm), _ptr(dH), _ptr(dHba), _ptr(nbr), a.real,
                                a.imag, PRECISIONS[precision], _ptr(out), _ptr(ws), ws.numel(), _stream(G.device))
        _raise(rc, "sse_forward_ex")
    elif Dm is D or Dm.data_ptr() == D.data_ptr():
        rc = lib.sse_forward(ctypes.byref(cd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr), a.real, a.imag,
                             PRECISIONS[precision], _ptr(out), _ptr(ws), ws.numel(), _stream(G.device))
        _raise(rc, "sse_forward")
    else:
        rc = lib.sse_forward_signed(ctypes.byref(cd), _ptr(G), _ptr(D), _ptr(Dm), _ptr(dH), _ptr(nbr), a.real, a.imag,
                                    PRECISIONS[precision], _ptr(out), _ptr(ws), ws.numel(), _stream(G.device))
        _raise(rc, "sse_forward_signed")
    return out


def phonon_forward(Gs, Go, dH, nbr, nqz: int, nw: int, beta=-1j, out=None) -> torch.Tensor:
    """Pi[nqz, nw, na, nb, 3, 3] = Eq. 4 for the nb off-diagonal blocks per atom.

    Gs is the electron Green's function of the same component as Pi, Go the
    opposite one (both [nkz, ne, na, slots, norb, norb]); beta carries -i and
    the energy quadrature weight."""
    Gs, Go, dH = _resolved(Gs), _resolved(Go), _resolved(dH)
    if Gs.dim() != 6 or dH.dim() != 5 or nbr.dim() != 2:
        raise ValueError("expected Gs/Go[nkz,ne,na,slots,norb,norb], dH[na,nb,3,norb,norb], nbr[na,nb]")
    nkz, ne, na, gs, norb, _ = Gs.shape
    d = Dims(nkz=nkz, ne=ne, nqz=int(nqz), nw=int(nw), na=na, nb=nbr.shape[1], norb=norb, g_slots=gs)
    if tuple(Go.shape) != tuple(Gs.shape) or tuple(Gs.shape) != d.g_shape:
        raise ValueError(f"Gs and Go must both be {d.g_shape}, got {tuple(Gs.shape)} and {tuple(Go.shape)}")
    if tuple(dH.shape) != d.dh_shape or tuple(nbr.shape) != d.nbr_shape:
        raise ValueError(f"dH must be {d.dh_shape} and nbr {d.nbr_shape}")
    for t, n in ((Gs, "Gs"), (Go, "Go"), (dH, "dH")):
        _check_tensor(t, n)
    _check_tensor(nbr, "nbr", torch.int32)
    if out is None:
        out = torch.empty(d.d_shape, dtype=torch.complex128, device=Gs.device)
    else:
        _check_tensor(out, "out")
        if tuple(out.shape) != d.d_shape:
            raise ValueError(f"out must be {d.d_shape}")
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    b = complex(beta)
    rc = lib.sse_phonon_forward(ctypes.byref(cd), _ptr(Gs), _ptr(Go), _ptr(dH), _ptr(nbr), b.real, b.imag, _ptr(out),
                                _stream(Gs.device))
    _raise(rc, "sse_phonon_forward")
    return out


def backward(G, D, dH, nbr, dSigma, alpha=1j, need=(True, True, True), ws=None):
    """(dL/dG, dL/dD, dL/d dH) for dSigma = dL/dSigma (PyTorch complex-gradient convention)."""
    G, D, dH, dSigma = _resolved(G), _resolved(D), _resolved(dH), _resolved(dSigma)
    d = dims_of(G, D, dH, nbr)
    for t, n in ((G, "G"), (D, "D"), (dH, "dH"), (dSigma, "dSigma")):
        _check_tensor(t, n)
    _check_tensor(nbr, "nbr", torch.int32)
    if tuple(dSigma.shape) != d.sigma_shape:
        raise ValueError(f"dSigma must be {d.sigma_shape}")
    dev = G.device
    dG = torch.empty(d.g_shape, dtype=torch.complex128, device=dev) if need[0] else None
    dD = torch.empty(d.d_shape, dtype=torch.complex128, device=dev) if need[1] else None
    ddH = torch.empty(d.dh_shape, dtype=torch.complex128, device=dev) if need[2] else None
    if ws is None:
        ws = workspace(d, backward=True, device=dev)
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    a = complex(alpha)
    rc = lib.sse_backward(ctypes.byref(cd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr), a.real, a.imag, _ptr(dSigma),
                          _ptr(dG), _ptr(dD), _ptr(ddH), _ptr(ws), ws.numel(), _stream(dev))
    _raise(rc, "sse_backward")
    return dG, dD, ddH


def backward_noalloc(G, D, dH, nbr, dSigma, alpha=1j, dG=None, dD=None, ddH=None):
    """sse_backward_noalloc: the adjoint into caller-provided outputs (any may be
    None to skip that gradient) with no device allocation in the library; the
    workspace is the library's own device array (at most
    sse_noalloc_scratch_bytes() bytes of workspace)."""
    G, D, dH, dSigma = _resolved(G), _resolved(D), _resolved(dH), _resolved(dSigma)
    d = dims_of(G, D, dH, nbr)
    for t, n in ((G, "G"), (D, "D"), (dH, "dH"), (dSigma, "dSigma")):
        _check_tensor(t, n)
    _check_tensor(nbr, "nbr", torch.int32)
    for t, n, shape in ((dG, "dG", d.g_shape), (dD, "dD", d.d_shape), (ddH, "ddH", d.dh_shape)):
        if t is not None:
            _check_tensor(t, n)
            if tuple(t.shape) != shape:
                raise ValueError(f"{n} must be {shape}")
    if tuple(dSigma.shape) != d.sigma_shape:
        raise ValueError(f"dSigma must be {d.sigma_shape}")
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    a = complex(alpha)
    rc = lib.sse_backward_noalloc(ctypes.byref(cd), _ptr(G), _ptr(D), _ptr(dH), _ptr(nbr), a.real, a.imag,
                                  _ptr(dSigma), _ptr(dG), _ptr(dD), _ptr(ddH), _stream(G.device))
    _raise(rc, "sse_backward_noalloc")
    return dG, dD, ddH


def backward_signed(G, Dp, Dm, dH, nbr, dSigma, alpha=1j, need=(True, True, True, True), ws=None):
    """(dL/dG, dL/dDp, dL/dDm, dL/d dH) through forward_signed, for dSigma = dL/dSigma."""
    G, Dp, Dm, dH, dSigma = (_resolved(t) for t in (G, Dp, Dm, dH, dSigma))
    d = dims_of(G, Dp, dH, nbr)
    for t, n in ((G, "G"), (Dp, "Dp"), (Dm, "Dm"), (dH, "dH"), (dSigma, "dSigma")):
        _check_tensor(t, n)
    _check_tensor(nbr, "nbr", torch.int32)
    if tuple(Dm.shape) != d.d_shape or tuple(dSigma.shape) != d.sigma_shape:
        raise ValueError(f"Dm must be {d.d_shape} and dSigma {d.sigma_shape}")
    dev = G.device
    dG = torch.empty(d.g_shape, dtype=torch.complex128, device=dev) if need[0] else None
    dDp = torch.empty(d.d_shape, dtype=torch.complex128, device=dev) if need[1] else None
    dDm = torch.empty(d.d_shape, dtype=torch.complex128, device=dev) if need[2] else None
    ddH = torch.empty(d.dh_shape, dtype=torch.complex128, device=dev) if need[3] else None
    if ws is None:
        ws = workspace(d, backward=True, device=dev)
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    a = complex(alpha)
    rc = lib.sse_backward_signed(ctypes.byref(cd), _ptr(G), _ptr(Dp), _ptr(Dm), _ptr(dH), _ptr(nbr), a.real, a.imag,
                                 _ptr(dSigma), _ptr(dG), _ptr(dDp), _ptr(dDm), _ptr(ddH), _ptr(ws), ws.numel(),
                                 _stream(dev))
    _raise(rc, "sse_backward_signed")
    return dG, dDp, dDm, ddH


class SSEFunction(torch.autograd.Function):
    """Sigma = SSE(G, D, dH) with the hand-written adjoint as backward.

    Saves only the inputs; the backward re-gathers the shifted G blocks.
    """

    @staticmethod
    def forward(ctx, G, D, dH, nbr, alpha=1j):
        ctx.save_for_backward(G, D, dH, nbr)
        ctx.alpha = complex(alpha)
        return forward(G, D, dH, nbr, alpha=alpha)

    @staticmethod
    def backward(ctx, gS):
        G, D, dH, nbr = ctx.saved_tensors
        need = ctx.needs_input_grad[:3]
        dG, dD, ddH = backward(G, D, dH, nbr, _resolved(gS).contiguous(), alpha=ctx.alpha, need=need)
        return dG, dD, ddH, None, None


def sse(G, D, dH, nbr, alpha=1j):
    """Differentiable Sigma (autograd through the hand-written adjoint)."""
    return SSEFunction.apply(G, D, dH, nbr, alpha)


class SSESignedFunction(torch.autograd.Function):
    """Sigma = SSE over signed frequencies (Dp at +w, Dm at -w) with the
    hand-written adjoint as backward; saves only the inputs."""

    @staticmethod
    def forward(ctx, G, Dp, Dm, dH, nbr, alpha=1j):
        ctx.save_for_backward(G, Dp, Dm, dH, nbr)
        ctx.alpha = complex(alpha)
        return forward_ex(G, Dp, dH, nbr, Dm=Dm, alpha=alpha)

    @staticmethod
    def backward(ctx, gS):
        G, Dp, Dm, dH, nbr = ctx.saved_tensors
        need = ctx.needs_input_grad[:4]
        dG, dDp, dDm, ddH = backward_signed(G, Dp, Dm, dH, nbr, _resolved(gS).contiguous(), alpha=ctx.alpha,
                                            need=need)
        return dG, dDp, dDm, ddH, None, None


def sse_signed(G, Dp, Dm, dH, nbr, alpha=1j):
    """Differentiable Sigma over signed frequencies (autograd through the hand-written adjoint)."""
    return SSESignedFunction.apply(G, Dp, Dm, dH, nbr, alpha)
