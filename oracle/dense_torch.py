"""Dense PyTorch (CPU, fp64) form of the scattering self-energy.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``).

Eq. 3 evaluated by materialising the whole gathered tensor of shifted
Green's-function blocks
    Gg[k, e, a, q, m, s, n] = G[(k-q) mod Nkz, e - s*m, nbr[a,n], 0]   (0 outside the energy grid)
and contracting it with one einsum.  This is a different evaluation order
from the loop nest in ``sse_oracle.c`` (one big contraction instead of
per-term 2-matrix products) and it is differentiable, so autograd gives a
reference for the adjoint.  Memory grows like Nkz*NE*Na*Nqz*Nw*2*NB*Norb^2,
so it is only for small inputs.
"""
from __future__ import annotations

import torch


def gather_shifted(G: torch.Tensor, nbr: torch.Tensor, nqz: int, nw: int) -> torch.Tensor:
    """Gg[k, e, a, q, m-1, s, n, t, u] with s index 0 -> s=+1 (E - w), 1 -> s=-1 (E + w)."""
    nkz, ne, na, _, norb, _ = G.shape
    nb = nbr.shape[1]
    k = torch.arange(nkz).view(nkz, 1)
    q = torch.arange(nqz).view(1, nqz)
    kp = torch.remainder(k - q, nkz)                                   # [nkz, nqz]
    e = torch.arange(ne).view(ne, 1, 1)
    m = torch.arange(1, nw + 1).view(1, nw, 1)
    s = torch.tensor([1, -1]).view(1, 1, 2)
    ep = e - s * m                                                     # [ne, nw, 2]
    valid = (ep >= 0) & (ep < ne)
    epc = ep.clamp(0, ne - 1)
    G0 = G[:, :, :, 0]                                                 # [nkz, ne, na, norb, norb]
    # index: [k, e, a, q, m, s, n]
    K = kp.view(nkz, 1, 1, nqz, 1, 1, 1)
    E = epc.view(1, ne, 1, 1, nw, 2, 1)
    B = nbr.long().view(1, 1, na, 1, 1, 1, nb)
    shape = (nkz, ne, na, nqz, nw, 2, nb)
    Gg = G0[K.expand(shape), E.expand(shape), B.expand(shape)]        # [..., norb, norb]
    mask = valid.view(1, ne, 1, 1, nw, 2, 1).expand(shape)
    return Gg * mask[..., None, None].to(Gg.dtype)


def sse_forward(G, D, dH, nbr, alpha=1j) -> torch.Tensor:
    nqz, nw = D.shape[0], D.shape[1]
    Gg = gather_shifted(G, nbr, nqz, nw)
    out = torch.einsum("qmanij,anirt,keaqmsntu,anjcu->kearc", D, dH, Gg, dH.conj())
    return alpha * out


def sse_forward_ex(G, Dp, Dm, dH, dHba, nbr, alpha=1j) -> torch.Tensor:
    """Eq. 3 over signed frequencies (Dp for the terms with G at E - w, Dm for
    those at E + w) with the stored right factor dHba[a, n, j] = grad_j H_ba
    (None: dH[a, n, j]^H), as one einsum over the gathered tensor."""
    nqz, nw = Dp.shape[0], Dp.shape[1]
    Gg = gather_shifted(G, nbr, nqz, nw)
    Ds = torch.stack([Dp, Dm], dim=2)                                  # [q, m, s, a, n, i, j]
    right = dHba if dHba is not None else dH.conj().transpose(-1, -2)  # [a, n, j, u, c]
    out = torch.einsum("qmsanij,anirt,keaqmsntu,anjuc->kearc", Ds, dH, Gg, right)
    return alpha * out
