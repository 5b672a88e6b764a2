"""Seeded synthetic inputs for the electron-phonon scattering self-energy.

This module only draws random numbers in the shapes and value distributions
of the paper's workloads; it contains none of the self-energy arithmetic.
Both the HIP path and the CPU oracle are fed from here, and nothing else is
shared between them.

Shapes (complex128, row-major, interleaved re/im):
  G    [nkz, ne, na, g_slots, norb, norb]   electron lesser/greater GF blocks;
       slot 0 is the diagonal block G_aa used by Eq. 3, slots 1.. are the
       neighbour blocks that the equation does not read (Sec. "Current State of
       the Art": the SSE needs [Nkz, NE, Na, Norb, Norb] for electrons).
  D    [nqz, nw, na, nb, 3, 3]              phonon GF coefficient per neighbour
       slot, already combined as D_ba - D_bb - D_aa + D_ab (Eq. 3 bracket).
  dH   [na, nb, 3, norb, norb]              grad_i H_ab for b = nbr[a, n].
  nbr  [na, nb] int32                       neighbour table (no self-loops).
  W    [nkz, ne, na, norb, norb]            weight of the scalar functional
       L = Re sum tr(W Sigma) used for the adjoint checks.

Value recipe: every real and imaginary part is drawn independently;
G ~ N(0,1) then each block is made anti-Hermitian, (X - X^H)/2, the property
lesser/greater Green's functions carry; D ~ N(0,1); dH ~ N(0, 0.1^2);
W ~ N(0,1).  Neighbours: for each atom, nb distinct other atoms drawn
uniformly without replacement (a random table has no spatial locality and is
the worst case for the gather).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Iterable, Optional

import numpy as np

N3D = 3
SEED_BASE = 1912
# order in which independent streams are spawned from one SeedSequence
STREAMS = ("nbr", "G<", "G>", "D<", "D>", "dH", "W")


@dataclasses.dataclass(frozen=True)
class Dims:
    nkz: int
    ne: int
    nqz: int
    nw: int
    na: int
    nb: int
    norb: int
    g_slots: int = 1

    def as_tuple(self):
        return (self.nkz, self.ne, self.nqz, self.nw, self.na, self.nb, self.norb, self.g_slots)

    # tensor shapes -------------------------------------------------------
    @property
    def g_shape(self):
        return (self.nkz, self.ne, self.na, self.g_slots, self.norb, self.norb)

    @property
    def d_shape(self):
        return (self.nqz, self.nw, self.na, self.nb, N3D, N3D)

    @property
    def dh_shape(self):
        return (self.na, self.nb, N3D, self.norb, self.norb)

    @property
    def sigma_shape(self):
        return (self.nkz, self.ne, self.na, self.norb, self.norb)

    @property
    def nbr_shape(self):
        return (self.na, self.nb)

    def replace(self, **kw) -> "Dims":
        return dataclasses.replace(self, **kw)


# Workloads: the tiny, mid and device-scale electron-phonon problems.  The
# device-scale one is one GPU's share of a ~5k-atom FinFET slice with the
# tight-binding-sized blocks the original OMEN runs used (Nb=4, Norb=10).
CONFIGS: Dict[str, Dims] = {
    "tiny": Dims(nkz=3, ne=16, nqz=3, nw=2, na=16, nb=4, norb=4, g_slots=5),
    "mid": Dims(nkz=7, ne=256, nqz=7, nw=10, na=1024, nb=4, norb=10, g_slots=5),
    # G is stored diagonal-only at this size (slot 0 is the only slot read)
    "device": Dims(nkz=7, ne=1024, nqz=7, nw=10, na=4864, nb=4, norb=10, g_slots=1),
}
CONFIG_INDEX = {"tiny": 0, "mid": 1, "device": 2}


def seed_streams(config_index: int) -> Dict[str, np.random.SeedSequence]:
    ss = np.random.SeedSequence(SEED_BASE + config_index)
    return dict(zip(STREAMS, ss.spawn(len(STREAMS))))


def _cnormal(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    out = np.empty(shape, dtype=np.complex128)
    v = out.view(np.float64).reshape(tuple(shape) + (2,))
    v[...] = rng.standard_normal(tuple(shape) + (2,)) * sigma
    return out


def make_nbr(rng: np.random.Generator, na: int, nb: int) -> np.ndarray:
    if nb > na - 1:
        raise ValueError("need nb <= na - 1 distinct neighbours")
    nbr = np.empty((na, nb), dtype=np.int32)
    for a in range(na):
        pick = rng.choice(na - 1, size=nb, replace=False)
        pick = pick + (pick >= a)  # skip the atom itself
        nbr[a] = pick
    return nbr


def make_symmetric_nbr(rng: np.random.Generator, na: int, nb: int) -> np.ndarray:
    """A symmetric nb-regular table (nb even): atoms on a random permutation of a
    ring, each linked to the nb/2 nearest ring positions on either side.  a is a
    neighbour of b exactly when b is a neighbour of a, as for a real structure."""
    if nb % 2 or nb > na - 1:
        raise ValueError("need an even nb <= na - 1")
    perm = rng.permutation(na)
    pos = np.empty(na, dtype=np.int64)
    pos[perm] = np.arange(na)
    nbr = np.empty((na, nb), dtype=np.int32)
    offs = [o for h in range(1, nb // 2 + 1) for o in (h, -h)]
    for a in range(na):
        nbr[a] = [perm[(pos[a] + o) % na] for o in offs]
    return nbr


def make_D_full(rng: np.random.Generator, dims: Dims) -> np.ndarray:
    """Phonon Green's function blocks [nqz, nw, na, nb+1, 3, 3]: slot 0 is D_aa,
    slot 1+n the block coupling a to its n-th neighbour; N(0,1) parts."""
    return _cnormal(rng, (dims.nqz, dims.nw, dims.na, dims.nb + 1, N3D, N3D), 1.0)


def anti_hermitian_blocks(x: np.ndarray) -> np.ndarray:
    """(X - X^H)/2 over the last two axes, in place."""
    xh = np.conj(np.swapaxes(x, -1, -2))
    x -= xh
    x *= 0.5
    return x


def make_G(rng: np.random.Generator, dims: Dims) -> np.ndarray:
    return anti_hermitian_blocks(_cnormal(rng, dims.g_shape, 1.0))


def make_D(rng: np.random.Generator, dims: Dims) -> np.ndarray:
    return _cnormal(rng, dims.d_shape, 1.0)


def make_dH(rng: np.random.Generator, dims: Dims) -> np.ndarray:
    return _cnormal(rng, dims.dh_shape, 0.1)


def make_W(rng: np.random.Generator, dims: Dims) -> np.ndarray:
    return _cnormal(rng, dims.sigma_shape, 1.0)


def generate(dims: Dims, config_index: int, which: Iterable[str] = ("nbr", "G<", "D<", "dH")) -> Dict[str, np.ndarray]:
    """Host-side inputs for one workload; each tensor has its own stream."""
    ss = seed_streams(config_index)
    out = {}
    for name in which:
        rng = np.random.default_rng(ss[name])
        if name == "nbr":
            out[name] = make_nbr(rng, dims.na, dims.nb)
        elif name in ("G<", "G>"):
            out[name] = make_G(rng, dims)
        elif name in ("D<", "D>"):
            out[name] = make_D(rng, dims)
        elif name == "dH":
            out[name] = make_dH(rng, dims)
        elif name == "W":
            out[name] = make_W(rng, dims)
        else:
            raise KeyError(name)
    return out


def generate_device(dims: Dims, config_index: int, device="cuda", which=("nbr", "G<", "D<", "dH"), chunk_elems: int = 1 << 27):
    """Device-side inputs for sizes that are impractical to draw on the host.

    Same distributions as :func:`generate`, drawn with torch's generator on
    the device (values differ from the host streams, which is fine: every
    check on these inputs copies what it needs back to the host).  The
    neighbour table is still drawn on the host with its numpy stream.
    """
    import torch

    ss = seed_streams(config_index)
    out = {}
    for name in which:
        idx = STREAMS.index(name)
        if name == "nbr":
            rng = np.random.default_rng(ss["nbr"])
            out[name] = torch.from_numpy(make_nbr(rng, dims.na, dims.nb)).to(device)
            continue
        gen = torch.Generator(device=device)
        gen.manual_seed(SEED_BASE + 1000 * config_index + idx)
        if name in ("G<", "G>"):
            shape, sigma = dims.g_shape, 1.0
        elif name in ("D<", "D>"):
            shape, sigma = dims.d_shape, 1.0
        elif name == "dH":
            shape, sigma = dims.dh_shape, 0.1
        elif name == "W":
            shape, sigma = dims.sigma_shape, 1.0
        else:
            raise KeyError(name)
        t = torch.empty(shape, dtype=torch.complex128, device=device)
        flat = torch.view_as_real(t).view(-1)
        for s in range(0, flat.numel(), chunk_elems):
            e = min(flat.numel(), s + chunk_elems)
            flat[s:e].normal_(0.0, sigma, generator=gen)
        if name in ("G<", "G>"):
            # anti-Hermitian blocks, processed one leading slice at a time
            for k in range(shape[0]):
                blk = t[k]
                for e0 in range(0, shape[1], 64):
                    x = blk[e0:e0 + 64]
                    xh = x.transpose(-1, -2).conj().clone()
                    x.sub_(xh).mul_(0.5)
        out[name] = t
    return out
