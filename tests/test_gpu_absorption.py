"""The absorption branch of Eq. 3 on the GPU: sse_absorption_d (coefficients at
-w from the opposite component's combined table) bit for bit against the
oracle's map, and the signed-frequency forward fed with it against the oracle's
signed form fed with the oracle's map (Sigma< with Dp = D<, Dm from D>)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_1912_10024_amd import _lib, sse
from paper_1912_10024_amd.inputs import Dims, anti_hermitian_blocks, make_nbr

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp16x2": 1e-6}


def _cn(rng, shape, s=1.0):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s


def _rel(x, y):
    return float(np.linalg.norm((x - y).ravel()) / max(np.linalg.norm(y.ravel()), 1e-300))


@pytest.mark.parametrize("dims", [Dims(nkz=7, ne=1, nqz=7, nw=10, na=9, nb=4, norb=1, g_slots=1),
                                  Dims(nkz=3, ne=1, nqz=3, nw=2, na=5, nb=3, norb=1, g_slots=1),
                                  Dims(nkz=1, ne=1, nqz=1, nw=3, na=2, nb=1, norb=1, g_slots=1)],
                         ids=["q7", "q3", "q1"])
def test_absorption_map_bitwise(dims):
    print(f"[gpu] absorption_d dims={dims.as_tuple()}", flush=True)
    D = _cn(np.random.default_rng(dims.nqz), dims.d_shape)
    got = sse.absorption_d(torch.from_numpy(D).cuda()).cpu().numpy()
    assert np.array_equal(got, oracle.absorption_d(dims, D))


SHAPES = [
    (Dims(nkz=7, ne=21, nqz=7, nw=10, na=6, nb=4, norb=10, g_slots=1), 1, ("fp64", "fp16x2")),   # matrix-core kernels
    (Dims(nkz=3, ne=11, nqz=3, nw=4, na=6, nb=3, norb=5, g_slots=2), 2, ("fp64",)),              # vector-ALU kernel
]
CASES = [(d, s, p) for d, s, ps in SHAPES for p in ps]


@pytest.mark.parametrize("dims,seed,precision", CASES, ids=[f"s{s}-{p}" for _, s, p in CASES])
def test_lesser_sigma_with_absorption_branch(dims, seed, precision):
    print(f"[gpu] Sigma< with the absorption branch dims={dims.as_tuple()} precision={precision}", flush=True)
    rng = np.random.default_rng(seed)
    G = anti_hermitian_blocks(_cn(rng, dims.g_shape))
    Dl, Dg = _cn(rng, dims.d_shape), _cn(rng, dims.d_shape)
    dH = _cn(rng, dims.dh_shape, 0.1)
    nbr = make_nbr(rng, dims.na, dims.nb)
    alpha = 0.2 + 0.9j
    t = {k: torch.from_numpy(v).cuda() for k, v in dict(G=G, Dl=Dl, Dg=Dg, dH=dH, nbr=nbr).items()}
    Dm = sse.absorption_d(t["Dg"])
    S = sse.forward_signed(t["G"], t["Dl"], Dm, t["dH"], t["nbr"], alpha=alpha, precision=precision).cpu().numpy()
    ref = oracle.sse_forward_signed(dims, G, Dl, oracle.absorption_d(dims, Dg), dH, nbr, alpha=alpha)
    err = _rel(S, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= TOL[precision]


def test_absorption_rejects_overlapping_buffers():
    """Checked before any launch: the same buffer, or one shifted by one entry."""
    d = Dims(nkz=3, ne=1, nqz=3, nw=2, na=4, nb=2, norb=1, g_slots=1)
    D = torch.zeros(d.d_shape, dtype=torch.complex128, device="cuda")
    lib = _lib.load()
    cd = _lib.SSEDims.of(d)
    for off in (0, 16):
        rc = lib.sse_absorption_d(ctypes.byref(cd), ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(D.data_ptr() + off),
                                  None)
        assert rc == _lib.SSE_ERR_DIMS
        assert "overlaps" in _lib.last_error()
