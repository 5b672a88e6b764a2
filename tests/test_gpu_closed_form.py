"""Closed-form cases on the GPU, compared bit for bit (fp64 path).

Sigma (Eq. 3): D a delta at (q0, w0, n0, i0, j0), grad H = I for (n0, i0) and
(n0, j0), alpha = 1: Sigma[k, E, a] = sum over s = +1, -1 of
G[(k - q0) mod Nkz, E - s w0, nbr[a, n0], 0] where that energy is on the grid.
Pi (Eq. 4): Gs one block X at (k1, e1, a0), Go one block Y at (k2, e2,
nbr[a0, n0]), grad H = I for (a0, n0, i0/j0): Pi[q, w-1, a0, n0][i][j] =
beta tr(X Y) where k1 = (k2 + q) mod Nkz and e1 = e2 + w, zero elsewhere.
Integer-valued blocks keep every product and sum exact, so both kernels
(matrix-core and vector-ALU) must reproduce these values exactly."""
import numpy as np
import pytest
import torch

from paper_1912_10024_amd import sse
from paper_1912_10024_amd.inputs import Dims, make_nbr

pytestmark = pytest.mark.gpu

SHAPES = [Dims(nkz=7, ne=23, nqz=7, nw=10, na=6, nb=4, norb=10, g_slots=2),   # matrix-core kernels
          Dims(nkz=7, ne=19, nqz=7, nw=10, na=6, nb=3, norb=10, g_slots=1),   # matrix-core kernels, nb 3
          Dims(nkz=3, ne=11, nqz=3, nw=4, na=6, nb=3, norb=5, g_slots=2)]     # vector-ALU kernels


def _int_blocks(rng, shape):
    return (rng.integers(-4, 5, shape) + 1j * rng.integers(-4, 5, shape)).astype(np.complex128)


@pytest.mark.parametrize("d", SHAPES, ids=["mfma", "mfma_nb3", "generic"])
@pytest.mark.parametrize("q0,w0,n0,i0,j0", [(0, 1, 0, 0, 0), (2, 3, 1, 2, 1)])
def test_sigma_delta_closed_form(d, q0, w0, n0, i0, j0):
    print(f"[gpu] sigma delta dims={d.as_tuple()} q0={q0} w0={w0}", flush=True)
    rng = np.random.default_rng(10 + q0)
    nbr = make_nbr(rng, d.na, d.nb)
    G = _int_blocks(rng, d.g_shape)
    D = np.zeros(d.d_shape, np.complex128)
    D[q0, w0 - 1, :, n0, i0, j0] = 1.0
    dH = np.zeros(d.dh_shape, np.complex128)
    dH[:, n0, i0] = np.eye(d.norb)
    dH[:, n0, j0] = np.eye(d.norb)
    t = [torch.from_numpy(x).cuda() for x in (G, D, dH, nbr)]
    S = sse.forward(*t, alpha=1.0).cpu().numpy()
    want = np.zeros(d.sigma_shape, np.complex128)
    for k in range(d.nkz):
        for e in range(d.ne):
            for a in range(d.na):
                b = nbr[a, n0]
                for s in (1, -1):
                    es = e - s * w0
                    if 0 <= es < d.ne:
                        want[k, e, a] += G[(k - q0) % d.nkz, es, b, 0]
    assert np.array_equal(S, want)


@pytest.mark.parametrize("d", SHAPES, ids=["mfma", "mfma_nb3", "generic"])
def test_phonon_delta_closed_form(d):
    print(f"[gpu] phonon delta dims={d.as_tuple()}", flush=True)
    rng = np.random.default_rng(21)
    nbr = make_nbr(rng, d.na, d.nb)
    a0, n0, i0, j0 = 4, 1, 2, 0
    b0 = int(nbr[a0, n0])
    k1, e1, k2, e2 = 2, 7, 1, 4
    X = _int_blocks(rng, (d.norb, d.norb))
    Y = _int_blocks(rng, (d.norb, d.norb))
    Gs = np.zeros(d.g_shape, np.complex128)
    Go = np.zeros(d.g_shape, np.complex128)
    Gs[k1, e1, a0, 0] = X
    Go[k2, e2, b0, 0] = Y
    Gs[:, :, :, 1:] = 7.0   # slots the equation does not read
    dH = np.zeros(d.dh_shape, np.complex128)
    dH[a0, n0, i0] = np.eye(d.norb)
    dH[a0, n0, j0] = np.eye(d.norb)
    t = [torch.from_numpy(x).cuda() for x in (Gs, Go, dH, nbr)]
    P = sse.phonon_forward(*t, d.nqz, d.nw, beta=1.0).cpu().numpy()
    want = np.zeros(d.d_shape, np.complex128)
    for q in range(d.nqz):
        w = e1 - e2
        if k1 == (k2 + q) % d.nkz and 1 <= w <= d.nw:
            for i in {i0, j0}:
                for j in {i0, j0}:
                    want[q, w - 1, a0, n0, i, j] = np.trace(X @ Y)
    assert np.count_nonzero(want) > 0
    assert np.array_equal(P, want)
