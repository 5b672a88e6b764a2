"""The paper's half-precision scheme without compensation, on the GPU.

Sec. "Mixed-Precision Computation" rounds the operands of the dense products to
one half-precision term after normalising them by magnitude factors, and
accumulates in double precision; Sec. "Mixed-Precision Convergence" compares
this with the same scheme without scaling D and G.  SSE_FP16 and
SSE_FP16_UNSCALED are those two legs (one fp16 term per operand, fp32 sums per
K chunk, fp64 reduction), run by the split 16-bit kernel with the lo terms
dropped.  Each test prints the measured error against the fp64 oracle.

The bar of the normalised single-term form: every Sigma term passes through four
roundings to fp16 (X = grad H . G, grad H, P = X . grad H^H, D), each with
relative error at most u = 2^-11 for normalised operands, so the relative error
stays below 4u (about 2e-3); the reduction itself is in fp64.
"""
import numpy as np
import pytest
import torch

from oracle import oracle
from paper_1912_10024_amd import sse
from paper_1912_10024_amd.inputs import CONFIGS, Dims, generate, make_nbr, anti_hermitian_blocks

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11
TOL_SINGLE = 4 * U16


def _rand(dims: Dims, seed: int):
    rng = np.random.default_rng(seed)

    def cn(shape, s=1.0):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s

    return dict(G=anti_hermitian_blocks(cn(dims.g_shape)), D=cn(dims.d_shape), dH=cn(dims.dh_shape, 0.1),
                nbr=make_nbr(rng, dims.na, dims.nb))


def _rel(S, ref):
    return float(np.linalg.norm(S - ref) / np.linalg.norm(ref))


def _run(inp, precision, sg=1.0, sd=1.0, sh=1.0):
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    return sse.forward(t["G"] * sg, t["D"] * sd, t["dH"] * sh, t["nbr"], alpha=1j, precision=precision).cpu().numpy()


@pytest.mark.parametrize("precision", ["fp16", "fp16_unscaled"])
@pytest.mark.parametrize("dims,seed", [
    (CONFIGS["tiny"], 0),
    (Dims(nkz=7, ne=29, nqz=7, nw=10, na=6, nb=4, norb=10, g_slots=5), 1),
    (Dims(nkz=7, ne=17, nqz=7, nw=10, na=5, nb=3, norb=10, g_slots=1), 2),
    (Dims(nkz=7, ne=5, nqz=7, nw=10, na=5, nb=4, norb=10, g_slots=1), 3),
], ids=["tiny", "ragged", "odd_nb", "ne5"])
def test_single_term_error_on_unit_inputs(precision, dims, seed):
    """Inputs of order one keep every operand in fp16's normal range, so both
    legs stay within the single-term bar and clearly above the two-term form's
    error (the lo terms are really dropped)."""
    inp = _rand(dims, seed)
    ref = oracle.sse_forward(dims, inp["G"], inp["D"], inp["dH"], inp["nbr"], alpha=1j)
    rel = _rel(_run(inp, precision), ref)
    rel2 = _rel(_run(inp, "fp16x2"), ref)
    print(f"[fp16 single] {precision} dims={dims.as_tuple()} rel_frob={rel:.3e} (fp16x2 {rel2:.3e})")
    assert rel <= TOL_SINGLE
    assert rel >= 20 * rel2


def test_single_term_mid_sampled():
    d = CONFIGS["mid"]
    inp = generate(d, 1)
    t = {k: torch.from_numpy(inp[k]).cuda() for k in ("G<", "D<", "dH", "nbr")}
    S = sse.forward(t["G<"], t["D<"], t["dH"], t["nbr"], precision="fp16")
    rng = np.random.default_rng(5)
    pts = [tuple(int(x) for x in (rng.integers(d.nkz), rng.integers(d.ne), rng.integers(d.na))) for _ in range(24)]
    ref = oracle.sse_points(d, inp["G<"], inp["D<"], inp["dH"], inp["nbr"], pts)
    got = np.stack([S[k, e, a].cpu().numpy() for k, e, a in pts])
    rel = _rel(got, ref)
    print(f"[fp16 single] fp16 mid sampled rel_frob={rel:.3e}")
    assert rel <= TOL_SINGLE


@pytest.mark.parametrize("sg,sd,sh", [(1e-5, 1.0, 1.0), (1e-3, 1e-6, 1.0), (1e3, 1e5, 1.0)],
                         ids=["small_G", "small_G_and_D", "large_G_and_D"])
def test_unscaled_is_far_worse(sg, sd, sh):
    """The paper's finding on the hardware: at magnitudes outside fp16's normal
    range (left products and P in the subnormal range, or D beyond 65504 and
    clamped), the unscaled leg loses accuracy by an order of magnitude or more
    while the normalised leg keeps its bar.  Sigma is linear in G and D and
    quadratic in grad H, so the reference is the oracle's result for the
    unscaled inputs times sg * sd * sh^2."""
    dims = Dims(nkz=7, ne=29, nqz=7, nw=10, na=6, nb=4, norb=10, g_slots=1)
    inp = _rand(dims, 21)
    ref = oracle.sse_forward(dims, inp["G"], inp["D"], inp["dH"], inp["nbr"], alpha=1j) * (sg * sd * sh * sh)
    e_norm = _rel(_run(inp, "fp16", sg, sd, sh), ref)
    e_raw = _rel(_run(inp, "fp16_unscaled", sg, sd, sh), ref)
    print(f"[fp16 single] G x{sg:g} D x{sd:g} dH x{sh:g}: normalised {e_norm:.3e}, unscaled {e_raw:.3e}")
    assert e_norm <= TOL_SINGLE
    assert e_raw >= 10 * e_norm


def test_single_term_refuses_two_tables():
    d = CONFIGS["tiny"]
    t = {k: torch.from_numpy(v).cuda() for k, v in _rand(d, 0).items()}
    with pytest.raises(RuntimeError, match="status 4"):
        sse.forward_signed(t["G"], t["D"], 0.5 * t["D"], t["dH"], t["nbr"], precision="fp16")
