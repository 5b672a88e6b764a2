"""The half-precision scheme on the CPU: why normalisation matters.

Sec. "Mixed-Precision Computation" and the mixed-precision convergence results
of the paper report that FP16 products with magnitude-based normalisation
stay within ~1e-6 of the double-precision result while unscaled FP16 is
orders of magnitude worse.  This test reproduces that finding for the
operand rounding of the fp16 hi/lo form, emulated in numpy: the P.D
regrouping of Eq. 3 is evaluated in float64 from operands rounded to
fp16 hi + lo, once with the power-of-two normalisation (per atom for D, per
source point for P) and once without, on inputs whose magnitudes put P in
the fp16 subnormal range.  The exact P.D evaluation is first pinned to the
oracle, so the differences come from the rounding alone.

The same is done for the single-term scheme as the paper describes it (one fp16
term per operand): the left products X = grad H . G, grad H, P and D are each
rounded once to fp16, after power-of-two factors (per atom for D and grad H, per
source point and row for X) or without them (magnitudes beyond fp16's range
clamped to 65504).  This is the arithmetic of the SSE_FP16 and
SSE_FP16_UNSCALED forms.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1912_10024_amd.inputs import Dims, anti_hermitian_blocks, make_nbr


def _inputs(dims, seed, g_scale):
    rng = np.random.default_rng(seed)

    def cn(shape, s=1.0):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s

    return dict(G=anti_hermitian_blocks(cn(dims.g_shape, g_scale)), D=cn(dims.d_shape),
                dH=cn(dims.dh_shape, 0.1), nbr=make_nbr(rng, dims.na, dims.nb))


def _split16(x):
    """x ~ hi + lo with hi = fp16(x), lo = fp16(x - hi), per real part."""
    def one(v):
        h = v.astype(np.float16).astype(np.float64)
        lo = (v - h).astype(np.float16).astype(np.float64)
        return h + lo
    return one(x.real) + 1j * one(x.imag)


def _pow2_scale(m, t):
    """Power of two s with m * s in [2^(t-1), 2^t), elementwise (1 where m == 0)."""
    m = np.asarray(m, dtype=np.float64)
    e = np.frexp(np.where(m > 0, m, 1.0))[1]
    return np.where(m > 0, np.ldexp(1.0, t - e), 1.0)


def _maxpart(x, axes):
    return np.maximum(np.abs(x.real), np.abs(x.imag)).max(axis=axes)


def _pd_sigma(inp, dims, alpha, mode):
    """P.D regrouping of Eq. 3 in float64; mode None (exact), 'unscaled' or 'scaled'."""
    G, D, dH, nbr = inp["G"], inp["D"], inp["dH"], inp["nbr"]
    Gb = G[:, :, nbr, 0]                                          # [k', e', a, n, t, u]
    P = np.einsum("anirt,keantu,anjcu->keanijrc", dH, Gb, dH.conj(), optimize=True)
    Dx = D
    if mode == "unscaled":
        P, Dx = _split16(P), _split16(D)
    elif mode == "scaled":
        sd = _pow2_scale(_maxpart(D, (0, 1, 3, 4, 5)), 7)[None, None, :, None, None, None]
        Dx = _split16(D * sd) / sd
        sp = _pow2_scale(_maxpart(P, (3, 4, 5, 6, 7)), 13)[:, :, :, None, None, None, None, None]
        P = _split16(P * sp) / sp
    return _stencil(P, Dx, dims, alpha)


def _stencil(P, Dx, dims, alpha):
    """Sigma from P[k', E', a, n, i, j, r, c] and D: the (q, w, +/-) sums of Eq. 3 in float64."""
    nkz, ne, nw = dims.nkz, dims.ne, dims.nw
    out = np.zeros(dims.sigma_shape, dtype=np.complex128)
    for q in range(dims.nqz):
        Pq = np.roll(P, q, axis=0)                                # P[(k - q) mod Nkz]
        for w in range(1, nw + 1):
            V = np.einsum("anij,keanijrc->kearc", Dx[q, w - 1], Pq, optimize=True)
            out[:, w:] += V[:, :ne - w]                           # E - w -> E
            out[:, :ne - w] += V[:, w:]                           # E + w -> E
    return alpha * out


def _r16(x, clamp=False):
    """Round each real part to fp16 through fp32; clamp=True first limits it to
    the largest finite fp16 value."""
    def one(v):
        v = v.astype(np.float32)
        if clamp:
            v = np.clip(v, -65504.0, 65504.0)
        return v.astype(np.float16).astype(np.float64)
    return one(x.real) + 1j * one(x.imag)


def _single_term_sigma(inp, dims, alpha, normalised):
    """Eq. 3 with every dense-product operand rounded once to fp16."""
    G, D, dH, nbr = inp["G"], inp["D"], inp["dH"], inp["nbr"]
    Gb = G[:, :, nbr, 0]                                          # [k', e', a, n, t, u]
    if normalised:
        sd = _pow2_scale(_maxpart(D, (0, 1, 3, 4, 5)), 7)[None, None, :, None, None, None]
        sh = _pow2_scale(_maxpart(dH, (1, 2, 3, 4)), 1)
    else:
        sd, sh = np.ones((1, 1, dims.na, 1, 1, 1)), np.ones(dims.na)
    Hs = dH * sh[:, None, None, None, None]
    X = np.einsum("anirt,keantu->keanriu", Hs, Gb, optimize=True)  # fp64 left products, row r
    if normalised:   # per (k', E', a, r): largest part over (n, i, u) below 2^XT
        xt = 14 - int(np.ceil(np.log2(4 * dims.norb)))
        sx = _pow2_scale(_maxpart(X, (3, 5, 6)), xt)               # [k', e', a, r]
    else:
        sx = np.ones(X.shape[:3] + (X.shape[4],))
    Xr = _r16(X * sx[:, :, :, None, :, None, None], not normalised)
    P = _r16(np.einsum("keanriu,anjcu->keanijrc", Xr, _r16(Hs, not normalised).conj(), optimize=True),
             not normalised)
    P = P / (sx[:, :, :, None, None, None, :, None] * (sh ** 2)[None, None, :, None, None, None, None, None])
    return _stencil(P, _r16(D * sd, not normalised) / sd, dims, alpha)


DIMS = Dims(nkz=3, ne=12, nqz=3, nw=2, na=6, nb=3, norb=4, g_slots=1)


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def test_pd_regrouping_matches_oracle(oracle_lib):
    inp = _inputs(DIMS, 3, 1.0)
    ref = oracle.sse_forward(DIMS, inp["G"], inp["D"], inp["dH"], inp["nbr"], alpha=1j)
    assert _rel(_pd_sigma(inp, DIMS, 1j, None), ref) <= 1e-13


@pytest.mark.parametrize("g_scale", [1e-4, 3e-5])
def test_unscaled_fp16_is_far_worse(oracle_lib, g_scale):
    inp = _inputs(DIMS, 4, g_scale)
    ref = oracle.sse_forward(DIMS, inp["G"], inp["D"], inp["dH"], inp["nbr"], alpha=1j)
    e_scaled = _rel(_pd_sigma(inp, DIMS, 1j, "scaled"), ref)
    e_unscaled = _rel(_pd_sigma(inp, DIMS, 1j, "unscaled"), ref)
    print(f"[fp16 scheme] G x{g_scale:g}: normalised {e_scaled:.2e}, unscaled {e_unscaled:.2e}")
    assert e_scaled <= 1e-6
    assert e_unscaled >= 1e-4
    assert e_unscaled >= 100 * e_scaled


@pytest.mark.parametrize("sg,sd", [(1.0, 1.0), (1e-5, 1.0), (1e-3, 1e-6), (1e3, 1e5)])
def test_single_term_scheme(oracle_lib, sg, sd):
    """One fp16 term per operand: with the factors, four roundings of at most
    2^-11 bound the error by 4 * 2^-11 at any magnitude; without them it is the
    same on inputs of order one and an order of magnitude worse or more once the
    left products fall into fp16's subnormal range or D passes 65504."""
    inp = _inputs(DIMS, 5, 1.0)
    inp["G"], inp["D"] = inp["G"] * sg, inp["D"] * sd
    ref = oracle.sse_forward(DIMS, inp["G"], inp["D"], inp["dH"], inp["nbr"], alpha=1j)
    e_norm = _rel(_single_term_sigma(inp, DIMS, 1j, True), ref)
    e_raw = _rel(_single_term_sigma(inp, DIMS, 1j, False), ref)
    print(f"[fp16 single-term scheme] G x{sg:g} D x{sd:g}: normalised {e_norm:.2e}, unscaled {e_raw:.2e}")
    assert 1e-5 <= e_norm <= 4 * 2.0 ** -11
    if sg == 1.0 and sd == 1.0:
        assert e_raw <= 4 * 2.0 ** -11
    else:
        assert e_raw >= 10 * e_norm
