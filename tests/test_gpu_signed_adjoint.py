"""GPU parity of the adjoint over signed frequencies (sse_backward_signed: dG,
dDp, dDm, d gradH) against the oracle's signed adjoint on every kernel family,
the reduction to the one-table adjoint, and central finite differences of the
autograd Function at h = 1e-6."""
import numpy as np
import pytest
import torch

from oracle import oracle
from paper_1912_10024_amd import sse
from paper_1912_10024_amd.inputs import Dims, anti_hermitian_blocks, make_nbr

pytestmark = pytest.mark.gpu


def _rand(d: Dims, seed: int):
    rng = np.random.default_rng(seed)

    def cn(shape, s=1.0):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s

    return dict(G=anti_hermitian_blocks(cn(d.g_shape)), Dp=cn(d.d_shape), Dm=cn(d.d_shape), dH=cn(d.dh_shape, 0.1),
                nbr=make_nbr(rng, d.na, d.nb), W=cn(d.sigma_shape))


def _rel(x, y):
    return float(np.linalg.norm((x - y).ravel()) / max(np.linalg.norm(y.ravel()), 1e-300))


SHAPES = [
    Dims(nkz=7, ne=17, nqz=7, nw=10, na=6, nb=4, norb=10, g_slots=2),   # matrix-core dD, nb 4
    Dims(nkz=7, ne=12, nqz=7, nw=10, na=5, nb=3, norb=10, g_slots=1),   # matrix-core dD, nb 3
    Dims(nkz=3, ne=16, nqz=3, nw=2, na=16, nb=4, norb=4, g_slots=3),    # tiny workload shape
    Dims(nkz=3, ne=11, nqz=3, nw=4, na=6, nb=3, norb=5, g_slots=2),     # odd shape
]


@pytest.mark.parametrize("dims", SHAPES, ids=[f"s{i}" for i in range(len(SHAPES))])
def test_signed_adjoint_matches_oracle(dims):
    print(f"[gpu] backward_signed dims={dims.as_tuple()}", flush=True)
    inp = _rand(dims, 3)
    alpha = 0.6 - 0.8j
    gS = np.ascontiguousarray(np.conj(np.swapaxes(inp["W"], -1, -2)))
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    got = sse.backward_signed(t["G"], t["Dp"], t["Dm"], t["dH"], t["nbr"], torch.from_numpy(gS).cuda(), alpha=alpha)
    ref = oracle.sse_backward_signed(dims, inp["G"], inp["Dp"], inp["Dm"], inp["dH"], inp["nbr"], gS, alpha=alpha)
    for name, g, r in zip(("dG", "dDp", "dDm", "ddH"), got, ref):
        err = _rel(g.cpu().numpy(), r)
        print(f"  {name} rel err {err:.3e}", flush=True)
        assert err <= 1e-12


def test_signed_adjoint_skips_and_reduces_to_one_table():
    d = SHAPES[0]
    inp = _rand(d, 4)
    gS = torch.from_numpy(np.ascontiguousarray(np.conj(np.swapaxes(inp["W"], -1, -2)))).cuda()
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    dG, dDp, dDm, ddH = sse.backward_signed(t["G"], t["Dp"], t["Dp"].clone(), t["dH"], t["nbr"], gS)
    rG, rD, rH = sse.backward(t["G"], t["Dp"], t["dH"], t["nbr"], gS)
    assert _rel(dG.cpu().numpy(), rG.cpu().numpy()) <= 1e-14
    assert _rel(ddH.cpu().numpy(), rH.cpu().numpy()) <= 1e-14
    assert _rel((dDp + dDm).cpu().numpy(), rD.cpu().numpy()) <= 1e-14
    only = sse.backward_signed(t["G"], t["Dp"], t["Dm"], t["dH"], t["nbr"], gS, need=(False, False, True, False))
    assert only[0] is None and only[1] is None and only[3] is None
    full = sse.backward_signed(t["G"], t["Dp"], t["Dm"], t["dH"], t["nbr"], gS)
    assert torch.equal(only[2], full[2])


def test_signed_autograd_central_differences():
    """The autograd Function against central differences at h = 1e-6: the Sigma
    blocks are differenced first and then contracted with W (the loss is linear
    in G, Dp, Dm and quadratic in grad H, so the only error is rounding)."""
    d = SHAPES[0]
    inp = _rand(d, 5)
    W = torch.from_numpy(inp["W"]).cuda()
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items() if k != "W"}
    leaves = {k: t[k].clone().requires_grad_(True) for k in ("G", "Dp", "Dm", "dH")}
    S = sse.sse_signed(leaves["G"], leaves["Dp"], leaves["Dm"], leaves["dH"], t["nbr"], alpha=1j)
    L = torch.einsum("kearc,keacr->", W, S).real
    L.backward()
    rng = np.random.default_rng(9)
    h = 1e-6
    for name in ("G", "Dp", "Dm", "dH"):
        grad = leaves[name].grad
        x = t[name]
        gmax, worst = 0.0, 0.0
        for _ in range(16):
            idx = tuple(int(rng.integers(s)) for s in x.shape)
            if name == "G":
                idx = idx[:3] + (0,) + idx[4:]  # slot 0 is the one the forward reads
            for part, unit in (("re", 1.0), ("im", 1j)):
                xp, xm = x.clone(), x.clone()
                xp[idx] += h * unit
                xm[idx] -= h * unit
                args = {k: t[k] for k in ("G", "Dp", "Dm", "dH")}
                args[name] = xp
                Sp = sse.forward_ex(args["G"], args["Dp"], args["dH"], t["nbr"], Dm=args["Dm"], alpha=1j)
                args[name] = xm
                Sm = sse.forward_ex(args["G"], args["Dp"], args["dH"], t["nbr"], Dm=args["Dm"], alpha=1j)
                fd = float(torch.einsum("kearc,keacr->", W, (Sp - Sm) / (2 * h)).real)
                g = grad[idx]
                an = float(g.real if part == "re" else g.imag)
                gmax = max(gmax, abs(an))
                worst = max(worst, abs(fd - an))
        print(f"  {name}: max |fd - grad| {worst:.3e} (max |grad| {gmax:.3e})", flush=True)
        assert worst <= 1e-7 * max(gmax, 1.0)
