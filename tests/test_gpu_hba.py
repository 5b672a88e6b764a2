"""GPU parity of the full Eq. 3 input contract (sse_forward_ex): a stored right
factor grad_j H_ba unrelated to grad_j H^H, on every kernel family and
precision, with one or two coefficient tables, against the oracle's
sse_forward_ex; and the explicit Hermitian right factor against sse_forward."""
import numpy as np
import pytest
import torch

from oracle import oracle
from paper_1912_10024_amd import sse
from paper_1912_10024_amd.inputs import CONFIGS, CONFIG_INDEX, Dims, anti_hermitian_blocks, generate, make_nbr

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6, "fp16x2": 1e-6, "bf16x2": 5e-5}


def _rand(d: Dims, seed: int):
    rng = np.random.default_rng(seed)

    def cn(shape, s=1.0):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s

    return dict(G=anti_hermitian_blocks(cn(d.g_shape)), Dp=cn(d.d_shape), Dm=cn(d.d_shape), dH=cn(d.dh_shape, 0.1),
                dHba=cn(d.dh_shape, 0.1), nbr=make_nbr(rng, d.na, d.nb))


def _rel(x, y):
    return float(np.linalg.norm((x - y).ravel()) / max(np.linalg.norm(y.ravel()), 1e-300))


SHAPES = [
    (Dims(nkz=7, ne=21, nqz=7, nw=10, na=5, nb=4, norb=10, g_slots=1), 1, ("fp64", "fp32", "bf16x2", "fp16x2")),
    (Dims(nkz=7, ne=13, nqz=7, nw=10, na=4, nb=3, norb=10, g_slots=2), 2, ("fp64", "fp16x2")),          # nb 3
    (Dims(nkz=3, ne=19, nqz=3, nw=2, na=9, nb=4, norb=4, g_slots=1), 3, ("fp64", "fp32", "bf16x2")),    # small instance
    (Dims(nkz=3, ne=11, nqz=3, nw=4, na=6, nb=3, norb=5, g_slots=2), 4, ("fp64",)),                      # vector-ALU kernel
]
CASES = [(d, s, p, two) for d, s, ps in SHAPES for p in ps for two in (False, True)]


@pytest.mark.parametrize("dims,seed,precision,two", CASES,
                         ids=[f"s{s}-{p}-{'two' if two else 'one'}" for _, s, p, two in CASES])
def test_stored_right_factor_matches_oracle(dims, seed, precision, two):
    print(f"[gpu] forward_ex dims={dims.as_tuple()} seed={seed} precision={precision} two_tables={two}", flush=True)
    inp = _rand(dims, seed)
    alpha = -0.4 + 0.9j
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    Dm = t["Dm"] if two else t["Dp"]
    out = torch.full(dims.sigma_shape, complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")
    S = sse.forward_ex(t["G"], t["Dp"], t["dH"], t["nbr"], Dm=Dm, dHba=t["dHba"], alpha=alpha, precision=precision,
                       out=out)
    torch.cuda.synchronize()
    got = S.cpu().numpy()
    ref = oracle.sse_forward_ex(dims, inp["G"], inp["Dp"], inp["Dm"] if two else inp["Dp"], inp["dH"], inp["dHba"],
                                inp["nbr"], alpha=alpha)
    err = _rel(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert np.isfinite(got).all()
    assert err <= TOL[precision]


@pytest.mark.parametrize("dims", [SHAPES[0][0], SHAPES[3][0]], ids=["mfma", "generic"])
def test_explicit_hermitian_right_factor(dims):
    inp = _rand(dims, 7)
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    herm = t["dH"].conj().transpose(-1, -2).contiguous()
    S1 = sse.forward(t["G"], t["Dp"], t["dH"], t["nbr"])
    S2 = sse.forward_ex(t["G"], t["Dp"], t["dH"], t["nbr"], dHba=herm)
    torch.cuda.synchronize()
    assert _rel(S2.cpu().numpy(), S1.cpu().numpy()) <= 1e-14


def test_mid_config_sampled_blocks():
    d = CONFIGS["mid"]
    print(f"[gpu] forward_ex mid sampled parity dims={d.as_tuple()}", flush=True)
    inp = generate(d, CONFIG_INDEX["mid"], which=("nbr", "G<", "D<", "D>", "dH"))
    rng = np.random.default_rng(41)
    dHba = 0.1 * (rng.standard_normal(d.dh_shape) + 1j * rng.standard_normal(d.dh_shape))
    t = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    tb = torch.from_numpy(dHba).cuda()
    pts = [(0, 0, 0), (d.nkz - 1, d.ne - 1, d.na - 1), (3, 5, 17), (6, d.ne - 3, 1000)]
    pts += [tuple(int(x) for x in (rng.integers(d.nkz), rng.integers(d.ne), rng.integers(d.na))) for _ in range(16)]
    ref = oracle.sse_points_ex(d, inp["G<"], inp["D<"], inp["D>"], inp["dH"], dHba, inp["nbr"], pts)
    idx = torch.tensor(pts, device="cuda")
    for precision in ("fp64", "fp16x2"):
        S = sse.forward_ex(t["G<"], t["D<"], t["dH"], t["nbr"], Dm=t["D>"], dHba=tb, precision=precision)
        got = S[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
        err = _rel(got, ref)
        print(f"  {precision} sampled rel err {err:.3e}", flush=True)
        assert err <= TOL[precision]
        del S
