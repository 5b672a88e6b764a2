"""Flop and byte counts of the scattering self-energy contraction.

Counting convention of the paper's computation model (Sec. "Performance
Model", "Computation Model"): one complex Norb x Norb matrix product costs
8*Norb^3 flops.
"""
from __future__ import annotations

N3D = 3


def f_eff(d) -> float:
    """Effective (algorithmic) flops of one Sigma component (one of lesser/greater).

    The regrouped form the paper arrives at after fission: one left product
    X = grad_i H . G per (k', E', a, n, i) and one product X . Y per
    (k, E, a, n, i, q, w, +/-):  8 Norb^3 * N3D * Nb * Na * Nkz * NE * (2 Nqz Nw + 1).
    """
    return 8.0 * d.norb ** 3 * N3D * d.nb * d.na * d.nkz * d.ne * (2 * d.nqz * d.nw + 1)


def omen_sse_flops(na, nb, nkz, nqz, ne, nw, norb) -> float:
    """The paper's count for the original OMEN SSE kernel (both components)."""
    return 64.0 * na * nb * N3D * nkz * nqz * ne * nw * norb ** 3


def dace_sse_flops(na, nb, nkz, nqz, ne, nw, norb, extra: int = 1) -> float:
    """OMEN count reduced by 2 Nqz Nw / (Nqz Nw + extra).

    The text states extra=1; the printed table is reproduced with extra=3.
    """
    return omen_sse_flops(na, nb, nkz, nqz, ne, nw, norb) * (nqz * nw + extra) / (2.0 * nqz * nw)


def pd_gemm_flops(d) -> float:
    """Real flops of the dense complex GEMM the HIP path runs on matrix cores.

    Per atom, V[(k, w), (E', r, c)] = sum_{(k', n, i, j)} D_a[k - k', w, n, i, j] P[k', E', n, i, j, r, c]:
    M = Nkz * Nw, K = Nkz * Nb * 9, N = NE * Norb^2, 8 flops per complex MAC.
    """
    return 8.0 * d.na * (d.nkz * d.nw) * (d.nkz * d.nb * 9) * (d.ne * d.norb ** 2)


def pd_left_flops(d) -> float:
    """Real flops of forming P = grad_i H . G . grad_j H^H (3 + 9 products per (k', E', a, n))."""
    return 8.0 * d.norb ** 3 * 12 * d.nb * d.na * d.nkz * d.ne


def pd_mfma_flops(d) -> float:
    """Useful real flops the forward issues on the matrix cores: the P.D GEMM plus
    the nine right products P_ij = X_i . grad_j H^H per (k', E', a, n)."""
    return pd_gemm_flops(d) + 8.0 * d.norb ** 3 * 9 * d.nb * d.na * d.nkz * d.ne


def pd_useful_flops(d) -> float:
    """The regrouped form's useful flops: the P.D GEMM plus the twelve Norb^3
    products per (k', E', a, n) that form P (X = grad_i H . G on the vector ALUs,
    P = X . grad_j H^H on the matrix cores); on MI355X the fp64 vector ALUs and
    matrix cores share the 78.6 TFLOP/s peak."""
    return pd_gemm_flops(d) + pd_left_flops(d)


def split16_mfma_flops(d) -> float:
    """Flops the split 16-bit forms issue on the 16-bit matrix cores: the four
    hi/lo partial products of the P.D GEMM and of the nine right products P =
    X . grad_j H^H (the X rows stay on the fp64 vector ALUs)."""
    return 4.0 * pd_mfma_flops(d)


def single16_mfma_flops(d) -> float:
    """Flops the single-term fp16 forms issue on the 16-bit matrix cores: they run
    the split kernel with the lo terms zero, so the P tiles issue the four partial
    products of the split forms and the P.D GEMM keeps one of its two
    instructions (hi parts of D against the (hi, lo) pairs of P: twice the GEMM's
    useful flops)."""
    return 2.0 * pd_gemm_flops(d) + 4.0 * (pd_mfma_flops(d) - pd_gemm_flops(d))


def pd_stencil_flops(d) -> float:
    """Real adds of the (w, +/-) energy stencil: 2 complex adds per valid (k, E, w, s, r, c)."""
    valid = 0
    for e in range(d.ne):
        for w in range(1, d.nw + 1):
            valid += (0 <= e - w < d.ne) + (0 <= e + w < d.ne)
    return 2.0 * d.na * d.nkz * valid * d.norb ** 2


def pd_executed_flops(d) -> float:
    return pd_gemm_flops(d) + pd_left_flops(d) + pd_stencil_flops(d)


def min_bytes(d) -> float:
    """Compulsory HBM traffic of one forward call: read G slot 0, D, grad H, nbr; write Sigma."""
    blk = d.norb * d.norb * 16
    g = d.nkz * d.ne * d.na * blk
    sig = g
    dd = d.nqz * d.nw * d.na * d.nb * 9 * 16
    dh = d.na * d.nb * N3D * blk
    return float(g + sig + dd + dh + d.na * d.nb * 4)


def pse_contraction_flops(d) -> float:
    """Real flops of the phonon self-energy contraction (Eq. 4): per valid
    (q, w, k, E, a, n), E + w < NE, the nine traces sum_{s,t} Gs[s][t] T_ij[t][s],
    9 Norb^2 complex MACs at 8 flops each."""
    valid = d.nkz * d.nqz * sum(max(d.ne - w, 0) for w in range(1, d.nw + 1))
    return 8.0 * 9 * d.norb ** 2 * d.na * d.nb * valid


def pse_formation_flops(d) -> float:
    """Real flops of T_ij = grad_j H . Go . grad_i H^H: 3 + 9 products per (k, E, a, n)."""
    return 8.0 * d.norb ** 3 * 12 * d.nb * d.na * d.nkz * d.ne


def pse_flops(d) -> float:
    """Useful fp64 flops of one phonon self-energy call (one of Pi< / Pi>)."""
    return pse_contraction_flops(d) + pse_formation_flops(d)


def adjoint_dgdh_flops(d) -> float:
    """Useful fp64 flops of the dG / d gradH part of one adjoint call: per edge
    (a, n), momentum k' and energy E', Y_ij = sum_{q,w} conj(alpha D_ij[q,w]) W[k'+q, w, E']
    (9 Nqz Nw complex products of Norb^2 entries) and the 27 complex Norb^3
    products built on it: U_m = sum_j Y_mj A_j (9), T_m = sum_i A_i^H Y_im (9),
    the dG term sum_j T_j A_j (3) and the d gradH terms U_m B^H and T_m^H B (6)."""
    per = 8.0 * d.norb ** 2 * (9 * d.nqz * d.nw + 27 * d.norb)
    return per * d.na * d.nb * d.nkz * d.ne
