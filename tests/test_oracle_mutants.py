"""The oracle's pins have teeth: plausible slips planted in a copy of the
oracle (on the CPU) each make at least one pin fail.

Every mutant is a one-line textual change of ``oracle/sse_oracle.c``
(applied to its first occurrence, which is the forward loop nest), compiled
with gcc into a temporary directory.  The mutated sources never leave the
temporary directory.
"""
import os

import pytest

from oracle import oracle
import test_oracle_pins as pins
import test_oracle_signed_pins as signed_pins

MUTANTS = {
    "k_plus_q": ("((k - q) % d->nkz + d->nkz) % d->nkz", "((k + q) % d->nkz + d->nkz) % d->nkz"),
    "one_energy_branch": ("for (int s = +1; s >= -1; s -= 2)", "for (int s = +1; s >= 1; s -= 2)"),
    "freq_index": ("c_at(D, off_D(d, q, m - 1, a, n, i, j))", "c_at(D, off_D(d, q, m % d->nw, a, n, i, j))"),
    "d_ij_swapped": ("c_at(D, off_D(d, q, m - 1, a, n, i, j))", "c_at(D, off_D(d, q, m - 1, a, n, j, i))"),
    "transpose_not_adjoint": ("c_conj(c_at(Y, c * N + u))", "c_at(Y, c * N + u)"),
    "adjoint_wrong_index": ("c_conj(c_at(Y, c * N + u))", "c_conj(c_at(Y, u * N + c))"),
    "self_not_neighbour": ("const int64_t b = nbr[a * d->nb + n];", "const int64_t b = a;"),
    "wrong_slot": ("* d->gs + 0)", "* d->gs + (d->gs > 1 ? 1 : 0))"),
    "no_alpha": ("cplx v = c_mul(alpha, acc[x]);", "cplx v = acc[x];"),
    "energy_edge": ("if (ep < 0 || ep >= d->ne) continue;", "if (ep < 1 || ep >= d->ne) continue;"),
    "first_neighbour_only": ("for (int64_t n = 0; n < d->nb; ++n) {", "for (int64_t n = 0; n < 1; ++n) {"),
    "right_product": ("mat_mul(N, A + 2 * off_A(d, a, n, i), Gb, T);", "mat_mul(N, Gb, A + 2 * off_A(d, a, n, i), T);"),
    "two_directions": ("for (int i = 0; i < 3; ++i) {\n                        mat_mul", "for (int i = 0; i < 2; ++i) {\n                        mat_mul"),
    "signed_tables_swapped": ("const double* D = s > 0 ? Dp : Dm;", "const double* D = s > 0 ? Dm : Dp;"),
    "signed_one_table": ("const double* D = s > 0 ? Dp : Dm;", "const double* D = Dp;"),
}


def _pin_checks(lib):
    """Run every forward pin against `lib`; return the names of the pins that fail."""
    failed = []
    checks = [
        ("closed_form_a", lambda: pins.test_shifted_delta_closed_form_bit_exact(lib, 0, 1, 0, 0, 0)),
        ("closed_form_b", lambda: pins.test_shifted_delta_closed_form_bit_exact(lib, 2, 3, 1, 1, 2)),
        ("closed_form_c", lambda: pins.test_shifted_delta_closed_form_bit_exact(lib, 1, 5, 0, 0, 2)),
        ("convolution_a", lambda: pins.test_single_ij_reduces_to_library_convolution(lib, 5, 1, 2, 2)),
        ("convolution_b", lambda: pins.test_single_ij_reduces_to_library_convolution(lib, 1, 2, 1, 1)),
        ("anti_hermitian", lambda: pins.test_anti_hermitian_output(lib, 1j, "anti")),
        ("homogeneity", lambda: pins.test_homogeneity_and_linearity(lib)),
        ("ne1_zero", lambda: pins.test_single_energy_point_is_zero(lib)),
        ("signed_closed_form", lambda: signed_pins.test_single_block_closed_form_bit_exact(lib, 0, 4, 1, 2, 0, 0, 1)),
        ("signed_reversal", lambda: signed_pins.test_energy_reversal_swaps_the_tables(lib)),
        ("signed_brute_force", lambda: signed_pins.test_brute_force_python_loops(lib)),
    ]
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_all_pins():
    assert _pin_checks(oracle.Bound(oracle.current_lib_path())) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert old in src, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    path = tmp_path / f"mut_{name}.c"
    path.write_text(mutated)
    so = str(tmp_path / f"libmut_{name}.so")
    oracle.build(src=str(path), out=so)
    failed = _pin_checks(oracle.Bound(so))
    assert failed, f"mutant {name} passed every pin"


# Slips in the phonon self-energy (Eq. 4) part of the oracle, checked against its own pins.
import test_oracle_pse_pins as pse_pins

PSE_MUTANTS = {
    "pse_k_minus_q": ("const int64_t ks = (k + q) % d->nkz;", "const int64_t ks = ((k - q) % d->nkz + d->nkz) % d->nkz;"),
    "pse_freq_off_by_one": ("const int64_t es = e + w;", "const int64_t es = e + w - 1;"),
    "pse_transpose_not_adjoint": ("c_conj(c_at(X, t * N + r))", "c_at(X, t * N + r)"),
    "pse_go_at_atom": ("const double* Gob = Go + 2 * off_G(d, k, e, b);", "const double* Gob = Go + 2 * off_G(d, k, e, a);"),
    "pse_same_component": ("const double* Gob = Go + 2 * off_G(d, k, e, b);", "const double* Gob = Gs + 2 * off_G(d, k, e, b);"),
    "pse_trace_transposed": ("c_at(Gob, u * N + r)", "c_at(Gob, r * N + u)"),
    "pse_no_beta": ("const cplx v = c_mul(beta, acc[x]);", "const cplx v = acc[x];"),
    "pse_energy_edge": ("if (es >= d->ne) continue;", "if (es >= d->ne - 1) continue;"),
    "pse_ij_swapped": ("acc[i * 3 + j] = c_add(acc[i * 3 + j], tr);", "acc[j * 3 + i] = c_add(acc[j * 3 + i], tr);"),
}


def _pse_pin_checks(lib):
    failed = []
    checks = [
        ("closed_form_a", lambda: pse_pins.test_delta_inputs_closed_form_bit_exact(lib, 2, 5, 1, 3, 1, 2, 1)),
        ("closed_form_b", lambda: pse_pins.test_delta_inputs_closed_form_bit_exact(lib, 0, 8, 2, 7, 2, 1, 2)),
        ("dense", lambda: pse_pins.test_brute_force_dense_einsum(lib)),
        ("correlate", lambda: pse_pins.test_textbook_reduction_to_correlate(lib)),
        ("anti_hermitian", lambda: pse_pins.test_anti_hermitian_for_anti_hermitian_inputs(lib)),
        ("homogeneity", lambda: pse_pins.test_linearity_and_homogeneity(lib)),
        ("ne1_zero", lambda: pse_pins.test_single_energy_point_is_zero(lib)),
    ]
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_pse_pins():
    assert _pse_pin_checks(oracle.Bound(oracle.current_lib_path())) == []


@pytest.mark.parametrize("name", sorted(PSE_MUTANTS))
def test_pse_mutant_is_caught(tmp_path, name):
    old, new = PSE_MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / f"libmut_{name}.so")
    oracle.build(src=str(path), out=so)
    failed = _pse_pin_checks(oracle.Bound(so))
    assert failed, f"mutant {name} passed every pin"


# Slips in the full Eq. 3 input contract (stored grad H_ba, adjoint over signed
# frequencies), checked against their own pins.
import test_oracle_f1_pins as f1_pins

F1_MUTANTS = {
    "ba_transposed": ("c_at(Y, u * N + c)", "c_at(Y, c * N + u)"),
    "ba_conjugated": ("c_at(Y, u * N + c)", "c_conj(c_at(Y, u * N + c))"),
    "ba_ignored": ("if (Aba)\n", "if (0)\n"),
    "adjoint_dD_tables_swapped": ("double* dD = s > 0 ? dDp : dDm;", "double* dD = s > 0 ? dDm : dDp;"),
    "adjoint_terms_tables_swapped": ("const double* D = s > 0 ? Dp : Dm;\n                        double* dD",
                                     "const double* D = s > 0 ? Dm : Dp;\n                        double* dD"),
    "adjoint_dG_tables_swapped": ("const double* D = s > 0 ? Dp : Dm;\n                                double* dB",
                                  "const double* D = s > 0 ? Dm : Dp;\n                                double* dB"),
}


def _f1_pin_checks(lib):
    failed = []
    checks = [
        ("explicit_hermitian", lambda: f1_pins.test_explicit_hermitian_right_factor_is_bitwise_the_default(lib)),
        ("closed_form_a", lambda: f1_pins.test_closed_form_with_independent_right_factor(lib, 0, 1, 0, 0, 2)),
        ("closed_form_b", lambda: f1_pins.test_closed_form_with_independent_right_factor(lib, 2, 3, 2, 1, 0)),
        ("linear", lambda: f1_pins.test_linear_in_right_factor(lib)),
        ("dense", lambda: f1_pins.test_right_factor_matches_dense_einsum(lib)),
        ("adjoint_dot", lambda: f1_pins.test_signed_adjoint_dot_products(lib, 1j)),
        ("adjoint_fd", lambda: f1_pins.test_signed_adjoint_grad_H_central_difference_exact(lib)),
        ("adjoint_dense", lambda: f1_pins.test_signed_adjoint_matches_dense_autograd(lib)),
        ("adjoint_one_table", lambda: f1_pins.test_signed_adjoint_reduces_to_one_table(lib)),
    ]
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_f1_pins():
    assert _f1_pin_checks(oracle.Bound(oracle.current_lib_path())) == []


@pytest.mark.parametrize("name", sorted(F1_MUTANTS))
def test_f1_mutant_is_caught(tmp_path, name):
    old, new = F1_MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / f"libmut_{name}.so")
    oracle.build(src=str(path), out=so)
    failed = _f1_pin_checks(oracle.Bound(so))
    assert failed, f"mutant {name} passed every pin"
