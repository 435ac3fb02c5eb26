"""Mutation check of the oracle pins: plausible mistakes planted in a temporary copy of the oracle's C
source (a transposed operand, a wrong sign, a dropped term, a wrong weight or index, one Taylor term too
few) must each make at least one pin fail. The planted copies live in a temporary directory and are
never used outside this test."""
import os
import subprocess

import pytest

import oracle
import test_curvilinear_oracle as CP
import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "stp_oracle.c")

MUTANTS = {
    "transposed_D": ("acc += M[i * n + j] * u[", "acc += M[j * n + i] * u["),
    "ncp_sign": ("            out[k * m + s] -= acc;", "            out[k * m + s] += acc;"),
    "dropped_flux_term": ("for (int k = 0; k < nn * m; ++k) out[k] -= grad[k] / h;",
                          "for (int k = 0; k < nn * m; ++k) out[k] -= 0.0 * grad[k] / h;"),
    "dropped_inverse_h": ("* (grad[k * m + r] / h);", "* (grad[k * m + r]);"),
    "integral_weight": ("wo *= dt / (double)(o + 2);", "wo *= dt / (double)(o + 1);"),
    "one_term_fewer": ("for (int o = 0; o <= N; ++o) {\n            const double* po",
                       "for (int o = 0; o < N; ++o) {\n            const double* po"),
    "swapped_face_vectors": ("(f % 2) ? e1v : e0v", "(f % 2) ? e0v : e1v"),
    "elastic_lambda_2mu": ("-(lam + 2.0 * mu)", "-(lam + mu)"),
    "elastic_shear_index": ("if (i != d) B[stress_index(d, i) * 9 + i] = -mu;",
                            "if (i != d) B[stress_index(d, i) * 9 + d] = -mu;"),
    "acoustic_rho": ("B[(1 + d) * 4 + 0] = 1.0 / rho;", "B[(1 + d) * 4 + 0] = rho;"),
    "axis_swap": ("int i = axis == 0 ? x : (axis == 1 ? y : z);", "int i = axis == 0 ? x : (axis == 1 ? z : y);"),
    "source_order_shift": ("src[nn + m + o];", "src[nn + m + (o > 0 ? o - 1 : 0)];"),
    "dmatrix_diag": ("diag -= v;", "diag += v;"),
    "face_axis": ("else if (axis == 1) { z = a; y = j; x = b; }", "else if (axis == 1) { z = b; y = j; x = a; }"),
    "curvilinear_metric_transposed": ("acc += G[d * 3 + j] * Mj[j * 81 + k];", "acc += G[j * 3 + d] * Mj[j * 81 + k];"),
    "curvilinear_diagonal_only": ("acc += G[d * 3 + j] * Mj[j * 81 + k];",
                                  "acc += (j == d) * G[d * 3 + j] * Mj[j * 81 + k];"),
    "curvilinear_metric_row": ("acc += G[d * 3 + j] * Mj[j * 81 + k];", "acc += G[d * 3 + j] * Mj[d * 81 + k];"),
}


def _pins():
    """(name, callable) pairs running pin tests against whatever library `oracle` currently uses."""
    o = oracle
    return [
        ("dmatrix", lambda: [P.test_dmatrix_differentiates_polynomials_exactly(o, N) for N in (1, 3, 6)]),
        ("faces", lambda: [P.test_face_vectors(o, N) for N in (1, 4)]),
        ("fig7", lambda: P.test_fig7_fused_y_contraction_layout(o)),
        ("kron", lambda: [P.test_contract_matches_kronecker(o, a) for a in range(3)]),
        ("spectra", lambda: P.test_preset_spectra(o)),
        ("denseV", lambda: [P.test_apply_Vd_matches_dense_kronecker(o, N, k)
                            for N in (1, 2) for k in ("acoustic", "elastic", "generic_A")]),
        ("taylor", lambda: [P.test_taylor_sum_vs_dense_series_and_expm(o, N, k)
                            for N in (1, 2) for k in ("acoustic", "elastic", "generic_A")]),
        ("planewave", lambda: [P.test_polynomial_plane_wave_exact(o, 3, ph, w)
                               for ph, w in ((0, "P"), (1, "P"), (1, "S"))]),
        ("source", lambda: [P.test_point_source_with_zero_operator(o, 3), P.test_point_source_enters_recursion(o)]),
        ("fface", lambda: P.test_fface_is_extrapolated_conservative_flux(o)),
        ("axisperm", lambda: P.test_axis_permutation(o)),
        ("curv_spectrum", lambda: CP.test_curvilinear_spectrum(o)),
        ("curv_affine", lambda: [CP.test_affine_element_polynomial_plane_wave_exact(o, 2, w) for w in ("P", "S")]),
    ]


def _failing_pins(libpath):
    failed = []
    with oracle.using(libpath):
        for name, fn in _pins():
            try:
                fn()
            except (AssertionError, ValueError, FloatingPointError):
                failed.append(name)
    return failed


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(src), "-lm",
                           "-lpthread"])
    return str(lib)


def test_unmutated_copy_passes_all_pins(tmp_path):
    assert _failing_pins(_build(tmp_path, "clean", open(SRC).read())) == []


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_each_planted_mistake_fails_a_pin(tmp_path, mutant):
    text = open(SRC).read()
    old, new = MUTANTS[mutant]
    assert text.count(old) == 1, f"mutation site for {mutant} not unique"
    failed = _failing_pins(_build(tmp_path, mutant, text.replace(old, new)))
    assert failed, f"planted mistake {mutant} was not caught by any pin"
