"""The oracle's pins catch plausible mistakes (no GPU).

Each case copies the oracle's C source to a temporary folder, plants one mistake there (a dropped
conjugate, a wrong sign, a transposed operand, a skipped step ...), builds the copy and runs a
selection of the pins against it. At least one pin must fail for every planted mistake, so the
pins would have caught that mistake in the oracle itself. The committed oracle is not touched.
"""
import os
import subprocess

import pytest

import test_nonhermitian_cpu as nh
import test_nonunitary_cpu as nu
import test_oracle_pins as pins
from oracle import build as obuild
from oracle import oracle as O

# (name, original text, planted text), or (name, [(original, planted), ...], None)
MUTANTS = [
    ("dot without conjugate", "s += conj(a[i]) * b[i];", "s += a[i] * b[i];"),
    ("derivative sign", "cplx cg = deriv ? -0.5 * I * c : -I * s;",
     "cplx cg = deriv ? 0.5 * I * c : -I * s;"),
    ("rotation sign alpha=+1/2", "cplx cg = deriv ? -0.5 * I * c : -I * s;",
     "cplx cg = deriv ? 0.5 * I * c : I * s;"),
    ("half angle dropped", "double c = cos(0.5 * theta), s = sin(0.5 * theta);",
     "double c = cos(theta), s = sin(theta);"),
    ("adjoint not applied", "if (adj) adjoint(nq == 1 ? 2 : 4, m);", "(void)adj;"),
    ("adjoint without conjugate", "t[a][b] = conj(m[b][a]);", "t[a][b] = m[b][a];"),
    ("lambda never un-applied", "if (k > 0) apply_gate(bra, n, g, theta, 1);", "(void)0;"),
    ("lambda un-applied before the product",
     [("    apply_gate_inverse(ket, n, g, theta);\n    for (int j = 0; j < gate_nparams(g->kind); ++j, ++slot) {",
       "    apply_gate_inverse(ket, n, g, theta); if (k > 0) apply_gate(bra, n, g, theta, 1);\n"
       "    for (int j = 0; j < gate_nparams(g->kind); ++j, ++slot) {"),
      ("    }\n    if (k > 0) apply_gate(bra, n, g, theta, 1);\n  }\n  free(ket); free(bra); free(work);\n  return ORC_OK;",
       "    }\n  }\n  free(ket); free(bra); free(work);\n  return ORC_OK;")], None),
    ("Pauli Y sign", "{{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},",
     "{{{0, 0}, {0, 1}}, {{0, -1}, {0, 0}}},"),
    ("two-qubit local index transposed", "int64_t idx[4] = {j, j | b1, j | b0, j | b0 | b1};",
     "int64_t idx[4] = {j, j | b0, j | b1, j | b0 | b1};"),
    ("factor 2 dropped", "grad[g->p[j]] += 2.0 * creal(z);", "grad[g->p[j]] += creal(z);"),
    ("imaginary part taken", "grad[g->p[j]] += 2.0 * creal(z);",
     "grad[g->p[j]] += 2.0 * cimag(z);"),
    ("repeated parameter overwritten", "grad[g->p[j]] += 2.0 * creal(z);",
     "grad[g->p[j]] = 2.0 * creal(z);"),
    ("Pauli coefficient dropped", "for (int64_t j = 0; j < dim; ++j) out[j] += c * tmp[j];",
     "for (int64_t j = 0; j < dim; ++j) out[j] += tmp[j];"),
    ("one-qubit row mixed up", "psi[j | bit] = m[1][0] * a + m[1][1] * b;",
     "psi[j | bit] = m[0][1] * a + m[1][1] * b;"),
    ("derivative on phi before the undo",
     [("    apply_gate_inverse(ket, n, g, theta);\n    for (int j = 0; j < gate_nparams(g->kind); ++j, ++slot) {",
       "    for (int j = 0; j < gate_nparams(g->kind); ++j, ++slot) {"),
      ("    }\n    if (k > 0) apply_gate(bra, n, g, theta, 1);\n  }\n  free(ket); free(bra); free(work);\n  return ORC_OK;",
       "    }\n    apply_gate_inverse(ket, n, g, theta);\n    if (k > 0) apply_gate(bra, n, g, theta, 1);\n"
       "  }\n  free(ket); free(bra); free(work);\n  return ORC_OK;")],
     None),
    ("reference gradient re-applies U_i",
     "apply_range(x, n, gates, i + 1, n_gates, theta);",
     "apply_range(x, n, gates, i, n_gates, theta);"),
    ("Hadamard sign", "m[1][1] = -M_SQRT1_2;", "m[1][1] = M_SQRT1_2;"),
    ("U3 phase", "m[0][0] = c; m[0][1] = -el * s; m[1][0] = ef * s; m[1][1] = efl * c;",
     "m[0][0] = c; m[0][1] = -ef * s; m[1][0] = el * s; m[1][1] = efl * c;"),
    ("controlled derivative keeps the control-0 block", "if (!d) m[0][0] = m[1][1] = 1;",
     "m[0][0] = m[1][1] = 1;"),
    ("phase derivative missing i", "if (d) m[1][1] = I * cexp(I * th[0]);",
     "if (d) m[1][1] = cexp(I * th[0]);"),
    ("inner product off by one", "for (int64_t i = 0; i < len; ++i) s += conj(a[i]) * b[i];",
     "for (int64_t i = 0; i + 1 < len; ++i) s += conj(a[i]) * b[i];"),
    ("non-Hermitian: conjugate on the A^dag run (the literal App. B.4 rule)",
     "const cplx d = conj(za[p]) + zd[p];", "const cplx d = za[p] + conj(zd[p]);"),
    ("non-Hermitian: second run with A instead of A^dag",
     "cim, -1.0, zd, &ed);", "cim, 1.0, zd, &ed);"),
    ("non-Hermitian: imaginary coefficients dropped",
     "const cplx c = cre[t] + I * (cim ? cim[t] : 0.0);", "const cplx c = cre[t];"),
    ("non-unitary: phi un-done by the adjoint", "  if (gate_unitary(g->kind)) {\n    adjoint(",
     "  if (1) {\n    adjoint("),
    ("non-unitary: lambda un-done by the inverse",
     "if (k > 0) apply_gate(bra, n, g, theta, 1);", "if (k > 0) apply_gate_inverse(bra, n, g, theta);"),
    ("non-unitary: derivative sign", "cg = d ? -0.5 * ch : -sh;", "cg = d ? 0.5 * ch : -sh;"),
]


def _pin_suite():
    """Pins run against each mutant (a cross-section of test_oracle_pins)."""
    suite = []
    for seed in (0, 1):
        suite.append((pins.test_closed_form_single_qubit, dict(seed=seed)))
    suite.append((pins.test_ry_under_z_and_x, dict(theta=1.0)))
    suite.append((pins.test_closed_form_two_qubits, dict(a=0.9)))
    suite.append((pins.test_scalable_closed_form, dict(n=5)))
    for kind in pins.ALL_KINDS:
        suite.append((pins.test_gate_matrix_vs_expm, dict(kind=kind)))
    for kind in (pins.W.PHASE, pins.W.CRY, pins.W.U3, pins.W.RZZ):
        suite.append((pins.test_derivative_matrix_vs_difference_quotient, dict(kind=kind)))
    suite.append((pins.test_pauli_sum_apply_vs_kron, dict(seed=0)))
    for seed in range(4):
        suite.append((pins.test_algorithms_vs_dense, dict(seed=seed)))
    suite.append((pins.test_repeated_parameters_sum, {}))
    suite.append((pins.test_hermitian_energy_is_real, {}))
    suite.append((nh.test_worked_example_rx_under_lowering, {}))
    suite.append((nh.test_linear_in_the_operator, dict(seed=0)))
    suite.append((nu.test_closed_forms, dict(t=0.3)))
    suite.append((nu.test_mixed_circuits_against_dense, dict(seed=0)))
    return suite


def _build_mutant(tmp_path, original, planted):
    src = open(obuild.SRC).read()
    edits = original if isinstance(original, list) else [(original, planted)]
    mutated = src
    for a, b in edits:
        assert mutated.count(a) >= 1, f"mutation anchor not found: {a!r}"
        mutated = mutated.replace(a, b, 1)
    c = tmp_path / "mut.c"
    c.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"],
                   check=True)
    return str(so)


def test_pristine_copy_passes_the_suite(tmp_path):
    so = _build_mutant(tmp_path, "int orc_num_threads(void) {", "int orc_num_threads(void) {")
    with O.using(so):
        for fn, kw in _pin_suite():
            fn(O, **kw)


@pytest.mark.parametrize("name,original,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, original, planted):
    so = _build_mutant(tmp_path, original, planted)
    failed = []
    with O.using(so):
        for fn, kw in _pin_suite():
            try:
                fn(O, **kw)
            except (AssertionError, ValueError, FloatingPointError):
                failed.append(fn.__name__)
                break
    assert failed, f"no pin caught the planted mistake '{name}'"
    os.remove(so)
