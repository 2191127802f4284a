/*
 * qsv_oracle.c -- CPU test oracle for the reverse-mode energy gradient.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, complex128 statement of what the GPU
 * library computes. Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it; the library never does, and the two share no code (this file includes no header of the
 * library and repeats the few interface codes it needs).
 *
 * Source: T. Jones and J. Gacon, "Efficient calculation of gradients in classical simulations of
 * variational quantum algorithms" (arXiv:2009.02823).
 *   - energy <E> = <in| U^dag H U |in>, U = U_G ... U_1 ......................... Sec. 2.2
 *   - reverse-mode gradient: the phi/lambda recurrence of Sec. 2.2, walked backwards . Algorithm 1
 *   - reference O(P^2) gradient, one re-simulation per entry .... Eq. (reference_gradient), Alg. 2
 *   - rotation derivative dR/dtheta = alpha i G R(theta), alpha = -1/2 ............ Appendix A
 *   - phase-gate and controlled-gate derivatives ................................. Appendix A
 *   - several parameters in one gate: one clone/derivative/product per parameter . Algorithm 3
 *   - repeated parameters: entries of one parameter are summed .......... App. B.2, Algorithm 4
 *   - non-Hermitian operator A: Algorithm 1 with the complex <lambda|mu> as the entry, run once
 *     with A and once with A^dag; d<A>/dtheta = conj(g_A) + g_{A^dag} .................. App. B.4
 *     (read with the conjugate on the A run: <dpsi|A|psi> = conj(<psi|A^dag|dpsi>))
 *   - non-unitary invertible gates: phi is un-done by M^-1, lambda by M^dag ......... App. B.3
 *     (here the imaginary-time rotations exp(-theta G/2), G = X, Y, Z; M^-1 by the 2x2 inverse)
 * Fixed (parameter-free) gates are un-applied from phi and lambda like any other gate and give no
 * gradient entry (the recurrences of Sec. 2.2 hold for any unitary).
 *
 * Conventions: qubit q is bit q of an amplitude index; a two-qubit gate on (q0, q1) uses the local
 * basis index 2*bit(q0) + bit(q1), q0 being the control of controlled gates; |in> defaults to
 * |0...0>. Gate matrices are built from their definitions and applied as dense 2x2 / 4x4 blocks;
 * the Hamiltonian is applied term by term, one Pauli factor (a 2x2 matrix) at a time.
 *
 * Inner products use pairwise summation over fixed power-of-two blocks, so the result does not
 * depend on the number of OpenMP threads.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* qsv_gate_kind codes of the C-ABI (an interface format; repeated, not included) */
enum {
  K_RX = 0, K_RY, K_RZ, K_H, K_X, K_Y, K_Z, K_S, K_CNOT, K_CZ,
  K_PHASE, K_CRX, K_CRY, K_CRZ, K_RXX, K_RYY, K_RZZ, K_U3, K_T, K_SDG,
  K_NRX, K_NRY, K_NRZ, K_NKINDS
};

typedef struct {
  int32_t kind, q0, q1, p[3];
} orc_gate;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* ------------------------------------------------------------------------------------------ */
/* Gate matrices                                                                              */
/* ------------------------------------------------------------------------------------------ */

static void pauli(int code, cplx m[2][2]) {
  /* 0 = I, 1 = X, 2 = Y, 3 = Z */
  static const double r[4][2][2][2] = {
      {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}},
      {{{0, 0}, {1, 0}}, {{1, 0}, {0, 0}}},
      {{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},
      {{{1, 0}, {0, 0}}, {{0, 0}, {-1, 0}}},
  };
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) m[a][b] = r[code][a][b][0] + I * r[code][a][b][1];
}

static void kron2(cplx a[2][2], cplx b[2][2], cplx out[4][4]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) out[2 * i + k][2 * j + l] = a[i][j] * b[k][l];
}

/* R_G(theta) = exp(-i theta G / 2) = cos(theta/2) 1 - i sin(theta/2) G for an involutory G
   (G^2 = 1), and its derivative -sin(theta/2)/2 1 - (i/2) cos(theta/2) G, which equals
   alpha i G R_G(theta) with alpha = -1/2 (Appendix A). dim = 2 or 4. */
static void rotation(int dim, cplx G[4][4], double theta, int deriv, cplx out[4][4]) {
  double c = cos(0.5 * theta), s = sin(0.5 * theta);
  double ci = deriv ? -0.5 * s : c;   /* coefficient of the identity */
  cplx cg = deriv ? -0.5 * I * c : -I * s; /* coefficient of G */
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) out[a][b] = (a == b ? ci : 0.0) + cg * G[a][b];
}

static int gate_nparams(int kind) {
  switch (kind) {
    case K_RX: case K_RY: case K_RZ: case K_PHASE: case K_CRX: case K_CRY: case K_CRZ:
    case K_RXX: case K_RYY: case K_RZZ: case K_NRX: case K_NRY: case K_NRZ:
      return 1;
    case K_U3:
      return 3;
    default:
      return 0;
  }
}

static int gate_unitary(int kind) { return kind != K_NRX && kind != K_NRY && kind != K_NRZ; }

static int gate_nqubits(int kind) {
  switch (kind) {
    case K_CNOT: case K_CZ: case K_CRX: case K_CRY: case K_CRZ: case K_RXX: case K_RYY:
    case K_RZZ:
      return 2;
    default:
      return 1;
  }
}

/* Matrix of gate g (deriv < 0) or of its partial derivative with respect to its deriv-th
   parameter, written into m (2x2 in the top-left corner for one-qubit gates). */
static int gate_matrix(const orc_gate* g, const double* theta, int deriv, cplx m[4][4]) {
  memset(m, 0, sizeof(cplx) * 16);
  double th[3] = {0, 0, 0};
  for (int j = 0; j < gate_nparams(g->kind); ++j) th[j] = theta[g->p[j]];
  int d = deriv >= 0;
  cplx P[2][2], Q[2][2], G4[4][4], R2[4][4];
  switch (g->kind) {
    case K_RX: case K_RY: case K_RZ: {
      pauli(g->kind - K_RX + 1, P);
      cplx G[4][4] = {{P[0][0], P[0][1]}, {P[1][0], P[1][1]}};
      rotation(2, G, th[0], d, m);
      return 1;
    }
    case K_NRX: case K_NRY: case K_NRZ: {
      /* exp(-theta G/2) = cosh(theta/2) 1 - sinh(theta/2) G (G involutory): invertible, not
         unitary; derivative sinh(theta/2)/2 1 - cosh(theta/2)/2 G = -(1/2) G M (App. B.3) */
      pauli(g->kind - K_NRX + 1, P);
      const double ch = cosh(0.5 * th[0]), sh = sinh(0.5 * th[0]);
      const double ci = d ? 0.5 * sh : ch, cg = d ? -0.5 * ch : -sh;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) m[a][b] = (a == b ? ci : 0.0) + cg * P[a][b];
      return 1;
    }
    case K_H:
      m[0][0] = m[0][1] = m[1][0] = M_SQRT1_2;
      m[1][1] = -M_SQRT1_2;
      return 1;
    case K_X: case K_Y: case K_Z:
      pauli(g->kind - K_X + 1, P);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) m[a][b] = P[a][b];
      return 1;
    case K_S:
      m[0][0] = 1; m[1][1] = I;
      return 1;
    case K_SDG:
      m[0][0] = 1; m[1][1] = -I;
      return 1;
    case K_T:
      m[0][0] = 1; m[1][1] = cexp(I * M_PI / 4);
      return 1;
    case K_PHASE:
      /* diag(1, e^{i theta}); derivative i e^{i theta} |1><1| (Appendix A) */
      if (d) m[1][1] = I * cexp(I * th[0]);
      else { m[0][0] = 1; m[1][1] = cexp(I * th[0]); }
      return 1;
    case K_U3: {
      /* U3(t, f, l) = [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]] */
      double t = th[0], f = th[1], l = th[2];
      double c = cos(0.5 * t), s = sin(0.5 * t);
      cplx ef = cexp(I * f), el = cexp(I * l), efl = cexp(I * (f + l));
      if (!d) {
        m[0][0] = c; m[0][1] = -el * s; m[1][0] = ef * s; m[1][1] = efl * c;
      } else if (deriv == 0) {
        m[0][0] = -0.5 * s; m[0][1] = -el * 0.5 * c; m[1][0] = ef * 0.5 * c; m[1][1] = -efl * 0.5 * s;
      } else if (deriv == 1) {
        m[1][0] = I * ef * s; m[1][1] = I * efl * c;
      } else {
        m[0][1] = -I * el * s; m[1][1] = I * efl * c;
      }
      return 1;
    }
    case K_CNOT:
      m[0][0] = m[1][1] = m[2][3] = m[3][2] = 1;
      return 2;
    case K_CZ:
      m[0][0] = m[1][1] = m[2][2] = 1; m[3][3] = -1;
      return 2;
    case K_CRX: case K_CRY: case K_CRZ: {
      /* |0><0| (x) 1 + |1><1| (x) R_G(theta); derivative |1><1| (x) dR_G (Appendix A) */
      pauli(g->kind - K_CRX + 1, P);
      cplx G[4][4] = {{P[0][0], P[0][1]}, {P[1][0], P[1][1]}};
      rotation(2, G, th[0], d, R2);
      if (!d) m[0][0] = m[1][1] = 1;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) m[2 + a][2 + b] = R2[a][b];
      return 2;
    }
    case K_RXX: case K_RYY: case K_RZZ: {
      /* exp(-i theta (s (x) s) / 2) for s = X, Y, Z (a rotation about a Pauli product) */
      pauli(g->kind - K_RXX + 1, P);
      pauli(g->kind - K_RXX + 1, Q);
      kron2(P, Q, G4);
      rotation(4, G4, th[0], d, m);
      return 2;
    }
    default:
      return 0;
  }
}

static void adjoint(int dim, cplx m[4][4]) {
  cplx t[4][4];
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) t[a][b] = conj(m[b][a]);
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) m[a][b] = t[a][b];
}

/* ------------------------------------------------------------------------------------------ */
/* State-vector primitives: apply a matrix, clone, inner product                              */
/* ------------------------------------------------------------------------------------------ */

/* psi <- M psi for M acting on qubit q (2x2). Every index j with bit q clear names one pair. */
static void apply_1q(cplx* psi, int n, int q, cplx m[4][4]) {
  const int64_t dim = (int64_t)1 << n, bit = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < dim; ++j) {
    if (j & bit) continue;
    cplx a = psi[j], b = psi[j | bit];
    psi[j] = m[0][0] * a + m[0][1] * b;
    psi[j | bit] = m[1][0] * a + m[1][1] * b;
  }
}

/* psi <- M psi for M acting on qubits (q0, q1) (4x4, local index 2 bit(q0) + bit(q1)). */
static void apply_2q(cplx* psi, int n, int q0, int q1, cplx m[4][4]) {
  const int64_t dim = (int64_t)1 << n, b0 = (int64_t)1 << q0, b1 = (int64_t)1 << q1;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < dim; ++j) {
    if (j & (b0 | b1)) continue;
    int64_t idx[4] = {j, j | b1, j | b0, j | b0 | b1};
    cplx v[4], w[4];
    for (int k = 0; k < 4; ++k) v[k] = psi[idx[k]];
    for (int r = 0; r < 4; ++r) {
      w[r] = 0;
      for (int k = 0; k < 4; ++k) w[r] += m[r][k] * v[k];
    }
    for (int k = 0; k < 4; ++k) psi[idx[k]] = w[k];
  }
}

static void apply_matrix(cplx* psi, int n, const orc_gate* g, int nq, cplx m[4][4]) {
  if (nq == 1) apply_1q(psi, n, g->q0, m);
  else apply_2q(psi, n, g->q0, g->q1, m);
}

/* psi <- U psi (adj = 0) or psi <- U^dag psi (adj = 1) */
static void apply_gate(cplx* psi, int n, const orc_gate* g, const double* theta, int adj) {
  cplx m[4][4];
  int nq = gate_matrix(g, theta, -1, m);
  if (adj) adjoint(nq == 1 ? 2 : 4, m);
  apply_matrix(psi, n, g, nq, m);
}

/* psi <- U^-1 psi: the adjoint for unitary gates; for the non-unitary one-qubit gates the 2x2
   inverse (1/(ad - bc)) [[d, -b], [-c, a]] of App. B.3 (the phi recurrence of Sec. 2.2). */
static void apply_gate_inverse(cplx* psi, int n, const orc_gate* g, const double* theta) {
  cplx m[4][4];
  int nq = gate_matrix(g, theta, -1, m);
  if (gate_unitary(g->kind)) {
    adjoint(nq == 1 ? 2 : 4, m);
  } else {
    const cplx a = m[0][0], b = m[0][1], c = m[1][0], d = m[1][1], det = a * d - b * c;
    m[0][0] = d / det; m[0][1] = -b / det; m[1][0] = -c / det; m[1][1] = a / det;
  }
  apply_matrix(psi, n, g, nq, m);
}

/* psi <- (dU/d theta_{p_j}) psi : a non-unitary matrix (Eq. recurrent_grad, App. A) */
static void apply_derivative(cplx* psi, int n, const orc_gate* g, const double* theta, int j) {
  cplx m[4][4];
  int nq = gate_matrix(g, theta, j, m);
  apply_matrix(psi, n, g, nq, m);
}

static void clone(cplx* dst, const cplx* src, int n) {
  memcpy(dst, src, sizeof(cplx) * ((size_t)1 << n));
}

static cplx dot_pairwise(const cplx* a, const cplx* b, int64_t len) {
  if (len <= 8) {
    cplx s = 0;
    for (int64_t i = 0; i < len; ++i) s += conj(a[i]) * b[i];
    return s;
  }
  int64_t h = len / 2;
  return dot_pairwise(a, b, h) + dot_pairwise(a + h, b + h, len - h);
}

/* <a|b> = sum_j conj(a_j) b_j. Blocks of 2^14 amplitudes are summed pairwise (in parallel), then
   the block sums pairwise; for power-of-two lengths this equals one pairwise sum. */
static cplx inner(const cplx* a, const cplx* b, int n) {
  const int64_t dim = (int64_t)1 << n;
  const int64_t blk = dim < (1 << 14) ? dim : (1 << 14);
  const int64_t nb = dim / blk;
  cplx* part = (cplx*)malloc(sizeof(cplx) * nb);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb; ++i) part[i] = dot_pairwise(a + i * blk, b + i * blk, blk);
  /* pairwise over the block sums */
  int64_t m = nb;
  while (m > 1) {
    int64_t h = m / 2;
    for (int64_t i = 0; i < h; ++i) part[i] = part[2 * i] + part[2 * i + 1];
    if (m & 1) part[h] = part[m - 1];
    m = h + (m & 1);
  }
  cplx s = part[0];
  free(part);
  return s;
}

/* out <- H psi = sum_t c_t P_t psi, each Pauli string applied one factor at a time to a copy of
   psi (tmp), then accumulated. The result is unnormalised (Sec. 2.1: the simulator applies the
   operator of interest to a state and keeps the unnormalised result). */
static void apply_pauli_sum(const cplx* psi, cplx* out, cplx* tmp, int n, int n_terms,
                            const uint8_t* codes, const double* coeffs) {
  const int64_t dim = (int64_t)1 << n;
  memset(out, 0, sizeof(cplx) * dim);
  for (int t = 0; t < n_terms; ++t) {
    clone(tmp, psi, n);
    for (int q = 0; q < n; ++q) {
      int code = codes[(int64_t)t * n + q];
      if (code == 0) continue;
      cplx p2[2][2], m[4][4] = {{0}};
      pauli(code, p2);
      m[0][0] = p2[0][0]; m[0][1] = p2[0][1]; m[1][0] = p2[1][0]; m[1][1] = p2[1][1];
      apply_1q(tmp, n, q, m);
    }
    const double c = coeffs[t];
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < dim; ++j) out[j] += c * tmp[j];
  }
}

/* out <- A psi for A = sum_t (cre_t + i cim_t) P_t, the complex-weighted sum of App. B.4 (Pauli
   strings as above; with cim = NULL the weights are real). */
static void apply_pauli_sum_complex(const cplx* psi, cplx* out, cplx* tmp, int n, int n_terms,
                                    const uint8_t* codes, const double* cre, const double* cim) {
  const int64_t dim = (int64_t)1 << n;
  memset(out, 0, sizeof(cplx) * dim);
  for (int t = 0; t < n_terms; ++t) {
    clone(tmp, psi, n);
    for (int q = 0; q < n; ++q) {
      int code = codes[(int64_t)t * n + q];
      if (code == 0) continue;
      cplx p2[2][2], m[4][4] = {{0}};
      pauli(code, p2);
      m[0][0] = p2[0][0]; m[0][1] = p2[0][1]; m[1][0] = p2[1][0]; m[1][1] = p2[1][1];
      apply_1q(tmp, n, q, m);
    }
    const cplx c = cre[t] + I * (cim ? cim[t] : 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < dim; ++j) out[j] += c * tmp[j];
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Validation                                                                                 */
/* ------------------------------------------------------------------------------------------ */

static int check_inputs(int n, const orc_gate* gates, int n_gates, int n_theta, int n_terms,
                        const uint8_t* codes, const double* coeffs) {
  if (n < 1 || n > 34 || n_gates < 0 || n_theta < 0 || n_terms < 0) return ORC_EINVAL;
  for (int k = 0; k < n_gates; ++k) {
    const orc_gate* g = &gates[k];
    if (g->kind < 0 || g->kind >= K_NKINDS) return ORC_EINVAL;
    int nq = gate_nqubits(g->kind);
    if (g->q0 < 0 || g->q0 >= n) return ORC_EINVAL;
    if (nq == 2 && (g->q1 < 0 || g->q1 >= n || g->q1 == g->q0)) return ORC_EINVAL;
    for (int j = 0; j < gate_nparams(g->kind); ++j)
      if (g->p[j] < 0 || g->p[j] >= n_theta) return ORC_EINVAL;
  }
  if (n_terms && (!codes || !coeffs)) return ORC_EINVAL;
  for (int64_t i = 0; i < (int64_t)n_terms * n; ++i)
    if (codes[i] > 3) return ORC_EINVAL;
  return ORC_OK;
}

static cplx* new_state(int n) { return (cplx*)malloc(sizeof(cplx) * ((size_t)1 << n)); }

static void set_input(cplx* psi, const cplx* in, int n) {
  if (in) {
    clone(psi, in, n);
  } else {
    memset(psi, 0, sizeof(cplx) * ((size_t)1 << n));
    psi[0] = 1;
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Exported entry points (called through ctypes by the tests)                                 */
/* ------------------------------------------------------------------------------------------ */

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* psi <- U_G ... U_1 psi, in place */
int orc_apply_circuit(int n, cplx* psi, const orc_gate* gates, int n_gates, const double* theta,
                      int n_theta, int adjoint_order) {
  if (check_inputs(n, gates, n_gates, n_theta, 0, NULL, NULL)) return ORC_EINVAL;
  if (!adjoint_order) {
    for (int k = 0; k < n_gates; ++k) apply_gate(psi, n, &gates[k], theta, 0);
  } else { /* psi <- U_1^dag ... U_G^dag psi, the inverse circuit */
    for (int k = n_gates - 1; k >= 0; --k) apply_gate(psi, n, &gates[k], theta, 1);
  }
  return ORC_OK;
}

/* psi <- (dU_k / d theta_{p_j}) psi, for tests of the derivative matrices */
int orc_apply_derivative(int n, cplx* psi, const orc_gate* g, const double* theta, int n_theta,
                         int j) {
  if (check_inputs(n, g, 1, n_theta, 0, NULL, NULL)) return ORC_EINVAL;
  if (j < 0 || j >= gate_nparams(g->kind)) return ORC_EINVAL;
  apply_derivative(psi, n, g, theta, j);
  return ORC_OK;
}

/* out <- H psi */
int orc_apply_pauli_sum(int n, const cplx* psi, cplx* out, int n_terms, const uint8_t* codes,
                        const double* coeffs) {
  if (check_inputs(n, NULL, 0, 0, n_terms, codes, coeffs)) return ORC_EINVAL;
  cplx* tmp = new_state(n);
  if (!tmp) return ORC_ENOMEM;
  apply_pauli_sum(psi, out, tmp, n, n_terms, codes, coeffs);
  free(tmp);
  return ORC_OK;
}

/* <a|b> */
int orc_inner(int n, const cplx* a, const cplx* b, double* out_re_im) {
  cplx s = inner(a, b, n);
  out_re_im[0] = creal(s);
  out_re_im[1] = cimag(s);
  return ORC_OK;
}

/* <E> = <psi|H|psi>, psi = U |in> (Sec. 2.2). energy = (Re, Im); Im is a Hermiticity check. */
int orc_energy(int n, const cplx* in, const orc_gate* gates, int n_gates, const double* theta,
               int n_theta, int n_terms, const uint8_t* codes, const double* coeffs,
               double* energy) {
  if (check_inputs(n, gates, n_gates, n_theta, n_terms, codes, coeffs)) return ORC_EINVAL;
  cplx *psi = new_state(n), *hpsi = new_state(n), *tmp = new_state(n);
  if (!psi || !hpsi || !tmp) { free(psi); free(hpsi); free(tmp); return ORC_ENOMEM; }
  set_input(psi, in, n);
  for (int k = 0; k < n_gates; ++k) apply_gate(psi, n, &gates[k], theta, 0);
  apply_pauli_sum(psi, hpsi, tmp, n, n_terms, codes, coeffs);
  cplx e = inner(psi, hpsi, n);
  energy[0] = creal(e);
  energy[1] = cimag(e);
  free(psi); free(hpsi); free(tmp);
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* The gradient through the recurrence of Sec. 2.2                                            */
/* ------------------------------------------------------------------------------------------ */
/*
 * Number the gates k = 1..G, |psi> = U_G ... U_1 |in>, and let B be the operator whose
 * expectation is differentiated (the Hamiltonian, or App. B.4's A or A^dag). Sec. 2.2 defines
 *
 *   |phi_k>    = (U_G ... U_k)^-1 |psi>       the state gate k acts on, U_{k-1} ... U_1 |in>
 *   |lambda_k> = (U_G ... U_{k+1})^dag B|psi>  B|psi> carried back to just after gate k
 *
 * and both follow from their k + 1 neighbours by one gate:
 *
 *   |phi_k> = U_k^-1 |phi_{k+1}>  (|phi_{G+1}> = |psi>),   |lambda_{k-1}> = U_k^dag |lambda_k>
 *   (|lambda_G> = B|psi>).
 *
 * The gradient entry of gate k and its parameter slot j is the product
 * <lambda_k| dU_k/dtheta_j |phi_k> (Eq. recurrent_grad), doubled and made real for a Hermitian B.
 * Walking k from G down to 1 keeps only two states alive plus one work copy for dU_k |phi_k>,
 * which is the reverse mode of Sec. 2.3. U_k^-1 is the adjoint for unitary gates and the 2x2
 * inverse for the non-unitary ones (App. B.3); lambda always takes the adjoint. Several slots in
 * one gate each get their own derivative product (Algorithm 3); products of one parameter are
 * summed (App. B.2).
 */

/* psi <- U_{to-1} ... U_{from} psi  (0-based gate indices, half-open range) */
static void apply_range(cplx* psi, int n, const orc_gate* gates, int from, int to,
                        const double* theta) {
  for (int k = from; k < to; ++k) apply_gate(psi, n, &gates[k], theta, 0);
}

/* <bra| (dU_g / dtheta_{p_j}) |ket>, with the derivative applied to a work copy of ket */
static cplx derivative_product(const cplx* bra, const cplx* ket, cplx* work, int n,
                               const orc_gate* g, const double* theta, int j) {
  clone(work, ket, n);
  apply_derivative(work, n, g, theta, j);
  return inner(bra, work, n);
}

/* Reverse mode for a Hermitian H (Algorithm 1). energy = <psi|H|psi> as (Re, Im), the imaginary
   part being a check only; grad[p] = sum over the slots that use p of 2 Re <lambda_k|dU_k|phi_k>.
   If prods is non-NULL it receives every complex product, gate G first, as (Re, Im) pairs. */
int orc_adjoint_gradient(int n, const cplx* in, const orc_gate* gates, int n_gates,
                         const double* theta, int n_theta, int n_terms, const uint8_t* codes,
                         const double* coeffs, double* energy, double* grad, double* prods) {
  if (check_inputs(n, gates, n_gates, n_theta, n_terms, codes, coeffs)) return ORC_EINVAL;
  cplx *ket = new_state(n), *bra = new_state(n), *work = new_state(n);
  if (!ket || !bra || !work) { free(ket); free(bra); free(work); return ORC_ENOMEM; }
  for (int p = 0; p < n_theta; ++p) grad[p] = 0.0;

  /* simulate psi in the bra buffer, keep it as phi_{G+1} and overwrite the bra with H psi */
  set_input(bra, in, n);
  apply_range(bra, n, gates, 0, n_gates, theta);
  clone(ket, bra, n);
  apply_pauli_sum(ket, bra, work, n, n_terms, codes, coeffs);
  const cplx e = inner(ket, bra, n);
  energy[0] = creal(e);
  energy[1] = cimag(e);

  int64_t slot = 0;
  for (int k = n_gates - 1; k >= 0; --k) {
    const orc_gate* g = &gates[k];
    apply_gate_inverse(ket, n, g, theta);
    for (int j = 0; j < gate_nparams(g->kind); ++j, ++slot) {
      const cplx z = derivative_product(bra, ket, work, n, g, theta, j);
      grad[g->p[j]] += 2.0 * creal(z);
      if (prods) { prods[2 * slot] = creal(z); prods[2 * slot + 1] = cimag(z); }
    }
    if (k > 0) apply_gate(bra, n, g, theta, 1);
  }
  free(ket); free(bra); free(work);
  return ORC_OK;
}

/* The same walk with B = sum (cre + i sign*cim) P and the complex products as entries (App. B.4
   keeps them complex): z[p] = sum of <lambda_k|dU_k|phi_k> over the slots that use p;
   *e = <psi|B|psi>. */
static int complex_products(int n, const cplx* in, const orc_gate* gates, int n_gates,
                            const double* theta, int n_theta, int n_terms, const uint8_t* codes,
                            const double* cre, const double* cim, double sign, cplx* z, cplx* e) {
  cplx *ket = new_state(n), *bra = new_state(n), *work = new_state(n);
  double* cb = (double*)malloc(sizeof(double) * (n_terms ? n_terms : 1));
  if (!ket || !bra || !work || !cb) {
    free(ket); free(bra); free(work); free(cb);
    return ORC_ENOMEM;
  }
  for (int t = 0; t < n_terms; ++t) cb[t] = sign * cim[t];
  for (int p = 0; p < n_theta; ++p) z[p] = 0;
  set_input(bra, in, n);
  apply_range(bra, n, gates, 0, n_gates, theta);
  clone(ket, bra, n);
  apply_pauli_sum_complex(ket, bra, work, n, n_terms, codes, cre, cb);
  *e = inner(ket, bra, n);
  for (int k = n_gates - 1; k >= 0; --k) {
    const orc_gate* g = &gates[k];
    apply_gate_inverse(ket, n, g, theta);
    for (int j = 0; j < gate_nparams(g->kind); ++j)
      z[g->p[j]] += derivative_product(bra, ket, work, n, g, theta, j);
    if (k > 0) apply_gate(bra, n, g, theta, 1);
  }
  free(ket); free(bra); free(work); free(cb);
  return ORC_OK;
}

/* The expectation <A> = <psi|A|psi> of a non-Hermitian A = sum (cre + i cim) P and its complex
   gradient (App. B.4): with g_B[p] the summed complex products of the walk run with operator B,
   d<A>/dtheta_p = <dpsi|A|psi> + <psi|A|dpsi> = conj(g_A[p]) + g_{A^dag}[p].
   energy = (Re, Im); grad = n_theta (Re, Im) pairs. */
int orc_adjoint_gradient_nonhermitian(int n, const cplx* in, const orc_gate* gates, int n_gates,
                                      const double* theta, int n_theta, int n_terms,
                                      const uint8_t* codes, const double* cre, const double* cim,
                                      double* energy, double* grad) {
  if (check_inputs(n, gates, n_gates, n_theta, n_terms, codes, cre)) return ORC_EINVAL;
  if (n_terms && !cim) return ORC_EINVAL;
  cplx *za = (cplx*)malloc(sizeof(cplx) * (n_theta ? n_theta : 1));
  cplx *zd = (cplx*)malloc(sizeof(cplx) * (n_theta ? n_theta : 1));
  if (!za || !zd) { free(za); free(zd); return ORC_ENOMEM; }
  cplx ea, ed;
  int rc = complex_products(n, in, gates, n_gates, theta, n_theta, n_terms, codes, cre,
                            cim, 1.0, za, &ea);                          /* B = A     */
  if (!rc)
    rc = complex_products(n, in, gates, n_gates, theta, n_theta, n_terms, codes, cre,
                          cim, -1.0, zd, &ed);                           /* B = A^dag */
  if (!rc) {
    energy[0] = creal(ea);
    energy[1] = cimag(ea);
    for (int p = 0; p < n_theta; ++p) {
      const cplx d = conj(za[p]) + zd[p];
      grad[2 * p] = creal(d);
      grad[2 * p + 1] = cimag(d);
    }
  }
  free(za); free(zd);
  return rc;
}

/* The reference gradient, Eq. (reference_gradient) evaluated as it stands: for every slot j of
   every gate i, the state U_G ... U_{i+1} (dU_i/dtheta_j) U_{i-1} ... U_1 |in> is simulated from
   scratch and its product with H|psi> taken (H Hermitian, so <psi|H|x> = <H psi|x>). This costs
   O(G) gates per entry, O(G^2) in all, the scheme Sec. 3 compares against. */
int orc_reference_gradient(int n, const cplx* in, const orc_gate* gates, int n_gates,
                           const double* theta, int n_theta, int n_terms, const uint8_t* codes,
                           const double* coeffs, double* grad) {
  if (check_inputs(n, gates, n_gates, n_theta, n_terms, codes, coeffs)) return ORC_EINVAL;
  cplx *hpsi = new_state(n), *x = new_state(n), *work = new_state(n);
  if (!hpsi || !x || !work) { free(hpsi); free(x); free(work); return ORC_ENOMEM; }
  for (int p = 0; p < n_theta; ++p) grad[p] = 0.0;

  set_input(work, in, n);
  apply_range(work, n, gates, 0, n_gates, theta);
  apply_pauli_sum(work, hpsi, x, n, n_terms, codes, coeffs);

  for (int i = 0; i < n_gates; ++i) {
    const orc_gate* g = &gates[i];
    for (int j = 0; j < gate_nparams(g->kind); ++j) {
      set_input(x, in, n);
      apply_range(x, n, gates, 0, i, theta);
      apply_derivative(x, n, g, theta, j);
      apply_range(x, n, gates, i + 1, n_gates, theta);
      grad[g->p[j]] += 2.0 * creal(inner(hpsi, x, n));
    }
  }
  free(hpsi); free(x); free(work);
  return ORC_OK;
}
