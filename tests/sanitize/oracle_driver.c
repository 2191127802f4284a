/* Drives the CPU oracle (test infrastructure) under AddressSanitizer and UndefinedBehaviorSanitizer:
   random small circuits over every gate kind, random Pauli sums, Algorithm 1, Algorithm 2, the
   complex-entry walk of App. B.4, invalid inputs. Built and run by tests/test_sanitize_cpu.py;
   exits non-zero if Algorithm 1 and Algorithm 2 disagree (the sanitizers abort on a finding). */
#include "../../oracle/qsv_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x2009002823ull;
static uint32_t rnd(void) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(rng_state >> 33);
}
static double urand(void) { return (rnd() + 0.5) / 2147483648.0; }

int main(void) {
  for (int trial = 0; trial < 40; ++trial) {
    const int n = 1 + (int)(rnd() % 6);
    const int ng = 1 + (int)(rnd() % 30), nt = 1 + (int)(rnd() % 6);
    orc_gate g[32];
    int np = 0;
    for (int k = 0; k < ng; ++k) {
      int kind = (int)(rnd() % K_NKINDS);
      if (n < 2 && gate_nqubits(kind) == 2) kind = K_RY;
      g[k].kind = kind;
      g[k].q0 = (int)(rnd() % n);
      g[k].q1 = -1;
      if (gate_nqubits(kind) == 2) {
        do g[k].q1 = (int)(rnd() % n); while (g[k].q1 == g[k].q0);
      }
      for (int j = 0; j < 3; ++j) g[k].p[j] = j < gate_nparams(kind) ? np++ : -1;
    }
    double theta[96];
    for (int p = 0; p < np; ++p) theta[p] = 6.283185307179586 * urand();
    uint8_t codes[6 * 6];
    double coeffs[6], cim[6];
    for (int t = 0; t < nt; ++t) {
      for (int q = 0; q < n; ++q) codes[t * n + q] = (uint8_t)(rnd() % 4);
      coeffs[t] = urand() - 0.5;
      cim[t] = urand() - 0.5;
    }
    double e[2], ga[96], gr[96], gc[192], prods[2 * 96];
    if (orc_adjoint_gradient(n, NULL, g, ng, theta, np, nt, codes, coeffs, e, ga, prods)) return 2;
    if (orc_reference_gradient(n, NULL, g, ng, theta, np, nt, codes, coeffs, gr)) return 2;
    if (orc_adjoint_gradient_nonhermitian(n, NULL, g, ng, theta, np, nt, codes, coeffs, cim, e,
                                          gc))
      return 2;
    /* compared on unitary circuits only: un-applying non-unitary gates (App. B.3) amplifies
       rounding by their condition numbers, so the two orders then agree only loosely */
    int unitary = 1;
    for (int k = 0; k < ng; ++k) unitary = unitary && gate_unitary(g[k].kind);
    double scale = 1.0;
    for (int p = 0; p < np; ++p) scale = fmax(scale, fabs(gr[p]));
    for (int p = 0; p < np && unitary; ++p)
      if (fabs(ga[p] - gr[p]) > 1e-10 * scale) {
        fprintf(stderr, "trial %d: Algorithm 1 and 2 differ at %d: %.17g vs %.17g (scale %g)\n",
                trial, p, ga[p], gr[p], scale);
        return 1;
      }
  }
  /* invalid inputs are rejected without reading past the tables */
  orc_gate bad = {K_CNOT, 0, 0, {-1, -1, -1}};
  double e[2], gsink[4];
  uint8_t code = 1;
  double c = 1.0;
  if (orc_adjoint_gradient(2, NULL, &bad, 1, NULL, 0, 1, &code, &c, e, gsink, NULL) != ORC_EINVAL)
    return 3;
  printf("oracle driver: ok\n");
  return 0;
}
