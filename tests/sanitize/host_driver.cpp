// Drives the library's host-only code under AddressSanitizer and UndefinedBehaviorSanitizer:
// the validators, the fused-pass scheduler (qsv_schedule_describe) over random circuits and every
// geometry, the Pauli planner (qsv_pauli_describe) over random sums, and the tuning cache reader
// on malformed files. Built (host-only) and run by tests/test_sanitize_cpu.py; no GPU is used.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qsv.h"

static uint64_t rng_state = 0x0902823ull;
static uint32_t rnd() {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(rng_state >> 33);
}

static int nparams(int k) {
  if (k == QSV_U3) return 3;
  if (k <= QSV_RZ || k == QSV_PHASE || (k >= QSV_CRX && k <= QSV_RZZ) || k >= QSV_NRX) return 1;
  return 0;
}
static bool two(int k) { return k == QSV_CNOT || k == QSV_CZ || (k >= QSV_CRX && k <= QSV_RZZ); }

int main() {
  const int geoms[][2] = {{2, 6}, {3, 6}, {2, 8}, {3, 8}, {4, 8}, {2, 9}, {3, 9}, {4, 9}};
  for (int trial = 0; trial < 60; ++trial) {
    const int n = 2 + (int)(rnd() % 20);
    const int ng = 1 + (int)(rnd() % 300);
    std::vector<qsv_gate> g(ng);
    int np = 0;
    for (auto& x : g) {
      int k = (int)(rnd() % 23);
      x.kind = k;
      x.q0 = (int)(rnd() % n);
      x.q1 = -1;
      if (two(k)) do x.q1 = (int)(rnd() % n); while (x.q1 == x.q0);
      for (int j = 0; j < 3; ++j) x.param[j] = j < nparams(k) ? np++ : -1;
    }
    if (qsv_validate_circuit(n, g.data(), ng, np) != QSV_OK) {
      std::fprintf(stderr, "valid circuit rejected: %s\n", qsv_last_error());
      return 1;
    }
    // one broken gate is rejected
    std::vector<qsv_gate> b = g;
    b[rnd() % ng].q0 = n + 3;
    if (qsv_validate_circuit(n, b.data(), ng, np) != QSV_ERR_INVALID_ARG) return 1;
    for (const auto& ge : geoms) {
      std::vector<int32_t> order(ng), pass_of(ng), phase_of(ng);
      std::vector<uint64_t> tile(ng), reg(ng);
      for (int back = 0; back < 2; ++back)
        for (int dt = 0; dt < 2; ++dt) {
          qsv_schedule_info info{0, 0, order.data(), pass_of.data(), phase_of.data(),
                                 tile.data(), reg.data(), 0, 0, 0};
          const qsv_status st =
              qsv_schedule_describe(n, g.data(), ng, back, ge[0], ge[1], (qsv_dtype)dt, &info);
          if (st != QSV_OK && st != QSV_ERR_UNSUPPORTED && st != QSV_ERR_INVALID_ARG) return 1;
        }
    }
    const int nt = 1 + (int)(rnd() % 80);
    std::vector<uint8_t> codes((size_t)nt * n);
    std::vector<double> coeffs(nt);
    for (auto& c : codes) c = (uint8_t)(rnd() % 4);
    for (auto& c : coeffs) c = (double)(rnd() % 1000) / 500.0 - 1.0;
    qsv_pauli_sum H{nt, codes.data(), coeffs.data()};
    if (qsv_validate_pauli_sum(n, &H) != QSV_OK) return 1;
    int32_t groups = 0, passes = 0, gather = 0, pg[64];
    uint64_t masks[64];
    for (int dt = 0; dt < 2; ++dt) {
      if (qsv_pauli_describe(n, (qsv_dtype)dt, &H, &groups, &passes, &gather, masks, pg, 64) !=
          QSV_OK)
        return 1;
      int sum = gather;
      for (int i = 0; i < passes && i < 64; ++i) sum += pg[i];
      if (sum != groups) return 1;
    }
    codes[0] = 9;
    if (qsv_validate_pauli_sum(n, &H) != QSV_ERR_INVALID_ARG) return 1;
  }
  // malformed tuning caches load nothing
  const char* path = "sanitize_tune.jsonl";
  FILE* f = std::fopen(path, "w");
  if (!f) return 1;
  std::fprintf(f, "{\"source\": \"%s\", \"key\": \"zz\"\n{bad\n\n", qsv_build_id());
  for (int i = 0; i < 3000; ++i) std::fputc('x', f);
  std::fprintf(f, "\n");
  std::fclose(f);
  int32_t loaded = -1;
  if (qsv_tune_cache_load(path, &loaded) != QSV_OK || loaded != 0) return 1;
  std::remove(path);
  std::printf("host driver: ok\n");
  return 0;
}
