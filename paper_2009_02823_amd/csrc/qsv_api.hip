// C-ABI of the qsv library: argument validation, handles, plan caching and the launch sequences
// of the forward pass, the Hamiltonian application and the reverse sweep (Algorithm 1).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qsv.h"
#include "fused.h"
#include "qsv_internal.h"
#include "sv_kernels.h"

using namespace qsv;

static_assert(sizeof(qsv_gate) == sizeof(GateDesc), "qsv_gate and GateDesc must match");

// ------------------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

static qsv_status fail(qsv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(QSV_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),        \
                  __FILE__, __LINE__);                                                       \
  } while (0)

#define QSV_TRY(expr)                 \
  do {                                \
    qsv_status s_ = (expr);           \
    if (s_ != QSV_OK) return s_;      \
  } while (0)

extern "C" const char* qsv_last_error(void) { return g_last_error.c_str(); }

static constexpr int kMaxQubits = 34;

// ------------------------------------------------------------------------------------------------
// validation (host only)
// ------------------------------------------------------------------------------------------------
extern "C" qsv_status qsv_validate_circuit(int32_t n, const qsv_gate* gates, int32_t n_gates,
                                           int32_t n_theta) {
  if (n < 1 || n > kMaxQubits)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits = %d outside [1, %d]", n, kMaxQubits);
  if (n_gates < 0) return fail(QSV_ERR_INVALID_ARG, "n_gates = %d < 0", n_gates);
  if (n_theta < 0) return fail(QSV_ERR_INVALID_ARG, "n_theta = %d < 0", n_theta);
  if (n_gates > 0 && !gates) return fail(QSV_ERR_INVALID_ARG, "gates is NULL");
  for (int32_t k = 0; k < n_gates; ++k) {
    const qsv_gate& g = gates[k];
    if (g.kind < 0 || g.kind >= K_NKINDS)
      return fail(QSV_ERR_INVALID_ARG, "gate %d: unknown kind %d", k, g.kind);
    if (g.q0 < 0 || g.q0 >= n)
      return fail(QSV_ERR_INVALID_ARG, "gate %d: qubit q0 = %d outside [0, %d)", k, g.q0, n);
    if (kind_nqubits(g.kind) == 2) {
      if (g.q1 < 0 || g.q1 >= n)
        return fail(QSV_ERR_INVALID_ARG, "gate %d: qubit q1 = %d outside [0, %d)", k, g.q1, n);
      if (g.q1 == g.q0)
        return fail(QSV_ERR_INVALID_ARG, "gate %d: two-qubit gate on one qubit %d", k, g.q0);
    } else if (g.q1 != -1) {
      return fail(QSV_ERR_INVALID_ARG, "gate %d: one-qubit kind with q1 = %d (must be -1)", k,
                  g.q1);
    }
    const int np = kind_nparams(g.kind);
    for (int j = 0; j < 3; ++j) {
      if (j < np && (g.param[j] < 0 || g.param[j] >= n_theta))
        return fail(QSV_ERR_INVALID_ARG, "gate %d: param[%d] = %d outside [0, %d)", k, j,
                    g.param[j], n_theta);
      if (j >= np && g.param[j] != -1)
        return fail(QSV_ERR_INVALID_ARG, "gate %d: unused param[%d] = %d (must be -1)", k, j,
                    g.param[j]);
    }
  }
  return QSV_OK;
}

extern "C" qsv_status qsv_validate_pauli_sum(int32_t n, const qsv_pauli_sum* H) {
  if (n < 1 || n > kMaxQubits)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits = %d outside [1, %d]", n, kMaxQubits);
  if (!H) return fail(QSV_ERR_INVALID_ARG, "Pauli sum is NULL");
  if (H->n_terms < 0) return fail(QSV_ERR_INVALID_ARG, "n_terms = %d < 0", H->n_terms);
  if (H->n_terms == 0) return QSV_OK;
  if (!H->codes || !H->coeffs) return fail(QSV_ERR_INVALID_ARG, "Pauli codes/coeffs NULL");
  for (int64_t i = 0; i < (int64_t)H->n_terms * n; ++i)
    if (H->codes[i] > 3)
      return fail(QSV_ERR_INVALID_ARG, "Pauli code %d at term %lld qubit %lld (must be 0..3)",
                  (int)H->codes[i], (long long)(i / n), (long long)(i % n));
  for (int32_t t = 0; t < H->n_terms; ++t)
    if (!std::isfinite(H->coeffs[t]))
      return fail(QSV_ERR_INVALID_ARG, "coefficient %d is not finite", t);
  return QSV_OK;
}

extern "C" size_t qsv_state_bytes(int32_t n, qsv_dtype dt) {
  if (n < 1 || n > kMaxQubits || (dt != QSV_C64 && dt != QSV_C128)) return 0;
  return ((size_t)1 << n) * (dt == QSV_C128 ? 16 : 8);
}

extern "C" size_t qsv_workspace_bytes(int32_t n, qsv_dtype dt) {
  return 2 * qsv_state_bytes(n, dt);
}

// ------------------------------------------------------------------------------------------------
// device buffers owned by the library
// ------------------------------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  // Grows to at least `bytes`; waits for `st` first so no queued kernel still uses the old one.
  qsv_status ensure(size_t bytes, hipStream_t st) {
    if (bytes <= cap) return QSV_OK;
    HIP_TRY(hipStreamSynchronize(st));
    if (p) HIP_TRY(hipFree(p));
    p = nullptr;
    cap = 0;
    size_t want = bytes < 256 ? 256 : bytes;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(QSV_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    cap = want;
    return QSV_OK;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

static uint64_t fnv1a(const void* data, size_t len, uint64_t h = 1469598103934665603ull) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < len; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// The fused schedules of one circuit for one tile geometry, with their device copies.
struct FusedSchedule {
  Schedule sched;
  DevBuf d_passes, d_phases, d_ops, d_slot_map;
};

// A circuit's fused schedules bound to one handle's buffers: one launch item per pass (forward
// into phi, forward in place on the state, reverse sweep), the reverse sweep's partials and the
// descriptors the final reduction reads them with.
struct FusedPlan {
  int r = 0, w = 0, t = 0;
  FusedSchedule fwd, bwd;
  int64_t tiles = 0, chunk = 1;
  int grid = 1, nb = 1;
  std::vector<PassItem> items_fwd_phi, items_fwd_state, items_bwd;
  std::vector<int64_t> occ_base;  // per global slot, relative to the partials buffer
  std::vector<int32_t> occ_nb;
  DevBuf d_items_fwd_phi, d_items_fwd_state, d_items_bwd, partials, d_occ_base, d_occ_nb,
      d_final;
  // When one tile covers the state, every pass of a sweep runs in one launch: a single
  // workgroup walks the passes in order (items with consecutive tile indices).
  DevBuf d_seq_fwd_phi, d_seq_fwd_state, d_seq_bwd;
  bool seq_gen_fwd = false, seq_gen_bwd = false;
  // non-Hermitian operators: the first sweep's partials, kept while the second sweep runs
  DevBuf partials_a, d_final_a;
};

// Reference-gradient (Algorithm 2) tables of one circuit for one tile geometry: for every
// parameter occurrence ("entry"), the forward passes with that occurrence's gate applied as its
// derivative, the last pass ending in Re <lambda|mu>. Entry e's K items are consecutive.
struct RefPlan {
  int K = 0;                // forward passes
  int64_t E = 0;            // entries
  bool single = false;      // one tile covers the state: entries in parallel, a workgroup each
  int64_t per_launch = 0;   // single: entries per launch (size of the mu pool)
  int nb = 1;               // partials per entry (workgroups of its last pass)
  FusedSchedule fwd;        // the forward schedule without rotation macros (ops one by one)
  DevBuf items, mu_pool, partials, d_occ_base, d_occ_nb, d_final;
};

// A circuit lowered for the device: gate table, matrix records, and the map from parameters to
// the reduction slots of their occurrences (in sweep order, last gate first).
// Serial numbers of plans: a cached batch names the plans it was built from by serial, so a plan
// freed by a cache flush and another allocated at the same address are never confused.
static uint64_t next_plan_serial() {
  static std::atomic<uint64_t> serial{0};
  return ++serial;
}

struct Plan {
  uint64_t serial = next_plan_serial();
  std::vector<GateDesc> gates;
  int n_theta = 0;
  int n_occ = 0;
  std::vector<int32_t> slot_of_gate;  // first reduction slot of gate k (-1 if none)
  std::vector<int32_t> param_ptr, occ;
  DevBuf d_gates, d_recs, d_param_ptr, d_occ;
  std::map<int, std::unique_ptr<FusedPlan>> fused;  // key r * 16 + w
  std::map<int, std::unique_ptr<RefPlan>> ref;      // key r * 16 + w
  // gate-granular reverse sweep: partials [slot][block] and their descriptors
  bool gg_ready = false;
  DevBuf gg_partials, d_gg_occ_base, d_gg_occ_nb, d_gg_final;
  // one-wave sweep (states of at most kWaveMaxQubits qubits): one product sum per slot
  DevBuf wave_slot_sum;
  bool all_unitary = true;
  bool wave_needs_recs = false;  // a gate the wave kernels read from its record
  // Algorithm 2 in waves: lambda, and the gate and parameter of each slot (k * 4 + j)
  bool wave_ready = false;
  DevBuf wave_ref_lam, wave_occ_gate;
  // chunked one-circuit sweep: chunk operators, boundary states, first slots, finish counter
  bool wc_ready = false;
  int wc_chunks = 0;
  DevBuf wc_A, wc_B, wc_phi, wc_lam, wc_slot0, wc_done;
};

struct PauliPlan {
  uint64_t serial = next_plan_serial();
  // the operator this plan was built from, compared in full on a cache hit
  std::vector<uint8_t> key_codes;
  std::vector<double> key_coeffs, key_im;
  double key_sign = 1.0;
  std::vector<PauliGroup> groups;
  std::vector<PauliTerm> terms;
  DevBuf d_groups, d_terms;
  // the handle's application of H: tiled passes (their groups and sign-folded terms) and the
  // groups left to the gather kernel
  std::vector<PauliTilePass> tpasses;
  std::vector<PauliTileGroup> tgroups;
  std::vector<PauliTerm> tterms;
  std::vector<PauliGroup> rgroups;
  std::vector<PauliTerm> rterms;
  DevBuf d_tgroups, d_tterms, d_rgroups, d_rterms;
};

// Chooses the tiled passes of the application of H on an n-qubit state: a pass holds TB tile
// qubits (the low run qubits plus TB - c free ones) and applies every X-mask group whose X bits
// lie in its tile, reading psi once for all of them; a gather reads psi once per group. Tiles are
// grown greedily (seeded by each remaining group, adding the qubit that completes the most
// remaining groups) and kept while a pass takes at least three groups; passes hold at most
// kPauliTileMaxTerms terms. Fills the plan's tiled and remaining (gather) tables.
static void plan_pauli_tiles(PauliPlan& P, int n, bool c128) {
  P.tpasses.clear();
  P.tgroups.clear();
  P.tterms.clear();
  P.rgroups.clear();
  P.rterms.clear();
  const int TB = pauli_tile_bits(c128);
  std::vector<int> unc;
  for (size_t g = 0; g < P.groups.size(); ++g) unc.push_back((int)g);
  if (n >= TB + 2) {
    const int c = run_qubits_for(c128, n);
    const uint64_t run = (1ull << c) - 1;
    const int F = TB - c;
    auto need = [&](int g) { return P.groups[g].x & ~run; };
    auto count_in = [&](uint64_t free) {
      int k = 0;
      for (int g : unc) k += (need(g) & ~free) == 0 ? 1 : 0;
      return k;
    };
    while (!unc.empty()) {
      uint64_t best_free = 0;
      int best = -1;
      std::vector<uint64_t> seeds;
      for (int g : unc) {
        const uint64_t x = need(g);
        if (__builtin_popcountll(x) <= F && std::find(seeds.begin(), seeds.end(), x) == seeds.end())
          seeds.push_back(x);
        if (seeds.size() >= 48) break;
      }
      for (uint64_t free : seeds) {
        while (__builtin_popcountll(free) < F) {
          int bq = -1, bgain = -1, bfreq = -1;
          for (int q = c; q < n; ++q) {
            const uint64_t b = 1ull << q;
            if (free & b) continue;
            int gain = 0, freq = 0;
            for (int g : unc) {
              const uint64_t x = need(g);
              if ((x & ~(free | b)) == 0 && (x & ~free) != 0) ++gain;
              if (x & b) ++freq;
            }
            if (gain > bgain || (gain == bgain && freq > bfreq)) {
              bq = q;
              bgain = gain;
              bfreq = freq;
            }
          }
          if (bq < 0) break;
          free |= 1ull << bq;
        }
        const int k = count_in(free);
        if (k > best) {
          best = k;
          best_free = free;
        }
      }
      if (best < 3) break;
      // the pass: its tile (run qubits, the free ones, padded with the lowest others)
      uint64_t tile = run | best_free;
      for (int q = c; q < n && __builtin_popcountll(tile) < TB; ++q) tile |= 1ull << q;
      PauliTilePass T;
      std::memset(&T, 0, sizeof T);
      int tb_of[64], s = 0;
      for (int q = 0; q < n; ++q) {
        tb_of[q] = -1;
        if ((tile >> q) & 1) {
          tb_of[q] = s;
          T.tile[s++] = (int8_t)q;
        } else {
          T.outer_mask |= 1ull << q;
        }
      }
      T.n_outer = n - TB;
      T.g0 = (int32_t)P.tgroups.size();
      T.t0 = (int32_t)P.tterms.size();
      std::vector<int> left;
      for (int g : unc) {
        const PauliGroup& G = P.groups[g];
        const int nt = G.t1 - G.t0;
        if ((need(g) & ~best_free) != 0 || T.n_terms + nt > kPauliTileMaxTerms) {
          left.push_back(g);
          continue;
        }
        PauliTileGroup TG{0, T.n_terms, T.n_terms + nt};
        for (uint64_t x = G.x; x; x &= x - 1) TG.xl |= 1u << tb_of[__builtin_ctzll(x)];
        for (int t = G.t0; t < G.t1; ++t) {
          PauliTerm term = P.terms[t];
          if (__builtin_popcountll(G.x & term.z) & 1) {  // (-1)^popcount(x & z) folded in
            term.cre = -term.cre;
            term.cim = -term.cim;
          }
          P.tterms.push_back(term);
        }
        T.n_terms += nt;
        P.tgroups.push_back(TG);
      }
      T.g1 = (int32_t)P.tgroups.size();
      if (T.g1 - T.g0 < 3) {  // the term limit left too little: undo and stop
        P.tgroups.resize(T.g0);
        P.tterms.resize(T.t0);
        break;
      }
      const int E = pauli_tile_elements(c128), LE = __builtin_ctz(E);
      for (int k = 0; k < E; ++k) {
        uint64_t off = 0;
        for (int b = 0; b < LE; ++b)
          if ((k >> b) & 1) off |= 1ull << T.tile[TB - LE + b];
        uint64_t bits = 0;
        for (int t = 0; t < T.n_terms; ++t)
          bits |= (uint64_t)(__builtin_popcountll(off & P.tterms[T.t0 + t].z) & 1) << t;
        T.kbits[k] = bits;
      }
      P.tpasses.push_back(T);
      unc.swap(left);
    }
  }
  for (int g : unc) {
    const PauliGroup& G = P.groups[g];
    PauliGroup R{G.x, (int32_t)P.rterms.size(), 0};
    for (int t = G.t0; t < G.t1; ++t) P.rterms.push_back(P.terms[t]);
    R.t1 = (int32_t)P.rterms.size();
    P.rgroups.push_back(R);
  }
}

// Per-launch HIP-event timing of selected kernel families (qsv_timing_enable / _read).
struct Timer {
  bool on = false;
  std::string filter;
  struct Pending {
    const char* name;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  std::map<std::string, qsv_kernel_stat> agg;
  ~Timer() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  bool wants(const char* name) const {
    return on && (filter.empty() || std::strstr(name, filter.c_str()) != nullptr);
  }
  hipError_t take(hipEvent_t* e) {
    if (!pool.empty()) {
      *e = pool.back();
      pool.pop_back();
      return hipSuccess;
    }
    return hipEventCreate(e);
  }
};

// A batch of circuits (one handle each) run level by level: level k of the forward pass (or of
// the reverse sweep) is one launch over the k-th pass of every circuit that has one.
struct BatchLevel {
  DevBuf d_items;
  double bytes = 0;  // algorithmic bytes of the launch (all its circuits)
  int n_items = 0;
  int64_t total = 0, chunk = 1;
  int grid = 1;
  bool general = false;
};
struct BatchPlan {
  uint64_t serial = next_plan_serial();
  std::vector<qsv_state*> states;
  std::vector<uint64_t> serials;  // of the circuits' plans and Pauli plans, in order
  std::vector<Plan*> plans;
  std::vector<PauliPlan*> paulis;
  int r = 0, w = 0;
  std::vector<std::unique_ptr<BatchLevel>> fwd, bwd;
  DevBuf partials, d_occ_base, d_occ_nb, d_final;
  int64_t total_params = 0;
  // every circuit's gates in one table (parameter indices into the flat theta) and records, so
  // one launch prepares the whole batch; one launch applies H to every circuit
  DevBuf d_gates_all, d_recs_all, d_jobs, partials_e;
  int total_gates = 0;
  // one-wave batch (every circuit of at most kWaveMaxQubits qubits): one wave per circuit
  bool wave = false;
  bool wave_needs_recs = false;
  DevBuf d_wave_jobs;
  uint64_t key = 0;  // the cache key (graph keys of its calls derive from it)
};

static constexpr int kBatchPauliBlocks = 128;  // blocks per circuit of the batched H apply

// Captured launch sequences, replayed with hipGraphLaunch when the same call repeats.
struct GraphCache {
  bool on = false;
  hipStream_t capture_stream = nullptr;  // library-owned, default priority
  struct Entry {
    int seen = 0;                // eager runs so far (capture on the second)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::unordered_map<uint64_t, Entry> entries;
  void clear() {
    for (auto& kv : entries) {
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    entries.clear();
  }
  ~GraphCache() {
    clear();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

struct qsv_state {
  int n = 0;
  qsv_dtype dt = QSV_C128;
  void* d_state = nullptr;
  void* d_work = nullptr;
  size_t work_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int nb = 1;
  int fusion_mode = -1;  // -1 automatic, 0 gate-granular, 1 fused with (fr, fw), 2 one wave,
                         // 3 chunked one-circuit sweep
  int fr = 0, fw = 0;
  std::unordered_map<uint64_t, std::unique_ptr<Plan>> plans;
  Plan* last_plan = nullptr;  // the plan of the last call: checked first, without hashing
  std::unordered_map<uint64_t, std::unique_ptr<PauliPlan>> paulis;
  DevBuf epartials, theta_scratch, energies;
  Timer timer;
  std::unordered_map<uint64_t, std::unique_ptr<BatchPlan>> batches;
  GraphCache graphs;
};

static constexpr size_t kMaxCachedPlans = 64;

static qsv_status check_handle(qsv_state* s) {
  if (!s) return fail(QSV_ERR_INVALID_ARG, "handle is NULL");
  HIP_TRY(hipSetDevice(s->device));
  return QSV_OK;
}

// Test hook (qsv_debug_fail_launch): counts down over launches made through `timed`; the launch
// that takes it from 1 to 0 is not enqueued and reports a HIP error instead.
static std::atomic<int32_t> g_fail_countdown{0};

static bool injected_failure() {
  int32_t k = g_fail_countdown.load();
  while (k > 0) {
    if (g_fail_countdown.compare_exchange_weak(k, k - 1)) return k == 1;
  }
  return false;
}

extern "C" qsv_status qsv_debug_fail_launch(int32_t k) {
  if (k < 0) return fail(QSV_ERR_INVALID_ARG, "k = %d < 0", k);
  g_fail_countdown.store(k);
  return QSV_OK;
}

// Runs `launch` (which enqueues exactly one kernel on s->stream) between two timing events when
// the kernel family `name` is being timed.
template <typename F>
static qsv_status timed(qsv_state* s, const char* name, double bytes, F&& launch) {
  if (injected_failure())
    return fail(QSV_ERR_HIP, "%s: launch failure injected by qsv_debug_fail_launch", name);
  const bool t = s->timer.wants(name);
  hipEvent_t a = nullptr, b = nullptr;
  if (t) {
    HIP_TRY(s->timer.take(&a));
    HIP_TRY(s->timer.take(&b));
    HIP_TRY(hipEventRecord(a, s->stream));
  }
  HIP_TRY(launch());
  if (t) {
    HIP_TRY(hipEventRecord(b, s->stream));
    s->timer.pending.push_back({name, bytes, a, b});
  }
  return QSV_OK;
}

// Algorithmic bytes of one gate-granular launch: unique state bytes read plus written.
static double forward_bytes(const GateDesc& g, double S) {
  if (g.kind == K_CNOT) return S;        // the control = 1 half, read and written
  if (g.kind == K_CZ) return 0.5 * S;    // the 11 quarter, read and written
  return 2 * S;
}
static double backward_bytes(const GateDesc& g, double S, bool undo_lam) {
  const bool reads_lam = kind_nparams(g.kind) > 0 || undo_lam;
  const double phi = forward_bytes(g, S);
  const double lam = undo_lam ? phi : (reads_lam ? 0.5 * phi : 0.0);
  return phi + lam;
}

static qsv_status get_plan(qsv_state* s, const qsv_gate* gates, int32_t n_gates, int32_t n_theta,
                           Plan** out) {
  // repeated calls with one circuit (the common case, and a batch's per-handle lookups) compare
  // the gate table with the last plan's copy instead of hashing it
  if (Plan* lp = s->last_plan) {
    if ((int32_t)lp->gates.size() == n_gates && lp->n_theta == n_theta &&
        (n_gates == 0 || std::memcmp(lp->gates.data(), gates, sizeof(qsv_gate) * n_gates) == 0)) {
      *out = lp;
      return QSV_OK;
    }
  }
  uint64_t h = fnv1a(gates, sizeof(qsv_gate) * (size_t)n_gates);
  h = fnv1a(&n_theta, sizeof n_theta, h);
  h = fnv1a(&n_gates, sizeof n_gates, h);
  auto it = s->plans.find(h);
  if (it != s->plans.end()) {
    Plan* p = it->second.get();
    if ((int32_t)p->gates.size() == n_gates && p->n_theta == n_theta &&
        (n_gates == 0 || std::memcmp(p->gates.data(), gates, sizeof(qsv_gate) * n_gates) == 0)) {
      *out = s->last_plan = p;
      return QSV_OK;
    }
  }
  if (s->plans.size() >= kMaxCachedPlans) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->plans.clear();
    s->last_plan = nullptr;
  }
  auto p = std::make_unique<Plan>();
  p->gates.assign(reinterpret_cast<const GateDesc*>(gates),
                  reinterpret_cast<const GateDesc*>(gates) + n_gates);
  p->n_theta = n_theta;
  p->slot_of_gate.assign(n_gates, -1);
  std::vector<std::vector<int32_t>> per_param(n_theta);
  int slot = 0;
  for (int k = n_gates - 1; k >= 0; --k) {
    const GateDesc& g = p->gates[k];
    const int np = kind_nparams(g.kind);
    if (!np) continue;
    p->slot_of_gate[k] = slot;
    for (int j = 0; j < np; ++j) per_param[g.p[j]].push_back(slot + j);
    slot += np;
  }
  p->n_occ = slot;
  for (const GateDesc& g : p->gates) {
    p->all_unitary = p->all_unitary && kind_unitary(g.kind);
    p->wave_needs_recs = p->wave_needs_recs || !wave_native_kind(g.kind);
  }
  p->param_ptr.assign(n_theta + 1, 0);
  for (int q = 0; q < n_theta; ++q) {
    p->param_ptr[q + 1] = p->param_ptr[q] + (int32_t)per_param[q].size();
    p->occ.insert(p->occ.end(), per_param[q].begin(), per_param[q].end());
  }
  const hipStream_t st = s->stream;
  QSV_TRY(p->d_gates.ensure(sizeof(GateDesc) * (n_gates ? n_gates : 1), st));
  QSV_TRY(p->d_recs.ensure(sizeof(GateRec) * (n_gates ? n_gates : 1), st));
  QSV_TRY(p->d_param_ptr.ensure(sizeof(int32_t) * (n_theta + 1), st));
  QSV_TRY(p->d_occ.ensure(sizeof(int32_t) * (p->occ.size() + 1), st));
  if (n_gates)
    HIP_TRY(hipMemcpyAsync(p->d_gates.p, p->gates.data(), sizeof(GateDesc) * n_gates,
                           hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(p->d_param_ptr.p, p->param_ptr.data(), sizeof(int32_t) * (n_theta + 1),
                         hipMemcpyHostToDevice, st));
  if (!p->occ.empty())
    HIP_TRY(hipMemcpyAsync(p->d_occ.p, p->occ.data(), sizeof(int32_t) * p->occ.size(),
                           hipMemcpyHostToDevice, st));
  *out = s->last_plan = p.get();
  s->plans[h] = std::move(p);
  return QSV_OK;
}

template <typename T>
static qsv_status upload_vec(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  QSV_TRY(b.ensure(sizeof(T) * (v.size() ? v.size() : 1), st));
  if (!v.empty())
    HIP_TRY(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  return QSV_OK;
}

// Terms grouped by X mask: (P psi)_j = i^{nY} (-1)^{popcount((j^x) & z)} psi_{j^x} with
// x = X|Y positions, z = Z|Y; each term's weight (c + i ci) i^{nY}.
static void build_pauli_groups(PauliPlan& P, int n, const qsv_pauli_sum* H,
                               const double* coeffs_im, double im_sign) {
  std::vector<uint64_t> xs;
  std::vector<std::vector<PauliTerm>> by_group;
  for (int t = 0; t < H->n_terms; ++t) {
    uint64_t x = 0, z = 0;
    int ny = 0;
    for (int q = 0; q < n; ++q) {
      const int c = H->codes[(size_t)t * n + q];
      if (c == 1 || c == 2) x |= 1ull << q;
      if (c == 3 || c == 2) z |= 1ull << q;
      if (c == 2) ++ny;
    }
    static const double ire[4] = {1, 0, -1, 0}, iim[4] = {0, 1, 0, -1};
    const double c = H->coeffs[t], ci = coeffs_im ? im_sign * coeffs_im[t] : 0.0;
    PauliTerm term{z, c * ire[ny & 3] - ci * iim[ny & 3], c * iim[ny & 3] + ci * ire[ny & 3]};
    size_t g = 0;
    while (g < xs.size() && xs[g] != x) ++g;
    if (g == xs.size()) {
      xs.push_back(x);
      by_group.emplace_back();
    }
    by_group[g].push_back(term);
  }
  for (size_t g = 0; g < xs.size(); ++g) {
    PauliGroup G{xs[g], (int32_t)P.terms.size(), 0};
    P.terms.insert(P.terms.end(), by_group[g].begin(), by_group[g].end());
    G.t1 = (int32_t)P.terms.size();
    P.groups.push_back(G);
  }
}

extern "C" qsv_status qsv_pauli_describe(int32_t n_qubits, qsv_dtype dt, const qsv_pauli_sum* H,
                                         int32_t* n_groups, int32_t* n_tiled_passes,
                                         int32_t* n_gather_groups, uint64_t* tile_masks,
                                         int32_t* pass_groups, int32_t max_passes) {
  if (dt != QSV_C64 && dt != QSV_C128) return fail(QSV_ERR_INVALID_ARG, "unknown dtype %d", dt);
  QSV_TRY(qsv_validate_pauli_sum(n_qubits, H));
  PauliPlan P;
  build_pauli_groups(P, n_qubits, H, nullptr, 1.0);
  plan_pauli_tiles(P, n_qubits, dt == QSV_C128);
  if (n_groups) *n_groups = (int32_t)P.groups.size();
  if (n_tiled_passes) *n_tiled_passes = (int32_t)P.tpasses.size();
  if (n_gather_groups) *n_gather_groups = (int32_t)P.rgroups.size();
  for (int i = 0; i < (int)P.tpasses.size() && i < max_passes; ++i) {
    const PauliTilePass& T = P.tpasses[i];
    if (tile_masks) tile_masks[i] = ~T.outer_mask & (n_qubits >= 64 ? ~0ull : (1ull << n_qubits) - 1);
    if (pass_groups) pass_groups[i] = T.g1 - T.g0;
  }
  return QSV_OK;
}

// coeffs_im (may be NULL): imaginary parts of the weights, taken times im_sign (-1 gives the
// adjoint of a non-Hermitian sum, the Pauli strings being Hermitian).
static qsv_status get_pauli_ex(qsv_state* s, const qsv_pauli_sum* H, const double* coeffs_im,
                               double im_sign, PauliPlan** out) {
  const int n = s->n;
  uint64_t h = fnv1a(H->codes, (size_t)H->n_terms * n);
  h = fnv1a(H->coeffs, sizeof(double) * H->n_terms, h);
  h = fnv1a(&H->n_terms, sizeof H->n_terms, h);
  if (coeffs_im) {
    h = fnv1a(coeffs_im, sizeof(double) * H->n_terms, h ^ 0x1a5ull);
    h = fnv1a(&im_sign, sizeof im_sign, h);
  }
  const size_t n_codes = (size_t)H->n_terms * n;
  auto it = s->paulis.find(h);
  if (it != s->paulis.end()) {
    const PauliPlan* q = it->second.get();
    const size_t cb = sizeof(double) * (size_t)H->n_terms;
    const bool same =
        q->key_codes.size() == n_codes && q->key_coeffs.size() == (size_t)H->n_terms &&
        (n_codes == 0 || std::memcmp(q->key_codes.data(), H->codes, n_codes) == 0) &&
        (H->n_terms == 0 || std::memcmp(q->key_coeffs.data(), H->coeffs, cb) == 0) &&
        (coeffs_im ? (q->key_im.size() == (size_t)H->n_terms && q->key_sign == im_sign &&
                      (H->n_terms == 0 || std::memcmp(q->key_im.data(), coeffs_im, cb) == 0))
                   : q->key_im.empty());
    if (same) {
      *out = it->second.get();
      return QSV_OK;
    }
  }
  if (s->paulis.size() >= kMaxCachedPlans) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->paulis.clear();
  }
  auto p = std::make_unique<PauliPlan>();
  p->key_codes.assign(H->codes, H->codes + n_codes);
  p->key_coeffs.assign(H->coeffs, H->coeffs + H->n_terms);
  if (coeffs_im) p->key_im.assign(coeffs_im, coeffs_im + H->n_terms);
  p->key_sign = im_sign;
  build_pauli_groups(*p, n, H, coeffs_im, im_sign);
  const hipStream_t st = s->stream;
  QSV_TRY(p->d_groups.ensure(sizeof(PauliGroup) * (p->groups.size() + 1), st));
  QSV_TRY(p->d_terms.ensure(sizeof(PauliTerm) * (p->terms.size() + 1), st));
  if (!p->groups.empty()) {
    HIP_TRY(hipMemcpyAsync(p->d_groups.p, p->groups.data(), sizeof(PauliGroup) * p->groups.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->d_terms.p, p->terms.data(), sizeof(PauliTerm) * p->terms.size(),
                           hipMemcpyHostToDevice, st));
  }
  plan_pauli_tiles(*p, n, s->dt == QSV_C128);
  QSV_TRY(upload_vec(p->d_tgroups, p->tgroups, st));
  QSV_TRY(upload_vec(p->d_tterms, p->tterms, st));
  QSV_TRY(upload_vec(p->d_rgroups, p->rgroups, st));
  QSV_TRY(upload_vec(p->d_rterms, p->rterms, st));
  *out = p.get();
  s->paulis[h] = std::move(p);
  return QSV_OK;
}

static qsv_status get_pauli(qsv_state* s, const qsv_pauli_sum* H, PauliPlan** out) {
  return get_pauli_ex(s, H, nullptr, 1.0, out);
}

// ------------------------------------------------------------------------------------------------
// handles
// ------------------------------------------------------------------------------------------------
template <typename R>
static hipError_t reset_state(qsv_state* s) {
  return launch_reset<R>(s->d_state, s->n, s->stream);
}

static hipError_t dispatch_reset(qsv_state* s) {
  return s->dt == QSV_C128 ? reset_state<double>(s) : reset_state<float>(s);
}

extern "C" qsv_status qsv_create(int32_t n, qsv_dtype dt, void* d_state, void* d_work,
                                 size_t work_bytes, void* stream, qsv_state** out) {
  if (!out) return fail(QSV_ERR_INVALID_ARG, "out is NULL");
  if (n < 1 || n > kMaxQubits)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits = %d outside [1, %d]", n, kMaxQubits);
  if (dt != QSV_C64 && dt != QSV_C128) return fail(QSV_ERR_INVALID_ARG, "unknown dtype %d", dt);
  if (!d_state || !d_work) return fail(QSV_ERR_INVALID_ARG, "state or workspace is NULL");
  if (((uintptr_t)d_state | (uintptr_t)d_work) & 255)
    return fail(QSV_ERR_INVALID_ARG, "state and workspace must be 256-byte aligned");
  if (work_bytes < qsv_workspace_bytes(n, dt))
    return fail(QSV_ERR_INVALID_ARG, "workspace of %zu bytes < %zu needed", work_bytes,
                qsv_workspace_bytes(n, dt));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  auto s = std::make_unique<qsv_state>();
  s->n = n;
  s->dt = dt;
  s->d_state = d_state;
  s->d_work = d_work;
  s->work_bytes = work_bytes;
  s->stream = static_cast<hipStream_t>(stream);
  s->device = dev;
  s->nb = sweep_blocks(n);
  HIP_TRY(dispatch_reset(s.get()));
  *out = s.release();
  return QSV_OK;
}

extern "C" qsv_status qsv_destroy(qsv_state* s) {
  if (!s) return QSV_OK;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  delete s;
  return QSV_OK;
}

extern "C" qsv_status qsv_set_stream(qsv_state* s, void* stream) {
  QSV_TRY(check_handle(s));
  // Work already queued on the old stream must finish before the new stream may touch the same
  // buffers.
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->stream = static_cast<hipStream_t>(stream);
  return QSV_OK;
}

extern "C" qsv_status qsv_reset(qsv_state* s) {
  QSV_TRY(check_handle(s));
  HIP_TRY(dispatch_reset(s));
  return QSV_OK;
}

extern "C" qsv_status qsv_sync(qsv_state* s) {
  QSV_TRY(check_handle(s));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// hipGraph capture and replay
// ------------------------------------------------------------------------------------------------
static constexpr size_t kMaxGraphs = 16;

// Runs `enqueue` (which puts a call's whole launch sequence on s->stream). With graphs on and no
// timing active, the first run with a given key is eager (it builds and allocates every plan), the
// second is captured on the library's capture stream into a graph, and every later run with that
// key replays the graph on s->stream. `key` must cover everything the launches bake in (plans,
// device pointers, geometry). `extra` lists further handles whose stream must follow during the
// capture (batches).
template <typename F>
static qsv_status run_graph(qsv_state* s, uint64_t key, F&& enqueue,
                            qsv_state* const* extra = nullptr, int n_extra = 0) {
  GraphCache& gc = s->graphs;
  if (!gc.on || s->timer.on) return enqueue();
  auto it = gc.entries.find(key);
  if (it == gc.entries.end()) {
    if (gc.entries.size() >= kMaxGraphs) {
      HIP_TRY(hipStreamSynchronize(s->stream));
      gc.clear();
    }
    it = gc.entries.emplace(key, GraphCache::Entry()).first;
  }
  GraphCache::Entry& e = it->second;
  if (e.exec) {
    HIP_TRY(hipGraphLaunch(e.exec, s->stream));
    return QSV_OK;
  }
  if (e.seen++ == 0) return enqueue();
  if (!gc.capture_stream) HIP_TRY(hipStreamCreateWithFlags(&gc.capture_stream, hipStreamNonBlocking));
  // the capture stream must not run ahead of work already queued on the caller's stream
  HIP_TRY(hipStreamSynchronize(s->stream));
  const hipStream_t user = s->stream;
  std::vector<std::pair<qsv_state*, hipStream_t>> saved;
  for (int i = 0; i < n_extra; ++i) {
    saved.push_back({extra[i], extra[i]->stream});
    extra[i]->stream = gc.capture_stream;
  }
  s->stream = gc.capture_stream;
  // every exit from here on puts the handles back on their own streams
  auto restore = [&] {
    s->stream = user;
    for (auto& kv : saved) kv.first->stream = kv.second;
  };
  const hipError_t eb = hipStreamBeginCapture(gc.capture_stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) {
    restore();
    return fail(QSV_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(eb));
  }
  const qsv_status st = enqueue();
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(gc.capture_stream, &graph);
  restore();
  if (st != QSV_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return fail(QSV_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(QSV_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  e.graph = graph;
  e.exec = exec;
  HIP_TRY(hipGraphLaunch(exec, s->stream));
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// computations
// ------------------------------------------------------------------------------------------------
static qsv_status check_theta(const Plan* p, const double* d_theta) {
  bool any = false;
  for (const GateDesc& g : p->gates) any = any || kind_nparams(g.kind) > 0;
  if (any && !d_theta) return fail(QSV_ERR_INVALID_ARG, "d_theta is NULL");
  return QSV_OK;
}

static double state_bytes_d(const qsv_state* s) { return (double)qsv_state_bytes(s->n, s->dt); }

// ------------------------------------------------------------------------------------------------
// fusion geometry and schedules
// ------------------------------------------------------------------------------------------------
static constexpr int kFusedGridCap = 1024;
// A batched level mixes passes of very different lengths (a small circuit may run all its gates
// in one pass): a workgroup per tile or two lets the hardware balance them.
static constexpr int kBatchGridCap = 1 << 20;

// Tile geometry for the handle: (r, w) with t = r + w tile qubits, or false for the gate-granular
// path (states too small for a tile, or fusion switched off).
static void auto_geometry(const qsv_state* s, int* r, int* w);

static bool fusion_geometry(const qsv_state* s, int* r, int* w) {
  if (s->fusion_mode == 0) return false;
  if (s->fusion_mode == 1) {
    *r = s->fr;
    *w = s->fw;
    return true;
  }
  auto_geometry(s, r, w);
  return true;
}

// Size-dependent default geometry (fusion mode -1).
static void auto_geometry(const qsv_state* s, int* r, int* w) {
  const bool c128 = s->dt == QSV_C128;
  const int rmax = c128 ? 3 : 4;
  for (int rr = rmax; rr >= 2; --rr)
    if (rr + 8 <= s->n) {
      *r = rr;
      *w = 8;
      return;
    }
  for (int rr = 3; rr >= 2; --rr)
    if (rr + 6 <= s->n) {
      *r = rr;
      *w = 6;
      return;
    }
  *r = 2;  // the state is smaller than the smallest tile: one tile with phantom bits
  *w = 6;
}

static qsv_status upload_schedule(FusedSchedule& fs, hipStream_t st) {
  const Schedule& sc = fs.sched;
  QSV_TRY(fs.d_passes.ensure(sizeof(PassDesc) * (sc.passes.size() + 1), st));
  QSV_TRY(fs.d_phases.ensure(sizeof(PhaseDesc) * (sc.phases.size() + 1), st));
  QSV_TRY(fs.d_ops.ensure(sizeof(FusedOp) * (sc.ops.size() + 1), st));
  QSV_TRY(fs.d_slot_map.ensure(sizeof(int32_t) * (sc.slot_map.size() + 1), st));
  if (!sc.passes.empty())
    HIP_TRY(hipMemcpyAsync(fs.d_passes.p, sc.passes.data(), sizeof(PassDesc) * sc.passes.size(),
                           hipMemcpyHostToDevice, st));
  if (!sc.phases.empty())
    HIP_TRY(hipMemcpyAsync(fs.d_phases.p, sc.phases.data(), sizeof(PhaseDesc) * sc.phases.size(),
                           hipMemcpyHostToDevice, st));
  if (!sc.ops.empty())
    HIP_TRY(hipMemcpyAsync(fs.d_ops.p, sc.ops.data(), sizeof(FusedOp) * sc.ops.size(),
                           hipMemcpyHostToDevice, st));
  if (!sc.slot_map.empty())
    HIP_TRY(hipMemcpyAsync(fs.d_slot_map.p, sc.slot_map.data(),
                           sizeof(int32_t) * sc.slot_map.size(), hipMemcpyHostToDevice, st));
  return QSV_OK;
}

// Launch geometry of `total` tiles: workgroups, tiles per workgroup, and for an item occupying
// tiles [begin, begin + count) the first workgroup reaching into it and how many do.
static void launch_shape(int64_t total, int* grid, int64_t* chunk, int64_t cap = kFusedGridCap) {
  const int64_t g = std::min<int64_t>(total, cap);
  *grid = (int)(g < 1 ? 1 : g);
  *chunk = (total + *grid - 1) / *grid;
  if (*chunk < 1) *chunk = 1;
}
static void item_span(int64_t begin, int64_t count, int64_t chunk, int32_t* first, int32_t* nb) {
  const int64_t f = begin / chunk, l = (begin + count - 1) / chunk;
  *first = (int32_t)f;
  *nb = (int32_t)(l - f + 1);
}

static PassItem make_item(const FusedSchedule& fs, size_t i, const Plan* p, const void* src,
                          void* dst, void* lam, int n_outer) {
  PassItem it;
  std::memset(&it, 0, sizeof it);
  it.pd = fs.sched.passes[i];
  it.phases = fs.d_phases.as<PhaseDesc>();
  it.ops = fs.d_ops.as<FusedOp>();
  it.recs = p->d_recs.as<GateRec>();
  it.slot_map = fs.d_slot_map.as<int32_t>();
  it.src = src;
  it.dst = dst;
  it.lam = lam;
  it.n_outer = n_outer;
  it.sub_op = -1;
  return it;
}

static qsv_status upload_final(DevBuf& d_final, const DevBuf& partials, const DevBuf& occ_base,
                               const DevBuf& occ_nb, const Plan* p, hipStream_t st) {
  FinalDesc fd;
  std::memset(&fd, 0, sizeof fd);
  fd.partials = partials.as<double2>();
  fd.occ_base = occ_base.as<int64_t>();
  fd.occ_nb = occ_nb.as<int32_t>();
  fd.param_ptr = p->d_param_ptr.as<int32_t>();
  fd.occ = p->d_occ.as<int32_t>();
  fd.grad_off = 0;
  fd.p_begin = 0;
  fd.n_theta = p->n_theta;
  std::vector<FinalDesc> v(1, fd);
  return upload_vec(d_final, v, st);
}

static qsv_status get_fused(qsv_state* s, Plan* p, int r, int w, FusedPlan** out) {
  const int key = r * 16 + w;
  auto it = p->fused.find(key);
  if (it != p->fused.end()) {
    *out = it->second.get();
    return QSV_OK;
  }
  if (!fused_config_supported(r, w, s->dt == QSV_C128))
    return fail(QSV_ERR_UNSUPPORTED, "fused geometry r=%d w=%d not available", r, w);
  const hipStream_t st = s->stream;
  auto fp = std::make_unique<FusedPlan>();
  fp->r = r;
  fp->w = w;
  fp->t = r + w;
  const int G = (int)p->gates.size();
  std::vector<int> seq(G);
  std::string msg;
  const int runq = run_qubits_for(s->dt == QSV_C128, s->n);
  for (int k = 0; k < G; ++k) seq[k] = G - 1 - k;
  if (!build_schedule(s->n, p->gates, seq, p->slot_of_gate, true, r + w, r, w, runq,
                      fp->bwd.sched, &msg))
    return fail(QSV_ERR_INTERNAL, "backward schedule: %s", msg.c_str());
  if (!build_forward_schedule(s->n, p->gates, r + w, r, w, runq, fp->bwd.sched, fp->fwd.sched,
                              &msg))
    return fail(QSV_ERR_INTERNAL, "forward schedule: %s", msg.c_str());
  QSV_TRY(upload_schedule(fp->fwd, st));
  QSV_TRY(upload_schedule(fp->bwd, st));

  // single-circuit launch items
  const int n_outer = std::max(0, s->n - fp->t);
  fp->tiles = 1ll << n_outer;
  launch_shape(fp->tiles, &fp->grid, &fp->chunk);
  int32_t first = 0, nb = 1;
  item_span(0, fp->tiles, fp->chunk, &first, &nb);
  fp->nb = nb;
  void* phi = s->d_work;
  void* lam = static_cast<char*>(s->d_work) + qsv_state_bytes(s->n, s->dt);
  for (size_t i = 0; i < fp->fwd.sched.passes.size(); ++i) {
    PassItem a = make_item(fp->fwd, i, p, i == 0 ? s->d_state : phi, phi, nullptr, n_outer);
    a.nb = nb;
    fp->items_fwd_phi.push_back(a);
    PassItem b = make_item(fp->fwd, i, p, s->d_state, s->d_state, nullptr, n_outer);
    b.nb = nb;
    fp->items_fwd_state.push_back(b);
  }
  const Schedule& bs = fp->bwd.sched;
  int64_t total_partials = 0;
  for (const PassDesc& pd : bs.passes) total_partials += (int64_t)pd.n_slots * nb;
  QSV_TRY(fp->partials.ensure(sizeof(double2) * (total_partials ? total_partials : 1), st));
  fp->occ_base.assign(p->n_occ ? p->n_occ : 1, 0);
  fp->occ_nb.assign(p->n_occ ? p->n_occ : 1, 0);
  int64_t off = 0;
  for (size_t i = 0; i < bs.passes.size(); ++i) {
    const PassDesc& pd = bs.passes[i];
    PassItem b = make_item(fp->bwd, i, p, nullptr, phi, lam, n_outer);
    b.nb = nb;
    b.partials = fp->partials.as<double2>() + off;
    fp->items_bwd.push_back(b);
    for (int j = 0; j < pd.n_slots; ++j) {
      const int gs = bs.slot_map[pd.slot_begin + j];
      fp->occ_base[gs] = off + (int64_t)j * nb;
      fp->occ_nb[gs] = nb;
    }
    off += (int64_t)pd.n_slots * nb;
  }
  QSV_TRY(upload_vec(fp->d_items_fwd_phi, fp->items_fwd_phi, st));
  QSV_TRY(upload_vec(fp->d_items_fwd_state, fp->items_fwd_state, st));
  QSV_TRY(upload_vec(fp->d_items_bwd, fp->items_bwd, st));
  if (fp->tiles == 1) {
    auto sequence = [](std::vector<PassItem> v) {
      for (size_t i = 0; i < v.size(); ++i) {
        v[i].tile_begin = (int64_t)i;
        v[i].first_wg = 0;
        v[i].nb = 1;
      }
      return v;
    };
    QSV_TRY(upload_vec(fp->d_seq_fwd_phi, sequence(fp->items_fwd_phi), st));
    QSV_TRY(upload_vec(fp->d_seq_fwd_state, sequence(fp->items_fwd_state), st));
    QSV_TRY(upload_vec(fp->d_seq_bwd, sequence(fp->items_bwd), st));
    for (const PassDesc& pd : fp->fwd.sched.passes) fp->seq_gen_fwd = fp->seq_gen_fwd || pd.general;
    for (const PassDesc& pd : bs.passes) fp->seq_gen_bwd = fp->seq_gen_bwd || pd.general;
  }
  QSV_TRY(upload_vec(fp->d_occ_base, fp->occ_base, st));
  QSV_TRY(upload_vec(fp->d_occ_nb, fp->occ_nb, st));
  QSV_TRY(upload_final(fp->d_final, fp->partials, fp->d_occ_base, fp->d_occ_nb, p, st));
  *out = fp.get();
  p->fused[key] = std::move(fp);
  return QSV_OK;
}

// Gate-granular reverse-sweep partials: slot o has nb consecutive block partials at o * nb.
static qsv_status get_gate_granular(qsv_state* s, Plan* p) {
  if (p->gg_ready) return QSV_OK;
  const hipStream_t st = s->stream;
  const int nb = s->nb, no = p->n_occ ? p->n_occ : 1;
  QSV_TRY(p->gg_partials.ensure(sizeof(double2) * (size_t)no * nb, st));
  std::vector<int64_t> base(no);
  std::vector<int32_t> cnt(no, nb);
  for (int o = 0; o < no; ++o) base[o] = (int64_t)o * nb;
  QSV_TRY(upload_vec(p->d_gg_occ_base, base, st));
  QSV_TRY(upload_vec(p->d_gg_occ_nb, cnt, st));
  QSV_TRY(upload_final(p->d_gg_final, p->gg_partials, p->d_gg_occ_base, p->d_gg_occ_nb, p, st));
  p->gg_ready = true;
  return QSV_OK;
}

// The one-wave sweep (launch_wave_adjoint): fusion mode 2, and the automatic mode's choice, for
// states of at most kWaveMaxQubits qubits.
static bool wave_path(const qsv_state* s) {
  return s->n <= kWaveMaxQubits &&
         (s->fusion_mode == 2 || s->fusion_mode == 3 || s->fusion_mode == -1);
}

// Circuits long enough for the chunked sweep to pay for forming the chunk operators (about
// 2^n gate applications per gate): the automatic mode takes it from this many gates on.
static constexpr int kWaveChunkMinGates = 96;

// The chunked variant (launch_wave_chunked) of a one-wave gradient: mode 3, or the automatic
// mode for long circuits; every gate unitary (phi is carried back by W_c^dag).
static bool wave_chunked(const qsv_state* s, const Plan* p) {
  const int G = (int)p->gates.size();
  return s->n <= kWaveChunkMaxQubits && p->all_unitary && G > 0 &&
         (s->fusion_mode == 3 || (s->fusion_mode == -1 && G >= kWaveChunkMinGates));
}

static qsv_status get_wave_chunks(qsv_state* s, Plan* p) {
  if (p->wc_ready) return QSV_OK;
  const hipStream_t st = s->stream;
  const int G = (int)p->gates.size();
  const int C = (G + kWaveChunk - 1) / kWaveChunk;
  const size_t N = (size_t)1 << s->n;
  QSV_TRY(p->wc_A.ensure(sizeof(double2) * C * N * N, st));
  QSV_TRY(p->wc_B.ensure(sizeof(double2) * C * N * N, st));
  QSV_TRY(p->wc_phi.ensure(sizeof(double2) * C * N, st));
  QSV_TRY(p->wc_lam.ensure(sizeof(double2) * C * N, st));
  // chunk c's first slot: the products of the gates after it (slots run in sweep order)
  std::vector<int32_t> slot0(C, 0);
  int after = 0;
  for (int c = C - 1; c >= 0; --c) {
    slot0[c] = after;
    for (int k = c * kWaveChunk; k < std::min(G, (c + 1) * kWaveChunk); ++k)
      after += kind_nparams(p->gates[k].kind);
  }
  QSV_TRY(upload_vec(p->wc_slot0, slot0, st));
  QSV_TRY(p->wc_done.ensure(sizeof(int32_t), st));
  HIP_TRY(hipMemsetAsync(p->wc_done.p, 0, sizeof(int32_t), st));
  p->wc_chunks = C;
  p->wc_ready = true;
  return QSV_OK;
}

static qsv_status get_wave(qsv_state* s, Plan* p) {
  if (p->wave_ready) return QSV_OK;
  const hipStream_t st = s->stream;
  QSV_TRY(p->wave_slot_sum.ensure(sizeof(double) * (size_t)std::max(p->n_occ, 1), st));
  QSV_TRY(p->wave_ref_lam.ensure(sizeof(double2) * 64, st));
  std::vector<int32_t> occ_gate(std::max(p->n_occ, 1), 0);
  for (size_t k = 0; k < p->gates.size(); ++k)
    for (int j = 0; j < kind_nparams(p->gates[k].kind); ++j)
      occ_gate[p->slot_of_gate[k] + j] = (int32_t)k * 4 + j;
  QSV_TRY(upload_vec(p->wave_occ_gate, occ_gate, st));
  p->wave_ready = true;
  return QSV_OK;
}

static WaveJob wave_job(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                        double* d_energy, double* d_grad) {
  WaveJob J;
  std::memset(&J, 0, sizeof J);
  J.gates = p->d_gates.as<GateDesc>();
  J.recs = p->d_recs.as<GateRec>();
  J.theta = d_theta;
  J.in = s->d_state;
  J.groups = hp->d_groups.as<PauliGroup>();
  J.terms = hp->d_terms.as<PauliTerm>();
  J.param_ptr = p->d_param_ptr.as<int32_t>();
  J.occ = p->d_occ.as<int32_t>();
  J.slot_sum = p->wave_slot_sum.as<double>();
  J.energy = d_energy;
  J.grad = d_grad;
  J.n_gates = (int32_t)p->gates.size();
  J.n = s->n;
  J.n_groups = (int32_t)hp->groups.size();
  J.n_theta = p->n_theta;
  J.ref_lam = p->wave_ref_lam.as<double2>();
  J.occ_gate = p->wave_occ_gate.as<int32_t>();
  J.n_occ = p->n_occ;
  return J;
}

// Algorithm 2 in waves (launch_wave_reference), after the launch that fills the gate records.
template <typename R>
static qsv_status wave_reference_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                                   double* d_energy, double* d_grad) {
  const hipStream_t st = s->stream;
  QSV_TRY(get_wave(s, p));
  if (p->wave_needs_recs)
    HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                        p->d_recs.as<GateRec>(), st));
  const WaveJob J = wave_job(s, p, hp, d_theta, d_energy, d_grad);
  return timed(s, "k_wave_reference", (p->n_occ + 1.0) * state_bytes_d(s), [&] {
    return launch_wave_reference<R>(nullptr, 1, p->n_occ, J, nullptr, d_energy, d_grad, st);
  });
}

// Algorithm 1 in one wave: the forward pass, H, the reverse sweep and the gradient entries in
// one launch (after the launch that fills the gate records).
template <typename R>
static qsv_status wave_adjoint_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                                 double* d_energy, double* d_grad) {
  const hipStream_t st = s->stream;
  QSV_TRY(get_wave(s, p));
  if (p->wave_needs_recs)
    HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                        p->d_recs.as<GateRec>(), st));
  const WaveJob J = wave_job(s, p, hp, d_theta, d_energy, d_grad);
  if (wave_chunked(s, p)) {
    QSV_TRY(get_wave_chunks(s, p));
    WaveChunks K;
    std::memset(&K, 0, sizeof K);
    K.A = p->wc_A.as<double2>();
    K.B = p->wc_B.as<double2>();
    K.phi = p->wc_phi.as<double2>();
    K.lam = p->wc_lam.as<double2>();
    K.slot0 = p->wc_slot0.as<int32_t>();
    K.done = p->wc_done.as<int32_t>();
    K.n_chunks = p->wc_chunks;
    return timed(s, "k_wave_chunked", 3 * state_bytes_d(s), [&] {
      return launch_wave_chunked<R>(J, K, st);
    });
  }
  return timed(s, "k_wave_adjoint", 3 * state_bytes_d(s), [&] {
    return launch_wave_adjoint<R>(nullptr, 1, J, nullptr, nullptr, nullptr, st);
  });
}

// dst <- U src (fused: into phi or in place on the state; gate-granular: any pair of buffers).
template <typename R>
static qsv_status forward(qsv_state* s, Plan* p, const void* src, void* dst) {
  const double S = state_bytes_d(s);
  const hipStream_t st = s->stream;
  int r = 0, w = 0;
  if (fusion_geometry(s, &r, &w) && !p->gates.empty() &&
      (src == dst ? dst == s->d_state : (src == s->d_state && dst == s->d_work))) {
    FusedPlan* fp = nullptr;
    QSV_TRY(get_fused(s, p, r, w, &fp));
    const Schedule& sc = fp->fwd.sched;
    if (fp->tiles == 1) {
      const PassItem* seq = (src == dst ? fp->d_seq_fwd_state : fp->d_seq_fwd_phi).as<PassItem>();
      const int K = (int)sc.passes.size();
      return timed(s, "k_pass_fwd", 2 * S * K, [&] {
        return launch_fused_forward<R>(seq, K, K, K, r, w, fp->seq_gen_fwd, 1, st);
      });
    }
    const PassItem* items = (src == dst ? fp->d_items_fwd_state : fp->d_items_fwd_phi).as<PassItem>();
    for (size_t i = 0; i < sc.passes.size(); ++i) {
      QSV_TRY(timed(s, "k_pass_fwd", 2 * S, [&] {
        return launch_fused_forward<R>(items + i, 1, fp->tiles, fp->chunk, r, w,
                                       sc.passes[i].general != 0, fp->grid, st);
      }));
    }
    return QSV_OK;
  }
  if (src != dst)
    QSV_TRY(timed(s, "k_copy", 2 * S, [&] { return launch_copy<R>(dst, src, s->n, st); }));
  for (size_t k = 0; k < p->gates.size(); ++k) {
    const GateDesc& g = p->gates[k];
    QSV_TRY(timed(s, forward_kernel_name(g), forward_bytes(g, S), [&] {
      return launch_forward_gate<R>(dst, s->n, g, p->d_recs.as<GateRec>() + k, false, st);
    }));
  }
  return QSV_OK;
}

// The reverse sweep of Algorithm 1 over (phi, lambda) = the workspace; *final_desc receives the
// descriptor table the final reduction reads the partials with.
template <typename R>
static qsv_status backward(qsv_state* s, Plan* p, const FinalDesc** final_desc,
                          bool cplx = false) {
  const double S = state_bytes_d(s);
  const hipStream_t st = s->stream;
  const int n = s->n;
  void* phi = s->d_work;
  void* lam = static_cast<char*>(s->d_work) + qsv_state_bytes(n, s->dt);
  int r = 0, w = 0;
  if (fusion_geometry(s, &r, &w) && !p->gates.empty()) {
    FusedPlan* fp = nullptr;
    QSV_TRY(get_fused(s, p, r, w, &fp));
    const Schedule& sc = fp->bwd.sched;
    *final_desc = fp->d_final.as<FinalDesc>();
    if (fp->tiles == 1) {
      const int K = (int)sc.passes.size();
      return timed(s, "k_pass_bwd", 4 * S * K, [&] {
        return launch_fused_backward<R>(fp->d_seq_bwd.as<PassItem>(), K, K, K, r, w,
                                        fp->seq_gen_bwd, 1, st, cplx);
      });
    }
    const PassItem* items = fp->d_items_bwd.as<PassItem>();
    for (size_t i = 0; i < sc.passes.size(); ++i) {
      QSV_TRY(timed(s, "k_pass_bwd", 4 * S, [&] {
        return launch_fused_backward<R>(items + i, 1, fp->tiles, fp->chunk, r, w,
                                        sc.passes[i].general != 0, fp->grid, st, cplx);
      }));
    }
    *final_desc = fp->d_final.as<FinalDesc>();
    return QSV_OK;
  }
  QSV_TRY(get_gate_granular(s, p));
  const int nb = s->nb;
  double2* part = p->gg_partials.as<double2>();
  for (int k = (int)p->gates.size() - 1; k >= 0; --k) {
    const int slot = p->slot_of_gate[k];
    const GateDesc& g = p->gates[k];
    QSV_TRY(timed(s, backward_kernel_name(g), backward_bytes(g, S, k > 0), [&] {
      return launch_backward_gate<R>(phi, lam, n, g, p->d_recs.as<GateRec>() + k, k > 0,
                                     slot >= 0 ? part + (size_t)slot * nb : nullptr, nb, st);
    }));
  }
  *final_desc = p->d_gg_final.as<FinalDesc>();
  return QSV_OK;
}

// out <- H psi (if out is set) and ep[0 .. nb) = the handle's energy partials: the gather kernel
// over the groups no tiled pass takes, then the tiled passes, each adding to out and to the
// partials (the first launch sets them).
template <typename R>
static qsv_status pauli(qsv_state* s, PauliPlan* hp, const void* psi, void* out, double2* ep) {
  const double S = state_bytes_d(s);
  if (hp->tpasses.empty())
    return timed(s, "k_pauli", out ? 2 * S : S, [&] {
      return launch_pauli<R>(psi, out, s->n, hp->d_groups.as<PauliGroup>(),
                             (int)hp->groups.size(), hp->d_terms.as<PauliTerm>(), ep, s->nb,
                             s->stream);
    });
  bool started = false;
  if (!hp->rgroups.empty()) {
    QSV_TRY(timed(s, "k_pauli", out ? 2 * S : S, [&] {
      return launch_pauli<R>(psi, out, s->n, hp->d_rgroups.as<PauliGroup>(),
                             (int)hp->rgroups.size(), hp->d_rterms.as<PauliTerm>(), ep, s->nb,
                             s->stream);
    }));
    started = true;
  }
  for (const PauliTilePass& T : hp->tpasses) {
    PauliTilePass P = T;
    P.lam_mode = out ? (started ? 1 : 0) : 2;
    P.e_accumulate = started ? 1 : 0;
    const double bytes = S + (P.lam_mode == 0 ? S : P.lam_mode == 1 ? 2 * S : 0.0);
    QSV_TRY(timed(s, "k_pauli_tile", bytes, [&] {
      return launch_pauli_tile<R>(psi, out, P, hp->d_tgroups.as<PauliTileGroup>(),
                                  hp->d_tterms.as<PauliTerm>(), ep, s->nb, s->stream);
    }));
    started = true;
  }
  return QSV_OK;
}

template <typename R>
static qsv_status apply_circuit_t(qsv_state* s, Plan* p, const double* d_theta) {
  HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                      p->d_recs.as<GateRec>(), s->stream));
  return forward<R>(s, p, s->d_state, s->d_state);
}

extern "C" qsv_status qsv_apply_circuit(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                        const double* d_theta, int32_t n_theta) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  QSV_TRY(check_theta(p, d_theta));
  return s->dt == QSV_C128 ? apply_circuit_t<double>(s, p, d_theta)
                           : apply_circuit_t<float>(s, p, d_theta);
}

extern "C" qsv_status qsv_expectation_pauli_sum(qsv_state* s, const qsv_pauli_sum* H,
                                                double* d_energy) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  PauliPlan* hp = nullptr;
  QSV_TRY(get_pauli(s, H, &hp));
  QSV_TRY(s->epartials.ensure(sizeof(double2) * s->nb, s->stream));
  double2* ep = s->epartials.as<double2>();
  if (s->dt == QSV_C128) QSV_TRY(pauli<double>(s, hp, s->d_state, nullptr, ep));
  else QSV_TRY(pauli<float>(s, hp, s->d_state, nullptr, ep));
  HIP_TRY(launch_final_energy(ep, s->nb, d_energy, nullptr, s->stream));
  return QSV_OK;
}

template <typename R>
static qsv_status energy_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                           double* d_energy) {
  QSV_TRY(s->epartials.ensure(sizeof(double2) * s->nb, s->stream));
  double2* ep = s->epartials.as<double2>();
  HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                      p->d_recs.as<GateRec>(), s->stream));
  void* phi = s->d_work;
  QSV_TRY(forward<R>(s, p, s->d_state, phi));
  QSV_TRY(pauli<R>(s, hp, phi, nullptr, ep));
  HIP_TRY(launch_final_energy(ep, s->nb, d_energy, nullptr, s->stream));
  return QSV_OK;
}

extern "C" qsv_status qsv_energy(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                 const double* d_theta, int32_t n_theta, const qsv_pauli_sum* H,
                                 double* d_energy) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  QSV_TRY(check_theta(p, d_theta));
  PauliPlan* hp = nullptr;
  QSV_TRY(get_pauli(s, H, &hp));
  return s->dt == QSV_C128 ? energy_t<double>(s, p, hp, d_theta, d_energy)
                           : energy_t<float>(s, p, hp, d_theta, d_energy);
}

template <typename R>
static qsv_status adjoint_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                            double* d_energy, double* d_grad) {
  const hipStream_t st = s->stream;
  const int nb = s->nb;
  void* phi = s->d_work;
  void* lam = static_cast<char*>(s->d_work) + qsv_state_bytes(s->n, s->dt);
  QSV_TRY(s->epartials.ensure(sizeof(double2) * nb, st));
  double2* ep = s->epartials.as<double2>();
  HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                      p->d_recs.as<GateRec>(), st));
  // Algorithm 1: the clone lambda := |in> and the forward pass build psi in the phi buffer (the
  // first pass reads |in> and writes phi); lambda is then written directly as H psi, which also
  // stands for the clone phi := psi. E = <psi|H psi>.
  QSV_TRY(forward<R>(s, p, s->d_state, phi));
  QSV_TRY(pauli<R>(s, hp, phi, lam, ep));
  const FinalDesc* fd = nullptr;
  QSV_TRY(backward<R>(s, p, &fd));
  // the outputs are written only once every pass has been enqueued
  HIP_TRY(launch_final_energy(ep, nb, d_energy, nullptr, st));
  HIP_TRY(launch_final_grad(fd, 1, p->n_theta, d_grad, st));
  return QSV_OK;
}

extern "C" qsv_status qsv_adjoint_gradient(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                           const double* d_theta, int32_t n_theta,
                                           const qsv_pauli_sum* H, double* d_energy,
                                           double* d_grad) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  if (n_theta > 0 && !d_grad) return fail(QSV_ERR_INVALID_ARG, "d_grad is NULL");
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  QSV_TRY(check_theta(p, d_theta));
  PauliPlan* hp = nullptr;
  QSV_TRY(get_pauli(s, H, &hp));
  int r = 0, w = 0;
  const bool fz = fusion_geometry(s, &r, &w);
  // plans are named by serial: a cache flush may reuse an address
  const uint64_t serials[2] = {p->serial, hp->serial};
  const void* key_parts[3] = {d_theta, d_energy, d_grad};
  uint64_t key = fnv1a(key_parts, sizeof key_parts, fnv1a(serials, sizeof serials));
  const bool wave = wave_path(s);
  const int geo[3] = {wave ? 2 : fz ? 1 : 0, r, w};
  key = fnv1a(geo, sizeof geo, key ^ 0xad301ull);
  return run_graph(s, key, [&] {
    if (wave)
      return s->dt == QSV_C128 ? wave_adjoint_t<double>(s, p, hp, d_theta, d_energy, d_grad)
                               : wave_adjoint_t<float>(s, p, hp, d_theta, d_energy, d_grad);
    return s->dt == QSV_C128 ? adjoint_t<double>(s, p, hp, d_theta, d_energy, d_grad)
                             : adjoint_t<float>(s, p, hp, d_theta, d_energy, d_grad);
  });
}
// ------------------------------------------------------------------------------------------------
// batches of independent circuits
// ------------------------------------------------------------------------------------------------
static constexpr size_t kMaxCachedBatches = 8;

// Routes the per-circuit helper launches of a batch onto one stream for the duration of a call.
struct StreamOverride {
  std::vector<std::pair<qsv_state*, hipStream_t>> saved;
  StreamOverride(qsv_state* const* states, int n, hipStream_t st) {
    for (int b = 0; b < n; ++b) {
      saved.push_back({states[b], states[b]->stream});
      states[b]->stream = st;
    }
  }
  ~StreamOverride() {
    for (auto& kv : saved) kv.first->stream = kv.second;
  }
};

// The batch's gate table (parameter indices into the flat theta) and matrix records, so that one
// launch prepares every circuit's records; gate_base[b] = circuit b's first gate.
static qsv_status build_batch_gates(const std::vector<Plan*>& plans, int B,
                                    const int64_t* theta_off, hipStream_t st, BatchPlan* bp,
                                    std::vector<int64_t>& gate_base) {
  std::vector<GateDesc> all;
  gate_base.assign(B, 0);
  for (int b = 0; b < B; ++b) {
    gate_base[b] = (int64_t)all.size();
    for (GateDesc g : plans[b]->gates) {
      for (int j = 0; j < 3; ++j)
        if (g.p[j] >= 0) g.p[j] += (int32_t)theta_off[b];
      all.push_back(g);
    }
  }
  bp->total_gates = (int)all.size();
  QSV_TRY(upload_vec(bp->d_gates_all, all, st));
  return bp->d_recs_all.ensure(sizeof(GateRec) * (all.size() ? all.size() : 1), st);
}

// A batch of small circuits: one wave each (see wave_adjoint_t).
static qsv_status build_batch_wave(qsv_state* const* states, const std::vector<Plan*>& plans,
                                   const std::vector<PauliPlan*>& hps, int B,
                                   const int64_t* theta_off, BatchPlan* bp) {
  const hipStream_t st = states[0]->stream;
  std::vector<int64_t> gate_base;
  QSV_TRY(build_batch_gates(plans, B, theta_off, st, bp, gate_base));
  bp->wave = true;
  std::vector<WaveJob> jobs(B);
  for (int b = 0; b < B; ++b) {
    QSV_TRY(get_wave(states[b], plans[b]));
    WaveJob J = wave_job(states[b], plans[b], hps[b], nullptr, nullptr, nullptr);
    bp->wave_needs_recs = bp->wave_needs_recs || plans[b]->wave_needs_recs;
    J.gates = bp->d_gates_all.as<GateDesc>() + gate_base[b];
    J.recs = bp->d_recs_all.as<GateRec>() + gate_base[b];
    J.grad_off = theta_off[b];
    jobs[b] = J;
  }
  QSV_TRY(upload_vec(bp->d_wave_jobs, jobs, st));
  bp->plans = plans;
  bp->paulis = hps;
  bp->states.assign(states, states + B);
  return QSV_OK;
}

template <typename R>
static qsv_status batched_wave_t(qsv_state* const* states, int B, BatchPlan* bp,
                                 const double* d_theta_flat, const int64_t* theta_off,
                                 double* d_energy, double* d_grad_flat) {
  qsv_state* s0 = states[0];
  const hipStream_t st = s0->stream;
  (void)theta_off;
  if (bp->wave_needs_recs)
    QSV_TRY(timed(s0, "k_prep", 0, [&] {
      return launch_prep(bp->d_gates_all.as<GateDesc>(), bp->total_gates, d_theta_flat,
                         bp->d_recs_all.as<GateRec>(), st);
    }));
  double bytes = 0;
  for (int b = 0; b < B; ++b) bytes += 3.0 * (double)qsv_state_bytes(states[b]->n, states[b]->dt);
  return timed(s0, "k_wave_adjoint", bytes, [&] {
    return launch_wave_adjoint<R>(bp->d_wave_jobs.as<WaveJob>(), B, WaveJob{}, d_theta_flat,
                                  d_energy, d_grad_flat, st);
  });
}

static qsv_status build_batch(qsv_state* const* states, const std::vector<Plan*>& plans,
                              const std::vector<PauliPlan*>& hps, int B, const int64_t* theta_off,
                              int r, int w, BatchPlan* bp) {
  qsv_state* s0 = states[0];
  const hipStream_t st = s0->stream;
  bp->r = r;
  bp->w = w;
  std::vector<FusedPlan*> fps(B);
  size_t lf = 0, lb = 0;
  for (int b = 0; b < B; ++b) {
    QSV_TRY(get_fused(states[b], plans[b], r, w, &fps[b]));
    lf = std::max(lf, fps[b]->fwd.sched.passes.size());
    lb = std::max(lb, fps[b]->bwd.sched.passes.size());
  }
  std::vector<int64_t> gate_base;
  QSV_TRY(build_batch_gates(plans, B, theta_off, st, bp, gate_base));
  GateRec* recs_all = bp->d_recs_all.as<GateRec>();
  // H applied to every circuit in one launch
  std::vector<PauliJob> jobs(B);
  for (int b = 0; b < B; ++b) {
    qsv_state* s = states[b];
    jobs[b].psi = s->d_work;
    jobs[b].out = static_cast<char*>(s->d_work) + qsv_state_bytes(s->n, s->dt);
    jobs[b].groups = hps[b]->d_groups.as<PauliGroup>();
    jobs[b].terms = hps[b]->d_terms.as<PauliTerm>();
    jobs[b].n = s->n;
    jobs[b].n_groups = (int32_t)hps[b]->groups.size();
  }
  QSV_TRY(upload_vec(bp->d_jobs, jobs, st));
  QSV_TRY(bp->partials_e.ensure(sizeof(double2) * (size_t)B * kBatchPauliBlocks, st));
  bp->paulis = hps;
  // forward levels
  for (size_t k = 0; k < lf; ++k) {
    auto L = std::make_unique<BatchLevel>();
    std::vector<PassItem> items;
    for (int b = 0; b < B; ++b) {
      if (k >= fps[b]->fwd.sched.passes.size()) continue;
      PassItem it = fps[b]->items_fwd_phi[k];
      it.recs = recs_all + gate_base[b];
      it.tile_begin = L->total;
      L->total += fps[b]->tiles;
      L->bytes += 2.0 * (double)qsv_state_bytes(states[b]->n, states[b]->dt);
      L->general = L->general || fps[b]->fwd.sched.passes[k].general;
      items.push_back(it);
    }
    launch_shape(L->total, &L->grid, &L->chunk, kBatchGridCap);
    for (PassItem& it : items) item_span(it.tile_begin, 1ll << it.n_outer, L->chunk, &it.first_wg, &it.nb);
    L->n_items = (int)items.size();
    QSV_TRY(upload_vec(L->d_items, items, st));
    bp->fwd.push_back(std::move(L));
  }
  // reverse-sweep levels: partial blocks [local slot][workgroup] per (level, circuit)
  std::vector<std::vector<PassItem>> level_items(lb);
  std::vector<std::vector<int>> level_owner(lb);
  int64_t total_partials = 0;
  for (size_t k = 0; k < lb; ++k) {
    auto L = std::make_unique<BatchLevel>();
    for (int b = 0; b < B; ++b) {
      if (k >= fps[b]->bwd.sched.passes.size()) continue;
      PassItem it = fps[b]->items_bwd[k];
      it.recs = recs_all + gate_base[b];
      it.tile_begin = L->total;
      L->total += fps[b]->tiles;
      L->bytes += 4.0 * (double)qsv_state_bytes(states[b]->n, states[b]->dt);
      L->general = L->general || fps[b]->bwd.sched.passes[k].general;
      level_items[k].push_back(it);
      level_owner[k].push_back(b);
    }
    launch_shape(L->total, &L->grid, &L->chunk, kBatchGridCap);
    for (PassItem& it : level_items[k])
      item_span(it.tile_begin, 1ll << it.n_outer, L->chunk, &it.first_wg, &it.nb);
    L->n_items = (int)level_items[k].size();
    bp->bwd.push_back(std::move(L));
  }
  std::vector<int64_t> occ_base;
  std::vector<int32_t> occ_nb;
  std::vector<int64_t> occ_off(B);
  for (int b = 0; b < B; ++b) {
    occ_off[b] = (int64_t)occ_base.size();
    const int no = plans[b]->n_occ ? plans[b]->n_occ : 1;
    occ_base.resize(occ_base.size() + no, 0);
    occ_nb.resize(occ_nb.size() + no, 0);
  }
  int64_t off = 0;
  std::vector<std::vector<int64_t>> item_off(lb);
  for (size_t k = 0; k < lb; ++k) {
    for (size_t i = 0; i < level_items[k].size(); ++i) {
      const int b = level_owner[k][i];
      const Schedule& bs = fps[b]->bwd.sched;
      const PassDesc& pd = bs.passes[k];
      const PassItem& it = level_items[k][i];
      item_off[k].push_back(off);
      for (int j = 0; j < pd.n_slots; ++j) {
        const int gs = bs.slot_map[pd.slot_begin + j];
        occ_base[occ_off[b] + gs] = off + (int64_t)j * it.nb;
        occ_nb[occ_off[b] + gs] = it.nb;
      }
      off += (int64_t)pd.n_slots * it.nb;
    }
  }
  total_partials = off;
  QSV_TRY(bp->partials.ensure(sizeof(double2) * (total_partials ? total_partials : 1), st));
  for (size_t k = 0; k < lb; ++k) {
    for (size_t i = 0; i < level_items[k].size(); ++i)
      level_items[k][i].partials = bp->partials.as<double2>() + item_off[k][i];
    QSV_TRY(upload_vec(bp->bwd[k]->d_items, level_items[k], st));
  }
  QSV_TRY(upload_vec(bp->d_occ_base, occ_base, st));
  QSV_TRY(upload_vec(bp->d_occ_nb, occ_nb, st));
  std::vector<FinalDesc> fds(B);
  int64_t pb = 0;
  for (int b = 0; b < B; ++b) {
    FinalDesc& fd = fds[b];
    std::memset(&fd, 0, sizeof fd);
    fd.partials = bp->partials.as<double2>();
    fd.occ_base = bp->d_occ_base.as<int64_t>() + occ_off[b];
    fd.occ_nb = bp->d_occ_nb.as<int32_t>() + occ_off[b];
    fd.param_ptr = plans[b]->d_param_ptr.as<int32_t>();
    fd.occ = plans[b]->d_occ.as<int32_t>();
    fd.grad_off = theta_off[b];
    fd.p_begin = pb;
    fd.n_theta = plans[b]->n_theta;
    pb += plans[b]->n_theta;
  }
  bp->total_params = pb;
  QSV_TRY(upload_vec(bp->d_final, fds, st));
  bp->plans = plans;
  bp->states.assign(states, states + B);
  return QSV_OK;
}

template <typename R>
static qsv_status batched_t(qsv_state* const* states, int B, const std::vector<Plan*>& plans,
                            const std::vector<PauliPlan*>& hps, BatchPlan* bp,
                            const double* d_theta_flat, const int64_t* theta_off,
                            double* d_energy, double* d_grad_flat) {
  qsv_state* s0 = states[0];
  const hipStream_t st = s0->stream;
  (void)plans;
  (void)hps;
  (void)theta_off;
  HIP_TRY(launch_prep(bp->d_gates_all.as<GateDesc>(), bp->total_gates, d_theta_flat,
                      bp->d_recs_all.as<GateRec>(), st));
  for (auto& L : bp->fwd)
    QSV_TRY(timed(s0, "k_pass_fwd", L->bytes, [&] {
      return launch_fused_forward<R>(L->d_items.as<PassItem>(), L->n_items, L->total, L->chunk,
                                     bp->r, bp->w, L->general, L->grid, st);
    }));
  double pauli_bytes = 0;
  for (int b = 0; b < B; ++b) pauli_bytes += 2.0 * (double)qsv_state_bytes(states[b]->n, states[b]->dt);
  QSV_TRY(timed(s0, "k_pauli", pauli_bytes, [&] {
    return launch_pauli_batched<R>(bp->d_jobs.as<PauliJob>(), B, kBatchPauliBlocks,
                                   bp->partials_e.as<double2>(), st);
  }));
  for (auto& L : bp->bwd)
    QSV_TRY(timed(s0, "k_pass_bwd", L->bytes, [&] {
      return launch_fused_backward<R>(L->d_items.as<PassItem>(), L->n_items, L->total, L->chunk,
                                      bp->r, bp->w, L->general, L->grid, st);
    }));
  HIP_TRY(launch_final_energy_batched(bp->partials_e.as<double2>(), kBatchPauliBlocks, B, d_energy,
                                      st));
  HIP_TRY(launch_final_grad(bp->d_final.as<FinalDesc>(), B, bp->total_params, d_grad_flat, st));
  return QSV_OK;
}

template <typename R>
static qsv_status reference_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                              double* d_energy, double* d_grad);

// Checks of a batch call (qsv_adjoint_gradient_batched, qsv_reference_gradient_batched).
static qsv_status batch_validate(int32_t n_batch, qsv_state* const* states,
                                 const qsv_gate* const* gates, const int32_t* n_gates,
                                 const double* d_theta_flat, const int64_t* theta_off,
                                 const int32_t* n_theta, const qsv_pauli_sum* H,
                                 const double* d_energy, const double* d_grad_flat) {
  if (n_batch < 1) return fail(QSV_ERR_INVALID_ARG, "n_batch = %d < 1", n_batch);
  if (!states || !gates || !n_gates || !theta_off || !n_theta || !H)
    return fail(QSV_ERR_INVALID_ARG, "NULL batch array");
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  qsv_state* s0 = states[0];
  QSV_TRY(check_handle(s0));
  bool any_theta = false;
  for (int b = 0; b < n_batch; ++b) {
    qsv_state* s = states[b];
    if (!s) return fail(QSV_ERR_INVALID_ARG, "states[%d] is NULL", b);
    if (s->device != s0->device || s->dt != s0->dt)
      return fail(QSV_ERR_INVALID_ARG, "states[%d]: device or dtype differs from states[0]", b);
    for (int c = 0; c < b; ++c)
      if (states[c] == s) return fail(QSV_ERR_INVALID_ARG, "states[%d] repeats states[%d]", b, c);
    QSV_TRY(qsv_validate_circuit(s->n, gates[b], n_gates[b], n_theta[b]));
    QSV_TRY(qsv_validate_pauli_sum(s->n, &H[b]));
    if (theta_off[b] < 0) return fail(QSV_ERR_INVALID_ARG, "theta_off[%d] < 0", b);
    any_theta = any_theta || n_theta[b] > 0;
  }
  if (any_theta && (!d_theta_flat || !d_grad_flat))
    return fail(QSV_ERR_INVALID_ARG, "d_theta_flat or d_grad_flat is NULL");
  return QSV_OK;
}

// The circuits' plans and Pauli plans (on states[0]'s stream, which the caller has set).
static qsv_status batch_plans(int32_t n_batch, qsv_state* const* states,
                              const qsv_gate* const* gates, const int32_t* n_gates,
                              const double* d_theta_flat, const int32_t* n_theta,
                              const qsv_pauli_sum* H, std::vector<Plan*>& plans,
                              std::vector<PauliPlan*>& hps) {
  plans.assign(n_batch, nullptr);
  hps.assign(n_batch, nullptr);
  for (int b = 0; b < n_batch; ++b) {
    QSV_TRY(get_plan(states[b], gates[b], n_gates[b], n_theta[b], &plans[b]));
    QSV_TRY(check_theta(plans[b], d_theta_flat));
    QSV_TRY(get_pauli(states[b], &H[b], &hps[b]));
  }
  return QSV_OK;
}

// The cached batch plan of these circuits (wave: one wave per circuit; else the fused levels of
// geometry (r, w)), built on first use.
static qsv_status get_batch_plan(int32_t n_batch, qsv_state* const* states,
                                 const std::vector<Plan*>& plans,
                                 const std::vector<PauliPlan*>& hps, const int64_t* theta_off,
                                 bool wave, int r, int w, BatchPlan** out) {
  qsv_state* s0 = states[0];
  uint64_t key = fnv1a(&n_batch, sizeof n_batch);
  key = fnv1a(states, sizeof(qsv_state*) * n_batch, key);
  key = fnv1a(plans.data(), sizeof(Plan*) * n_batch, key);
  key = fnv1a(theta_off, sizeof(int64_t) * n_batch, key);
  key = fnv1a(&r, sizeof r, key);
  key = fnv1a(&w, sizeof w, key);
  key = fnv1a(&wave, sizeof wave, key);
  std::vector<uint64_t> serials;
  for (int b = 0; b < n_batch; ++b) {
    serials.push_back(plans[b]->serial);
    serials.push_back(hps[b]->serial);
  }
  key = fnv1a(serials.data(), sizeof(uint64_t) * serials.size(), key);
  auto it = s0->batches.find(key);
  if (it != s0->batches.end() && it->second->serials == serials &&
      std::equal(it->second->states.begin(), it->second->states.end(), states)) {
    *out = it->second.get();
    return QSV_OK;
  }
  if (s0->batches.size() >= kMaxCachedBatches) {
    HIP_TRY(hipStreamSynchronize(s0->stream));
    s0->batches.clear();
  }
  auto nbp = std::make_unique<BatchPlan>();
  if (wave)
    QSV_TRY(build_batch_wave(states, plans, hps, n_batch, theta_off, nbp.get()));
  else
    QSV_TRY(build_batch(states, plans, hps, n_batch, theta_off, r, w, nbp.get()));
  nbp->serials = serials;
  nbp->key = key;
  *out = nbp.get();
  s0->batches[key] = std::move(nbp);
  return QSV_OK;
}

static bool batch_is_wave(int32_t n_batch, qsv_state* const* states) {
  bool wave = true;
  for (int b = 0; b < n_batch && wave; ++b) wave = wave_path(states[b]);
  return wave;
}

extern "C" qsv_status qsv_adjoint_gradient_batched(int32_t n_batch, qsv_state* const* states,
                                                   const qsv_gate* const* gates,
                                                   const int32_t* n_gates,
                                                   const double* d_theta_flat,
                                                   const int64_t* theta_off,
                                                   const int32_t* n_theta,
                                                   const qsv_pauli_sum* H, double* d_energy,
                                                   double* d_grad_flat) {
  QSV_TRY(batch_validate(n_batch, states, gates, n_gates, d_theta_flat, theta_off, n_theta, H,
                         d_energy, d_grad_flat));
  qsv_state* s0 = states[0];
  StreamOverride so(states, n_batch, s0->stream);
  std::vector<Plan*> plans;
  std::vector<PauliPlan*> hps;
  QSV_TRY(batch_plans(n_batch, states, gates, n_gates, d_theta_flat, n_theta, H, plans, hps));
  // every circuit small enough for one wave: one launch of one wave per circuit
  const bool wave = batch_is_wave(n_batch, states);
  // a common tile geometry that fits every circuit; otherwise one circuit after the other
  int r = 0, w = 0;
  bool fused = !wave && fusion_geometry(s0, &r, &w);
  for (int b = 0; b < n_batch && fused; ++b) {
    int rb = 0, wb = 0;
    fused = fusion_geometry(states[b], &rb, &wb) && r + w <= states[b]->n &&
            !plans[b]->gates.empty();
  }
  if (!fused && !wave) {
    for (int b = 0; b < n_batch; ++b) {
      qsv_state* s = states[b];
      double* g = d_grad_flat ? d_grad_flat + theta_off[b] : nullptr;
      if (s->dt == QSV_C128)
        QSV_TRY(adjoint_t<double>(s, plans[b], hps[b], d_theta_flat + theta_off[b], d_energy + b, g));
      else
        QSV_TRY(adjoint_t<float>(s, plans[b], hps[b], d_theta_flat + theta_off[b], d_energy + b, g));
    }
    return QSV_OK;
  }
  BatchPlan* bp = nullptr;
  QSV_TRY(get_batch_plan(n_batch, states, plans, hps, theta_off, wave, r, w, &bp));
  const void* key_parts[3] = {d_theta_flat, d_energy, d_grad_flat};
  const uint64_t gkey =
      fnv1a(key_parts, sizeof key_parts, fnv1a(&bp->serial, sizeof bp->serial, bp->key));
  return run_graph(
      s0, gkey,
      [&] {
        if (bp->wave)
          return s0->dt == QSV_C128 ? batched_wave_t<double>(states, n_batch, bp, d_theta_flat,
                                                             theta_off, d_energy, d_grad_flat)
                                    : batched_wave_t<float>(states, n_batch, bp, d_theta_flat,
                                                            theta_off, d_energy, d_grad_flat);
        return s0->dt == QSV_C128
                   ? batched_t<double>(states, n_batch, plans, hps, bp, d_theta_flat, theta_off,
                                       d_energy, d_grad_flat)
                   : batched_t<float>(states, n_batch, plans, hps, bp, d_theta_flat, theta_off,
                                      d_energy, d_grad_flat);
      },
      states + 1, n_batch - 1);
}

template <typename R>
static qsv_status batched_wave_reference_t(qsv_state* const* states, int B, BatchPlan* bp,
                                           const double* d_theta_flat, double* d_energy,
                                           double* d_grad_flat) {
  qsv_state* s0 = states[0];
  const hipStream_t st = s0->stream;
  if (bp->wave_needs_recs)
    QSV_TRY(timed(s0, "k_prep", 0, [&] {
      return launch_prep(bp->d_gates_all.as<GateDesc>(), bp->total_gates, d_theta_flat,
                         bp->d_recs_all.as<GateRec>(), st);
    }));
  double bytes = 0;
  int max_occ = 0;
  for (int b = 0; b < B; ++b) {
    bytes += (bp->plans[b]->n_occ + 1.0) * (double)qsv_state_bytes(states[b]->n, states[b]->dt);
    max_occ = std::max(max_occ, bp->plans[b]->n_occ);
  }
  return timed(s0, "k_wave_reference", bytes, [&] {
    return launch_wave_reference<R>(bp->d_wave_jobs.as<WaveJob>(), B, max_occ, WaveJob{},
                                    d_theta_flat, d_energy, d_grad_flat, st);
  });
}

extern "C" qsv_status qsv_reference_gradient_batched(int32_t n_batch, qsv_state* const* states,
                                                     const qsv_gate* const* gates,
                                                     const int32_t* n_gates,
                                                     const double* d_theta_flat,
                                                     const int64_t* theta_off,
                                                     const int32_t* n_theta,
                                                     const qsv_pauli_sum* H, double* d_energy,
                                                     double* d_grad_flat) {
  QSV_TRY(batch_validate(n_batch, states, gates, n_gates, d_theta_flat, theta_off, n_theta, H,
                         d_energy, d_grad_flat));
  qsv_state* s0 = states[0];
  StreamOverride so(states, n_batch, s0->stream);
  std::vector<Plan*> plans;
  std::vector<PauliPlan*> hps;
  QSV_TRY(batch_plans(n_batch, states, gates, n_gates, d_theta_flat, n_theta, H, plans, hps));
  if (!batch_is_wave(n_batch, states)) {
    for (int b = 0; b < n_batch; ++b) {
      qsv_state* s = states[b];
      double* g = d_grad_flat ? d_grad_flat + theta_off[b] : nullptr;
      const double* th = d_theta_flat ? d_theta_flat + theta_off[b] : nullptr;
      if (s->dt == QSV_C128)
        QSV_TRY(reference_t<double>(s, plans[b], hps[b], th, d_energy + b, g));
      else
        QSV_TRY(reference_t<float>(s, plans[b], hps[b], th, d_energy + b, g));
    }
    return QSV_OK;
  }
  BatchPlan* bp = nullptr;
  QSV_TRY(get_batch_plan(n_batch, states, plans, hps, theta_off, true, 0, 0, &bp));
  return s0->dt == QSV_C128
             ? batched_wave_reference_t<double>(states, n_batch, bp, d_theta_flat, d_energy,
                                                d_grad_flat)
             : batched_wave_reference_t<float>(states, n_batch, bp, d_theta_flat, d_energy,
                                               d_grad_flat);
}

// ------------------------------------------------------------------------------------------------
// GPU parameter-shift baseline
// ------------------------------------------------------------------------------------------------
template <typename R>
static qsv_status param_shift_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                                int first, int count, double* d_grad) {
  const hipStream_t st = s->stream;
  const int n = s->n, nb = s->nb, nt = p->n_theta;
  QSV_TRY(s->theta_scratch.ensure(sizeof(double) * (nt ? nt : 1), st));
  QSV_TRY(s->energies.ensure(sizeof(double) * 2 * (count ? count : 1), st));
  QSV_TRY(s->epartials.ensure(sizeof(double2) * nb, st));
  double* th = s->theta_scratch.as<double>();
  double* e = s->energies.as<double>();
  double2* ep = s->epartials.as<double2>();
  void* phi = s->d_work;
  const double half_pi = 1.57079632679489661923;
  for (int i = 0; i < count; ++i) {
    for (int side = 0; side < 2; ++side) {
      HIP_TRY(launch_shift_theta(th, d_theta, nt, first + i, side ? -half_pi : half_pi, st));
      HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), th,
                          p->d_recs.as<GateRec>(), st));
      QSV_TRY(forward<R>(s, p, s->d_state, phi));
      QSV_TRY(pauli<R>(s, hp, phi, nullptr, ep));
      HIP_TRY(launch_final_energy(ep, nb, e + 2 * i + side, nullptr, st));
    }
  }
  HIP_TRY(launch_ps_combine(d_grad, e, first, count, st));
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// non-Hermitian operators (App. B.4)
// ------------------------------------------------------------------------------------------------
template <typename R>
static qsv_status nonherm_t(qsv_state* s, Plan* p, PauliPlan* ha, PauliPlan* hd,
                            const double* d_theta, double* d_energy, double* d_grad) {
  const hipStream_t st = s->stream;
  const int nb = s->nb;
  void* phi = s->d_work;
  void* lam = static_cast<char*>(s->d_work) + qsv_state_bytes(s->n, s->dt);
  QSV_TRY(s->epartials.ensure(sizeof(double2) * nb, st));
  double2* ep = s->epartials.as<double2>();
  int r = 0, w = 0;
  if (!fusion_geometry(s, &r, &w)) auto_geometry(s, &r, &w);  // complex entries: fused only
  const int saved[3] = {s->fusion_mode, s->fr, s->fw};
  s->fusion_mode = 1;
  s->fr = r;
  s->fw = w;
  FusedPlan* fp = nullptr;
  qsv_status rc = get_fused(s, p, r, w, &fp);
  if (rc == QSV_OK && fp->partials_a.cap < fp->partials.cap) {
    rc = fp->partials_a.ensure(fp->partials.cap, st);
    if (rc == QSV_OK)
      rc = upload_final(fp->d_final_a, fp->partials_a, fp->d_occ_base, fp->d_occ_nb, p, st);
  }
  auto run = [&]() -> qsv_status {
    HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                        p->d_recs.as<GateRec>(), st));
    // run with A: psi in phi, lambda = A psi, <A> = <psi|A psi>, complex entries
    QSV_TRY(forward<R>(s, p, s->d_state, phi));
    QSV_TRY(pauli<R>(s, ha, phi, lam, ep));
    HIP_TRY(launch_final_energy(ep, nb, d_energy, d_energy + 1, st));
    const FinalDesc* fd = nullptr;
    QSV_TRY(backward<R>(s, p, &fd, true));
    HIP_TRY(hipMemcpyAsync(fp->partials_a.p, fp->partials.p, fp->partials.cap,
                           hipMemcpyDeviceToDevice, st));
    // run with A^dag
    QSV_TRY(forward<R>(s, p, s->d_state, phi));
    QSV_TRY(pauli<R>(s, hd, phi, lam, ep));
    QSV_TRY(backward<R>(s, p, &fd, true));
    HIP_TRY(launch_final_grad_nonherm(fp->d_final_a.as<FinalDesc>(), fd, p->n_theta, d_grad, st));
    return QSV_OK;
  };
  if (rc == QSV_OK) rc = run();
  s->fusion_mode = saved[0];
  s->fr = saved[1];
  s->fw = saved[2];
  return rc;
}

extern "C" qsv_status qsv_adjoint_gradient_nonhermitian(qsv_state* s, const qsv_gate* gates,
                                                        int32_t n_gates, const double* d_theta,
                                                        int32_t n_theta, const qsv_pauli_sum* A,
                                                        const double* coeffs_im,
                                                        double* d_energy, double* d_grad) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  QSV_TRY(qsv_validate_pauli_sum(s->n, A));
  if (A->n_terms > 0 && !coeffs_im) return fail(QSV_ERR_INVALID_ARG, "coeffs_im is NULL");
  for (int t = 0; t < A->n_terms; ++t)
    if (!std::isfinite(coeffs_im[t]))
      return fail(QSV_ERR_INVALID_ARG, "coeffs_im[%d] is not finite", t);
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  if (n_theta > 0 && !d_grad) return fail(QSV_ERR_INVALID_ARG, "d_grad is NULL");
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  QSV_TRY(check_theta(p, d_theta));
  PauliPlan *ha = nullptr, *hd = nullptr;
  QSV_TRY(get_pauli_ex(s, A, coeffs_im, 1.0, &ha));
  QSV_TRY(get_pauli_ex(s, A, coeffs_im, -1.0, &hd));
  if (p->gates.empty()) {  // <A> of |in> and an all-zero gradient
    QSV_TRY(s->epartials.ensure(sizeof(double2) * s->nb, s->stream));
    double2* ep = s->epartials.as<double2>();
    if (s->dt == QSV_C128) QSV_TRY(pauli<double>(s, ha, s->d_state, nullptr, ep));
    else QSV_TRY(pauli<float>(s, ha, s->d_state, nullptr, ep));
    HIP_TRY(launch_final_energy(ep, s->nb, d_energy, d_energy + 1, s->stream));
    QSV_TRY(get_gate_granular(s, p));
    const FinalDesc* fd = p->d_gg_final.as<FinalDesc>();
    HIP_TRY(launch_final_grad_nonherm(fd, fd, p->n_theta, d_grad, s->stream));
    return QSV_OK;
  }
  return s->dt == QSV_C128 ? nonherm_t<double>(s, p, ha, hd, d_theta, d_energy, d_grad)
                           : nonherm_t<float>(s, p, ha, hd, d_theta, d_energy, d_grad);
}

// ------------------------------------------------------------------------------------------------
// reference gradient (Algorithm 2)
// ------------------------------------------------------------------------------------------------
static constexpr size_t kRefPoolBytes = size_t(1) << 30;  // mu pool of the parallel entries

static qsv_status get_ref(qsv_state* s, Plan* p, FusedPlan* fp, RefPlan** out) {
  const int key = fp->r * 16 + fp->w;
  auto it = p->ref.find(key);
  if (it != p->ref.end()) {
    *out = it->second.get();
    return QSV_OK;
  }
  const hipStream_t st = s->stream;
  auto rp = std::make_unique<RefPlan>();
  {
    std::string msg;
    // the derivative substitution addresses every op of the pass on its own
    if (!build_forward_schedule(s->n, p->gates, fp->t, fp->r, fp->w,
                                run_qubits_for(s->dt == QSV_C128, s->n), fp->bwd.sched,
                                rp->fwd.sched, &msg, false))
      return fail(QSV_ERR_INTERNAL, "forward schedule: %s", msg.c_str());
    QSV_TRY(upload_schedule(rp->fwd, st));
  }
  const FusedSchedule& fs = rp->fwd;
  const Schedule& sc = fs.sched;
  const int K = (int)sc.passes.size(), G = (int)p->gates.size();
  const size_t S = qsv_state_bytes(s->n, s->dt);
  rp->K = K;
  rp->E = p->n_occ;
  rp->single = fp->tiles == 1;
  rp->nb = rp->single ? 1 : fp->nb;
  std::vector<int> op_of_gate(G, -1);
  for (size_t i = 0; i < sc.order.size(); ++i) op_of_gate[sc.order[i]] = (int)i;
  if (rp->single) {
    rp->per_launch = std::max<int64_t>(1, std::min<int64_t>(rp->E, (int64_t)(kRefPoolBytes / S)));
    QSV_TRY(rp->mu_pool.ensure(S * (size_t)std::max<int64_t>(rp->per_launch, 1), st));
  }
  QSV_TRY(rp->partials.ensure(sizeof(double2) * (size_t)std::max<int64_t>(rp->E * rp->nb, 1), st));
  const int n_outer = std::max(0, s->n - fp->t);
  void* lam = static_cast<char*>(s->d_work) + S;
  std::vector<PassItem> items((size_t)rp->E * K);
  for (int g = 0; g < G; ++g) {
    const int np = kind_nparams(p->gates[g].kind);
    if (!np) continue;
    const int i = op_of_gate[g];
    const int pk = sc.pass_of[i];
    const int kloc = i - sc.passes[pk].op_begin;
    for (int j = 0; j < np; ++j) {
      const int64_t o = p->slot_of_gate[g] + j;
      // mu: a pool slot (parallel entries) or the phi buffer, free once lambda = H psi is built
      const int64_t slot = rp->single ? o % rp->per_launch : 0;
      void* mu = rp->single ? static_cast<char*>(rp->mu_pool.p) + (size_t)slot * S : s->d_work;
      for (int k = 0; k < K; ++k) {
        PassItem it = make_item(fs, k, p, k == 0 ? s->d_state : mu, mu, nullptr, n_outer);
        if (rp->single) {
          it.tile_begin = slot * K + k;
          it.first_wg = (int32_t)slot;
          it.nb = 1;
        } else {
          it.nb = fp->nb;
        }
        if (k == pk) {
          it.sub_op = kloc;
          it.sub_param = j;
        }
        if (k == K - 1) {
          it.lam = lam;
          it.partials = rp->partials.as<double2>() + o * rp->nb;
        }
        items[(size_t)o * K + k] = it;
      }
    }
  }
  QSV_TRY(upload_vec(rp->items, items, st));
  std::vector<int64_t> base((size_t)std::max<int64_t>(rp->E, 1), 0);
  std::vector<int32_t> cnt((size_t)std::max<int64_t>(rp->E, 1), rp->nb);
  for (int64_t o = 0; o < rp->E; ++o) base[o] = o * rp->nb;
  QSV_TRY(upload_vec(rp->d_occ_base, base, st));
  QSV_TRY(upload_vec(rp->d_occ_nb, cnt, st));
  QSV_TRY(upload_final(rp->d_final, rp->partials, rp->d_occ_base, rp->d_occ_nb, p, st));
  *out = rp.get();
  p->ref[key] = std::move(rp);
  return QSV_OK;
}

template <typename R>
static qsv_status reference_t(qsv_state* s, Plan* p, PauliPlan* hp, const double* d_theta,
                              double* d_energy, double* d_grad) {
  const hipStream_t st = s->stream;
  const int nb = s->nb;
  const double S = state_bytes_d(s);
  void* phi = s->d_work;
  void* lam = static_cast<char*>(s->d_work) + qsv_state_bytes(s->n, s->dt);
  QSV_TRY(s->epartials.ensure(sizeof(double2) * nb, st));
  double2* ep = s->epartials.as<double2>();
  HIP_TRY(launch_prep(p->d_gates.as<GateDesc>(), (int)p->gates.size(), d_theta,
                      p->d_recs.as<GateRec>(), st));
  // lambda := |in>, lambda <- U lambda (in the phi buffer), lambda <- H lambda; E = <psi|H psi>
  QSV_TRY(forward<R>(s, p, s->d_state, phi));
  QSV_TRY(pauli<R>(s, hp, phi, lam, ep));
  HIP_TRY(launch_final_energy(ep, nb, d_energy, nullptr, st));
  if (p->n_occ == 0) {  // no gate carries a parameter: every entry is 0
    QSV_TRY(get_gate_granular(s, p));
    HIP_TRY(launch_final_grad(p->d_gg_final.as<FinalDesc>(), 1, p->n_theta, d_grad, st));
    return QSV_OK;
  }
  int r = 0, w = 0;
  if (!fusion_geometry(s, &r, &w)) auto_geometry(s, &r, &w);
  FusedPlan* fp = nullptr;
  QSV_TRY(get_fused(s, p, r, w, &fp));
  RefPlan* rp = nullptr;
  QSV_TRY(get_ref(s, p, fp, &rp));
  const int K = rp->K;
  const PassItem* items = rp->items.as<PassItem>();
  if (rp->single) {
    for (int64_t e0 = 0; e0 < rp->E; e0 += rp->per_launch) {
      const int64_t m = std::min<int64_t>(rp->per_launch, rp->E - e0);
      QSV_TRY(timed(s, "k_pass_fwd_ref", 2 * S * K * m, [&] {
        return launch_fused_forward<R>(items + e0 * K, (int)(m * K), m * K, K, r, w, true,
                                       (int)m, st);
      }));
    }
  } else {
    for (int64_t o = 0; o < rp->E; ++o)
      for (int k = 0; k < K; ++k)
        QSV_TRY(timed(s, "k_pass_fwd_ref", 2 * S, [&] {
          return launch_fused_forward<R>(items + o * K + k, 1, fp->tiles, fp->chunk, r, w, true,
                                         fp->grid, st);
        }));
  }
  HIP_TRY(launch_final_grad(rp->d_final.as<FinalDesc>(), 1, p->n_theta, d_grad, st));
  return QSV_OK;
}

extern "C" qsv_status qsv_reference_gradient(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                             const double* d_theta, int32_t n_theta,
                                             const qsv_pauli_sum* H, double* d_energy,
                                             double* d_grad) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  if (n_theta > 0 && !d_grad) return fail(QSV_ERR_INVALID_ARG, "d_grad is NULL");
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  QSV_TRY(check_theta(p, d_theta));
  PauliPlan* hp = nullptr;
  QSV_TRY(get_pauli(s, H, &hp));
  if (wave_path(s))
    return s->dt == QSV_C128 ? wave_reference_t<double>(s, p, hp, d_theta, d_energy, d_grad)
                             : wave_reference_t<float>(s, p, hp, d_theta, d_energy, d_grad);
  return s->dt == QSV_C128 ? reference_t<double>(s, p, hp, d_theta, d_energy, d_grad)
                           : reference_t<float>(s, p, hp, d_theta, d_energy, d_grad);
}

extern "C" qsv_status qsv_param_shift_gradient(qsv_state* s, const qsv_gate* gates,
                                               int32_t n_gates, const double* d_theta,
                                               int32_t n_theta, const qsv_pauli_sum* H,
                                               int32_t first, int32_t count, double* d_grad) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (first < 0 || count < 0 || (int64_t)first + count > n_theta)
    return fail(QSV_ERR_INVALID_ARG, "entry range [%d, %d + %d) outside [0, %d)", first, first,
                count, n_theta);
  if (count > 0 && !d_grad) return fail(QSV_ERR_INVALID_ARG, "d_grad is NULL");
  if (count > 0 && !d_theta) return fail(QSV_ERR_INVALID_ARG, "d_theta is NULL");
  std::vector<int> uses(n_theta, 0);
  for (int32_t k = 0; k < n_gates; ++k) {
    const qsv_gate& g = gates[k];
    if (g.kind == K_CRX || g.kind == K_CRY || g.kind == K_CRZ)
      return fail(QSV_ERR_UNSUPPORTED, "gate %d: the two-term shift rule is not exact for "
                  "controlled rotations", k);
    for (int j = 0; j < kind_nparams(g.kind); ++j)
      if (++uses[g.param[j]] > 1)
        return fail(QSV_ERR_UNSUPPORTED, "parameter %d is used by more than one gate",
                    g.param[j]);
  }
  for (int32_t k = 0; k < n_gates; ++k)
    if (!kind_unitary(gates[k].kind))
      return fail(QSV_ERR_UNSUPPORTED,
                  "gate %d: the parameter-shift rule does not hold for non-unitary gates", k);
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  PauliPlan* hp = nullptr;
  QSV_TRY(get_pauli(s, H, &hp));
  return s->dt == QSV_C128 ? param_shift_t<double>(s, p, hp, d_theta, first, count, d_grad)
                           : param_shift_t<float>(s, p, hp, d_theta, first, count, d_grad);
}

// ------------------------------------------------------------------------------------------------
// measurement
// ------------------------------------------------------------------------------------------------
static qsv_status drain_timer(qsv_state* s) {
  Timer& t = s->timer;
  if (t.pending.empty()) return QSV_OK;
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (auto& pnd : t.pending) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, pnd.a, pnd.b));
    qsv_kernel_stat& a = t.agg[pnd.name];
    if (a.launches == 0) {
      std::memset(&a, 0, sizeof a);
      std::snprintf(a.name, sizeof a.name, "%s", pnd.name);
    }
    a.launches += 1;
    a.total_ms += ms;
    a.bytes += pnd.bytes;
    t.pool.push_back(pnd.a);
    t.pool.push_back(pnd.b);
  }
  t.pending.clear();
  return QSV_OK;
}

extern "C" qsv_status qsv_timing_enable(qsv_state* s, const char* name_filter) {
  QSV_TRY(check_handle(s));
  QSV_TRY(drain_timer(s));
  s->timer.agg.clear();
  s->timer.on = name_filter != nullptr;
  s->timer.filter = name_filter ? name_filter : "";
  return QSV_OK;
}

extern "C" qsv_status qsv_timing_read(qsv_state* s, qsv_kernel_stat* out, int32_t max_out,
                                      int32_t* n_out) {
  QSV_TRY(check_handle(s));
  if (max_out < 0 || (max_out > 0 && !out) || !n_out)
    return fail(QSV_ERR_INVALID_ARG, "bad output array");
  QSV_TRY(drain_timer(s));
  std::vector<qsv_kernel_stat> v;
  for (auto& kv : s->timer.agg) v.push_back(kv.second);
  std::sort(v.begin(), v.end(), [](const qsv_kernel_stat& a, const qsv_kernel_stat& b) {
    return a.total_ms > b.total_ms;
  });
  const int32_t m = std::min<int32_t>(max_out, (int32_t)v.size());
  for (int32_t i = 0; i < m; ++i) out[i] = v[i];
  *n_out = m;
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// fusion control and schedule inspection
// ------------------------------------------------------------------------------------------------
extern "C" qsv_status qsv_set_fusion(qsv_state* s, int32_t mode, int32_t reg_qubits,
                                     int32_t threads_log2) {
  QSV_TRY(check_handle(s));
  if (mode < -1 || mode > 3) return fail(QSV_ERR_INVALID_ARG, "fusion mode %d", mode);
  if (mode == 2 && s->n > kWaveMaxQubits)
    return fail(QSV_ERR_UNSUPPORTED, "the one-wave sweep holds at most %d qubits (state has %d)",
                kWaveMaxQubits, s->n);
  if (mode == 3 && s->n > kWaveChunkMaxQubits)
    return fail(QSV_ERR_UNSUPPORTED, "the chunked sweep holds at most %d qubits (state has %d)",
                kWaveChunkMaxQubits, s->n);
  if (mode == 1) {
    if (!fused_config_supported(reg_qubits, threads_log2, s->dt == QSV_C128))
      return fail(QSV_ERR_UNSUPPORTED, "no fused kernel for reg_qubits=%d threads_log2=%d",
                  reg_qubits, threads_log2);
  }
  s->fusion_mode = mode;
  s->fr = mode == 1 ? reg_qubits : 0;
  s->fw = mode == 1 ? threads_log2 : 0;
  return QSV_OK;
}

extern "C" qsv_status qsv_get_fusion(qsv_state* s, int32_t* mode, int32_t* reg_qubits,
                                     int32_t* threads_log2) {
  QSV_TRY(check_handle(s));
  if (!mode || !reg_qubits || !threads_log2) return fail(QSV_ERR_INVALID_ARG, "NULL output");
  if (wave_path(s)) {  // the gradient runs the one-wave sweep (mode 3: its chunked variant)
    *mode = s->fusion_mode == 3 ? 3 : 2;
    *reg_qubits = *threads_log2 = 0;
    return QSV_OK;
  }
  int r = 0, w = 0;
  const bool f = fusion_geometry(s, &r, &w);
  *mode = f ? 1 : 0;
  *reg_qubits = r;
  *threads_log2 = w;
  return QSV_OK;
}

extern "C" qsv_status qsv_schedule_describe(int32_t n, const qsv_gate* gates, int32_t n_gates,
                                            int32_t backward, int32_t reg_qubits,
                                            int32_t threads_log2, qsv_dtype dt,
                                            qsv_schedule_info* out) {
  QSV_TRY(qsv_validate_circuit(n, gates, n_gates, 1 << 30));
  if (!out || (n_gates > 0 && (!out->order || !out->pass_of || !out->phase_of ||
                               !out->tile_mask || !out->reg_mask)))
    return fail(QSV_ERR_INVALID_ARG, "NULL output array");
  if (reg_qubits < 1 || reg_qubits > kMaxRegBits || threads_log2 < 1 ||
      reg_qubits + threads_log2 > kMaxTileBits)
    return fail(QSV_ERR_INVALID_ARG, "tile geometry r=%d w=%d invalid for n=%d", reg_qubits,
                threads_log2, n);
  std::vector<GateDesc> g(reinterpret_cast<const GateDesc*>(gates),
                          reinterpret_cast<const GateDesc*>(gates) + n_gates);
  std::vector<int32_t> slot(n_gates, -1);
  int sl = 0;
  for (int k = n_gates - 1; k >= 0; --k)
    if (kind_nparams(g[k].kind)) {
      slot[k] = sl;
      sl += kind_nparams(g[k].kind);
    }
  std::vector<int> seq(n_gates);
  for (int k = 0; k < n_gates; ++k) seq[k] = n_gates - 1 - k;
  Schedule sc;
  std::string msg;
  if (dt != QSV_C64 && dt != QSV_C128) return fail(QSV_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
  const int t = reg_qubits + threads_log2, runq = run_qubits_for(dt == QSV_C128, n);
  // the forward schedule is derived with the reverse sweep's at hand, as the library does
  if (!build_schedule(n, g, seq, slot, true, t, reg_qubits, threads_log2, runq, sc, &msg))
    return fail(QSV_ERR_INTERNAL, "schedule: %s", msg.c_str());
  if (!backward) {
    Schedule fw;
    if (!build_forward_schedule(n, g, t, reg_qubits, threads_log2, runq, sc, fw, &msg))
      return fail(QSV_ERR_INTERNAL, "schedule: %s", msg.c_str());
    sc = std::move(fw);
  }
  out->n_passes = (int32_t)sc.passes.size();
  out->n_phases = (int32_t)sc.phases.size();
  for (int i = 0; i < n_gates; ++i) {
    out->order[i] = sc.order[i];
    out->pass_of[i] = sc.pass_of[i];
    out->phase_of[i] = sc.phase_of[i];
  }
  for (size_t i = 0; i < sc.passes.size(); ++i) out->tile_mask[i] = sc.tile_mask[i];
  for (size_t i = 0; i < sc.phases.size(); ++i) out->reg_mask[i] = sc.reg_mask[i];
  out->n_macros = 0;
  for (const FusedOp& op : sc.ops) out->n_macros += (op.flags & FOPF_MACRO) ? 1 : 0;
  out->n_folded_cnots = sc.n_folded;
  out->n_diag_blocks = 0;
  for (const FusedOp& op : sc.ops)
    out->n_diag_blocks += op.opc == QSV_OPC(FOP_RZ, QSV_V_DIAG) ? 1 : 0;
  out->n_direct_loads = out->n_direct_stores = 0;
  for (const PassDesc& pd : sc.passes) {
    out->n_direct_loads += (pd.io_flags & PASS_LOAD_FIRST_PHASE) ? 1 : 0;
    out->n_direct_stores += (pd.io_flags & PASS_STORE_LAST_PHASE) ? 1 : 0;
  }
  return QSV_OK;
}

extern "C" qsv_status qsv_set_graphs(qsv_state* s, int32_t on) {
  QSV_TRY(check_handle(s));
  if (!on) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->graphs.clear();
  }
  s->graphs.on = on != 0;
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// autotuner
// ------------------------------------------------------------------------------------------------
struct TuneKey {
  uint64_t h;
  bool operator==(const TuneKey& o) const { return h == o.h; }
};
struct TuneHash {
  size_t operator()(const TuneKey& k) const { return (size_t)k.h; }
};
struct TuneEntry {
  std::array<int, 3> best;  // mode, r, w
  int32_t n, dt;
  double ms;                // measured time of the choice, -1 if unknown
};
// Process-wide: handles on different threads may tune concurrently, so every access holds the
// lock (the timing runs themselves do not).
static std::mutex g_tune_mu;
static std::unordered_map<TuneKey, TuneEntry, TuneHash> g_tuned;

#ifndef QSV_SOURCE_ID
#define QSV_SOURCE_ID "unversioned"
#endif

// Circuit structure (kinds and qubits, not angles), qubit count and storage type.
static uint64_t tune_key(const qsv_state* s, const Plan* p) {
  uint64_t h = fnv1a(&s->n, sizeof s->n);
  h = fnv1a(&s->dt, sizeof s->dt, h);
  for (const GateDesc& g : p->gates) {
    const int32_t v[3] = {g.kind, g.q0, g.q1};
    h = fnv1a(v, sizeof v, h);
  }
  return h;
}

extern "C" qsv_status qsv_autotune(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                   const double* d_theta, int32_t n_theta, const qsv_pauli_sum* H,
                                   int32_t repeats, int32_t* out_mode, int32_t* out_reg_qubits,
                                   int32_t* out_threads_log2, double* out_ms) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_circuit(s->n, gates, n_gates, n_theta));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (repeats < 1) repeats = 1;
  Plan* p = nullptr;
  QSV_TRY(get_plan(s, gates, n_gates, n_theta, &p));
  QSV_TRY(check_theta(p, d_theta));
  const TuneKey key{tune_key(s, p)};
  std::array<int, 3> best = {0, 0, 0};
  double best_ms = -1;
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto found = g_tuned.find(key);
    if (found != g_tuned.end() && found->second.n == s->n && found->second.dt == (int32_t)s->dt) {
      best = found->second.best;
      best_ms = found->second.ms;
      cached = true;
    }
  }
  if (!cached) {
    std::vector<std::array<int, 3>> cands;
    if (s->n <= kWaveMaxQubits) cands.push_back({2, 0, 0});
    if (s->n <= kWaveChunkMaxQubits) cands.push_back({3, 0, 0});
    if (s->n <= 20) cands.push_back({0, 0, 0});
    const int ws[3] = {9, 8, 6};
    for (int w : ws)
      for (int r = 2; r <= kMaxRegBits; ++r)
        if (fused_config_supported(r, w, s->dt == QSV_C128) && r + w <= std::max(s->n, 8))
          cands.push_back({1, r, w});
    DevBuf e, g;
    QSV_TRY(e.ensure(sizeof(double), s->stream));
    QSV_TRY(g.ensure(sizeof(double) * (n_theta ? n_theta : 1), s->stream));
    const int saved[3] = {s->fusion_mode, s->fr, s->fw};
    const bool graphs = s->graphs.on;
    s->graphs.on = false;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    qsv_status st = QSV_OK;
    for (const auto& c : cands) {
      s->fusion_mode = c[0];
      s->fr = c[1];
      s->fw = c[2];
      st = qsv_adjoint_gradient(s, gates, n_gates, d_theta, n_theta, H, e.as<double>(),
                                g.as<double>());  // warm-up: builds the schedules
      if (st != QSV_OK) break;
      if (hipEventRecord(a, s->stream) != hipSuccess) { st = QSV_ERR_HIP; break; }
      for (int i = 0; i < repeats && st == QSV_OK; ++i)
        st = qsv_adjoint_gradient(s, gates, n_gates, d_theta, n_theta, H, e.as<double>(),
                                  g.as<double>());
      if (st != QSV_OK) break;
      if (hipEventRecord(b, s->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
        st = QSV_ERR_HIP;
        break;
      }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, a, b);
      ms /= repeats;
      if (best_ms < 0 || ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    s->fusion_mode = saved[0];
    s->fr = saved[1];
    s->fw = saved[2];
    s->graphs.on = graphs;
    (void)hipStreamSynchronize(s->stream);  // the temporary outputs are freed on return
    if (st != QSV_OK) return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = TuneEntry{best, s->n, (int32_t)s->dt, best_ms};
  }
  s->fusion_mode = best[0];
  s->fr = best[1];
  s->fw = best[2];
  if (out_mode) *out_mode = best[0];
  if (out_reg_qubits) *out_reg_qubits = best[1];
  if (out_threads_log2) *out_threads_log2 = best[2];
  if (out_ms) *out_ms = best_ms;
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// persisted tuning choices: one JSON object per line, tagged with the library's source id so
// that choices timed on other kernel sources are never reused
// ------------------------------------------------------------------------------------------------
extern "C" const char* qsv_build_id(void) { return QSV_SOURCE_ID; }

extern "C" qsv_status qsv_tune_cache_save(const char* path) {
  if (!path) return fail(QSV_ERR_INVALID_ARG, "path is NULL");
  std::vector<std::pair<TuneKey, TuneEntry>> all;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    all.assign(g_tuned.begin(), g_tuned.end());
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(QSV_ERR_INVALID_ARG, "cannot write %s", tmp.c_str());
  for (const auto& kv : all) {
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 "{\"source\": \"%s\", \"key\": \"%016llx\", \"n\": %d, \"dtype\": %d, "
                 "\"mode\": %d, \"r\": %d, \"w\": %d, \"ms\": %.6f}\n",
                 QSV_SOURCE_ID, (unsigned long long)kv.first.h, e.n, e.dt, e.best[0], e.best[1],
                 e.best[2], e.ms);
  }
  const bool ok = std::fflush(f) == 0 && !std::ferror(f);
  std::fclose(f);
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(QSV_ERR_INVALID_ARG, "cannot write %s", path);
  }
  return QSV_OK;
}

extern "C" qsv_status qsv_tune_cache_load(const char* path, int32_t* out_loaded) {
  if (!path) return fail(QSV_ERR_INVALID_ARG, "path is NULL");
  if (out_loaded) *out_loaded = 0;
  FILE* f = std::fopen(path, "r");
  if (!f) return QSV_OK;  // no cache yet
  char line[512];
  int loaded = 0;
  std::vector<std::pair<TuneKey, TuneEntry>> got;
  while (std::fgets(line, sizeof line, f)) {
    char src[64] = {0};
    unsigned long long h = 0;
    int n = 0, dt = 0, m = 0, r = 0, w = 0;
    double ms = -1;
    const int k = std::sscanf(line,
                              "{\"source\": \"%63[^\"]\", \"key\": \"%llx\", \"n\": %d, "
                              "\"dtype\": %d, \"mode\": %d, \"r\": %d, \"w\": %d, "
                              "\"ms\": %lf}",
                              src, &h, &n, &dt, &m, &r, &w, &ms);
    if (k != 8 || std::strcmp(src, QSV_SOURCE_ID) != 0) continue;
    if (n < 1 || n > kMaxQubits || (dt != QSV_C64 && dt != QSV_C128)) continue;
    if (m == 1 ? !fused_config_supported(r, w, dt == QSV_C128)
               : (m == 2 ? n > kWaveMaxQubits : (m == 3 ? n > kWaveChunkMaxQubits : m != 0)))
      continue;
    got.push_back({TuneKey{(uint64_t)h}, TuneEntry{{m, r, w}, n, dt, ms}});
    ++loaded;
  }
  std::fclose(f);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : got) g_tuned[kv.first] = kv.second;
  }
  if (out_loaded) *out_loaded = loaded;
  return QSV_OK;
}

// ------------------------------------------------------------------------------------------------
// allocation-free expectation: the energy partials and the Pauli tables live in a fixed device
// array (one per GPU, kept until the process ends); nothing is allocated on the device or the host
// ------------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = 1u << 20;
constexpr int kNoAllocMaxTerms = 16384;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;             // guards the per-device addresses and the host tables
static void* g_scratch_ptr[64] = {nullptr};  // device address of `scratch` on each GPU
// host-side grouping tables (static: no heap use per call)
static PauliGroup g_na_groups[kNoAllocMaxTerms];
static PauliTerm g_na_terms[kNoAllocMaxTerms];
static int32_t g_na_group_of[kNoAllocMaxTerms];
static int32_t g_na_fill[kNoAllocMaxTerms];
static PauliTerm g_na_sorted[kNoAllocMaxTerms];

// Copies host words into device memory through kernel arguments (captured by value), so that no
// host buffer has to outlive the call and no staging allocation is made.
constexpr int kStageWords = 896;
struct StageChunk {
  uint32_t off, n;
  uint32_t w[kStageWords];
};
__global__ void k_stage_words(uint32_t* dst, StageChunk c) {
  for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[c.off + i] = c.w[i];
}

static qsv_status stage_words(uint32_t* dst, const void* src, size_t n_words, hipStream_t st) {
  const uint32_t* w = static_cast<const uint32_t*>(src);
  StageChunk c;
  for (size_t off = 0; off < n_words; off += kStageWords) {
    c.off = (uint32_t)off;
    c.n = (uint32_t)std::min<size_t>(kStageWords, n_words - off);
    std::memcpy(c.w, w + off, sizeof(uint32_t) * c.n);
    hipLaunchKernelGGL(k_stage_words, dim3(1), dim3(256), 0, st, dst, c);
    HIP_TRY(hipGetLastError());
  }
  return QSV_OK;
}

extern "C" qsv_status qsv_expectation_pauli_sum_noalloc(qsv_state* s, const qsv_pauli_sum* H,
                                                        double* d_energy) {
  QSV_TRY(check_handle(s));
  QSV_TRY(qsv_validate_pauli_sum(s->n, H));
  if (!d_energy) return fail(QSV_ERR_INVALID_ARG, "d_energy is NULL");
  if (H->n_terms > kNoAllocMaxTerms)
    return fail(QSV_ERR_INVALID_ARG, "%d Pauli terms exceed the allocation-free limit of %d",
                H->n_terms, kNoAllocMaxTerms);
  if (s->device < 0 || s->device >= 64)
    return fail(QSV_ERR_UNSUPPORTED, "device %d beyond the allocation-free table", s->device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[s->device]) {  // once per device, with that device current
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[s->device] = p;
  }
  char* base = static_cast<char*>(g_scratch_ptr[s->device]);
  // group the terms by X mask, as the cached path does, into the static host tables
  const int n = s->n, T = H->n_terms;
  int G = 0;
  static const double ire[4] = {1, 0, -1, 0}, iim[4] = {0, 1, 0, -1};
  for (int t = 0; t < T; ++t) {
    uint64_t x = 0, z = 0;
    int ny = 0;
    for (int q = 0; q < n; ++q) {
      const int c = H->codes[(size_t)t * n + q];
      if (c == 1 || c == 2) x |= 1ull << q;
      if (c == 3 || c == 2) z |= 1ull << q;
      if (c == 2) ++ny;
    }
    int g = 0;
    while (g < G && g_na_groups[g].x != x) ++g;
    if (g == G) g_na_groups[G++] = PauliGroup{x, 0, 0};
    ++g_na_groups[g].t1;  // count
    g_na_group_of[t] = g;
    const double c = H->coeffs[t];
    g_na_terms[t] = PauliTerm{z, c * ire[ny & 3], c * iim[ny & 3]};  // temporary, term order
  }
  // terms ordered by group (prefix sums, then place)
  int acc = 0;
  for (int g = 0; g < G; ++g) {
    const int cnt = g_na_groups[g].t1;
    g_na_groups[g].t0 = acc;
    g_na_groups[g].t1 = acc + cnt;
    g_na_fill[g] = acc;
    acc += cnt;
  }
  for (int t = 0; t < T; ++t) g_na_sorted[g_na_fill[g_na_group_of[t]]++] = g_na_terms[t];
  // scratch layout: [energy partials | groups | terms], 256-byte aligned parts
  const size_t part_bytes = sizeof(double2) * (size_t)s->nb;
  const size_t groups_off = (part_bytes + 255) & ~(size_t)255;
  const size_t terms_off = (groups_off + sizeof(PauliGroup) * (size_t)G + 255) & ~(size_t)255;
  const size_t need = terms_off + sizeof(PauliTerm) * (size_t)T;
  if (need > kNoAllocScratchBytes)
    return fail(QSV_ERR_INVALID_ARG,
                "allocation-free expectation needs %zu bytes of device scratch, the limit is %zu",
                need, kNoAllocScratchBytes);
  const hipStream_t st = s->stream;
  static_assert(sizeof(PauliGroup) % 4 == 0 && sizeof(PauliTerm) % 4 == 0, "word tables");
  QSV_TRY(stage_words(reinterpret_cast<uint32_t*>(base + groups_off), g_na_groups,
                      sizeof(PauliGroup) * (size_t)G / 4, st));
  QSV_TRY(stage_words(reinterpret_cast<uint32_t*>(base + terms_off), g_na_sorted,
                      sizeof(PauliTerm) * (size_t)T / 4, st));
  double2* ep = reinterpret_cast<double2*>(base);
  const PauliGroup* dg = reinterpret_cast<const PauliGroup*>(base + groups_off);
  const PauliTerm* dt = reinterpret_cast<const PauliTerm*>(base + terms_off);
  if (s->dt == QSV_C128)
    HIP_TRY(launch_pauli<double>(s->d_state, nullptr, n, dg, G, dt, ep, s->nb, st));
  else
    HIP_TRY(launch_pauli<float>(s->d_state, nullptr, n, dg, G, dt, ep, s->nb, st));
  HIP_TRY(launch_final_energy(ep, s->nb, d_energy, nullptr, st));
  return QSV_OK;
}
