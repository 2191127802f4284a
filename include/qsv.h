/*
 * qsv.h -- C-ABI of the MI355X state-vector library for reverse-mode ("adjoint") energy gradients.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the energy
 *     E(theta) = <psi|H|psi>,   |psi> = U_G(theta) ... U_1(theta) |in>            (paper Sec. 2.2)
 * of a parameterised circuit of one- and two-qubit gates under a Hamiltonian given as a real-
 * weighted sum of Pauli strings, and its full gradient in one forward pass, one application of H
 * and one backward sweep that un-applies every gate from two states phi and lambda, applies the
 * gate derivative to (a register copy of) phi and accumulates 2 Re <lambda|mu> per parameter
 * (paper Algorithm 1, Eq. recurrent_grad). Paper: T. Jones, J. Gacon, "Efficient calculation of
 * gradients in classical simulations of variational quantum algorithms", arXiv:2009.02823.
 *
 * Conventions
 *   - Qubit q is bit q of an amplitude index (little-endian). A state of n qubits is 2^n
 *     contiguous interleaved complex amplitudes: (re, im) doubles for QSV_C128 (16 B each) or
 *     floats for QSV_C64 (8 B each).
 *   - Rotations are R_G(t) = exp(-i t G / 2) for a Pauli G (the paper's alpha = -1/2, App. A).
 *   - A two-qubit gate on (q0, q1) has the local basis index 2 bit(q0) + bit(q1); q0 is the
 *     control of controlled gates.
 *   - Parameters, energies and gradients are float64 in both storage types.
 *
 * Memory and streams
 *   - Every state and every array whose name starts with d_ is DEVICE memory owned by the caller;
 *     gate tables and Pauli sums are HOST memory, copied (and cached by content) before return.
 *   - Small internal tables (gate matrices, schedules, reduction partials) are allocated by the
 *     library on first use and reused; a call that has to grow them allocates device memory.
 *   - All work is enqueued on the handle's stream (a hipStream_t passed as void*; NULL = the
 *     default stream) and is asynchronous: outputs are valid once the stream reaches the point
 *     of the call (qsv_sync, or any later stream-ordered consumer).
 *
 * Errors
 *   - Every entry point validates its arguments on the host before enqueueing anything; on an
 *     error it returns a nonzero qsv_status, enqueues nothing, leaves every output untouched and
 *     records a message readable with qsv_last_error() (thread-local).
 *   - QSV_ERR_HIP reports a failed HIP call; faults of earlier asynchronous work surface there or
 *     at qsv_sync. No call aborts the process or throws across the ABI.
 *   - A handle must not be used by two threads at once; distinct handles are independent.
 */
#ifndef QSV_PUBLIC_API_H
#define QSV_PUBLIC_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QSV_OK = 0,
  QSV_ERR_INVALID_ARG = 1,
  QSV_ERR_UNSUPPORTED = 2,
  QSV_ERR_OUT_OF_MEMORY = 3,
  QSV_ERR_HIP = 4,
  QSV_ERR_INTERNAL = 5
} qsv_status;

typedef enum { QSV_C64 = 0, QSV_C128 = 1 } qsv_dtype;

/* Gate kinds. Parameterised kinds read theta[param[j]] for j < (number of parameters). */
typedef enum {
  QSV_RX = 0,     /* exp(-i t X/2) on q0                           1 parameter            */
  QSV_RY = 1,     /* exp(-i t Y/2) on q0                           1 parameter            */
  QSV_RZ = 2,     /* exp(-i t Z/2) on q0                           1 parameter            */
  QSV_H = 3,      /* Hadamard on q0                                                       */
  QSV_X = 4,      /* Pauli X on q0                                                        */
  QSV_Y = 5,      /* Pauli Y on q0                                                        */
  QSV_Z = 6,      /* Pauli Z on q0                                                        */
  QSV_S = 7,      /* diag(1, i) on q0                                                     */
  QSV_CNOT = 8,   /* control q0, target q1                                                */
  QSV_CZ = 9,     /* diag(1, 1, 1, -1) on (q0, q1)                                        */
  QSV_PHASE = 10, /* diag(1, e^{i t}) on q0                        1 parameter            */
  QSV_CRX = 11,   /* control q0, exp(-i t X/2) on target q1        1 parameter            */
  QSV_CRY = 12,   /* control q0, exp(-i t Y/2) on target q1        1 parameter            */
  QSV_CRZ = 13,   /* control q0, exp(-i t Z/2) on target q1        1 parameter            */
  QSV_RXX = 14,   /* exp(-i t X(x)X/2) on (q0, q1)                 1 parameter            */
  QSV_RYY = 15,   /* exp(-i t Y(x)Y/2) on (q0, q1)                 1 parameter            */
  QSV_RZZ = 16,   /* exp(-i t Z(x)Z/2) on (q0, q1)                 1 parameter            */
  QSV_U3 = 17,    /* [[c, -e^{il} s], [e^{if} s, e^{i(f+l)} c]], c = cos(t/2), s = sin(t/2),
                     parameters (t, f, l) = theta[param[0..2]]   3 parameters            */
  QSV_T = 18,     /* diag(1, e^{i pi/4}) on q0                                            */
  QSV_SDG = 19,   /* diag(1, -i) on q0                                                    */
  /* Non-unitary, invertible gates (paper App. B.3): imaginary-time rotations
     M(t) = exp(-t G/2) = cosh(t/2) 1 - sinh(t/2) G. The reverse sweep un-does phi by
     M^-1 = exp(+t G/2) and lambda by M^dag; the energy <psi|H|psi> is then not normalised.
     The parameter-shift rule does not hold for them (qsv_param_shift_gradient rejects them). */
  QSV_NRX = 20,   /* exp(-t X/2) on q0                             1 parameter            */
  QSV_NRY = 21,   /* exp(-t Y/2) on q0                             1 parameter            */
  QSV_NRZ = 22    /* exp(-t Z/2) on q0                             1 parameter            */
} qsv_gate_kind;

/* One gate of a circuit. Circuits are arrays applied in index order (U_1 first).
   q1 = -1 for one-qubit kinds. param[j] = index into theta for the j-th parameter of the kind,
   -1 for the unused slots. Several gates may name the same parameter; its gradient entry is then
   the sum over its occurrences (paper App. B.2). */
typedef struct {
  int32_t kind;
  int32_t q0;
  int32_t q1;
  int32_t param[3];
} qsv_gate;

/* H = sum_t coeffs[t] P_t with P_t = (x)_q sigma(codes[t * n_qubits + q]) and the codes
   0 = I, 1 = X, 2 = Y, 3 = Z. Coefficients are real (H Hermitian, paper Sec. 2.2). Host memory. */
typedef struct {
  int32_t n_terms;
  const uint8_t* codes;   /* [n_terms * n_qubits] */
  const double* coeffs;   /* [n_terms]            */
} qsv_pauli_sum;

typedef struct qsv_state qsv_state;

/* ---- host-only validation (no GPU needed) ------------------------------------------------- */

/* Checks a gate table against n_qubits and n_theta: known kinds, qubits in range and distinct,
   q1 = -1 for one-qubit kinds, parameter slots in [0, n_theta) where used and -1 elsewhere. */
qsv_status qsv_validate_circuit(int32_t n_qubits, const qsv_gate* gates, int32_t n_gates,
                                int32_t n_theta);

/* Checks a Pauli sum: n_terms >= 0, codes <= 3, finite coefficients, non-NULL arrays. */
qsv_status qsv_validate_pauli_sum(int32_t n_qubits, const qsv_pauli_sum* H);

/* Bytes of caller-provided device workspace qsv_create needs: two states (phi and lambda of
   Algorithm 1). Returns 0 for an invalid (n_qubits, dtype). */
size_t qsv_workspace_bytes(int32_t n_qubits, qsv_dtype dtype);

/* Bytes of one state of n_qubits in dtype (2^n amplitudes). 0 if invalid. */
size_t qsv_state_bytes(int32_t n_qubits, qsv_dtype dtype);

/* Message of the last failed call on this thread ("" if none). Valid until the next call. */
const char* qsv_last_error(void);

/* ---- handles ------------------------------------------------------------------------------ */

/* Creates a handle for an n_qubits state (1 <= n_qubits <= 34) on the current HIP device.
   d_state: caller-owned device buffer of qsv_state_bytes(n_qubits, dtype) bytes holding the
            immutable input state |in> of Algorithm 1; qsv_create writes |0...0> into it.
   d_work:  caller-owned device buffer of at least qsv_workspace_bytes(n_qubits, dtype) bytes.
   stream:  hipStream_t (as void*) all work of this handle is ordered on.
   Both buffers must be 256-byte aligned and stay valid until qsv_destroy. */
qsv_status qsv_create(int32_t n_qubits, qsv_dtype dtype, void* d_state, void* d_work,
                      size_t work_bytes, void* stream, qsv_state** out);

/* Releases the library-owned tables of the handle; never frees caller buffers. NULL is a no-op. */
qsv_status qsv_destroy(qsv_state* s);

/* Changes the stream later calls of this handle enqueue on. */
qsv_status qsv_set_stream(qsv_state* s, void* stream);

/* Writes |0...0> into the handle's state. */
qsv_status qsv_reset(qsv_state* s);

/* Blocks until all work enqueued on the handle's stream has finished; reports asynchronous
   HIP errors. */
qsv_status qsv_sync(qsv_state* s);

/* ---- the computation ---------------------------------------------------------------------- */

/* state <- U_G(theta) ... U_1(theta) state   (Algorithm 1, apply-circuit step; Sec. 2.2).
   d_theta: device float64[n_theta] (may be NULL if no gate has a parameter). */
qsv_status qsv_apply_circuit(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                             const double* d_theta, int32_t n_theta);

/* *d_energy <- <state|H|state> (real part; the state is not modified, nothing is written into the
   workspace). d_energy: device float64[1]. (Sec. 2.2, the energy functional.) */
qsv_status qsv_expectation_pauli_sum(qsv_state* s, const qsv_pauli_sum* H, double* d_energy);

/* The same as qsv_expectation_pauli_sum, for callers that cannot allocate (code under graph
   capture, tight serving loops, harnesses that forbid allocation): nothing is allocated on the
   device or the host. The energy partials and the Pauli tables live in a fixed device array of
   1 MiB per GPU (kept until the process ends); the terms are grouped on the host in static
   tables and copied to the device through kernel arguments. Limits: at most 16384 terms, and
   16 bytes per gather block plus 16 bytes per X-mask group plus 24 bytes per term within the
   1 MiB; beyond them QSV_ERR_INVALID_ARG with a message, nothing enqueued. All X-mask groups are
   gathered (no tiled passes), so the result agrees with qsv_expectation_pauli_sum to rounding.
   Every call on a GPU shares that GPU's array, and host grouping is serialised by a lock:
   calls that overlap on one GPU (on different streams) race on the array. */
qsv_status qsv_expectation_pauli_sum_noalloc(qsv_state* s, const qsv_pauli_sum* H,
                                             double* d_energy);

/* *d_energy <- <psi|H|psi> with psi = U(theta)|in>, computed in the workspace (the handle's state
   |in> is left unchanged): the forward pass and expectation of Sec. 2.2 without the sweep. */
qsv_status qsv_energy(qsv_state* s, const qsv_gate* gates, int32_t n_gates, const double* d_theta,
                      int32_t n_theta, const qsv_pauli_sum* H, double* d_energy);

/* Reverse-mode gradient (Algorithm 1) with the handle's state as |in> (left unchanged):
     psi = U |in>,  lambda = H psi,  E = <psi|lambda>;
     for i = G..1:  phi <- U_i^dag phi;  grad[param_i] += 2 Re <lambda| dU_i/dtheta |phi>;
                    lambda <- U_i^dag lambda (for i > 1).
   d_energy: device float64[1] <- E.   d_grad: device float64[n_theta], overwritten (entries of
   parameters no gate uses are 0). Uses the workspace as phi and lambda. */
qsv_status qsv_adjoint_gradient(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                const double* d_theta, int32_t n_theta, const qsv_pauli_sum* H,
                                double* d_energy, double* d_grad);

/* Algorithm 1 for a batch of independent circuits, one handle each (their states are the inputs
   |in>, left unchanged; every handle uses its own workspace).
   gates[b], n_gates[b], n_theta[b], H[b]: circuit b (host arrays, as for qsv_adjoint_gradient).
   d_theta_flat: device float64; circuit b reads theta_off[b] .. theta_off[b] + n_theta[b] - 1.
   d_energy: device float64[n_batch] <- E_b.  d_grad_flat: device float64, circuit b's gradient
   is written at theta_off[b] ..; segments must not overlap.
   All handles must be distinct, on one device, with one dtype; all work is ordered on the stream
   of states[0] (the other handles must have no work pending on other streams). When every
   circuit holds a tile of the common geometry, the k-th fused pass of all circuits runs as one
   launch (levels of the forward pass and of the reverse sweep), else circuits run one after the
   other. */
qsv_status qsv_adjoint_gradient_batched(int32_t n_batch, qsv_state* const* states,
                                        const qsv_gate* const* gates, const int32_t* n_gates,
                                        const double* d_theta_flat, const int64_t* theta_off,
                                        const int32_t* n_theta, const qsv_pauli_sum* H,
                                        double* d_energy, double* d_grad_flat);

/* Faithful O(P^2) baseline on the same GPU (the re-simulation the paper's introduction calls
   "faithful" emulation, here in its parameter-shift form): for p in [first, first + count),
     grad[p] = ( E(theta + (pi/2) e_p) - E(theta - (pi/2) e_p) ) / 2,
   each E a full reset + forward pass + expectation with the same kernels as the adjoint path.
   Exact for parameters used by exactly one gate whose generator has two eigenvalues that differ
   by 1 (RX RY RZ RXX RYY RZZ PHASE U3); returns QSV_ERR_UNSUPPORTED for controlled rotations or
   repeated parameters. Entries outside the range are not written. Uses the workspace. */
qsv_status qsv_param_shift_gradient(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                    const double* d_theta, int32_t n_theta, const qsv_pauli_sum* H,
                                    int32_t first, int32_t count, double* d_grad);

/* The same energy and gradient by the reference scheme of Algorithm 2 (Sec. 3): lambda = H U |in>,
   then for every parameter occurrence i a separate simulation mu = U_G..U_{i+1} dU_i/dtheta
   U_{i-1}..U_1 |in> and the entry 2 Re <lambda|mu> (summed over the occurrences of a repeated
   parameter); O(P^2) gate applications. Arguments and results as qsv_adjoint_gradient. States of
   at most 6 qubits (automatic fusion mode, or mode 2 or 3) run in waves: one wave forms lambda,
   then one wave per parameter occurrence its simulation and entry, all at once. Larger states
   that fit one fused tile (see qsv_set_fusion) run all entries in parallel, one workgroup each,
   with a library-allocated pool of up to 1 GiB of mu states; larger states run the entries one
   after another in the phi buffer. Meant as the faithful comparison baseline for small
   circuits. */
qsv_status qsv_reference_gradient(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                  const double* d_theta, int32_t n_theta, const qsv_pauli_sum* H,
                                  double* d_energy, double* d_grad);

/* Algorithm 2 (as qsv_reference_gradient) for a batch of independent circuits; arguments and
   results as qsv_adjoint_gradient_batched. When every state has at most 6 qubits (and the
   automatic fusion mode or mode 2 or 3), one launch runs lambda = H U |in> of every circuit (one
   wave each), one launch the simulation of every (circuit, parameter occurrence) pair (one wave
   each) and one launch the gradient entries; otherwise the circuits run one after the other.
   The batch counterpart of the O(P^2) baseline, for throughput comparisons with
   qsv_adjoint_gradient_batched. */
qsv_status qsv_reference_gradient_batched(int32_t n_batch, qsv_state* const* states,
                                          const qsv_gate* const* gates, const int32_t* n_gates,
                                          const double* d_theta_flat, const int64_t* theta_off,
                                          const int32_t* n_theta, const qsv_pauli_sum* H,
                                          double* d_energy, double* d_grad_flat);

/* Non-Hermitian operator A = sum_t (A->coeffs[t] + i coeffs_im[t]) P_t (App. B.4): the complex
   expectation <A> = <psi|A|psi>, psi = U |in>, and its complex gradient. Algorithm 1 runs twice
   with the complex <lambda|mu> as the entry of each occurrence: once with A (entries g_A) and
   once with A^dag = sum conj(c_t) P_t (entries g_{A^dag}); d<A>/dtheta_p = conj(g_A[p]) +
   g_{A^dag}[p]. (The appendix conjugates the A^dag run instead, which gives the conjugate of the
   derivative; here the conjugate is on the A run, since <dpsi|A|psi> = conj(<psi|A^dag|dpsi>).)
   coeffs_im: host float64[A->n_terms]. d_energy: device float64[2] = (Re, Im). d_grad: device
   float64[2 * n_theta], (Re, Im) per parameter. Runs the fused passes (the handle's geometry, or
   the automatic one if the handle is set to gate-granular). Real coeffs_im = 0 reproduces
   qsv_adjoint_gradient with zero imaginary parts. */
qsv_status qsv_adjoint_gradient_nonhermitian(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                                             const double* d_theta, int32_t n_theta,
                                             const qsv_pauli_sum* A, const double* coeffs_im,
                                             double* d_energy, double* d_grad);

/* ---- graphs and tuning ------------------------------------------------------------------- */

/* on != 0: qsv_adjoint_gradient and qsv_adjoint_gradient_batched capture their launch sequence
   into a hipGraph on the second call with the same circuit, Hamiltonian, geometry and device
   pointers (the first call builds every plan eagerly) and replay it on every later such call.
   Capture happens on a library-owned stream after the handle's stream has drained; replays are
   ordered on the handle's stream. Graphs are bypassed while kernel timing is on. on = 0 frees
   them. */
qsv_status qsv_set_graphs(qsv_state* s, int32_t on);

/* Times qsv_adjoint_gradient `repeats` times for every available execution mode (gate-granular
   for states up to 20 qubits, every fused geometry that fits the state), keeps the fastest as
   the handle's mode and caches the choice per (qubit count, storage type, gate kinds and qubits)
   for the process; later calls with the same structure reuse it without timing. Writes the
   chosen mode and geometry and the measured ms per gradient (for a cached choice, the time it
   was measured with, -1 if unknown). Uses the workspace; outputs may be NULL. The process-wide
   cache is guarded by a lock, so handles on different threads may tune concurrently. */
qsv_status qsv_autotune(qsv_state* s, const qsv_gate* gates, int32_t n_gates,
                        const double* d_theta, int32_t n_theta, const qsv_pauli_sum* H,
                        int32_t repeats, int32_t* out_mode, int32_t* out_reg_qubits,
                        int32_t* out_threads_log2, double* out_ms);

/* Host-only description of how a handle of n_qubits qubits and storage dt applies H (no GPU
   needed). Terms are grouped by X mask (*n_groups groups). Groups whose X bits fit one tile of
   2^12 (complex128) or 2^13 (complex64) amplitudes that holds the low run qubits are applied in
   tiled passes that read psi once for all of their groups (*n_tiled_passes, each kept only if it
   takes at least three groups); the other groups (*n_gather_groups) are applied by a gather that
   reads psi once per group. For the first max_passes passes, tile_masks[i] = the pass's qubits
   and pass_groups[i] = its groups (both arrays caller-owned, may be NULL). Every group is applied
   exactly once. QSV_ERR_INVALID_ARG for an invalid sum or dtype. */
qsv_status qsv_pauli_describe(int32_t n_qubits, qsv_dtype dt, const qsv_pauli_sum* H,
                              int32_t* n_groups, int32_t* n_tiled_passes,
                              int32_t* n_gather_groups, uint64_t* tile_masks,
                              int32_t* pass_groups, int32_t max_passes);

/* Persisted tuning choices. qsv_tune_cache_save writes every cached choice to `path` (one JSON
   object per line: source id of this library build, structure key, qubit count, storage type,
   mode, geometry, measured ms), replacing the file atomically; QSV_ERR_INVALID_ARG if it cannot
   be written. qsv_tune_cache_load merges the lines of `path` that carry this library's source
   id into the process cache (choices timed on other kernel sources are skipped, as are
   malformed lines and geometries this build lacks); *out_loaded (may be NULL) = lines taken.
   A missing file loads nothing and returns QSV_OK. Host-only: no GPU is touched. */
qsv_status qsv_tune_cache_save(const char* path);
qsv_status qsv_tune_cache_load(const char* path, int32_t* out_loaded);

/* The source id the persisted tuning choices of this build are tagged with (a hash of the
   library's sources, fixed at build time). Static storage; never NULL. */
const char* qsv_build_id(void);

/* Test hook for the error path: the k-th kernel launch of the computations from now (k >= 1,
   counted over all handles; the final reductions are not counted) is not enqueued and its call
   returns QSV_ERR_HIP, as a failed launch would; k = 0 disarms. A computation that fails this
   way has enqueued only launches before the failed one, and its outputs (energy, gradient) are
   written by final reductions that come after every counted launch, so they stay untouched. */
qsv_status qsv_debug_fail_launch(int32_t k);

/* ---- measurement -------------------------------------------------------------------------- */

/* Per-kernel-family statistics gathered from HIP events recorded on the handle's stream right
   before and after every timed launch. */
typedef struct {
  char name[48];     /* kernel family: a substring of the kernel's symbol name                  */
  int64_t launches;  /* timed launches                                                          */
  double total_ms;   /* sum of the launches' event-to-event durations                           */
  double bytes;      /* sum of their algorithmic bytes: unique state bytes read plus written    */
} qsv_kernel_stat;

/* Starts timing launches whose family name contains name_filter ("" = every kernel) and clears
   earlier statistics; name_filter = NULL stops timing. */
qsv_status qsv_timing_enable(qsv_state* s, const char* name_filter);

/* Waits for the handle's stream, folds the recorded events into per-family statistics and copies
   up to max_out of them (sorted by total time, largest first) to out; *n_out = number copied. */
qsv_status qsv_timing_read(qsv_state* s, qsv_kernel_stat* out, int32_t max_out, int32_t* n_out);

/* ---- fusion ------------------------------------------------------------------------------- */

/* Execution mode of a handle's forward pass and reverse sweep:
     mode = 0   one HBM pass per gate (gate-granular kernels);
     mode = 1   fused passes: each pass loads every tile of 2^(reg_qubits + threads_log2)
                amplitudes once (workgroups of 2^threads_log2 threads, 2^reg_qubits amplitudes of
                each state per thread), applies a scheduled run of gates in registers and LDS, and
                stores it once; supported (reg_qubits, threads_log2): (2..4, 8) and (2..3, 9) for
                complex128, (2..4, 8) and (2..4, 9) for complex64, (2..3, 6) for both. A tile
                may exceed the state: its extra ("phantom") bits hold amplitudes that are never
                loaded or stored, and a state within one tile runs every pass of a sweep in a
                single launch (one workgroup walks the passes in order);
     mode = 2   (states of at most 6 qubits) the gradient runs Algorithm 1 in one wave: amplitude
                j in lane j, gates applied across lanes by lane permutations, the forward pass,
                H, the reverse sweep and the gradient entries in one launch; the other calls run
                fused passes; qsv_adjoint_gradient_batched runs one such wave per circuit;
     mode = 3   (states of at most 5 qubits) as mode 2, with the gradient's gates taken in chunks
                of 64: the product W_c of each chunk is formed in parallel (the chunk applied to
                the basis states), psi, phi and lambda are carried across chunk boundaries by W_c
                and W_c^dag on one wave, and the steps of Algorithm 1 inside the chunks run for
                all chunks at once. Circuits with a non-unitary gate run mode 2;
     mode = -1  automatic (the default): for the gradient of states of at most 6 qubits mode 3
                from 96 gates on (at most 5 qubits, unitary gates), else mode 2; otherwise fused
                with a size-dependent geometry. qsv_autotune picks among all modes by
                measurement. */
qsv_status qsv_set_fusion(qsv_state* s, int32_t mode, int32_t reg_qubits, int32_t threads_log2);

/* The geometry the handle's gradient currently runs with: *mode = 2 (one wave, chosen or
   automatic; the automatic mode runs long circuits chunked) or 3 (chunked one wave), with
   *reg_qubits = *threads_log2 = 0; 1 (fused, with *reg_qubits and *threads_log2) or 0
   (gate-granular). */
qsv_status qsv_get_fusion(qsv_state* s, int32_t* mode, int32_t* reg_qubits, int32_t* threads_log2);

/* Host-only description of the fused schedule of a circuit (no GPU needed): the order gates run
   in, and for each executed gate its pass and register phase; the physical-qubit masks of every
   pass's tile and every phase's register qubits. backward != 0 describes the reverse sweep (gates
   taken from last to first). The storage type matters: every tile holds the lowest qubits
   (0..2 for complex128 and for complex64 states of up to 24 qubits, 0..3 for larger complex64
   states), so that loads and stores move contiguous runs. All arrays are caller-owned with
   n_gates entries. n_macros counts
   the rotation macros (runs of reg_qubits same-axis rotations, one per register qubit, that run
   as one op; formed for reg_qubits <= 4). n_direct_loads / n_direct_stores count the passes whose
   tiles move between HBM and registers in their first / last phase's layout (those phases keep
   the low run qubits off the register bits), which saves the relayout after the loads / before
   the stores. */
typedef struct {
  int32_t n_passes;
  int32_t n_phases;
  int32_t* order;
  int32_t* pass_of;
  int32_t* phase_of;
  uint64_t* tile_mask;
  uint64_t* reg_mask;
  int32_t n_macros;
  int32_t n_direct_loads;   /* passes that load their tiles in the first phase's layout        */
  int32_t n_direct_stores;  /* passes that store their tiles from the last phase's layout      */
  int32_t n_diag_blocks;    /* diagonal blocks (RZ and CZ gates on register bits run as one
                               diagonal matrix per thread; formed for reg_qubits <= 4)         */
  int32_t n_folded_cnots;   /* reverse sweep: CNOTs with both bits in registers that open a
                               phase entered by a relayout (its reads permute the registers) */
} qsv_schedule_info;

qsv_status qsv_schedule_describe(int32_t n_qubits, const qsv_gate* gates, int32_t n_gates,
                                 int32_t backward, int32_t reg_qubits, int32_t threads_log2,
                                 qsv_dtype dt, qsv_schedule_info* out);

#ifdef __cplusplus
}
#endif

#endif /* QSV_PUBLIC_API_H */
