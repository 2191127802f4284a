// Launchers of the gate-granular HIP kernels (one HBM pass per gate).
#pragma once

#include "qsv_internal.h"

namespace qsv {

// Per-gate matrices U and dU/dtheta_j from the device parameter vector (one thread per gate).
hipError_t launch_prep(const GateDesc* d_gates, int n_gates, const double* d_theta, GateRec* d_rec,
                       hipStream_t st);

// Blocks used by every gate-granular launch on an n-qubit state (the partials stride).
int sweep_blocks(int n);

// psi <- U psi (adj = false) or U^dag psi for one gate.
template <typename R>
hipError_t launch_forward_gate(void* psi, int n, const GateDesc& g, const GateRec* d_rec, bool adj,
                               hipStream_t st);

// One step of the reverse sweep for gate g, in one pass over phi and lambda:
//   phi <- U^dag phi;  for each parameter j of g: partial_j[block] = sum conj(lambda) dU_j phi;
//   lambda <- U^dag lambda if undo_lam.
// partial points at slot 0 of the gate's kind_nparams(g.kind) consecutive slots of nb entries.
template <typename R>
hipError_t launch_backward_gate(void* phi, void* lam, int n, const GateDesc& g,
                                const GateRec* d_rec, bool undo_lam, double2* partial, int nb,
                                hipStream_t st);

// out <- H psi (if out != nullptr) and partial[block] = sum_j conj(psi_j) (H psi)_j.
template <typename R>
hipError_t launch_pauli(const void* psi, void* out, int n, const PauliGroup* d_groups, int n_groups,
                        const PauliTerm* d_terms, double2* partial, int nb, hipStream_t st);

// Tiled application of H (Algorithm 1, step lambda <- H psi): the 2^TB amplitudes that share
// the values of the qubits outside a tile are loaded into LDS once, and every X-mask group whose
// X bits lie in the tile is applied there (one HBM read of psi for all of them). TB = 12 for
// complex128, 13 for complex64 (64 KiB of LDS); 2^TB / 8 threads, each owning E = 8
// amplitudes, element k of thread tid being tile index tid + k * 2^TB / E.
constexpr int kPauliTileMaxTerms = 64;
struct PauliTileGroup {
  uint32_t xl;        // X bits as a tile-local bit mask
  int32_t t0, t1;     // its terms [t0, t1) in the pass's term table (sign bit t - pass t0)
};
struct PauliTilePass {
  uint64_t outer_mask;            // qubits outside the tile
  uint64_t kbits[16];             // element k < E: bit t = parity of (k's tile offset & z_t)
  int8_t tile[16];                // physical qubit of tile bit s (ascending)
  int32_t n_outer;
  int32_t g0, g1;                 // groups [g0, g1) of the tiled group table
  int32_t t0, n_terms;            // terms [t0, t0 + n_terms), n_terms <= kPauliTileMaxTerms
  int32_t lam_mode;               // 0: lambda = (H psi) part, 1: lambda += it, 2: no lambda
  int32_t e_accumulate;           // 0: partial[block] = sum, 1: partial[block] += sum
};

// One tiled pass over psi (and lambda): terms' coefficients already carry the sign
// (-1)^popcount(x & z) of their group's X mask. partial[block] as set by e_accumulate; grid
// blocks stride over the tiles. tile_bits: 12 (complex128) or 13 (complex64).
template <typename R>
hipError_t launch_pauli_tile(const void* psi, void* lam, const PauliTilePass& P,
                             const PauliTileGroup* d_groups, const PauliTerm* d_terms,
                             double2* partial, int grid, hipStream_t st);

// Tile bits and amplitudes per thread of the tiled application for the storage type.
constexpr int pauli_tile_bits(bool c128) { return c128 ? 12 : 13; }
constexpr int pauli_tile_elements(bool) { return 8; }

// Algorithm 1 for states of at most kWaveMaxQubits qubits, one wave (64 threads) per circuit:
// amplitude j in lane j. The wave writes the energy, the per-slot sums of the products
// Re <lambda|mu> (slots in sweep order, last gate first) and the gradient itself.
constexpr int kWaveMaxQubits = 6;
struct WaveJob {
  const GateDesc* gates;
  const GateRec* recs;            // read for the gates other than RX, RY, RZ, CNOT, CZ
  const double* theta;            // RX, RY, RZ take cos and sin of half their angle from here
  const void* in;                 // |in>, 2^n amplitudes of the storage type
  const PauliGroup* groups;
  const PauliTerm* terms;
  const int32_t* param_ptr;       // parameter p owns slots occ[param_ptr[p] .. param_ptr[p+1])
  const int32_t* occ;
  double* slot_sum;               // [slots] workspace: Re <lambda|mu> per slot
  double* energy;                 // [1] <- E (one circuit)
  double* grad;                   // [n_theta] <- dE/dtheta (one circuit)
  int64_t grad_off;               // batch: the gradient goes to grad_base + grad_off (the
                                  // batch's gate tables index the flat theta_base)
  // Algorithm 2 (launch_wave_reference): lambda = H U|in> and the gate and parameter of each
  // slot, k * 4 + j
  double2* ref_lam;               // [64]
  const int32_t* occ_gate;        // [slots]
  int32_t n_gates, n, n_groups, n_theta;
  int32_t n_occ, pad;
};

// Algorithm 2 in waves: one wave per circuit forms lambda = H U|in> and E, then one wave per
// (circuit, slot) runs the forward pass with that slot's gate replaced by its derivative and
// forms Re <lambda|mu> (lanes summed in order), then one wave per circuit the gradient entries.
// max_occ: the largest slot count of the circuits.
template <typename R>
hipError_t launch_wave_reference(const WaveJob* d_jobs, int n_jobs, int max_occ,
                                 const WaveJob& single, const double* theta_base,
                                 double* energy_base, double* grad_base, hipStream_t st);

// The chunked sweep of one circuit (every gate unitary, at most kWaveChunkMaxQubits qubits): the
// gates in chunks of 64, each chunk's operator W_c formed in parallel, the states at the chunk
// boundaries carried by W_c, and the steps inside all chunks run at once (launch_wave_chunked).
constexpr int kWaveChunk = 64;
constexpr int kWaveChunkMaxQubits = 5;
struct WaveChunks {
  double2* A;               // [n_chunks][N][N]: A[c][j * N + r] = W_c[r][j]
  double2* B;               // [n_chunks][N][N]: B[c][j * N + r] = W_c[j][r]
  double2* phi;             // [n_chunks][N]: phi at the end of chunk c
  double2* lam;             // [n_chunks][N]: lambda at the end of chunk c
  const int32_t* slot0;     // [n_chunks]: first product slot of chunk c
  int32_t* done;            // chunks finished (0 between calls)
  int32_t n_chunks;
  int32_t pad;
};
template <typename R>
hipError_t launch_wave_chunked(const WaveJob& J, const WaveChunks& K, hipStream_t st);

// d_jobs = NULL: one circuit, `single`; else n_jobs circuits from the device table, job b writing
// energy_base[b] and its gradient at grad_base + grad_off (the output pointers are launch
// arguments, so a table serves any outputs).
template <typename R>
hipError_t launch_wave_adjoint(const WaveJob* d_jobs, int n_jobs, const WaveJob& single,
                               const double* theta_base, double* energy_base, double* grad_base,
                               hipStream_t st);

// Gates the one-wave kernels take from their parameters alone (no record needed).
__host__ __device__ inline bool wave_native_kind(int k) {
  return k == K_RX || k == K_RY || k == K_RZ || k == K_CNOT || k == K_CZ;
}

template <typename R>
hipError_t launch_copy(void* dst, const void* src, int n, hipStream_t st);

template <typename R>
hipError_t launch_reset(void* psi, int n, hipStream_t st);

// Where the partial sums of one circuit's products live: occurrence o (a reduction slot) has
// occ_nb[o] consecutive partials starting at partials[occ_base[o]]; parameter p owns the
// occurrences occ[param_ptr[p] .. param_ptr[p+1]) (in sweep order). Gradient entries are written
// to grad[grad_off + p].
struct FinalDesc {
  const double2* partials;
  const int64_t* occ_base;
  const int32_t* occ_nb;
  const int32_t* param_ptr;
  const int32_t* occ;
  int64_t grad_off;
  int64_t p_begin;   // first block of this circuit in the launch
  int32_t n_theta;
  int32_t pad;
};

// One block per gradient entry over n_desc circuits (total_params = sum of n_theta):
// grad[grad_off + p] = 2 Re sum over the occurrences of p of their partials, in a fixed order.
// grad[p] = conj(Z_A[p]) + Z_{A^dag}[p] as (Re, Im) pairs, Z the complex entry sums of two sweeps
// sharing one occurrence layout (a: with A, b: with A^dag).
hipError_t launch_final_grad_nonherm(const FinalDesc* d_a, const FinalDesc* d_b, int n_theta,
                                     double* d_grad, hipStream_t st);
hipError_t launch_final_grad(const FinalDesc* d_desc, int n_desc, int64_t total_params,
                             double* d_grad, hipStream_t st);

// *energy = Re sum_b partials[b]; energy_im (optional) = Im.
// One circuit of a batched H application: lambda = H psi with E partials (Algorithm 1, the application of H).
struct PauliJob {
  const void* psi;
  void* out;
  const PauliGroup* groups;
  const PauliTerm* terms;
  int32_t n, n_groups;
};

// Every job in one launch: partials[job * blocks_per_job + block].
template <typename R>
hipError_t launch_pauli_batched(const PauliJob* d_jobs, int n_jobs, int blocks_per_job,
                                double2* partials, hipStream_t st);

// energy[job] = Re of the sum of the job's nb partials (one block per job).
hipError_t launch_final_energy_batched(const double2* partials, int nb, int n_jobs,
                                       double* d_energy, hipStream_t st);

hipError_t launch_final_energy(const double2* partials, int nb, double* d_energy,
                               double* d_energy_im, hipStream_t st);

// Kernel family names (substrings of the symbol names rocprof reports) of the launches above.
const char* forward_kernel_name(const GateDesc& g);
const char* backward_kernel_name(const GateDesc& g);

// dst = src with dst[p] += delta (one block; n_theta >= 1).
hipError_t launch_shift_theta(double* dst, const double* src, int n_theta, int p, double delta,
                              hipStream_t st);

// grad[first + i] = (e[2i] - e[2i + 1]) / 2 for i < count.
hipError_t launch_ps_combine(double* grad, const double* e, int first, int count, hipStream_t st);

}  // namespace qsv
