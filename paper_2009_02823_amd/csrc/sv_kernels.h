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
