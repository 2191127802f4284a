// Internal types shared by the HIP kernels and the host runtime of the qsv library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qsv {

enum Kind : int32_t {
  K_RX = 0, K_RY, K_RZ, K_H, K_X, K_Y, K_Z, K_S, K_CNOT, K_CZ,
  K_PHASE, K_CRX, K_CRY, K_CRZ, K_RXX, K_RYY, K_RZZ, K_U3, K_T, K_SDG,
  K_NRX, K_NRY, K_NRZ, K_NKINDS
};

__host__ __device__ inline int kind_nparams(int k) {
  switch (k) {
    case K_RX: case K_RY: case K_RZ: case K_PHASE: case K_CRX: case K_CRY: case K_CRZ:
    case K_RXX: case K_RYY: case K_RZZ: case K_NRX: case K_NRY: case K_NRZ:
      return 1;
    case K_U3:
      return 3;
    default:
      return 0;
  }
}

__host__ __device__ inline int kind_nqubits(int k) {
  switch (k) {
    case K_CNOT: case K_CZ: case K_CRX: case K_CRY: case K_CRZ: case K_RXX: case K_RYY:
    case K_RZZ:
      return 2;
    default:
      return 1;
  }
}

// Non-unitary (invertible) kinds: un-done by their inverse on phi, their adjoint on lambda.
__host__ __device__ inline bool kind_unitary(int k) {
  return k != K_NRX && k != K_NRY && k != K_NRZ;
}

// Gates whose matrix is diagonal in the computational basis (they commute with every
// diagonal operator and act on single amplitudes).
__host__ __device__ inline bool kind_diagonal(int k) {
  return k == K_RZ || k == K_Z || k == K_S || k == K_T || k == K_SDG || k == K_PHASE ||
         k == K_CZ || k == K_RZZ || k == K_CRZ;
}

// Same layout as qsv_gate.
struct GateDesc {
  int32_t kind, q0, q1, p[3];
};

// Matrices of one gate at the current parameters, written on the device by the prep kernel.
//   one-qubit kinds: m[0..3] = U (row-major 2x2), m[4 + 4j .. 7 + 4j] = dU / dtheta_j;
//                    non-unitary kinds also m[8..11] = U^-1
//   two-qubit kinds: m[0..15] = U (4x4, local index 2 bit(q0) + bit(q1)), m[16..31] = dU/dtheta
struct GateRec {
  double2 m[32];
};

// Pauli sum lowered for the device: P = i^{nY} X^x Z^z, so
//   (P psi)_j = i^{nY} (-1)^{popcount((j ^ x) & z)} psi_{j ^ x}.
// Terms are grouped by their X mask; coef = c * i^{nY}.
struct PauliGroup {
  uint64_t x;
  int32_t t0, t1;  // terms [t0, t1)
};
struct PauliTerm {
  uint64_t z;
  double cre, cim;
};

constexpr int kBlock = 256;        // threads per block of the gate-granular kernels
constexpr int kMaxBlocks = 2048;   // grid cap (grid-stride loops beyond)

// Device-side addresses of one gradient sweep's reduction partials.
struct Partials {
  double2* data;  // [slots][nb]
  int nb;         // blocks per launch (stride)
};

}  // namespace qsv
