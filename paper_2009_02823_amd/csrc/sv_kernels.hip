// Gate-granular HIP kernels for gfx950: one HBM pass per gate over amplitude pairs (one-qubit
// gates), quadruples (two-qubit gates) or single amplitudes (diagonal gates), with grid-stride
// loops over 64-bit indices so consecutive lanes touch consecutive amplitudes.
//
// The backward kernels implement one iteration of the reverse sweep of Algorithm 1 in a single
// pass: phi is un-applied, the derivative is applied to a register copy of phi (the clone mu
// never reaches memory), the products conj(lambda) mu are accumulated in FP64, and lambda is
// un-applied. Partial sums go to one slot per block (no atomics) and are reduced in a fixed order.
#include <cmath>

#include "qsv_device.h"
#include "sv_kernels.h"

namespace qsv {

// ----------------------------------------------------------------------------------------------
// Gate matrices at the current parameters (App. A): R_G(t) = exp(-i t G/2) = cos(t/2) - i
// sin(t/2) G, dR_G/dt = -(i/2) G R_G(t) = -sin(t/2)/2 - (i/2) cos(t/2) G.
// ----------------------------------------------------------------------------------------------
__device__ void set2(double2* m, double2 a, double2 b, double2 c, double2 d) {
  m[0] = a;
  m[1] = b;
  m[2] = c;
  m[3] = d;
}

// One-qubit Pauli g (1 = X, 2 = Y, 3 = Z): U = c 1 - i s G (deriv = false) or -s/2 1 - i c/2 G.
__device__ void pauli_rotation_2x2(double2* m, int g, double t, bool deriv) {
  double s, c;
  sincos(0.5 * t, &s, &c);
  const double a = deriv ? -0.5 * s : c;  // identity coefficient (real)
  const double b = deriv ? -0.5 * c : -s;  // G coefficient is i * b
  const double2 z = make_double2(0, 0);
  if (g == 1) set2(m, make_double2(a, 0), make_double2(0, b), make_double2(0, b), make_double2(a, 0));
  else if (g == 2) set2(m, make_double2(a, 0), make_double2(b, 0), make_double2(-b, 0), make_double2(a, 0));
  else set2(m, make_double2(a, b), z, z, make_double2(a, -b));
}

// Imaginary-time rotation exp(-t G/2) = ch 1 - sh G (ch = cosh(t/2), sh = sinh(t/2)), G = X, Y, Z
// (g = 1, 2, 3): which = 0 the matrix, 1 its derivative sh/2 1 - ch/2 G, 2 its inverse ch 1 + sh G.
__device__ void imag_rotation_2x2(double2* m, int g, double t, int which) {
  const double ch = cosh(0.5 * t), sh = sinh(0.5 * t);
  const double a = which == 1 ? 0.5 * sh : ch;                       // identity coefficient
  const double b = which == 0 ? -sh : which == 1 ? -0.5 * ch : sh;    // G coefficient
  const double2 z = make_double2(0, 0);
  if (g == 1) set2(m, make_double2(a, 0), make_double2(b, 0), make_double2(b, 0), make_double2(a, 0));
  else if (g == 2) set2(m, make_double2(a, 0), make_double2(0, -b), make_double2(0, b), make_double2(a, 0));
  else set2(m, make_double2(a + b, 0), z, z, make_double2(a - b, 0));
}

// Two-qubit Pauli product s(x)s (1 = XX, 2 = YY, 3 = ZZ) rotation, 4x4 row-major.
__device__ void pauli2_rotation_4x4(double2* m, int g, double t, bool deriv) {
  double s, c;
  sincos(0.5 * t, &s, &c);
  const double a = deriv ? -0.5 * s : c;
  const double b = deriv ? -0.5 * c : -s;  // coefficient of s(x)s is i * b
  for (int k = 0; k < 16; ++k) m[k] = make_double2(0, 0);
  for (int r = 0; r < 4; ++r) m[5 * r] = make_double2(a, 0);
  if (g == 3) {  // ZZ = diag(1, -1, -1, 1)
    const double sign[4] = {1, -1, -1, 1};
    for (int r = 0; r < 4; ++r) m[5 * r].y = b * sign[r];
  } else {       // XX: antidiagonal of ones; YY: antidiagonal (-1, 1, 1, -1)
    const double sign[4] = {g == 1 ? 1.0 : -1.0, 1, 1, g == 1 ? 1.0 : -1.0};
    for (int r = 0; r < 4; ++r) m[4 * r + (3 - r)] = make_double2(0, b * sign[r]);
  }
}

__global__ void k_prep(const GateDesc* gates, int n_gates, const double* theta, GateRec* recs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_gates) return;
  const GateDesc g = gates[k];
  GateRec r;
  for (int i = 0; i < 32; ++i) r.m[i] = make_double2(0, 0);
  double th[3] = {0, 0, 0};
  for (int j = 0; j < kind_nparams(g.kind); ++j) th[j] = theta[g.p[j]];
  const double h = 0.70710678118654752440;
  const double2 z = make_double2(0, 0), one = make_double2(1, 0);
  switch (g.kind) {
    case K_RX: case K_RY: case K_RZ:
      pauli_rotation_2x2(r.m, g.kind - K_RX + 1, th[0], false);
      pauli_rotation_2x2(r.m + 4, g.kind - K_RX + 1, th[0], true);
      break;
    case K_NRX: case K_NRY: case K_NRZ:
      imag_rotation_2x2(r.m, g.kind - K_NRX + 1, th[0], 0);
      imag_rotation_2x2(r.m + 4, g.kind - K_NRX + 1, th[0], 1);
      imag_rotation_2x2(r.m + 8, g.kind - K_NRX + 1, th[0], 2);
      break;
    case K_H: set2(r.m, make_double2(h, 0), make_double2(h, 0), make_double2(h, 0), make_double2(-h, 0)); break;
    case K_X: set2(r.m, z, one, one, z); break;
    case K_Y: set2(r.m, z, make_double2(0, -1), make_double2(0, 1), z); break;
    case K_Z: set2(r.m, one, z, z, make_double2(-1, 0)); break;
    case K_S: set2(r.m, one, z, z, make_double2(0, 1)); break;
    case K_SDG: set2(r.m, one, z, z, make_double2(0, -1)); break;
    case K_T: set2(r.m, one, z, z, make_double2(h, h)); break;
    case K_PHASE: {
      double s, c;
      sincos(th[0], &s, &c);
      set2(r.m, one, z, z, make_double2(c, s));
      set2(r.m + 4, z, z, z, make_double2(-s, c));  // i e^{it} |1><1|
      break;
    }
    case K_U3: {
      // [[c, -e^{il} s], [e^{if} s, e^{i(f+l)} c]] and its partial derivatives in (t, f, l)
      double s, c, sf, cf, sl, cl, sfl, cfl;
      sincos(0.5 * th[0], &s, &c);
      sincos(th[1], &sf, &cf);
      sincos(th[2], &sl, &cl);
      sincos(th[1] + th[2], &sfl, &cfl);
      set2(r.m, make_double2(c, 0), make_double2(-cl * s, -sl * s), make_double2(cf * s, sf * s),
           make_double2(cfl * c, sfl * c));
      set2(r.m + 4, make_double2(-0.5 * s, 0), make_double2(-0.5 * cl * c, -0.5 * sl * c),
           make_double2(0.5 * cf * c, 0.5 * sf * c), make_double2(-0.5 * cfl * s, -0.5 * sfl * s));
      set2(r.m + 8, z, z, make_double2(-sf * s, cf * s), make_double2(-sfl * c, cfl * c));
      set2(r.m + 12, z, make_double2(sl * s, -cl * s), z, make_double2(-sfl * c, cfl * c));
      break;
    }
    case K_CNOT:
      r.m[0] = r.m[5] = r.m[11] = r.m[14] = one;
      break;
    case K_CZ:
      r.m[0] = r.m[5] = r.m[10] = one;
      r.m[15] = make_double2(-1, 0);
      break;
    case K_CRX: case K_CRY: case K_CRZ: {
      // |0><0| (x) 1 + |1><1| (x) R; derivative |1><1| (x) dR
      double2 u[4], d[4];
      pauli_rotation_2x2(u, g.kind - K_CRX + 1, th[0], false);
      pauli_rotation_2x2(d, g.kind - K_CRX + 1, th[0], true);
      r.m[0] = r.m[5] = one;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          r.m[(2 + a) * 4 + 2 + b] = u[2 * a + b];
          r.m[16 + (2 + a) * 4 + 2 + b] = d[2 * a + b];
        }
      break;
    }
    case K_RXX: case K_RYY: case K_RZZ:
      pauli2_rotation_4x4(r.m, g.kind - K_RXX + 1, th[0], false);
      pauli2_rotation_4x4(r.m + 16, g.kind - K_RXX + 1, th[0], true);
      break;
    default:
      break;
  }
  recs[k] = r;
}

hipError_t launch_prep(const GateDesc* d_gates, int n_gates, const double* d_theta, GateRec* d_rec,
                       hipStream_t st) {
  if (n_gates <= 0) return hipSuccess;
  const int blk = 64;
  hipLaunchKernelGGL(k_prep, dim3((n_gates + blk - 1) / blk), dim3(blk), 0, st, d_gates, n_gates,
                     d_theta, d_rec);
  return hipGetLastError();
}

int sweep_blocks(int n) {
  const uint64_t pairs = n >= 1 ? (1ull << (n - 1)) : 1;
  uint64_t nb = (pairs + kBlock - 1) / kBlock;
  if (nb > (uint64_t)kMaxBlocks) nb = kMaxBlocks;
  return (int)(nb < 1 ? 1 : nb);
}

// ----------------------------------------------------------------------------------------------
// Forward (and inverse) gate kernels
// ----------------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_fwd_1q(typename Vec2<R>::T* psi, int n, int q, const GateRec* rec, int adj) {
  cx<R> u00 = mat<R>(rec, 0), u01 = mat<R>(rec, 1), u10 = mat<R>(rec, 2), u11 = mat<R>(rec, 3);
  if (adj) {
    const cx<R> t = u01;
    u00 = conj(u00); u11 = conj(u11); u01 = conj(u10); u10 = conj(t);
  }
  const uint64_t pairs = 1ull << (n - 1), bit = 1ull << q;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pairs;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i0 = insert_zero(g, q), i1 = i0 | bit;
    const cx<R> a = load<R>(psi, i0), b = load<R>(psi, i1);
    store<R>(psi, i0, u00 * a + u01 * b);
    store<R>(psi, i1, u10 * a + u11 * b);
  }
}

// Diagonal one-qubit gate: psi_j *= d[bit q of j].
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_fwd_diag1(typename Vec2<R>::T* psi, int n, int q, const GateRec* rec, int adj) {
  cx<R> d0 = mat<R>(rec, 0), d1 = mat<R>(rec, 3);
  if (adj) { d0 = conj(d0); d1 = conj(d1); }
  const uint64_t dim = 1ull << n;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < dim;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const cx<R> a = load<R>(psi, j);
    store<R>(psi, j, sel(((j >> q) & 1) != 0, d1, d0) * a);
  }
}

// Index of the g-th quadruple base of qubits (lo < hi): both bits cleared.
__device__ __forceinline__ uint64_t quad_base(uint64_t g, int lo, int hi) {
  return insert_zero(insert_zero(g, lo), hi);
}

// CNOT (self-inverse): swap the target pair inside the control = 1 half.
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_fwd_cnot(typename Vec2<R>::T* psi, int n, int c, int t) {
  const int lo = c < t ? c : t, hi = c < t ? t : c;
  const uint64_t quads = 1ull << (n - 2), bc = 1ull << c, bt = 1ull << t;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < quads;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i0 = quad_base(g, lo, hi) | bc, i1 = i0 | bt;
    const cx<R> a = load<R>(psi, i0), b = load<R>(psi, i1);
    store<R>(psi, i0, b);
    store<R>(psi, i1, a);
  }
}

// CZ (self-inverse): negate the amplitude with both bits set.
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_fwd_cz(typename Vec2<R>::T* psi, int n, int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  const uint64_t quads = 1ull << (n - 2), m = (1ull << a) | (1ull << b);
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < quads;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = quad_base(g, lo, hi) | m;
    store<R>(psi, i, neg(load<R>(psi, i)));
  }
}

template <typename R>
__device__ __forceinline__ void load_quad(const typename Vec2<R>::T* psi, const uint64_t* idx,
                                          cx<R>* v) {
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = load<R>(psi, idx[k]);
}

// w = M v (adj: M^dag v) for a 4x4 matrix stored row-major at rec->m[off ..].
template <typename R>
__device__ __forceinline__ void matvec4(const GateRec* rec, int off, bool adj, const cx<R>* v,
                                        cx<R>* w) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cx<R> s = {0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const cx<R> m = sel(adj, conj(mat<R>(rec, off + 4 * k + r)), mat<R>(rec, off + 4 * r + k));
      s = s + m * v[k];
    }
    w[r] = s;
  }
}

__device__ __forceinline__ void quad_indices(uint64_t g, int q0, int q1, uint64_t* idx) {
  const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  const uint64_t base = quad_base(g, lo, hi), b0 = 1ull << q0, b1 = 1ull << q1;
  idx[0] = base;
  idx[1] = base | b1;
  idx[2] = base | b0;
  idx[3] = base | b0 | b1;
}

// Generic two-qubit gate (4x4 matrix).
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_fwd_2q(typename Vec2<R>::T* psi, int n, int q0, int q1, const GateRec* rec, int adj) {
  const uint64_t quads = 1ull << (n - 2);
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < quads;
       g += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t idx[4];
    quad_indices(g, q0, q1, idx);
    cx<R> v[4], w[4];
    load_quad<R>(psi, idx, v);
    matvec4<R>(rec, 0, adj != 0, v, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) store<R>(psi, idx[k], w[k]);
  }
}

static unsigned grid_for(uint64_t items) {
  uint64_t nb = (items + kBlock - 1) / kBlock;
  if (nb > (uint64_t)kMaxBlocks) nb = kMaxBlocks;
  return (unsigned)(nb < 1 ? 1 : nb);
}

template <typename R>
hipError_t launch_forward_gate(void* psi_, int n, const GateDesc& g, const GateRec* d_rec, bool adj,
                               hipStream_t st) {
  using V = typename Vec2<R>::T;
  V* psi = static_cast<V*>(psi_);
  const int nq = kind_nqubits(g.kind);
  if (nq == 1) {
    if (kind_diagonal(g.kind))
      hipLaunchKernelGGL(k_fwd_diag1<R>, dim3(grid_for(1ull << n)), dim3(kBlock), 0, st, psi, n,
                         g.q0, d_rec, adj ? 1 : 0);
    else
      hipLaunchKernelGGL(k_fwd_1q<R>, dim3(grid_for(1ull << (n - 1))), dim3(kBlock), 0, st, psi,
                         n, g.q0, d_rec, adj ? 1 : 0);
  } else if (g.kind == K_CNOT) {
    hipLaunchKernelGGL(k_fwd_cnot<R>, dim3(grid_for(1ull << (n - 2))), dim3(kBlock), 0, st, psi, n,
                       g.q0, g.q1);
  } else if (g.kind == K_CZ) {
    hipLaunchKernelGGL(k_fwd_cz<R>, dim3(grid_for(1ull << (n - 2))), dim3(kBlock), 0, st, psi, n,
                       g.q0, g.q1);
  } else {
    hipLaunchKernelGGL(k_fwd_2q<R>, dim3(grid_for(1ull << (n - 2))), dim3(kBlock), 0, st, psi, n,
                       g.q0, g.q1, d_rec, adj ? 1 : 0);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Backward-sweep kernels (Algorithm 1, loop body): phi <- U^dag phi; mu = dU phi (registers);
// acc += conj(lambda) mu; lambda <- U^dag lambda.
// ----------------------------------------------------------------------------------------------
template <typename R, int NP>
__global__ void __launch_bounds__(kBlock)
k_bwd_1q(typename Vec2<R>::T* phi, typename Vec2<R>::T* lam, int n, int q, const GateRec* rec,
         int undo_lam, double2* partial, int nb, int inverse_rec) {
  const cx<R> u00 = mat<R>(rec, 0), u01 = mat<R>(rec, 1), u10 = mat<R>(rec, 2),
              u11 = mat<R>(rec, 3);
  // phi is un-done by U^-1: U^dag for unitary gates, the stored inverse m[8..11] otherwise
  const cx<R> v00 = inverse_rec ? mat<R>(rec, 8) : conj(u00);
  const cx<R> v01 = inverse_rec ? mat<R>(rec, 9) : conj(u10);
  const cx<R> v10 = inverse_rec ? mat<R>(rec, 10) : conj(u01);
  const cx<R> v11 = inverse_rec ? mat<R>(rec, 11) : conj(u11);
  double2 acc[NP > 0 ? NP : 1];
#pragma unroll
  for (int j = 0; j < (NP > 0 ? NP : 1); ++j) acc[j] = make_double2(0, 0);
  const uint64_t pairs = 1ull << (n - 1), bit = 1ull << q;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pairs;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i0 = insert_zero(g, q), i1 = i0 | bit;
    const cx<R> p0 = load<R>(phi, i0), p1 = load<R>(phi, i1);
    // phi <- U^-1 phi
    const cx<R> f0 = v00 * p0 + v01 * p1;
    const cx<R> f1 = v10 * p0 + v11 * p1;
    store<R>(phi, i0, f0);
    store<R>(phi, i1, f1);
    if (NP > 0 || undo_lam) {
      const cx<R> l0 = load<R>(lam, i0), l1 = load<R>(lam, i1);
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const cx<R> m0 = mat<R>(rec, 4 + 4 * j) * f0 + mat<R>(rec, 5 + 4 * j) * f1;
        const cx<R> m1 = mat<R>(rec, 6 + 4 * j) * f0 + mat<R>(rec, 7 + 4 * j) * f1;
        acc_dot<R>(acc[j], l0, m0);
        acc_dot<R>(acc[j], l1, m1);
      }
      if (undo_lam) {
        store<R>(lam, i0, conj(u00) * l0 + conj(u10) * l1);
        store<R>(lam, i1, conj(u01) * l0 + conj(u11) * l1);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) block_sum_store<kBlock>(acc[j], partial + (size_t)j * nb + blockIdx.x);
}

template <typename R, int NP>
__global__ void __launch_bounds__(kBlock)
k_bwd_diag1(typename Vec2<R>::T* phi, typename Vec2<R>::T* lam, int n, int q, const GateRec* rec,
            int undo_lam, double2* partial, int nb) {
  const cx<R> d0 = conj(mat<R>(rec, 0)), d1 = conj(mat<R>(rec, 3));  // U^dag
  const cx<R> e0 = mat<R>(rec, 4), e1 = mat<R>(rec, 7);              // dU (diagonal)
  double2 acc = make_double2(0, 0);
  const uint64_t dim = 1ull << n;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < dim;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const bool b = (j >> q) & 1;
    const cx<R> f = sel(b, d1, d0) * load<R>(phi, j);
    store<R>(phi, j, f);
    if (NP > 0 || undo_lam) {
      const cx<R> l = load<R>(lam, j);
      if (NP > 0) acc_dot<R>(acc, l, sel(b, e1, e0) * f);
      if (undo_lam) store<R>(lam, j, sel(b, d1, d0) * l);
    }
  }
  if (NP > 0) block_sum_store<kBlock>(acc, partial + blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_bwd_cnot(typename Vec2<R>::T* phi, typename Vec2<R>::T* lam, int n, int c, int t, int undo_lam) {
  const int lo = c < t ? c : t, hi = c < t ? t : c;
  const uint64_t quads = 1ull << (n - 2), bc = 1ull << c, bt = 1ull << t;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < quads;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i0 = quad_base(g, lo, hi) | bc, i1 = i0 | bt;
    const cx<R> a = load<R>(phi, i0), b = load<R>(phi, i1);
    store<R>(phi, i0, b);
    store<R>(phi, i1, a);
    if (undo_lam) {
      const cx<R> x = load<R>(lam, i0), y = load<R>(lam, i1);
      store<R>(lam, i0, y);
      store<R>(lam, i1, x);
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_bwd_cz(typename Vec2<R>::T* phi, typename Vec2<R>::T* lam, int n, int a, int b, int undo_lam) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  const uint64_t quads = 1ull << (n - 2), m = (1ull << a) | (1ull << b);
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < quads;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = quad_base(g, lo, hi) | m;
    store<R>(phi, i, neg(load<R>(phi, i)));
    if (undo_lam) store<R>(lam, i, neg(load<R>(lam, i)));
  }
}

template <typename R, int NP>
__global__ void __launch_bounds__(kBlock)
k_bwd_2q(typename Vec2<R>::T* phi, typename Vec2<R>::T* lam, int n, int q0, int q1,
         const GateRec* rec, int undo_lam, double2* partial, int nb) {
  double2 acc = make_double2(0, 0);
  const uint64_t quads = 1ull << (n - 2);
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < quads;
       g += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t idx[4];
    quad_indices(g, q0, q1, idx);
    cx<R> v[4], f[4];
    load_quad<R>(phi, idx, v);
    matvec4<R>(rec, 0, true, v, f);
#pragma unroll
    for (int k = 0; k < 4; ++k) store<R>(phi, idx[k], f[k]);
    if (NP > 0 || undo_lam) {
      cx<R> l[4];
      load_quad<R>(lam, idx, l);
      if (NP > 0) {
        cx<R> m[4];
        matvec4<R>(rec, 16, false, f, m);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc_dot<R>(acc, l[k], m[k]);
      }
      if (undo_lam) {
        cx<R> w[4];
        matvec4<R>(rec, 0, true, l, w);
#pragma unroll
        for (int k = 0; k < 4; ++k) store<R>(lam, idx[k], w[k]);
      }
    }
  }
  if (NP > 0) block_sum_store<kBlock>(acc, partial + blockIdx.x);
}

template <typename R>
hipError_t launch_backward_gate(void* phi_, void* lam_, int n, const GateDesc& g,
                                const GateRec* d_rec, bool undo_lam, double2* partial, int nb,
                                hipStream_t st) {
  using V = typename Vec2<R>::T;
  V* phi = static_cast<V*>(phi_);
  V* lam = static_cast<V*>(lam_);
  const int np = kind_nparams(g.kind), ul = undo_lam ? 1 : 0, inv = kind_unitary(g.kind) ? 0 : 1;
  const dim3 grid(nb), blk(kBlock);
  if (kind_nqubits(g.kind) == 1) {
    if (kind_diagonal(g.kind)) {
      if (np) hipLaunchKernelGGL((k_bwd_diag1<R, 1>), grid, blk, 0, st, phi, lam, n, g.q0, d_rec, ul, partial, nb);
      else hipLaunchKernelGGL((k_bwd_diag1<R, 0>), grid, blk, 0, st, phi, lam, n, g.q0, d_rec, ul, partial, nb);
    } else if (np == 3) {
      hipLaunchKernelGGL((k_bwd_1q<R, 3>), grid, blk, 0, st, phi, lam, n, g.q0, d_rec, ul, partial, nb,
                         inv);
    } else if (np == 1) {
      hipLaunchKernelGGL((k_bwd_1q<R, 1>), grid, blk, 0, st, phi, lam, n, g.q0, d_rec, ul, partial, nb,
                         inv);
    } else {
      hipLaunchKernelGGL((k_bwd_1q<R, 0>), grid, blk, 0, st, phi, lam, n, g.q0, d_rec, ul, partial, nb,
                         inv);
    }
  } else if (g.kind == K_CNOT) {
    hipLaunchKernelGGL(k_bwd_cnot<R>, grid, blk, 0, st, phi, lam, n, g.q0, g.q1, ul);
  } else if (g.kind == K_CZ) {
    hipLaunchKernelGGL(k_bwd_cz<R>, grid, blk, 0, st, phi, lam, n, g.q0, g.q1, ul);
  } else if (np) {
    hipLaunchKernelGGL((k_bwd_2q<R, 1>), grid, blk, 0, st, phi, lam, n, g.q0, g.q1, d_rec, ul, partial, nb);
  } else {
    hipLaunchKernelGGL((k_bwd_2q<R, 0>), grid, blk, 0, st, phi, lam, n, g.q0, g.q1, d_rec, ul, partial, nb);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Hamiltonian: (H psi)_j = sum_groups psi_{j^x} sum_{t in group} coef_t (-1)^{popc((j^x) & z_t)}
// ----------------------------------------------------------------------------------------------
// (H psi) at the V consecutive indices j0 .. j0 + V - 1 (j0 a multiple of V = 1, 2 or 4). For a
// group with X mask x the sources (j0 + k) ^ x form the aligned block j0 ^ (x & ~(V - 1)), in the
// order k ^ (x & (V - 1)): one contiguous load per group, permuted in registers. The sum over
// the groups is kept in FP64 whatever the storage precision (rounded only where it is stored).
template <typename R, int V>
__device__ __forceinline__ void pauli_block(const typename Vec2<R>::T* psi, uint64_t j0,
                                            const PauliGroup* groups, int n_groups,
                                            const PauliTerm* terms, cx<double>* acc) {
#pragma unroll
  for (int k = 0; k < V; ++k) acc[k] = {0, 0};
#pragma unroll 2
  for (int gi = 0; gi < n_groups; ++gi) {
    const PauliGroup G = groups[gi];
    const uint64_t base = j0 ^ (G.x & ~(uint64_t)(V - 1));
    cx<R> a[V];
#pragma unroll
    for (int k = 0; k < V; ++k) a[k] = load<R>(psi, base + k);
    const int xl = (int)(G.x & (V - 1));  // uniform
    if constexpr (V >= 2) {
      if (xl & 1) {
#pragma unroll
        for (int k = 0; k < V; k += 2) {
          const cx<R> t = a[k];
          a[k] = a[k + 1];
          a[k + 1] = t;
        }
      }
    }
    if constexpr (V >= 4) {
      if (xl & 2) {
#pragma unroll
        for (int k = 0; k < V; k += 4) {
          cx<R> t = a[k];
          a[k] = a[k + 2];
          a[k + 2] = t;
          t = a[k + 1];
          a[k + 1] = a[k + 3];
          a[k + 3] = t;
        }
      }
    }
    // a[k] = psi[(j0 + k) ^ x]; its coefficient sums the group's terms with their Z signs
    // (-1)^popcount(((j0 + k) ^ x) & z). j0 is a multiple of V, so the parity splits into the
    // block's part, popcount((j0 ^ x) & z) (once per term), and k's, popcount(k & z) (uniform).
    double sr[V], si[V];
#pragma unroll
    for (int k = 0; k < V; ++k) sr[k] = si[k] = 0.0;
    for (int t = G.t0; t < G.t1; ++t) {
      const PauliTerm T = terms[t];
      const uint32_t pb = (uint32_t)__popcll((j0 ^ G.x) & T.z & ~(uint64_t)(V - 1)) & 1u;
      const uint32_t zl = (uint32_t)(T.z & (V - 1));
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const uint32_t pk = (uint32_t)__popc((uint32_t)(k ^ (uint32_t)(G.x & (V - 1))) & zl) & 1u;
        const bool odd = (pb ^ pk) != 0;
        sr[k] += odd ? -T.cre : T.cre;
        si[k] += odd ? -T.cim : T.cim;
      }
    }
#pragma unroll
    for (int k = 0; k < V; ++k)
      acc[k] = acc[k] + cx<double>{sr[k], si[k]} * cx<double>{(double)a[k].r, (double)a[k].i};
  }
}

template <typename R>
__device__ __forceinline__ cx<double> widen(cx<R> a) {
  return {(double)a.r, (double)a.i};
}
template <typename R>
__device__ __forceinline__ cx<R> narrow(cx<double> a) {
  return {(R)a.r, (R)a.i};
}

template <typename R, bool WRITE, int V>
__global__ void __launch_bounds__(kBlock)
k_pauli(const typename Vec2<R>::T* psi, typename Vec2<R>::T* out, int n, const PauliGroup* groups,
        int n_groups, const PauliTerm* terms, double2* partial) {
  double2 e = make_double2(0, 0);
  const uint64_t blocks = (1ull << n) / V;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < blocks;
       b += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j0 = b * V;
    cx<double> acc[V];
    pauli_block<R, V>(psi, j0, groups, n_groups, terms, acc);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (WRITE) store<R>(out, j0 + k, narrow<R>(acc[k]));
      acc_dot<double>(e, widen<R>(load<R>(psi, j0 + k)), acc[k]);
    }
  }
  block_sum_store<kBlock>(e, partial + blockIdx.x);
}

// Every circuit of a batch in one launch: blockIdx.y selects the job, blockIdx.x strides over its
// amplitudes; partials[job * gridDim.x + blockIdx.x].
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_pauli_batched(const PauliJob* __restrict__ jobs, double2* partials) {
  constexpr int V = 4;  // a batched level needs a fused tile: every circuit has at least 8 qubits
  const PauliJob J = jobs[blockIdx.y];
  const typename Vec2<R>::T* psi = static_cast<const typename Vec2<R>::T*>(J.psi);
  typename Vec2<R>::T* out = static_cast<typename Vec2<R>::T*>(J.out);
  double2 e = make_double2(0, 0);
  const uint64_t blocks = (1ull << J.n) / V;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < blocks;
       b += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j0 = b * V;
    cx<double> acc[V];
    pauli_block<R, V>(psi, j0, J.groups, J.n_groups, J.terms, acc);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      store<R>(out, j0 + k, narrow<R>(acc[k]));
      acc_dot<double>(e, widen<R>(load<R>(psi, j0 + k)), acc[k]);
    }
  }
  block_sum_store<kBlock>(e, partials + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

template <typename R>
hipError_t launch_pauli_batched(const PauliJob* d_jobs, int n_jobs, int blocks_per_job,
                                double2* partials, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pauli_batched<R>, dim3(blocks_per_job, n_jobs), dim3(kBlock), 0, st,
                     d_jobs, partials);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pauli(const void* psi_, void* out_, int n, const PauliGroup* d_groups,
                        int n_groups, const PauliTerm* d_terms, double2* partial, int nb,
                        hipStream_t st) {
  using V = typename Vec2<R>::T;
  const V* psi = static_cast<const V*>(psi_);
  V* out = static_cast<V*>(out_);
#define QSV_PAULI(VV)                                                                         \
  if (out)                                                                                    \
    hipLaunchKernelGGL((k_pauli<R, true, VV>), dim3(nb), dim3(kBlock), 0, st, psi, out, n,    \
                       d_groups, n_groups, d_terms, partial);                                 \
  else                                                                                        \
    hipLaunchKernelGGL((k_pauli<R, false, VV>), dim3(nb), dim3(kBlock), 0, st, psi, out, n,   \
                       d_groups, n_groups, d_terms, partial);
  if (n >= 2) {
    QSV_PAULI(4)
  } else {
    QSV_PAULI(1)
  }
#undef QSV_PAULI
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Tiled application of H
// ----------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t parity64(uint64_t v) { return (uint32_t)__popcll(v) & 1u; }

template <typename R, int TB, int LE>
__global__ void __launch_bounds__(1 << (TB - LE))
k_pauli_tile(const typename Vec2<R>::T* __restrict__ psi, typename Vec2<R>::T* lam,
             PauliTilePass P, const PauliTileGroup* __restrict__ groups,
             const PauliTerm* __restrict__ terms, double2* partial) {
  using V = typename Vec2<R>::T;
  constexpr int NT = 1 << (TB - LE), EPT = 1 << LE, HALF = EPT / 2;
  __shared__ V tile[1 << TB];
  __shared__ PauliTerm sterm[kPauliTileMaxTerms];
  __shared__ PauliTileGroup sgroup[kPauliTileMaxTerms];
  __shared__ double2 red[NT / 64];
  const uint32_t tid = threadIdx.x;
  const int lane = tid & 63;
  const int n_terms = P.n_terms, n_groups = P.g1 - P.g0;
  // the pass's terms and groups, staged once
  for (int t = tid; t < n_terms; t += NT) sterm[t] = terms[P.t0 + t];
  for (int g = tid; g < n_groups; g += NT) sgroup[g] = groups[P.g0 + g];
  // thread part of the amplitude index (tile bits 0 .. TB-LE-1); element offsets (bits TB-LE ..
  // TB-1) are uniform
  uint64_t gthr = 0;
#pragma unroll
  for (int s = 0; s < TB - LE; ++s) gthr |= (uint64_t)((tid >> s) & 1u) << P.tile[s];
  uint64_t greg[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    uint64_t o = 0;
#pragma unroll
    for (int b = 0; b < LE; ++b)
      if ((k >> b) & 1) o |= 1ull << P.tile[TB - LE + b];
    greg[k] = o;
  }
  __syncthreads();
  // sign bits of the thread part, one per term of the pass
  uint64_t tb = 0;
  for (int t = 0; t < n_terms; ++t) tb |= (uint64_t)parity64(gthr & sterm[t].z) << t;
  // lane t holds term t's Z mask for the per-tile sign bits (one ballot per tile)
  const uint64_t zl = lane < n_terms ? sterm[lane].z : 0ull;
  double2 e = make_double2(0, 0);
  const uint64_t n_tiles = 1ull << P.n_outer;
  for (uint64_t g = blockIdx.x; g < n_tiles; g += gridDim.x) {
    uint64_t obase = 0;
    {
      uint64_t x = g;
      for (uint64_t m = P.outer_mask; m && x; m &= m - 1, x >>= 1)
        if (x & 1) obase |= m & (~m + 1);
    }
    const uint64_t ob = __ballot(parity64(obase & zl) != 0);
    const uint64_t base = obase | gthr;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const cx<R> v = load<R>(psi, base | greg[k]);
      V w;
      w.x = v.r;
      w.y = v.i;
      tile[tid + NT * k] = w;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cx<R> lv[HALF];
      if (P.lam_mode == 1) {
#pragma unroll
        for (int k = 0; k < HALF; ++k) lv[k] = load<R>(lam, base | greg[h * HALF + k]);
      }
      uint64_t sb[HALF];
#pragma unroll
      for (int k = 0; k < HALF; ++k) sb[k] = tb ^ ob ^ P.kbits[h * HALF + k];
      double ar[HALF], ai[HALF];
#pragma unroll
      for (int k = 0; k < HALF; ++k) ar[k] = ai[k] = 0.0;
      for (int gi = 0; gi < n_groups; ++gi) {
        const PauliTileGroup G = sgroup[gi];
        double cr[HALF], ci[HALF];
#pragma unroll
        for (int k = 0; k < HALF; ++k) cr[k] = ci[k] = 0.0;
        for (int t = G.t0; t < G.t1; ++t) {
          const PauliTerm T = sterm[t];
          // the sign flips the weight's sign bit; a Hermitian term's weight is real or imaginary
          const int sh = 31 - (t & 31);
          const bool hi = t >= 32, has_re = T.cre != 0.0, has_im = T.cim != 0.0;
#pragma unroll
          for (int k = 0; k < HALF; ++k) {
            const uint32_t word = hi ? (uint32_t)(sb[k] >> 32) : (uint32_t)sb[k];
            const uint32_t flip = (word << sh) & 0x80000000u;
            if (has_re) cr[k] += __hiloint2double(__double2hiint(T.cre) ^ (int)flip, __double2loint(T.cre));
            if (has_im) ci[k] += __hiloint2double(__double2hiint(T.cim) ^ (int)flip, __double2loint(T.cim));
          }
        }
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
          const V w = tile[(tid + NT * (h * HALF + k)) ^ G.xl];
          const double wr = (double)w.x, wi = (double)w.y;
          ar[k] += cr[k] * wr - ci[k] * wi;
          ai[k] += cr[k] * wi + ci[k] * wr;
        }
      }
#pragma unroll
      for (int k = 0; k < HALF; ++k) {
        // E part: conj(psi_j) (H psi)_j, FP64
        const V w = tile[tid + NT * (h * HALF + k)];
        const double pr = (double)w.x, pi = (double)w.y;
        e.x += pr * ar[k] + pi * ai[k];
        e.y += pr * ai[k] - pi * ar[k];
        const uint64_t idx = base | greg[h * HALF + k];
        if (P.lam_mode == 0)
          store<R>(lam, idx, cx<R>{(R)ar[k], (R)ai[k]});
        else if (P.lam_mode == 1)
          store<R>(lam, idx, cx<R>{(R)((double)lv[k].r + ar[k]), (R)((double)lv[k].i + ai[k])});
      }
    }
    __syncthreads();  // the tile buffer is rewritten by the next tile
  }
  // block sum in a fixed order: waves, then the waves in index order
  const double re = wave_sum(e.x), im = wave_sum(e.y);
  if (lane == 0) red[tid >> 6] = make_double2(re, im);
  __syncthreads();
  if (tid == 0) {
    double2 s = red[0];
    for (int w = 1; w < NT / 64; ++w) {
      s.x += red[w].x;
      s.y += red[w].y;
    }
    if (P.e_accumulate) {
      s.x = partial[blockIdx.x].x + s.x;
      s.y = partial[blockIdx.x].y + s.y;
    }
    partial[blockIdx.x] = s;
  }
}

template <typename R>
hipError_t launch_pauli_tile(const void* psi, void* lam, const PauliTilePass& P,
                             const PauliTileGroup* d_groups, const PauliTerm* d_terms,
                             double2* partial, int grid, hipStream_t st) {
  using V = typename Vec2<R>::T;
  constexpr bool C128 = sizeof(R) == 8;
  constexpr int TB = C128 ? 12 : 13, LE = 3;
  static_assert(TB == pauli_tile_bits(C128) && (1 << LE) == pauli_tile_elements(C128), "tile shape");
  hipLaunchKernelGGL((k_pauli_tile<R, TB, LE>), dim3(grid), dim3(1 << (TB - LE)), 0, st,
                     static_cast<const V*>(psi), static_cast<V*>(lam), P, d_groups, d_terms,
                     partial);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Clone and reset
// ----------------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_copy(typename Vec2<R>::T* dst, const typename Vec2<R>::T* src, uint64_t count) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
       j += (uint64_t)gridDim.x * blockDim.x)
    dst[j] = src[j];
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_reset(typename Vec2<R>::T* psi, uint64_t count) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
       j += (uint64_t)gridDim.x * blockDim.x) {
    typename Vec2<R>::T v;
    v.x = j == 0 ? (R)1 : (R)0;
    v.y = 0;
    psi[j] = v;
  }
}

template <typename R>
hipError_t launch_copy(void* dst, const void* src, int n, hipStream_t st) {
  using V = typename Vec2<R>::T;
  hipLaunchKernelGGL(k_copy<R>, dim3(grid_for(1ull << n)), dim3(kBlock), 0, st,
                     static_cast<V*>(dst), static_cast<const V*>(src), 1ull << n);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_reset(void* psi, int n, hipStream_t st) {
  using V = typename Vec2<R>::T;
  hipLaunchKernelGGL(k_reset<R>, dim3(grid_for(1ull << n)), dim3(kBlock), 0, st,
                     static_cast<V*>(psi), 1ull << n);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Second reduction stage (fixed order): one block per parameter.
// ----------------------------------------------------------------------------------------------
__device__ double2 block_sum_range(const double2* p, int count) {
  __shared__ double2 sm[kBlock];
  double2 s = make_double2(0, 0);
  for (int b = threadIdx.x; b < count; b += kBlock) {
    s.x += p[b].x;
    s.y += p[b].y;
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sm[threadIdx.x].x += sm[threadIdx.x + w].x;
      sm[threadIdx.x].y += sm[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  const double2 r = sm[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kBlock)
k_final_grad(const FinalDesc* __restrict__ descs, int n_desc, double* grad) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = n_desc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].p_begin <= blk) lo = mid;
    else hi = mid - 1;
  }
  const FinalDesc d = descs[lo];
  const int p = (int)(blk - d.p_begin);
  double total = 0;
  for (int k = d.param_ptr[p]; k < d.param_ptr[p + 1]; ++k) {
    const int o = d.occ[k];
    const double2 s = block_sum_range(d.partials + d.occ_base[o], d.occ_nb[o]);
    total += s.x;
  }
  if (threadIdx.x == 0) grad[d.grad_off + p] = 2.0 * total;
}

// Complex gradient of a non-Hermitian operator A (App. B.4) from the complex entries of the two
// sweeps, with A (descriptor a) and A^dag (descriptor b): grad[p] = conj(Z_A[p]) + Z_{A^dag}[p],
// Z[p] the sum of the entries of the occurrences of p. grad holds (Re, Im) pairs.
__global__ void __launch_bounds__(kBlock)
k_final_grad_nonherm(const FinalDesc* __restrict__ a, const FinalDesc* __restrict__ b,
                     double* grad) {
  const int p = blockIdx.x;
  double2 za = make_double2(0, 0), zb = make_double2(0, 0);
  for (int k = a->param_ptr[p]; k < a->param_ptr[p + 1]; ++k) {
    const int o = a->occ[k];
    const double2 sa = block_sum_range(a->partials + a->occ_base[o], a->occ_nb[o]);
    const double2 sb = block_sum_range(b->partials + b->occ_base[o], b->occ_nb[o]);
    za.x += sa.x;
    za.y += sa.y;
    zb.x += sb.x;
    zb.y += sb.y;
  }
  if (threadIdx.x == 0) {
    grad[2 * p] = za.x + zb.x;
    grad[2 * p + 1] = zb.y - za.y;
  }
}

hipError_t launch_final_grad_nonherm(const FinalDesc* d_a, const FinalDesc* d_b, int n_theta,
                                     double* d_grad, hipStream_t st) {
  if (n_theta <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_final_grad_nonherm, dim3((unsigned)n_theta), dim3(kBlock), 0, st, d_a, d_b,
                     d_grad);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_final_energy_batched(const double2* partials, int nb, double* energy) {
  const double2 s = block_sum_range(partials + (size_t)blockIdx.x * nb, nb);
  if (threadIdx.x == 0) energy[blockIdx.x] = s.x;
}

hipError_t launch_final_energy_batched(const double2* partials, int nb, int n_jobs,
                                       double* d_energy, hipStream_t st) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_final_energy_batched, dim3(n_jobs), dim3(kBlock), 0, st, partials, nb,
                     d_energy);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_final_energy(const double2* partials, int nb, double* energy, double* energy_im) {
  const double2 s = block_sum_range(partials, nb);
  if (threadIdx.x == 0) {
    *energy = s.x;
    if (energy_im) *energy_im = s.y;
  }
}

hipError_t launch_final_grad(const FinalDesc* d_desc, int n_desc, int64_t total_params,
                             double* d_grad, hipStream_t st) {
  if (total_params <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_final_grad, dim3((unsigned)total_params), dim3(kBlock), 0, st, d_desc,
                     n_desc, d_grad);
  return hipGetLastError();
}

hipError_t launch_final_energy(const double2* partials, int nb, double* d_energy,
                               double* d_energy_im, hipStream_t st) {
  hipLaunchKernelGGL(k_final_energy, dim3(1), dim3(kBlock), 0, st, partials, nb, d_energy,
                     d_energy_im);
  return hipGetLastError();
}

const char* forward_kernel_name(const GateDesc& g) {
  if (kind_nqubits(g.kind) == 1) return kind_diagonal(g.kind) ? "k_fwd_diag1" : "k_fwd_1q";
  if (g.kind == K_CNOT) return "k_fwd_cnot";
  if (g.kind == K_CZ) return "k_fwd_cz";
  return "k_fwd_2q";
}

const char* backward_kernel_name(const GateDesc& g) {
  if (kind_nqubits(g.kind) == 1) return kind_diagonal(g.kind) ? "k_bwd_diag1" : "k_bwd_1q";
  if (g.kind == K_CNOT) return "k_bwd_cnot";
  if (g.kind == K_CZ) return "k_bwd_cz";
  return "k_bwd_2q";
}

// ----------------------------------------------------------------------------------------------
// Parameter-shift helpers
// ----------------------------------------------------------------------------------------------
__global__ void k_shift_theta(double* dst, const double* src, int n_theta, int p, double delta) {
  for (int i = threadIdx.x; i < n_theta; i += blockDim.x) dst[i] = src[i] + (i == p ? delta : 0.0);
}

__global__ void k_ps_combine(double* grad, const double* e, int first, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) grad[first + i] = 0.5 * (e[2 * i] - e[2 * i + 1]);
}

hipError_t launch_shift_theta(double* dst, const double* src, int n_theta, int p, double delta,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_shift_theta, dim3(1), dim3(256), 0, st, dst, src, n_theta, p, delta);
  return hipGetLastError();
}

hipError_t launch_ps_combine(double* grad, const double* e, int first, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ps_combine, dim3(1), dim3(256), 0, st, grad, e, first, count);
  return hipGetLastError();
}

// Explicit instantiations for the two storage precisions.
#define QSV_INSTANTIATE(R)                                                                        \
  template hipError_t launch_forward_gate<R>(void*, int, const GateDesc&, const GateRec*, bool,    \
                                             hipStream_t);                                         \
  template hipError_t launch_backward_gate<R>(void*, void*, int, const GateDesc&, const GateRec*,  \
                                              bool, double2*, int, hipStream_t);                   \
  template hipError_t launch_pauli_batched<R>(const PauliJob*, int, int, double2*, hipStream_t); \
  template hipError_t launch_pauli<R>(const void*, void*, int, const PauliGroup*, int,             \
                                      const PauliTerm*, double2*, int, hipStream_t);               \
  template hipError_t launch_pauli_tile<R>(const void*, void*, const PauliTilePass&,               \
                                           const PauliTileGroup*, const PauliTerm*, double2*, int,   \
                                           hipStream_t);                                             \
  template hipError_t launch_copy<R>(void*, const void*, int, hipStream_t);                        \
  template hipError_t launch_reset<R>(void*, int, hipStream_t);
QSV_INSTANTIATE(double)
QSV_INSTANTIATE(float)

}  // namespace qsv
