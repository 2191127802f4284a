// Fused pass kernels for gfx950 (see fused.h for the tile/phase model).
//
// One workgroup of 2^W threads processes tiles of 2^(RB+W) amplitudes; every thread keeps 2^RB
// amplitudes of each state in registers. Loads and stores use the direct layout (consecutive lanes
// on consecutive tile bits, the low tile bits being the lowest physical qubits), so every wave
// reads and writes runs of contiguous amplitudes. Register phases are changed by a transpose
// through LDS with an XOR swizzle of the element index against bank conflicts.
//
// The reverse-sweep kernel applies, per gate, the loop body of Algorithm 1 to both states held in
// registers: the product of lambda with the gate derivative applied to phi, then
// phi <- U^dag phi and lambda <- U^dag lambda. For the rotations R = exp(-i t G/2) the product
// uses dR/dt = -(i/2) G R (paper App. A): Re <lambda|dR phi'> = (1/2) Im <lambda|G|phi> with phi
// taken before un-applying R; other parameterised gates use their explicit derivative matrices.
// Per-thread products (FP64) are summed over the wave with DPP row operations and accumulated in a
// register of the wave, lane j holding product slot j, over all tiles of the workgroup; the waves'
// sums are combined through LDS and written as one partial per workgroup and product slot; no
// atomics, fixed order.
//
// At the start of a pass every workgroup copies the pass's op records, with the cos/sin of the
// rotation angles, and its phase descriptors into LDS in one round of loads issued behind the
// first tile's loads. Ops are then read from LDS one ahead of their execution, so no op waits for a
// dependent global load.
//
// Two instances per geometry: the lean one handles RX, RY, RZ, CNOT, CZ and fixed one-qubit
// gates, with every control/diagonal bit resolved either at compile time (register bit) or once
// per thread (thread bit); the general one adds parameterised dense/diagonal gates with explicit
// derivatives, controlled rotations and two-qubit rotations.
#include <cstddef>

#include "fused.h"
#include "qsv_device.h"

namespace qsv {

template <typename R>
struct Swz;
// 64 banks x 4 bytes: fold higher index bits into the bank-selecting bits
template <>
struct Swz<double> {  // 16-byte elements, 16 per bank row
  static __device__ __forceinline__ uint32_t f(uint32_t x) {
    return x ^ (((x >> 4) ^ (x >> 8) ^ (x >> 12)) & 15u);
  }
};
template <>
struct Swz<float> {  // 8-byte elements, 32 per bank row
  static __device__ __forceinline__ uint32_t f(uint32_t x) { return x ^ (((x >> 5) ^ (x >> 10)) & 31u); }
};

// s_waitcnt immediate for vmcnt(0) lgkmcnt(0) (expcnt not waited for).
constexpr int kWaitVmLgkm = 0x0070;

// Workgroup barrier for LDS traffic: waits for this wave's LDS (and scalar) operations only, so
// global loads already issued stay in flight across it. The memory clobber keeps the compiler
// from moving memory accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------------------------
// Layouts
// ---------------------------------------------------------------------------------------------
template <int RB>
struct Layout {
  int8_t rb[RB];   // tile bit of each register position (ascending)
  uint32_t tdep;   // thread part of the tile index
  uint32_t tsw;    // its swizzled LDS element index
};

// The thread index deposited into the tile bits that are not register bits (lowest first): a
// zero inserted at every register bit, in ascending order.
template <int RB>
__device__ __forceinline__ uint32_t insert_zeros(const int8_t* regbit, uint32_t tid) {
  uint32_t x = tid;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const uint32_t b = (uint32_t)regbit[k];
    x = ((x >> b) << (b + 1)) | (x & ((1u << b) - 1u));
  }
  return x;
}


template <int RB>
__device__ __forceinline__ uint32_t reg_deposit(const Layout<RB>& L, int ri) {
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < RB; ++k) x |= (uint32_t)((ri >> k) & 1) << L.rb[k];
  return x;
}

// The swizzle is linear over GF(2) (an XOR of shifted copies), and the thread and register
// parts of an element index have disjoint bits, so the LDS index of element ri is the XOR of the
// swizzled thread part (once per layout and thread) and the swizzled register part (uniform).
template <typename R, int RB>
__device__ __forceinline__ void make_layout(Layout<RB>& L, const int8_t* regbit, uint32_t tid) {
#pragma unroll
  for (int k = 0; k < RB; ++k) L.rb[k] = regbit[k];
  L.tdep = insert_zeros<RB>(regbit, tid);
  L.tsw = Swz<R>::f(L.tdep);
}
template <typename R, int RB>
__device__ __forceinline__ uint32_t lds_index(const Layout<RB>& L, int ri) {
  return L.tsw ^ Swz<R>::f(reg_deposit<RB>(L, ri));
}

// Register index ri through a phase's rperm (PhaseDesc): 0 is the identity; otherwise the XOR of
// the images Q(e_k) (bits 4k .. 4k + 3) of ri's set bits. Uniform.
template <int RB>
__device__ __forceinline__ int perm_index(uint32_t rperm, int ri) {
  if (rperm == 0) return ri;
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < RB; ++k)
    if ((ri >> k) & 1) v ^= (rperm >> (4 * k)) & 15u;
  return (int)v;
}

// rperm: the reads take element Q(ri) into register ri (CNOTs on register bits folded into the
// relayout; 0 for none).
template <typename R, int RB>
__device__ __forceinline__ void relayout(cx<R>* a, const Layout<RB>& from, const Layout<RB>& to,
                                         typename Vec2<R>::T* lds, uint32_t rperm = 0) {
  constexpr int NA = 1 << RB;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    typename Vec2<R>::T v;
    v.x = a[ri].r;
    v.y = a[ri].i;
    lds[lds_index<R, RB>(from, ri)] = v;
  }
  lds_barrier();
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    const typename Vec2<R>::T v = lds[lds_index<R, RB>(to, perm_index<RB>(rperm, ri))];
    a[ri].r = v.x;
    a[ri].i = v.y;
  }
  lds_barrier();
}

// Both states of the reverse sweep through one pair of barriers (two LDS halves).
template <typename R, int RB>
__device__ __forceinline__ void relayout2(cx<R>* a, cx<R>* b, const Layout<RB>& from,
                                          const Layout<RB>& to, typename Vec2<R>::T* lds,
                                          int half, uint32_t rperm = 0) {
  constexpr int NA = 1 << RB;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    const uint32_t x = lds_index<R, RB>(from, ri);
    typename Vec2<R>::T v, w;
    v.x = a[ri].r;
    v.y = a[ri].i;
    w.x = b[ri].r;
    w.y = b[ri].i;
    lds[x] = v;
    lds[half + x] = w;
  }
  lds_barrier();
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    const uint32_t x = lds_index<R, RB>(to, perm_index<RB>(rperm, ri));
    const typename Vec2<R>::T v = lds[x], w = lds[half + x];
    a[ri].r = v.x;
    a[ri].i = v.y;
    b[ri].r = w.x;
    b[ri].i = w.y;
  }
  lds_barrier();
}

template <int RB>
__device__ __forceinline__ bool same_layout(const Layout<RB>& a, const int8_t* rb) {
  bool s = true;
#pragma unroll
  for (int k = 0; k < RB; ++k) s = s && a.rb[k] == rb[k];
  return s;
}

// ---------------------------------------------------------------------------------------------
// Lean ops. ADJ selects U^dag (reverse sweep) instead of U.
// ---------------------------------------------------------------------------------------------

// x <- x + m t with the result in x's own register (a tied operand): left to itself the compiler
// accumulates into a temporary and copies the result back at the switch join.
__device__ __forceinline__ void fmac_inplace(double& x, double m, double t) {
  asm("v_fma_f64 %0, %1, %2, %0" : "+v"(x) : "v"(m), "v"(t));
}
__device__ __forceinline__ void fmac_inplace(float& x, float m, float t) {
  asm("v_fma_f32 %0, %1, %2, %0" : "+v"(x) : "v"(m), "v"(t));
}
// (x, y) <- the plane rotation [[cos phi, -sin phi], [sin phi, cos phi]] (x, y) as three shears
// (alpha = -tan(phi/2), beta = sin phi), in place: three FMAs per pair of components.
template <typename R>
__device__ __forceinline__ void shear3(R& x, R& y, R al, R be) {
  fmac_inplace(x, al, y);
  fmac_inplace(y, be, x);
  fmac_inplace(x, al, y);
}

// Rotations on register position K from the staged shear factors (al, be); ADJ rotates by -phi.
// RY = [[c, -s], [s, c]] rotates (re a0, re a1) and (im a0, im a1).
template <typename R, int NA, int K, bool ADJ>
__device__ __forceinline__ void ry_k(cx<R>* a, R al, R be) {
  if constexpr (ADJ) { al = -al; be = -be; }
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    shear3(a[ri].r, a[rj].r, al, be);
    shear3(a[ri].i, a[rj].i, al, be);
  }
}

// RX = [[c, -i s], [-i s, c]] rotates (im a1, re a0) and (im a0, re a1).
template <typename R, int NA, int K, bool ADJ>
__device__ __forceinline__ void rx_k(cx<R>* a, R al, R be) {
  if constexpr (ADJ) { al = -al; be = -be; }
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    shear3(a[rj].i, a[ri].r, al, be);
    shear3(a[ri].i, a[rj].r, al, be);
  }
}

// RZ = diag(c - i s, c + i s): bit 0 rotates (im z, re z), bit 1 rotates (re z, im z).
template <typename R, int NA, int K, bool ADJ>
__device__ __forceinline__ void rz_k(cx<R>* a, R al, R be) {
  if constexpr (ADJ) { al = -al; be = -be; }
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if ((ri >> K) & 1) shear3(a[ri].r, a[ri].i, al, be);
    else shear3(a[ri].i, a[ri].r, al, be);
  }
}

// RZ on a thread bit b: every amplitude rotates (re z, im z) by phi (b = 1) or -phi (b = 0).
template <typename R, int NA, bool ADJ>
__device__ __forceinline__ void rz_thr(cx<R>* a, R al, R be, bool b) {
  if (b == ADJ) { al = -al; be = -be; }
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) shear3(a[ri].r, a[ri].i, al, be);
}

// a <- -a (the sign carried by rotations staged with FOPF_FLIP)
template <typename R, int NA>
__device__ __forceinline__ void negate_all(cx<R>* a) {
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) a[ri] = cx<R>{-a[ri].r, -a[ri].i};
}

// Exchange two values in their registers (v_swap_b32). Written as an exchange of SSA values, a
// swap inside one case of the op switch permutes the amplitude array at the switch join; the
// register allocator then splits every amplitude's live range and copies all of them on every
// op's path. The tied asm operands keep each register holding "its" array element.
__device__ __forceinline__ void swap_inplace(double& x, double& y) {
  int xl = __double2loint(x), xh = __double2hiint(x);
  int yl = __double2loint(y), yh = __double2hiint(y);
  asm("v_swap_b32 %0, %1" : "+v"(xl), "+v"(yl));
  asm("v_swap_b32 %0, %1" : "+v"(xh), "+v"(yh));
  x = __hiloint2double(xh, xl);
  y = __hiloint2double(yh, yl);
}
__device__ __forceinline__ void swap_inplace(float& x, float& y) {
  asm("v_swap_b32 %0, %1" : "+v"(x), "+v"(y));
}

// CNOT with control and target both register positions: swaps chosen at compile time.
template <typename R, int NA, int KC, int KT>
__device__ __forceinline__ void cnot_rr(cx<R>* a) {
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if ((ri & (1 << KT)) || !(ri & (1 << KC))) continue;
    swap_inplace(a[ri].r, a[ri | (1 << KT)].r);
    swap_inplace(a[ri].i, a[ri | (1 << KT)].i);
  }
}

// CNOT with the control on a thread bit: swap the target pairs of the threads whose bit is set.
// A branch on the thread's bit (the swaps run under the exec mask of those lanes): one v_swap_b32
// per word instead of two selects.
template <typename R, int NA, int KT>
__device__ __forceinline__ void cnot_tr(cx<R>* a, bool on) {
  if (on) {
#pragma unroll
    for (int ri = 0; ri < NA; ++ri) {
      if (ri & (1 << KT)) continue;
      const int rj = ri | (1 << KT);
      swap_inplace(a[ri].r, a[rj].r);
      swap_inplace(a[ri].i, a[rj].i);
    }
  }
}

// Flips the sign of x when sign = 0x80000000 (an XOR of the sign bit).
__device__ __forceinline__ double flip_sign(double x, uint32_t sign) {
  return __hiloint2double(__double2hiint(x) ^ (int)sign, __double2loint(x));
}
__device__ __forceinline__ float flip_sign(float x, uint32_t sign) {
  return __int_as_float(__float_as_int(x) ^ (int)sign);
}

// Negate the amplitudes whose register bits in MASK are all set, when `on`.
template <typename R, int NA, int MASK>
__device__ __forceinline__ void neg_where(cx<R>* a, bool on) {
  const uint32_t sign = on ? 0x80000000u : 0u;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if ((ri & MASK) != MASK) continue;
    a[ri] = cx<R>{flip_sign(a[ri].r, sign), flip_sign(a[ri].i, sign)};
  }
}

template <typename R, int NA, int K>
__device__ __forceinline__ void dense1_k(cx<R>* a, cx<R> m00, cx<R> m01, cx<R> m10, cx<R> m11) {
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    const cx<R> x = a[ri], y = a[rj];
    a[ri] = m00 * x + m01 * y;
    a[rj] = m10 * x + m11 * y;
  }
}

template <typename R, int NA, int K>
__device__ __forceinline__ void diag1_k(cx<R>* a, cx<R> d0, cx<R> d1) {
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) a[ri] = (((ri >> K) & 1) ? d1 : d0) * a[ri];
}

// ---- runtime register position -> compile-time template instance (general ops)
template <typename R, int RB, bool ADJ, int K = 0, typename... Args>
__device__ __forceinline__ void dense1_at(int k, cx<R>* a, Args... args) {
  if constexpr (K < RB) {
    if (k == K) dense1_k<R, 1 << RB, K>(a, args...);
    else dense1_at<R, RB, ADJ, K + 1>(k, a, args...);
  }
}

__device__ __forceinline__ bool thread_bit(uint32_t tdep, int s) { return (tdep >> s) & 1u; }

// ---------------------------------------------------------------------------------------------
// Products of the lean parameterised ops: Re <lambda|dR phi'> = (1/2) Im <lambda|G|phi>, phi
// before the un-application. Per-pair terms are summed as a balanced tree.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double im_cm(double lr, double li, double fr, double fi) {
  return lr * fi - li * fr;  // Im(conj(l) f)
}
__device__ __forceinline__ double re_cm(double lr, double li, double fr, double fi) {
  return lr * fr + li * fi;  // Re(conj(l) f)
}

template <int N>
__device__ __forceinline__ double tree_sum(const double* t) {
  if constexpr (N == 1) return t[0];
  else return tree_sum<N / 2>(t) + tree_sum<N - N / 2>(t + N / 2);
}

// Complex64: per pair a product difference, then a tree sum over the pairs.
template <typename R, int NA, int K>
__device__ __forceinline__ double prod_ry_pairs(const cx<R>* f, const cx<R>* l) {
  double t[NA / 2];  // Y f = (-i f1, i f0)
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    t[j++] = re_cm(l[rj].r, l[rj].i, f[ri].r, f[ri].i) - re_cm(l[ri].r, l[ri].i, f[rj].r, f[rj].i);
  }
  return 0.5 * tree_sum<NA / 2>(t);
}

template <typename R, int NA, int K>
__device__ __forceinline__ double prod_rx_pairs(const cx<R>* f, const cx<R>* l) {
  double t[NA / 2];  // X f = (f1, f0)
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    t[j++] = im_cm(l[ri].r, l[ri].i, f[rj].r, f[rj].i) + im_cm(l[rj].r, l[rj].i, f[ri].r, f[ri].i);
  }
  return 0.5 * tree_sum<NA / 2>(t);
}

template <typename R, int NA, int K>
__device__ __forceinline__ double prod_rz_pairs(const cx<R>* f, const cx<R>* l) {
  double t[NA / 2];  // Z f = (-1)^bit f
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    t[j++] = im_cm(l[ri].r, l[ri].i, f[ri].r, f[ri].i) - im_cm(l[rj].r, l[rj].i, f[rj].r, f[rj].i);
  }
  return 0.5 * tree_sum<NA / 2>(t);
}

// Half the sum of x[i] y[i] over the T terms, as two interleaved FMA chains (fewer instructions
// than a product, a difference and a tree sum per pair; two chains keep the dependence short).
template <int T>
__device__ __forceinline__ double half_dot(const double* x, const double* y) {
  static_assert(T % 2 == 0 && T >= 4, "two chains of at least two terms");
  double a = x[0] * y[0], b = x[T / 2] * y[T / 2];
#pragma unroll
  for (int i = 1; i < T / 2; ++i) {
    a = __builtin_fma(x[i], y[i], a);
    b = __builtin_fma(x[T / 2 + i], y[T / 2 + i], b);
  }
  return 0.5 * (a + b);
}

// Rotation products (1/2) Im<lambda|G|phi> over the pairs of register position K, written as
// sums of real products (the sign of each term folded into x); complex128 only (in complex64 the
// FP64 term arrays cost registers).
template <typename R, int NA, int K>
__device__ __forceinline__ double prod_ry_k(const cx<R>* f, const cx<R>* l) {
  if constexpr (sizeof(R) != 8) return prod_ry_pairs<R, NA, K>(f, l);
  // Y f = (-i f1, i f0): per pair Re(conj(l1) f0) - Re(conj(l0) f1)
  double x[2 * NA], y[2 * NA];
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    x[j] = l[rj].r;   y[j++] = f[ri].r;
    x[j] = l[rj].i;   y[j++] = f[ri].i;
    x[j] = -l[ri].r;  y[j++] = f[rj].r;
    x[j] = -l[ri].i;  y[j++] = f[rj].i;
  }
  return half_dot<2 * NA>(x, y);
}

template <typename R, int NA, int K>
__device__ __forceinline__ double prod_rx_k(const cx<R>* f, const cx<R>* l) {
  if constexpr (sizeof(R) != 8) return prod_rx_pairs<R, NA, K>(f, l);
  // X f = (f1, f0): per pair Im(conj(l0) f1) + Im(conj(l1) f0)
  double x[2 * NA], y[2 * NA];
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    x[j] = l[ri].r;   y[j++] = f[rj].i;
    x[j] = -l[ri].i;  y[j++] = f[rj].r;
    x[j] = l[rj].r;   y[j++] = f[ri].i;
    x[j] = -l[rj].i;  y[j++] = f[ri].r;
  }
  return half_dot<2 * NA>(x, y);
}

template <typename R, int NA, int K>
__device__ __forceinline__ double prod_rz_k(const cx<R>* f, const cx<R>* l) {
  if constexpr (sizeof(R) != 8) return prod_rz_pairs<R, NA, K>(f, l);
  // Z f = (-1)^bit f: per pair Im(conj(l0) f0) - Im(conj(l1) f1)
  double x[2 * NA], y[2 * NA];
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    x[j] = l[ri].r;   y[j++] = f[ri].i;
    x[j] = -l[ri].i;  y[j++] = f[ri].r;
    x[j] = -l[rj].r;  y[j++] = f[rj].i;
    x[j] = l[rj].i;   y[j++] = f[rj].r;
  }
  return half_dot<2 * NA>(x, y);
}

template <typename R, int NA>
__device__ __forceinline__ double prod_im_all(const cx<R>* f, const cx<R>* l) {
  double t[NA];
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) t[ri] = im_cm(l[ri].r, l[ri].i, f[ri].r, f[ri].i);
  return tree_sum<NA>(t);
}

// ---------------------------------------------------------------------------------------------
// Lean ops, one fully specialised function per (op, register positions). With BWD the op runs
// as a step of the reverse sweep on (phi = f, lambda = l): the product with phi taken before the
// un-application, then U^dag on both states; otherwise U on f alone.
// ---------------------------------------------------------------------------------------------
template <typename R, int RB, bool BWD, int K>
__device__ __forceinline__ double op_ry(R al, R be, cx<R>* f, cx<R>* l) {
  constexpr int NA = 1 << RB;
  double p = 0.0;
  if constexpr (K < RB) {
    if constexpr (BWD) p = prod_ry_k<R, NA, K>(f, l);
    ry_k<R, NA, K, BWD>(f, al, be);
    if constexpr (BWD) ry_k<R, NA, K, true>(l, al, be);
  }
  return p;
}

template <typename R, int RB, bool BWD, int K>
__device__ __forceinline__ double op_rx(R al, R be, cx<R>* f, cx<R>* l) {
  constexpr int NA = 1 << RB;
  double p = 0.0;
  if constexpr (K < RB) {
    if constexpr (BWD) p = prod_rx_k<R, NA, K>(f, l);
    rx_k<R, NA, K, BWD>(f, al, be);
    if constexpr (BWD) rx_k<R, NA, K, true>(l, al, be);
  }
  return p;
}

template <typename R, int RB, bool BWD, int K>
__device__ __forceinline__ double op_rz(R al, R be, cx<R>* f, cx<R>* l) {
  constexpr int NA = 1 << RB;
  double p = 0.0;
  if constexpr (K < RB) {
    if constexpr (BWD) p = prod_rz_k<R, NA, K>(f, l);
    rz_k<R, NA, K, BWD>(f, al, be);
    if constexpr (BWD) rz_k<R, NA, K, true>(l, al, be);
  }
  return p;
}

// RZ on a thread bit b: Z = (-1)^b on all of the thread's amplitudes
template <typename R, int RB, bool BWD>
__device__ __forceinline__ double op_rz_thr(R al, R be, cx<R>* f, cx<R>* l, bool b) {
  constexpr int NA = 1 << RB;
  double p = 0.0;
  if constexpr (BWD) {
    const double v = 0.5 * prod_im_all<R, NA>(f, l);
    p = b ? -v : v;
  }
  rz_thr<R, NA, BWD>(f, al, be, b);
  if constexpr (BWD) rz_thr<R, NA, true>(l, al, be, b);
  return p;
}

template <typename R, int RB, bool BWD, int KC, int KT>
__device__ __forceinline__ double op_cnot_rr(cx<R>* f, cx<R>* l) {
  if constexpr (KC < RB && KT < RB && KC != KT) {  // self-inverse
    cnot_rr<R, 1 << RB, KC, KT>(f);
    if constexpr (BWD) cnot_rr<R, 1 << RB, KC, KT>(l);
  }
  return 0.0;
}

template <typename R, int RB, bool BWD, int KT>
__device__ __forceinline__ double op_cnot_tr(cx<R>* f, cx<R>* l, bool on) {
  if constexpr (KT < RB) {
    cnot_tr<R, 1 << RB, KT>(f, on);
    if constexpr (BWD) cnot_tr<R, 1 << RB, KT>(l, on);
  }
  return 0.0;
}

template <typename R, int RB, bool BWD, int KA, int KB>
__device__ __forceinline__ double op_cz_rr(cx<R>* f, cx<R>* l) {
  if constexpr (KA < RB && KB < RB && KA != KB) {  // self-inverse
    neg_where<R, 1 << RB, (1 << KA) | (1 << KB)>(f, true);
    if constexpr (BWD) neg_where<R, 1 << RB, (1 << KA) | (1 << KB)>(l, true);
  }
  return 0.0;
}

// CZ with one register bit K and one thread bit (on = its value)
template <typename R, int RB, bool BWD, int K>
__device__ __forceinline__ double op_cz_r(cx<R>* f, cx<R>* l, bool on) {
  if constexpr (K < RB) {
    neg_where<R, 1 << RB, 1 << K>(f, on);
    if constexpr (BWD) neg_where<R, 1 << RB, 1 << K>(l, on);
  }
  return 0.0;
}

template <typename R, int RB, bool BWD>
__device__ __forceinline__ double op_cz_tt(cx<R>* f, cx<R>* l, bool on) {
  neg_where<R, 1 << RB, 0>(f, on);
  if constexpr (BWD) neg_where<R, 1 << RB, 0>(l, on);
  return 0.0;
}

template <typename R, int RB, bool BWD, int K>
__device__ __forceinline__ double op_dense1(const GateRec* rec, cx<R>* f, cx<R>* l) {
  if constexpr (K < RB) {
    cx<R> m00 = mat<R>(rec, 0), m01 = mat<R>(rec, 1), m10 = mat<R>(rec, 2), m11 = mat<R>(rec, 3);
    if constexpr (BWD) {
      const cx<R> t = m01;
      m00 = conj(m00); m11 = conj(m11); m01 = conj(m10); m10 = conj(t);
    }
    dense1_k<R, 1 << RB, K>(f, m00, m01, m10, m11);
    if constexpr (BWD) dense1_k<R, 1 << RB, K>(l, m00, m01, m10, m11);
  }
  return 0.0;
}

template <typename R, int RB, bool BWD, int K>
__device__ __forceinline__ double op_diag1(const GateRec* rec, cx<R>* f, cx<R>* l) {
  if constexpr (K < RB) {
    cx<R> d0 = mat<R>(rec, 0), d1 = mat<R>(rec, 3);
    if constexpr (BWD) { d0 = conj(d0); d1 = conj(d1); }
    diag1_k<R, 1 << RB, K>(f, d0, d1);
    if constexpr (BWD) diag1_k<R, 1 << RB, K>(l, d0, d1);
  }
  return 0.0;
}

template <typename R, int RB, bool BWD>
__device__ __forceinline__ double op_diag1_thr(const GateRec* rec, cx<R>* f, cx<R>* l, bool b) {
  constexpr int NA = 1 << RB;
  cx<R> d = sel(b, mat<R>(rec, 3), mat<R>(rec, 0));
  if constexpr (BWD) d = conj(d);
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) f[ri] = d * f[ri];
  if constexpr (BWD) {
#pragma unroll
    for (int ri = 0; ri < NA; ++ri) l[ri] = d * l[ri];
  }
  return 0.0;
}

// Re <lambda|G|phi> of a lean rotation on register position K (G = Y, X or Z), all indices
// compile-time.
template <typename R, int NA, int K>
__device__ __forceinline__ double re_w_k(int type, const cx<R>* f, const cx<R>* l) {
  double t[NA / 2];
  int j = 0;
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & (1 << K)) continue;
    const int rj = ri | (1 << K);
    if (type == FOP_RY)  // Y f = (-i f1, i f0): Re w = -Im(conj(l1) f0 - conj(l0) f1)
      t[j++] = im_cm(l[ri].r, l[ri].i, f[rj].r, f[rj].i) - im_cm(l[rj].r, l[rj].i, f[ri].r, f[ri].i);
    else if (type == FOP_RX)  // X f = (f1, f0)
      t[j++] = re_cm(l[ri].r, l[ri].i, f[rj].r, f[rj].i) + re_cm(l[rj].r, l[rj].i, f[ri].r, f[ri].i);
    else  // Z f = (-1)^bit f
      t[j++] = re_cm(l[ri].r, l[ri].i, f[ri].r, f[ri].i) - re_cm(l[rj].r, l[rj].i, f[rj].r, f[rj].i);
  }
  return tree_sum<NA / 2>(t);
}

// A rotation macro: RB rotations about one axis, one per register position, in straight-line
// code. Position 0 is the head (shear factors al0, be0); the factors of positions 1 .. RB - 1
// are staged from record `mem` of the pass on (with their FOPF_FLIP, toggled into flip). The
// product of position K goes to prod[K] (reverse sweep).
template <typename R, int RB, bool BWD, int AXIS, int K = 0>
__device__ __forceinline__ void rot_macro_k(R al0, R be0, const OpStage* mem, cx<R>* f, cx<R>* l,
                                            double* prod, int& flip) {
  if constexpr (K < RB) {
    R al = al0, be = be0;
    if constexpr (K > 0) {
      const double2 ab = *reinterpret_cast<const double2*>(&mem[K - 1].alpha);
      al = (R)ab.x;
      be = (R)ab.y;
      const uint32_t w1 = __builtin_amdgcn_readfirstlane(
          reinterpret_cast<const uint32_t*>(&mem[K - 1].op)[1]);
      flip ^= ((w1 >> 24) & FOPF_FLIP) ? 1 : 0;
    }
    if constexpr (AXIS == FOP_RY) prod[K] = op_ry<R, RB, BWD, K>(al, be, f, l);
    else if constexpr (AXIS == FOP_RX) prod[K] = op_rx<R, RB, BWD, K>(al, be, f, l);
    else prod[K] = op_rz<R, RB, BWD, K>(al, be, f, l);
    rot_macro_k<R, RB, BWD, AXIS, K + 1>(al0, be0, mem, f, l, prod, flip);
  }
}

// Sums S[k] = sum over ri of (-1)^(bit k of ri) w[ri] for every register position k, by halving
// butterflies: at level k the partial sums over the lower bits pair up by bit k.
template <int NA, int K = 0>
__device__ __forceinline__ void walsh_singles(const double* w, double* S) {
  if constexpr (NA >= 2) {
    double a[NA / 2], d[NA / 2];
#pragma unroll
    for (int j = 0; j < NA / 2; ++j) {
      a[j] = w[2 * j] + w[2 * j + 1];
      d[j] = w[2 * j] - w[2 * j + 1];
    }
    S[K] = tree_sum<NA / 2>(d);
    walsh_singles<NA / 2, K + 1>(a, S);
  }
}

// A diagonal block (FOPF_DIAG head): amplitude ri times entry d[ri] of the block's staged table
// (the product of its RZ and CZ gates); the reverse sweep multiplies phi and lambda by the
// conjugate. The product of RZ member j, on register position p_j (four bits each in op.gate),
// is (1/2) sum over ri of (-1)^(bit p_j of ri) Im(conj(lambda) phi) (see prod_rz_k).
template <typename R, int RB, bool BWD>
__device__ __forceinline__ void diag_block(const FusedOp& op, const typename Vec2<R>::T* d,
                                           cx<R>* f, cx<R>* l, double* prod) {
  constexpr int NA = 1 << RB;
  if constexpr (BWD) {
    double w[NA], S[RB];
#pragma unroll
    for (int ri = 0; ri < NA; ++ri) w[ri] = im_cm(l[ri].r, l[ri].i, f[ri].r, f[ri].i);
    walsh_singles<NA>(w, S);
#pragma unroll
    for (int j = 0; j < kMaxMacroRegBits; ++j) {
      if (j >= op.np) break;
      const int pj = (op.gate >> (4 * j)) & 15;
      double v = S[0];
#pragma unroll
      for (int k = 1; k < RB; ++k) v = pj == k ? S[k] : v;
      prod[j] = 0.5 * v;
    }
  }
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    const typename Vec2<R>::T e = d[ri];
    const R er = e.x, ei = BWD ? -e.y : e.y;
    const cx<R> a = f[ri];
    f[ri] = cx<R>{a.r * er - a.i * ei, a.r * ei + a.i * er};
    if constexpr (BWD) {
      const cx<R> b = l[ri];
      l[ri] = cx<R>{b.r * er - b.i * ei, b.r * ei + b.i * er};
    }
  }
}

// One lean op, dispatched on its op code by a single switch whose cases are all fully
// specialised: no nested per-position branches whose joins would copy the amplitude registers.
// The op's products (reverse sweep) go to prod[0], or prod[0 .. RB) for a rotation macro, whose
// records (with their cos/sin) start at st.
#define QSV_K5(T, V0, FN, ...)                                                      \
  case QSV_OPC(T, (V0) + 0): p = FN<R, RB, BWD, 0>(__VA_ARGS__); break;           \
  case QSV_OPC(T, (V0) + 1): p = FN<R, RB, BWD, 1>(__VA_ARGS__); break;           \
  case QSV_OPC(T, (V0) + 2): p = FN<R, RB, BWD, 2>(__VA_ARGS__); break;           \
  case QSV_OPC(T, (V0) + 3): p = FN<R, RB, BWD, 3>(__VA_ARGS__); break;           \
  case QSV_OPC(T, (V0) + 4): p = FN<R, RB, BWD, 4>(__VA_ARGS__); break;
#define QSV_KK1(T, A, FN, ...)                                                      \
  case QSV_OPC(T, 8 * (A) + 0): p = FN<R, RB, BWD, A, 0>(__VA_ARGS__); break;     \
  case QSV_OPC(T, 8 * (A) + 1): p = FN<R, RB, BWD, A, 1>(__VA_ARGS__); break;     \
  case QSV_OPC(T, 8 * (A) + 2): p = FN<R, RB, BWD, A, 2>(__VA_ARGS__); break;     \
  case QSV_OPC(T, 8 * (A) + 3): p = FN<R, RB, BWD, A, 3>(__VA_ARGS__); break;     \
  case QSV_OPC(T, 8 * (A) + 4): p = FN<R, RB, BWD, A, 4>(__VA_ARGS__); break;
#define QSV_KK5(T, FN, ...)                                                         \
  QSV_KK1(T, 0, FN, __VA_ARGS__) QSV_KK1(T, 1, FN, __VA_ARGS__)                     \
  QSV_KK1(T, 2, FN, __VA_ARGS__) QSV_KK1(T, 3, FN, __VA_ARGS__)                     \
  QSV_KK1(T, 4, FN, __VA_ARGS__)

// (c, s) are a rotation's staged shear factors; flip collects the sign of the rotations run as
// -1 times a rotation (FOPF_FLIP).
template <typename R, int RB, bool BWD>
__device__ __forceinline__ void lean_step(const FusedOp& op, R c, R s, const GateRec* rec,
                                          const OpStage* sops, const typename Vec2<R>::T* sdiag,
                                          cx<R>* f, cx<R>* l, uint32_t tdep, double* prod,
                                          int& flip) {
  static_assert(RB <= 5, "op codes hold register positions below 5");
  double& p = prod[0];
  if (op.type <= FOP_RZ && (op.flags & FOPF_FLIP)) flip ^= 1;
  switch (op.opc) {
    QSV_K5(FOP_RY, 0, op_ry, c, s, f, l)
    QSV_K5(FOP_RX, 0, op_rx, c, s, f, l)
    QSV_K5(FOP_RZ, 0, op_rz, c, s, f, l)
    case QSV_OPC(FOP_RZ, QSV_V_THREAD):
      p = op_rz_thr<R, RB, BWD>(c, s, f, l, thread_bit(tdep, op.s0));
      break;
    QSV_KK5(FOP_CNOT, op_cnot_rr, f, l)
    QSV_K5(FOP_CNOT, QSV_V_CTL_THREAD, op_cnot_tr, f, l, thread_bit(tdep, op.s0))
    QSV_KK5(FOP_CZ, op_cz_rr, f, l)
    QSV_K5(FOP_CZ, QSV_V_REG0, op_cz_r, f, l, thread_bit(tdep, op.s1))
    QSV_K5(FOP_CZ, QSV_V_REG1, op_cz_r, f, l, thread_bit(tdep, op.s0))
    case QSV_OPC(FOP_CZ, QSV_V_THREAD):
      p = op_cz_tt<R, RB, BWD>(f, l, thread_bit(tdep, op.s0) && thread_bit(tdep, op.s1));
      break;
    QSV_K5(FOP_DENSE1, 0, op_dense1, rec, f, l)
    QSV_K5(FOP_DIAG1, 0, op_diag1, rec, f, l)
    case QSV_OPC(FOP_DIAG1, QSV_V_THREAD):
      p = op_diag1_thr<R, RB, BWD>(rec, f, l, thread_bit(tdep, op.s0));
      break;
    case QSV_OPC(FOP_RY, QSV_V_MACRO):
      if constexpr (RB <= kMaxMacroRegBits)
        rot_macro_k<R, RB, BWD, FOP_RY>(c, s, sops + op.k1, f, l, prod, flip);
      break;
    case QSV_OPC(FOP_RX, QSV_V_MACRO):
      if constexpr (RB <= kMaxMacroRegBits)
        rot_macro_k<R, RB, BWD, FOP_RX>(c, s, sops + op.k1, f, l, prod, flip);
      break;
    case QSV_OPC(FOP_RZ, QSV_V_MACRO):
      if constexpr (RB <= kMaxMacroRegBits)
        rot_macro_k<R, RB, BWD, FOP_RZ>(c, s, sops + op.k1, f, l, prod, flip);
      break;
    case QSV_OPC(FOP_RZ, QSV_V_DIAG):
      if constexpr (RB <= kMaxMacroRegBits)
        diag_block<R, RB, BWD>(op, sdiag + op.ks1 * (1 << RB), f, l, prod);
      break;
    default:
      break;
  }
}
#undef QSV_K5
#undef QSV_KK1
#undef QSV_KK5

// ---------------------------------------------------------------------------------------------
// General ops (tile bits evaluated per amplitude)
// ---------------------------------------------------------------------------------------------
template <int RB>
__device__ __forceinline__ bool bit_of(int s, const Layout<RB>& L, int ri) {
  return ((L.tdep | reg_deposit<RB>(L, ri)) >> s) & 1u;
}

template <typename R, int NA, int K0, int K1>
__device__ __forceinline__ void dense2_k(cx<R>* a, const GateRec* rec, int off, bool adj) {
  cx<R> m[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      m[4 * i + j] = sel(adj, conj(mat<R>(rec, off + 4 * j + i)), mat<R>(rec, off + 4 * i + j));
#pragma unroll
  for (int ri = 0; ri < NA; ++ri) {
    if (ri & ((1 << K0) | (1 << K1))) continue;
    const int idx[4] = {ri, ri | (1 << K1), ri | (1 << K0), ri | (1 << K0) | (1 << K1)};
    cx<R> v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = a[idx[k]];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      cx<R> s = {0, 0};
#pragma unroll
      for (int k = 0; k < 4; ++k) s = s + m[4 * rr + k] * v[k];
      a[idx[rr]] = s;
    }
  }
}

template <typename R, int RB, int K0 = 0, int K1 = 0>
__device__ __forceinline__ void dense2_at(int k0, int k1, cx<R>* a, const GateRec* rec, int off,
                                          bool adj) {
  if constexpr (K0 < RB) {
    if constexpr (K1 < RB) {
      if constexpr (K0 != K1) {
        if (k0 == K0 && k1 == K1) {
          dense2_k<R, 1 << RB, K0, K1>(a, rec, off, adj);
          return;
        }
      }
      dense2_at<R, RB, K0, K1 + 1>(k0, k1, a, rec, off, adj);
    } else {
      dense2_at<R, RB, K0 + 1, 0>(k0, k1, a, rec, off, adj);
    }
  }
}

template <typename R, int RB>
__device__ __forceinline__ cx<R> pick_diag4(const cx<R>* d, bool b0, bool b1) {
  const cx<R> lo = sel(b1, d[1], d[0]);
  const cx<R> hi = sel(b1, d[3], d[2]);
  return sel(b0, hi, lo);
}

// ADJ: the reverse sweep's un-do, U^dag; for a non-unitary op (FOP_NDENSE1) on phi (phi_side) the
// stored inverse instead (App. B.3).
template <typename R, int RB, bool ADJ>
__device__ __forceinline__ void apply_general(const FusedOp& op, const GateRec* rec, cx<R>* a,
                                              const Layout<RB>& L, bool phi_side = false) {
  constexpr int NA = 1 << RB;
  switch (op.type) {
    case FOP_NDENSE1: {
      cx<R> m00 = mat<R>(rec, 0), m01 = mat<R>(rec, 1), m10 = mat<R>(rec, 2), m11 = mat<R>(rec, 3);
      if (ADJ && phi_side) {
        m00 = mat<R>(rec, 8); m01 = mat<R>(rec, 9); m10 = mat<R>(rec, 10); m11 = mat<R>(rec, 11);
      } else if (ADJ) {
        const cx<R> t = m01;
        m00 = conj(m00); m11 = conj(m11); m01 = conj(m10); m10 = conj(t);
      }
      dense1_at<R, RB, ADJ>(op.k0, a, m00, m01, m10, m11);
      break;
    }
    case FOP_PDENSE1: case FOP_CDENSE1: {
      const bool ctl = op.type == FOP_CDENSE1;
      const int o = ctl ? 10 : 0, st = ctl ? 4 : 2;  // 2x2 block and its row stride
      cx<R> m00 = mat<R>(rec, o), m01 = mat<R>(rec, o + 1), m10 = mat<R>(rec, o + st),
            m11 = mat<R>(rec, o + st + 1);
      if (ADJ) {
        const cx<R> t = m01;
        m00 = conj(m00); m11 = conj(m11); m01 = conj(m10); m10 = conj(t);
      }
      cx<R> b[NA];
#pragma unroll
      for (int ri = 0; ri < NA; ++ri) b[ri] = a[ri];
      dense1_at<R, RB, ADJ>(op.k0, b, m00, m01, m10, m11);
#pragma unroll
      for (int ri = 0; ri < NA; ++ri) a[ri] = sel(!ctl || bit_of<RB>(op.s0, L, ri), b[ri], a[ri]);
      break;
    }
    case FOP_PDIAG1: {
      cx<R> d0 = mat<R>(rec, 0), d1 = mat<R>(rec, 3);
      if (ADJ) { d0 = conj(d0); d1 = conj(d1); }
#pragma unroll
      for (int ri = 0; ri < NA; ++ri) a[ri] = sel(bit_of<RB>(op.s0, L, ri), d1, d0) * a[ri];
      break;
    }
    case FOP_DIAG2: {
      cx<R> d[4] = {mat<R>(rec, 0), mat<R>(rec, 5), mat<R>(rec, 10), mat<R>(rec, 15)};
      if (ADJ) {
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = conj(d[k]);
      }
#pragma unroll
      for (int ri = 0; ri < NA; ++ri)
        a[ri] = pick_diag4<R, RB>(d, bit_of<RB>(op.s0, L, ri), bit_of<RB>(op.s1, L, ri)) * a[ri];
      break;
    }
    case FOP_DENSE2:
      dense2_at<R, RB>(op.k0, op.k1, a, rec, 0, ADJ);
      break;
    default:
      break;
  }
}

// mu <- D_j mu, D_j the derivative of the op's matrix in its j-th parameter, from the op's record:
// rotations and one-qubit parameterised gates m[4 + 4j ..], controlled rotations the |1><1| (x) dR
// block (amplitudes with control 0 zeroed), two-qubit gates m[16 ..].
template <typename R, int RB>
__device__ __forceinline__ void apply_derivative(const FusedOp& op, const GateRec* rec, int j,
                                                 cx<R>* mu, const Layout<RB>& L) {
  constexpr int NA = 1 << RB;
  switch (op.type) {
    case FOP_RY: case FOP_RX: case FOP_PDENSE1: case FOP_NDENSE1: {
      const int o = 4 + 4 * j;
      dense1_at<R, RB, false>(op.k0, mu, mat<R>(rec, o), mat<R>(rec, o + 1), mat<R>(rec, o + 2),
                              mat<R>(rec, o + 3));
      break;
    }
    case FOP_RZ: case FOP_PDIAG1: {
      const cx<R> e0 = mat<R>(rec, 4), e1 = mat<R>(rec, 7);
#pragma unroll
      for (int ri = 0; ri < NA; ++ri) mu[ri] = sel(bit_of<RB>(op.s0, L, ri), e1, e0) * mu[ri];
      break;
    }
    case FOP_CDENSE1:
      dense1_at<R, RB, false>(op.k0, mu, mat<R>(rec, 26), mat<R>(rec, 27), mat<R>(rec, 30),
                              mat<R>(rec, 31));
#pragma unroll
      for (int ri = 0; ri < NA; ++ri) mu[ri] = sel(bit_of<RB>(op.s0, L, ri), mu[ri], cx<R>{0, 0});
      break;
    case FOP_DIAG2: {
      const cx<R> e[4] = {mat<R>(rec, 16), mat<R>(rec, 21), mat<R>(rec, 26), mat<R>(rec, 31)};
#pragma unroll
      for (int ri = 0; ri < NA; ++ri)
        mu[ri] = pick_diag4<R, RB>(e, bit_of<RB>(op.s0, L, ri), bit_of<RB>(op.s1, L, ri)) * mu[ri];
      break;
    }
    case FOP_DENSE2:
      dense2_at<R, RB>(op.k0, op.k1, mu, rec, 16, false);
      break;
    default:
      break;
  }
}

// <l|D_j f> for the explicit derivative matrices of a general op (f already un-applied): the
// real parts in out, the imaginary parts in out_im when want_im is set (complex entries), else
// zeros. Both arrays are the caller's register arrays (a pointer select between one of them and
// a null pointer would put it on the stack).
template <typename R, int RB>
__device__ __forceinline__ void general_products(const FusedOp& op, const GateRec* rec,
                                                 const cx<R>* f, const cx<R>* l,
                                                 const Layout<RB>& L, double* out,
                                                 double* out_im, bool want_im) {
  constexpr int NA = 1 << RB;
  cx<R> mu[NA];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j >= op.np) break;
#pragma unroll
    for (int ri = 0; ri < NA; ++ri) mu[ri] = f[ri];
    apply_derivative<R, RB>(op, rec, j, mu, L);
    double s = 0, si = 0;
#pragma unroll
    for (int ri = 0; ri < NA; ++ri) {
      s += re_cm(l[ri].r, l[ri].i, mu[ri].r, mu[ri].i);
      if (want_im) si += im_cm(l[ri].r, l[ri].i, mu[ri].r, mu[ri].i);
    }
    out[j] = s;
    out_im[j] = si;
  }
}

template <typename R, int RB, int K = 0>
__device__ __forceinline__ double re_w_at(int type, int k, const cx<R>* f, const cx<R>* l) {
  if constexpr (K < RB) {
    if (k == K) return re_w_k<R, 1 << RB, K>(type, f, l);
    return re_w_at<R, RB, K + 1>(type, k, f, l);
  } else {
    return 0.0;
  }
}

// Im <lambda|dR phi'> of a lean rotation (complex entries, App. B.4), from the states before
// the un-application: with w = <lambda|G|phi>, <lambda|dR phi'> = -(i/2) w, so its imaginary
// part is -Re(w)/2 (its real part, Im(w)/2, is the lean product).
template <typename R, int RB>
__device__ __forceinline__ double lean_product_im(const FusedOp& op, const cx<R>* f,
                                                  const cx<R>* l, uint32_t tdep) {
  constexpr int NA = 1 << RB;
  double re_w = 0;
  if (op.type == FOP_RY || op.type == FOP_RX) {
    re_w = re_w_at<R, RB>(op.type, op.k0, f, l);
  } else if (op.type == FOP_RZ) {
    if (op.flags & FOPF_S0_REG) {
      re_w = re_w_at<R, RB>(FOP_RZ, op.ks0, f, l);
    } else {
      double t[NA];
#pragma unroll
      for (int ri = 0; ri < NA; ++ri) t[ri] = re_cm(l[ri].r, l[ri].i, f[ri].r, f[ri].i);
      re_w = tree_sum<NA>(t);
      if (thread_bit(tdep, op.s0)) re_w = -re_w;
    }
  }
  return -0.5 * re_w;
}

// ---------------------------------------------------------------------------------------------
// Wave sum with DPP row operations (inclusive scan; the total ends in lane 63).
// ---------------------------------------------------------------------------------------------
template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWM, BANKM, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWM, BANKM, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_total_lane63(double v) {
  double t = v + dpp_f64<0x111, 0xf, 0xf>(v);  // row_shr:1
  t += dpp_f64<0x112, 0xf, 0xf>(v);             // row_shr:2
  t += dpp_f64<0x113, 0xf, 0xf>(v);             // row_shr:3
  t += dpp_f64<0x114, 0xf, 0xe>(t);             // row_shr:4, banks 1-3
  t += dpp_f64<0x118, 0xf, 0xc>(t);             // row_shr:8, banks 2-3
  t += dpp_f64<0x142, 0xa, 0xf>(t);             // row_bcast:15, rows 1 and 3
  t += dpp_f64<0x143, 0xc, 0xf>(t);             // row_bcast:31, rows 2 and 3
  return t;
}

// ---------------------------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------------------------
template <int RB, int W>
struct Geometry {
  static constexpr int NA = 1 << RB;
  static constexpr int NT = 1 << W;
  static constexpr int T = RB + W;
  static constexpr int NW = NT / 64;
};

// Global amplitude offsets of a layout's elements in a pass: a thread part and one offset per
// register position; element ri sits at gthr | greg[k] for every set bit k of ri.
template <int RB>
struct TileMap {
  uint64_t gthr;
  uint64_t greg[RB];
};

template <int RB>
__device__ __forceinline__ uint64_t map_off(const TileMap<RB>& M, int ri) {
  uint64_t o = 0;
#pragma unroll
  for (int k = 0; k < RB; ++k)
    if ((ri >> k) & 1) o |= M.greg[k];
  return o;
}

// The direct layout's map: thread bits = tile bits 0..W-1, register bits = tile bits W..T-1.
// Phantom tile bits (tile[s] < 0, states smaller than the tile) contribute no address bit;
// amplitudes with a phantom bit set are not live (never loaded or stored, zero in registers).
// live: the thread's phantom bits are all zero; preg: register positions on phantom bits.
template <int RB, int W>
__device__ __forceinline__ void direct_map(const PassDesc& pd, uint32_t tid, TileMap<RB>& M,
                                           bool& live, uint32_t& preg) {
  M.gthr = 0;
  live = true;
#pragma unroll
  for (int s = 0; s < W; ++s) {
    const uint32_t b = (tid >> s) & 1u;
    if (pd.tile[s] >= 0) M.gthr |= (uint64_t)b << pd.tile[s];
    else live = live && !b;
  }
  preg = 0;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    M.greg[k] = pd.tile[W + k] >= 0 ? 1ull << pd.tile[W + k] : 0ull;
    if (pd.tile[W + k] < 0) preg |= 1u << k;
  }
}

// The map of any layout of a pass without phantom bits (tile bit indices resolved at compile
// time: the register bits select among the T tile qubits).
template <int RB, int T>
__device__ __forceinline__ void layout_map(const PassDesc& pd, const Layout<RB>& L, TileMap<RB>& M) {
  M.gthr = 0;
#pragma unroll
  for (int s = 0; s < T; ++s) M.gthr |= (uint64_t)((L.tdep >> s) & 1u) << pd.tile[s];
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    uint64_t g = 0;
#pragma unroll
    for (int s = 0; s < T; ++s)
      if (L.rb[k] == s) g = 1ull << pd.tile[s];
    M.greg[k] = g;
  }
}

// Register bits of phase ph of a pass, read from the global phase table (uniform).
template <int RB>
__device__ __forceinline__ void global_phase_regbits(const PhaseDesc* phases, int ph, int8_t* rb) {
  const QSV_GLOBAL uint32_t* p = (const QSV_GLOBAL uint32_t*)(phases + ph);
  const uint32_t w1 = __builtin_amdgcn_readfirstlane(p[1]);
  const uint32_t w2 = __builtin_amdgcn_readfirstlane(p[2]);
#pragma unroll
  for (int k = 0; k < RB; ++k) rb[k] = (int8_t)(((k < 4 ? w1 >> (8 * k) : w2 >> (8 * (k - 4)))) & 0xffu);
}

// The layouts (and maps) a pass loads its tiles in and stores them from: the first and last
// phase's layouts where the scheduler marked them as keeping the contiguous runs on the low lane
// bits (PASS_LOAD_FIRST_PHASE, PASS_STORE_LAST_PHASE), otherwise the direct layout.
template <typename R, int RB, int T>
__device__ __forceinline__ void io_layouts(const PassItem& I, uint32_t tid, const Layout<RB>& D,
                                           const TileMap<RB>& MD, Layout<RB>& LL, TileMap<RB>& ML,
                                           Layout<RB>& LS, TileMap<RB>& MS) {
  LL = D;
  ML = MD;
  LS = D;
  MS = MD;
  const uint32_t fl = I.pd.io_flags;
  int8_t rb[RB];
  if (fl & PASS_LOAD_FIRST_PHASE) {
    global_phase_regbits<RB>(I.phases, I.pd.phase_begin, rb);
    make_layout<R, RB>(LL, rb, tid);
    layout_map<RB, T>(I.pd, LL, ML);
  }
  if (fl & PASS_STORE_LAST_PHASE) {
    global_phase_regbits<RB>(I.phases, I.pd.phase_end - 1, rb);
    make_layout<R, RB>(LS, rb, tid);
    layout_map<RB, T>(I.pd, LS, MS);
  }
}

template <typename R, int RB, int W>
__device__ __forceinline__ void direct_layout(Layout<RB>& L, uint32_t tid) {
  int8_t rb[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) rb[k] = (int8_t)(W + k);
  make_layout<R, RB>(L, rb, tid);
}

// Item of the chunk-local tile g: the last item whose first tile is <= g (binary search).
__device__ __forceinline__ int find_item(const PassItem* __restrict__ items, int n_items, int64_t g) {
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_begin <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The low bits of x deposited into the set bits of mask, lowest first (the amplitude offset of
// tile x of a pass whose outer qubits are mask).
__device__ __forceinline__ uint64_t deposit_bits(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t m = mask; m && x; m &= m - 1, x >>= 1)
    if (x & 1) r |= m & (~m + 1);
  return r;
}

// The next subset of mask after b in increasing order (the offset of the next tile).
__device__ __forceinline__ uint64_t next_in_mask(uint64_t b, uint64_t mask) {
  return (b - mask) & mask;
}

// An RZ member of a diagonal block, run on its own (complex-entry sweeps): its staged (c, s)
// become the shear factors and FOPF_FLIP as the staging gives them to other rotations.
__device__ __forceinline__ void diag_member_shears(FusedOp& op, double2& cs) {
  if (op.type != FOP_RZ || !(op.flags & FOPF_DIAG)) return;
  const double c = cs.x, s = cs.y;
  if (c >= 0.0) {
    cs = make_double2(-s / (1.0 + c), s);
    op.flags &= (uint8_t)~FOPF_FLIP;
  } else {
    cs = make_double2(s / (1.0 - c), -s);
    op.flags |= FOPF_FLIP;
  }
}

// Raw words of staged op k (issued early; made uniform when the op is executed).
__device__ __forceinline__ uint4 staged_words(const OpStage* sops, int k) {
  return *reinterpret_cast<const uint4*>(&sops[k].op);
}
__device__ __forceinline__ double2 staged_cs(const OpStage* sops, int k) {
  return *reinterpret_cast<const double2*>(&sops[k].alpha);
}

// Copies the pass's op records (with the cos/sin of the rotation angles) and phase descriptors to
// LDS; every thread loads a share, so the whole op stream arrives in one round of loads.
template <int RB, typename V>
__device__ __forceinline__ void stage_pass(const PassItem& I, OpStage* sops, PhaseDesc* sph,
                                           V* sdiag, int tid, int nt) {
  const int n_ops = I.pd.n_ops, n_ph = I.pd.phase_end - I.pd.phase_begin;
  for (int i = tid; i < n_ops; i += nt) {
    // the 16-byte op record moves as one word quadruple (type in the low byte of the first)
    // (global-address-space reads: see load())
    using U4 = uint32_t __attribute__((ext_vector_type(4)));
    const U4 w = ((const QSV_GLOBAL U4*)(I.ops + I.pd.op_begin))[i];
    const uint4 raw = make_uint4(w.x, w.y, w.z, w.w);
    const int type = (int)(raw.x & 0xffu);
    double al = 0.0, be = 0.0;
    uint4 staged = raw;
    if (type <= FOP_RZ && (raw.z >> 16) != QSV_OPC(FOP_RZ, QSV_V_DIAG)) {
      // RY m[2] = s, RX m[1] = -i s, RZ m[0] = c - i s
      const QSV_GLOBAL double* m = rec_words(I.recs + (int32_t)raw.w);
      const double c = m[0];
      const double s = type == FOP_RY ? m[4] : type == FOP_RX ? -m[3] : -m[1];
      // shear factors of the rotation by phi (cos phi = c >= 0), or of -1 times the rotation by
      // phi - pi (cos = -c, sin = -s): alpha = -tan(phi/2) = -s / (1 + c), beta = sin(phi).
      // An RZ member of a diagonal block keeps (c, s) (see diag_member_shears).
      if ((raw.y >> 24) & FOPF_DIAG) {
        al = c;
        be = s;
      } else if (c >= 0.0) {
        al = -s / (1.0 + c);
        be = s;
      } else {
        al = s / (1.0 - c);
        be = -s;
        staged.y |= (uint32_t)FOPF_FLIP << 24;
      }
    }
    *reinterpret_cast<uint4*>(&sops[i].op) = staged;
    *reinterpret_cast<double2*>(&sops[i].alpha) = make_double2(al, be);
  }
  static_assert(sizeof(PhaseDesc) == 12, "PhaseDesc moves as three words");
  const QSV_GLOBAL uint32_t* ph = (const QSV_GLOBAL uint32_t*)(I.phases + I.pd.phase_begin);
  for (int i = tid; i < 3 * n_ph; i += nt) reinterpret_cast<uint32_t*>(sph)[i] = ph[i];
  // diagonal blocks: entry ri of a head's table is the product over its members of
  // exp(-i t Z/2)[bit] = c -+ i s (RZ on position ks0) and (-1)^(b0 b1) (CZ on ks0, ks1), from
  // the members' staged (c, s) (a second round over LDS)
  if constexpr (RB <= kMaxMacroRegBits) {
    if (I.pd.n_diag > 0) {
      lds_barrier();
      constexpr int NA = 1 << RB;
      for (int x = tid; x < n_ops * NA; x += nt) {
        const int i = x / NA, ri = x % NA;
        const uint4 h = staged_words(sops, i);
        if ((h.z >> 16) != QSV_OPC(FOP_RZ, QSV_V_DIAG)) continue;
        const int first = (int)((h.x >> 16) & 0xffu), n_mem = (int)(h.x >> 24);
        double dr = 1.0, di = 0.0;
        int sign = 0;
        for (int m = 0; m < n_mem; ++m) {
          const uint4 w = staged_words(sops, first + m);
          const int ks0 = (int)(w.z & 0xffu), ks1 = (int)((w.z >> 8) & 0xffu);
          if ((w.x & 0xffu) == FOP_RZ) {
            const double2 cs = staged_cs(sops, first + m);
            const double c = cs.x, sn = ((ri >> ks0) & 1) ? cs.y : -cs.y;
            const double t = dr * c - di * sn;
            di = dr * sn + di * c;
            dr = t;
          } else {
            sign ^= (ri >> ks0) & (ri >> ks1) & 1;
          }
        }
        V e;
        e.x = sign ? -dr : dr;
        e.y = sign ? -di : di;
        sdiag[((h.z >> 8) & 0xffu) * NA + ri] = e;
      }
    }
  }
}

static_assert(sizeof(FusedOp) == 16 && offsetof(FusedOp, s0) == 3 && offsetof(FusedOp, flags) == 7 &&
                  offsetof(FusedOp, ks1) == 9 && offsetof(FusedOp, opc) == 10 &&
                  offsetof(FusedOp, gate) == 12,
              "FusedOp is read from LDS as four words");

__device__ __forceinline__ FusedOp uniform_op(uint4 raw) {
  const uint32_t w0 = __builtin_amdgcn_readfirstlane(raw.x);
  const uint32_t w1 = __builtin_amdgcn_readfirstlane(raw.y);
  const uint32_t w2 = __builtin_amdgcn_readfirstlane(raw.z);
  FusedOp op;
  op.type = (uint8_t)w0;
  op.k0 = (uint8_t)(w0 >> 8);
  op.k1 = (uint8_t)(w0 >> 16);
  op.s0 = (uint8_t)(w0 >> 24);
  op.s1 = (uint8_t)w1;
  op.np = (uint8_t)(w1 >> 8);
  op.lslot = (uint8_t)(w1 >> 16);
  op.flags = (uint8_t)(w1 >> 24);
  op.ks0 = (uint8_t)w2;
  op.ks1 = (uint8_t)(w2 >> 8);
  op.opc = (uint16_t)(w2 >> 16);
  op.gate = (int32_t)__builtin_amdgcn_readfirstlane(raw.w);
  return op;
}

// Phase ph of the staged pass: its op end and register bits, as uniform values.
template <int RB>
__device__ __forceinline__ int uniform_phase(const PhaseDesc* sph, int ph, int8_t* rb,
                                             uint32_t* rperm) {
  static_assert(sizeof(PhaseDesc) == 12, "PhaseDesc is read from LDS as three words");
  const uint32_t* p = reinterpret_cast<const uint32_t*>(sph + ph);
  const uint32_t w0 = __builtin_amdgcn_readfirstlane(p[0]);
  const uint32_t w1 = __builtin_amdgcn_readfirstlane(p[1]);
  const uint32_t w2 = __builtin_amdgcn_readfirstlane(p[2]);
#pragma unroll
  for (int k = 0; k < RB; ++k) rb[k] = (int8_t)(((k < 4 ? w1 >> (8 * k) : w2 >> (8 * (k - 4)))) & 0xffu);
  static_assert(offsetof(PhaseDesc, rperm) == 10, "rperm is the high half of the third word");
  *rperm = w2 >> 16;
  return (int)w0;
}

// Wave totals of four values at once: a lane-half exchange (permlane32_swap) pairs p0 with p1
// and p2 with p3, a row exchange (permlane16_swap) leaves each row with one value's 16 partial
// sums, and a butterfly inside the rows (quad_perm, half-row and row mirrors) puts each row's
// total in all its lanes: row 0 holds p0's total, row 1 p2's, row 2 p1's, row 3 p3's. A fixed
// order of additions, as in wave_total_lane63.
__device__ __forceinline__ void swap_halves(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double(hi[0], lo[0]);
  b = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ void swap_rows(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double(hi[0], lo[0]);
  b = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double wave_totals4(double p0, double p1, double p2, double p3) {
  swap_halves(p0, p1);  // p0: (p0 lanes 0-31 | p1 lanes 0-31), p1: (p0 lanes 32-63 | p1 lanes 32-63)
  swap_halves(p2, p3);
  double a = p0 + p1, b = p2 + p3;
  swap_rows(a, b);
  double t = a + b;
  t += dpp_f64<0xb1, 0xf, 0xf>(t);   // quad_perm [1, 0, 3, 2]
  t += dpp_f64<0x4e, 0xf, 0xf>(t);   // quad_perm [2, 3, 0, 1]
  t += dpp_f64<0x141, 0xf, 0xf>(t);  // row_half_mirror
  t += dpp_f64<0x140, 0xf, 0xf>(t);  // row_mirror
  return t;
}

template <int LANE>
__device__ __forceinline__ double lane_value(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), LANE);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), LANE);
  return __hiloint2double(hi, lo);
}

// Adds a wave total v (uniform) to product slot `slot` of the two-register accumulator whose
// lane j holds slot j (a0) and slot 64 + j (a1).
__device__ __forceinline__ void add_to_slot(double& a0, double& a1, int slot, int lane, double v) {
  const double add = lane == (slot & 63) ? v : 0.0;
  if (slot < 64) a0 += add;
  else a1 += add;
}

// Product batches of the reverse sweep: the products of four consecutive slots 4b .. 4b + 3 are
// buffered per thread and reduced together (wave_totals4); their wave totals stay in the rows
// that wave_totals4 leaves them in, so slot 4b + k accumulates in register b / 16, in the lanes
// of row rowof(k) = (0, 2, 1, 3)[k] and column b % 16 (each lane of a row adds only in its own
// column). slot_of_lane inverts the map for the end of a pass.
struct ProductBatch {
  double p[4];
};

__device__ __forceinline__ void batch_put(ProductBatch& B, int k, double v) {
  switch (k) {  // uniform
    case 0: B.p[0] = v; break;
    case 1: B.p[1] = v; break;
    case 2: B.p[2] = v; break;
    default: B.p[3] = v; break;
  }
}

__device__ __forceinline__ void batch_flush(ProductBatch& B, int b, int lane, double& a0,
                                            double& a1) {
  const double t = wave_totals4(B.p[0], B.p[1], B.p[2], B.p[3]);
  const double add = (lane & 15) == (b & 15) ? t : 0.0;
  if (b < 16) a0 += add;
  else a1 += add;
  B.p[0] = B.p[1] = B.p[2] = B.p[3] = 0.0;
}

__device__ __forceinline__ int slot_of_lane(int reg, int lane) {
  const int row = lane >> 4;
  return 4 * (16 * reg + (lane & 15)) + (((row & 1) << 1) | (row >> 1));
}

__device__ __forceinline__ double lane63_value(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// The lean forward pass of 512-thread workgroups fits 128 VGPRs: four waves per SIMD, so two
// workgroups share a CU (one's loads and stores overlap the other's gates).
template <typename R, int RB, int W, bool GEN>
__global__ void __launch_bounds__(1 << W) __attribute__((amdgpu_waves_per_eu(W == 9 && !GEN ? 4 : 1)))
k_pass_fwd(const PassItem* __restrict__ items, int n_items, int64_t total, int64_t chunk) {
  using G = Geometry<RB, W>;
  using V = typename Vec2<R>::T;
  __shared__ V lds[1 << G::T];
  __shared__ OpStage sops[kMaxOpsPerPass + 1];
  __shared__ PhaseDesc sph[kMaxPhasesPerPass];
  __shared__ V sdiag[RB <= kMaxMacroRegBits ? kMaxDiagBlocks << RB : 1];
  __shared__ double wsum[G::NW];
  const uint32_t tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int64_t g0 = (int64_t)blockIdx.x * chunk;
  const int64_t g1 = g0 + chunk < total ? g0 + chunk : total;
  if (g0 >= g1) return;
  int it = find_item(items, n_items, g0);
  Layout<RB> D;
  direct_layout<R, RB, W>(D, tid);
  while (g0 < g1) {
    const PassItem I = items[it];
    const int64_t stop = I.tile_begin + (1ll << I.n_outer) < g1 ? I.tile_begin + (1ll << I.n_outer) : g1;
    const V* src = static_cast<const V*>(I.src);
    V* dst = static_cast<V*>(I.dst);
    const int n_ph = I.pd.phase_end - I.pd.phase_begin;
    TileMap<RB> MD, ML, MS;
    bool live;
    uint32_t preg;
    direct_map<RB, W>(I.pd, tid, MD, live, preg);
    Layout<RB> LL, LS;
    io_layouts<R, RB, G::T>(I, tid, D, MD, LL, ML, LS, MS);
    const bool phantom = I.pd.tile[G::T - 1] < 0;  // phantom bits are the top tile bits
    uint64_t obase = deposit_bits((uint64_t)(g0 - I.tile_begin), I.pd.outer_mask);
    // reference gradient (Algorithm 2): an item with lam set ends its entry with Re <lambda|mu>
    // in place of storing mu
    const V* lamv = static_cast<const V*>(I.lam);
    double dot = 0.0;
    for (int64_t g = g0; g < stop; ++g, obase = next_in_mask(obase, I.pd.outer_mask)) {
      const uint64_t obl = obase | ML.gthr, obs = obase | MS.gthr;
      cx<R> a[G::NA];
      if (!phantom) {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) a[ri] = load<R>(src, obl | map_off<RB>(ML, ri));
      } else {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) {
          a[ri] = cx<R>{0, 0};
          if (live && !(ri & preg)) a[ri] = load<R>(src, obl | map_off<RB>(ML, ri));
        }
      }
      if (g == g0) {  // staged while the first tile's loads are in flight
        stage_pass<RB, V>(I, sops, sph, sdiag, (int)tid, G::NT);
        lds_barrier();
      }
      Layout<RB> cur = LL;
      int k = 0;
      int flip = 0;
      uint4 nraw = staged_words(sops, 0);
      double2 ncs = staged_cs(sops, 0);
      for (int ph = 0; ph < n_ph; ++ph) {
        int8_t rb[RB];
        uint32_t rperm;  // 0: the forward schedule folds no CNOTs
        const int op_end = uniform_phase<RB>(sph, ph, rb, &rperm);
        if (!same_layout<RB>(cur, rb)) {
          Layout<RB> nxt;
          make_layout<R, RB>(nxt, rb, tid);
          relayout<R, RB>(a, cur, nxt, lds);
          cur = nxt;
        }
        // every load in flight is complete before the ops: without this the compiler's wait
        // analysis (the op loop is rotated, so its blocks are also entered from the relayout)
        // keeps a wait on the LDS counter in every op, which also waits for the op prefetch
        __builtin_amdgcn_s_waitcnt(kWaitVmLgkm);
        for (; k < op_end; ++k) {
          const FusedOp op = uniform_op(nraw);
          const double2 cs = ncs;
          nraw = staged_words(sops, k + 1);
          ncs = staged_cs(sops, k + 1);
          const GateRec* rec = I.recs + op.gate;
          if (GEN && k == I.sub_op) {
            apply_derivative<R, RB>(op, rec, I.sub_param, a, cur);
          } else if (GEN && op.type >= FOP_FIRST_GENERAL) {
            apply_general<R, RB, false>(op, rec, a, cur);
          } else {
            double unused[kMaxMacroRegBits];
            lean_step<R, RB, false>(op, (R)cs.x, (R)cs.y, rec, sops, sdiag, a, nullptr, cur.tdep, unused,
                                    flip);
          }
        }
      }
      if (flip) negate_all<R, G::NA>(a);
      if (!same_layout<RB>(cur, LS.rb)) relayout<R, RB>(a, cur, LS, lds);
      if (lamv) {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri)
          if (live && !(ri & preg)) {
            const cx<R> l = load<R>(lamv, obs | map_off<RB>(MS, ri));
            dot += re_cm(l.r, l.i, a[ri].r, a[ri].i);
          }
      } else if (!phantom) {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) store<R>(dst, obs | map_off<RB>(MS, ri), a[ri]);
      } else {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri)
          if (live && !(ri & preg)) store<R>(dst, obs | map_off<RB>(MS, ri), a[ri]);
      }
    }
    if (lamv) {
      const double t = wave_total_lane63(dot);
      if (lane == 63) wsum[wave] = t;
      lds_barrier();
      if (tid == 0) {
        double sum = 0;
#pragma unroll
        for (int w = 0; w < G::NW; ++w) sum += wsum[w];
        I.partials[(int)blockIdx.x - I.first_wg] = make_double2(sum, 0.0);
      }
    }
    // the next item may be the next pass over the same tile (a circuit whose state is one tile
    // runs all its passes in one launch): this thread's stores precede its loads there
    __threadfence_block();
    lds_barrier();  // the staged tables are rewritten for the next item
    g0 = stop;
    ++it;
  }
}

// cplx (general instance only): complex entries <lambda|mu> (App. B.4); partials hold (Re, Im).
template <typename R, int RB, int W, bool GEN>
__global__ void __launch_bounds__(1 << W)
k_pass_bwd(const PassItem* __restrict__ items, int n_items, int64_t total, int64_t chunk,
           int cplx) {
  using G = Geometry<RB, W>;
  using V = typename Vec2<R>::T;
  // Workgroups of at most four waves re-lay out phi and lambda one after the other through one
  // tile-sized buffer when a buffer for both would exceed 80 KiB: two such workgroups then fit
  // in a CU's LDS and run independently, one's loads and stores overlapping the other's gates.
  constexpr bool SPLIT = W <= 8 && (2u << G::T) * sizeof(V) > (80u << 10);
  __shared__ V lds[SPLIT ? (1 << G::T) : (2 << G::T)];
  __shared__ OpStage sops[kMaxOpsPerPass + 1];
  __shared__ PhaseDesc sph[kMaxPhasesPerPass];
  __shared__ V sdiag[RB <= kMaxMacroRegBits ? kMaxDiagBlocks << RB : 1];
  // per-wave slot sums, written after the item's last tile: they share the relayout buffer
  // (every wave has passed the barrier that ends its last relayout by then)
  static_assert(sizeof(lds) >= 2 * sizeof(double) * kMaxSlotsPerPass * G::NW,
                "slot sums fit the relayout buffer");
  double (*wacc)[G::NW] = reinterpret_cast<double (*)[G::NW]>(lds);
  double (*wacc_im)[G::NW] = wacc + kMaxSlotsPerPass;
  const uint32_t tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int64_t g0 = (int64_t)blockIdx.x * chunk;
  const int64_t g1 = g0 + chunk < total ? g0 + chunk : total;
  if (g0 >= g1) return;
  int it = find_item(items, n_items, g0);
  Layout<RB> D;
  direct_layout<R, RB, W>(D, tid);
  while (g0 < g1) {
    const PassItem I = items[it];
    const int64_t stop = I.tile_begin + (1ll << I.n_outer) < g1 ? I.tile_begin + (1ll << I.n_outer) : g1;
    V* phi = static_cast<V*>(I.dst);
    V* lam = static_cast<V*>(I.lam);
    const int n_ph = I.pd.phase_end - I.pd.phase_begin;
    TileMap<RB> MD, ML, MS;
    bool live;
    uint32_t preg;
    direct_map<RB, W>(I.pd, tid, MD, live, preg);
    Layout<RB> LL, LS;
    io_layouts<R, RB, G::T>(I, tid, D, MD, LL, ML, LS, MS);
    const bool phantom = I.pd.tile[G::T - 1] < 0;  // phantom bits are the top tile bits
    uint64_t obase = deposit_bits((uint64_t)(g0 - I.tile_begin), I.pd.outer_mask);
    // every wave accumulates the product slots over its share of the tiles, in two registers:
    // batched (ProductBatch) for real entries; for complex entries lane j of acc0 holds slot j,
    // lane j of acc1 slot 64 + j
    double acc0 = 0.0, acc1 = 0.0, acc0_im = 0.0, acc1_im = 0.0;
    const bool cx_entries = GEN && cplx;
    ProductBatch pb;
    pb.p[0] = pb.p[1] = pb.p[2] = pb.p[3] = 0.0;
    for (int64_t g = g0; g < stop; ++g, obase = next_in_mask(obase, I.pd.outer_mask)) {
      const uint64_t obl = obase | ML.gthr, obs = obase | MS.gthr;
      cx<R> f[G::NA], l[G::NA];
      if (!phantom) {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) {
          f[ri] = load<R>(phi, obl | map_off<RB>(ML, ri));
          l[ri] = load<R>(lam, obl | map_off<RB>(ML, ri));
        }
      } else {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) {
          f[ri] = cx<R>{0, 0};
          l[ri] = cx<R>{0, 0};
          if (live && !(ri & preg)) {
            f[ri] = load<R>(phi, obl | map_off<RB>(ML, ri));
            l[ri] = load<R>(lam, obl | map_off<RB>(ML, ri));
          }
        }
      }
      if (g == g0) {  // staged while the first tile's loads are in flight
        stage_pass<RB, V>(I, sops, sph, sdiag, (int)tid, G::NT);
        lds_barrier();
      }
      Layout<RB> cur = LL;
      int k = 0;
      // phi and lambda carry the same sign from flipped rotations, so products are unaffected
      int flip = 0;
      uint4 nraw = staged_words(sops, 0);
      double2 ncs = staged_cs(sops, 0);
      for (int ph = 0; ph < n_ph; ++ph) {
        int8_t rb[RB];
        uint32_t rperm;
        const int op_end = uniform_phase<RB>(sph, ph, rb, &rperm);
        if (!same_layout<RB>(cur, rb)) {
          Layout<RB> nxt;
          make_layout<R, RB>(nxt, rb, tid);
          if constexpr (SPLIT) {
            relayout<R, RB>(f, cur, nxt, lds, rperm);
            relayout<R, RB>(l, cur, nxt, lds, rperm);
          } else {
            relayout2<R, RB>(f, l, cur, nxt, lds, 1 << G::T, rperm);
          }
          cur = nxt;
        }
        // every load in flight is complete before the ops: without this the compiler's wait
        // analysis (the op loop is rotated, so its blocks are also entered from the relayout)
        // keeps a wait on the LDS counter in every op, which also waits for the op prefetch
        __builtin_amdgcn_s_waitcnt(kWaitVmLgkm);
        for (; k < op_end; ++k) {
          FusedOp op = uniform_op(nraw);
          double2 cs = ncs;
          nraw = staged_words(sops, k + 1);
          ncs = staged_cs(sops, k + 1);
          // complex entries take a rotation macro apart: its RB records run one by one (the head
          // as the plain rotation on position 0)
          int n_sub = 1;
          const int mem = op.k1;
          if (cx_entries && (op.flags & FOPF_MACRO)) {
            n_sub = RB;
            op.opc = QSV_OPC(op.type, 0);
            op.np = 1;
          } else if (cx_entries && op.opc == QSV_OPC(FOP_RZ, QSV_V_DIAG)) {
            n_sub = 1 + op.s0;  // the members one by one; the head itself does nothing
            op.opc = 0xffff;
            op.np = 0;
          }
          for (int sub = 0; sub < n_sub; ++sub) {
            if (sub > 0) {
              op = uniform_op(staged_words(sops, mem + sub - 1));
              cs = staged_cs(sops, mem + sub - 1);
              diag_member_shears(op, cs);
            }
            const GateRec* rec = I.recs + op.gate;
            double prod[kMaxMacroRegBits] = {}, prod_im[kMaxMacroRegBits] = {};
            if (GEN && op.type >= FOP_FIRST_GENERAL) {
              apply_general<R, RB, true>(op, rec, f, cur, true);
              if (op.np)
                general_products<R, RB>(op, rec, f, l, cur, prod, prod_im, cx_entries);
              apply_general<R, RB, true>(op, rec, l, cur);
            } else {
              if (cx_entries && op.np) prod_im[0] = lean_product_im<R, RB>(op, f, l, cur.tdep);
              lean_step<R, RB, true>(op, (R)cs.x, (R)cs.y, rec, sops, sdiag, f, l, cur.tdep,
                                     prod, flip);
            }
            if (!cx_entries) {
#pragma unroll
              for (int j = 0; j < kMaxMacroRegBits; ++j) {
                if (j >= op.np) break;
                const int slot = op.lslot + j;
                batch_put(pb, slot & 3, prod[j]);
                if ((slot & 3) == 3) batch_flush(pb, slot >> 2, lane, acc0, acc1);
              }
            } else {
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                if (j >= op.np) break;
                const double s = lane63_value(wave_total_lane63(prod[j]));
                add_to_slot(acc0, acc1, op.lslot + j, lane, s);
                if (cx_entries) {
                  const double si = lane63_value(wave_total_lane63(prod_im[j]));
                  add_to_slot(acc0_im, acc1_im, op.lslot + j, lane, si);
                }
              }
            }
          }
        }
      }
      // the tile's last, partial batch
      if (!cx_entries && (I.pd.n_slots & 3)) batch_flush(pb, (I.pd.n_slots - 1) >> 2, lane, acc0, acc1);
      if (flip) {
        negate_all<R, G::NA>(f);
        negate_all<R, G::NA>(l);
      }
      if (!same_layout<RB>(cur, LS.rb)) {
        if constexpr (SPLIT) {
          relayout<R, RB>(f, cur, LS, lds);
          relayout<R, RB>(l, cur, LS, lds);
        } else {
          relayout2<R, RB>(f, l, cur, LS, lds, 1 << G::T);
        }
      }
      if (!phantom) {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) {
          store<R>(phi, obs | map_off<RB>(MS, ri), f[ri]);
          store<R>(lam, obs | map_off<RB>(MS, ri), l[ri]);
        }
      } else {
#pragma unroll
        for (int ri = 0; ri < G::NA; ++ri) {
          if (live && !(ri & preg)) {
            store<R>(phi, obs | map_off<RB>(MS, ri), f[ri]);
            store<R>(lam, obs | map_off<RB>(MS, ri), l[ri]);
          }
        }
      }
    }
    if (cx_entries) {
      wacc[lane][wave] = acc0;
      wacc[64 + lane][wave] = acc1;
      wacc_im[lane][wave] = acc0_im;
      wacc_im[64 + lane][wave] = acc1_im;
    } else {
      wacc[slot_of_lane(0, lane)][wave] = acc0;
      wacc[slot_of_lane(1, lane)][wave] = acc1;
    }
    lds_barrier();
    const int col = (int)blockIdx.x - I.first_wg;
    for (int j = tid; j < I.pd.n_slots; j += G::NT) {
      double s = 0, si = 0;
#pragma unroll
      for (int w = 0; w < G::NW; ++w) {
        s += wacc[j][w];
        if (cx_entries) si += wacc_im[j][w];
      }
      I.partials[(size_t)j * I.nb + col] = make_double2(s, si);
    }
    __threadfence_block();  // see k_pass_fwd
    lds_barrier();  // wacc and the staged tables are rewritten for the next item
    g0 = stop;
    ++it;
  }
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
// The cases below are the geometries fused_config_supported (fused.h) names.
#define QSV_FUSED_CASES(X, R) X(R, 2, 8) X(R, 3, 8) X(R, 3, 9) X(R, 2, 9) X(R, 2, 6) X(R, 3, 6)

template <typename R>
hipError_t launch_fused_forward(const PassItem* d_items, int n_items, int64_t total, int64_t chunk,
                                int r, int w, bool general, int grid, hipStream_t st) {
#define X(RR, RB, WW)                                                                          \
  if (r == RB && w == WW) {                                                                    \
    if (general)                                                                               \
      hipLaunchKernelGGL((k_pass_fwd<RR, RB, WW, true>), dim3(grid), dim3(1 << WW), 0, st,     \
                         d_items, n_items, total, chunk);                                      \
    else                                                                                       \
      hipLaunchKernelGGL((k_pass_fwd<RR, RB, WW, false>), dim3(grid), dim3(1 << WW), 0, st,    \
                         d_items, n_items, total, chunk);                                      \
    return hipGetLastError();                                                                  \
  }
  QSV_FUSED_CASES(X, R)
  X(R, 4, 8)
  if constexpr (sizeof(R) == 4) { X(R, 4, 9) }
#undef X
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_fused_backward(const PassItem* d_items, int n_items, int64_t total,
                                 int64_t chunk, int r, int w, bool general, int grid,
                                 hipStream_t st, bool cplx) {
#define X(RR, RB, WW)                                                                          \
  if (r == RB && w == WW) {                                                                    \
    if (general || cplx)                                                                       \
      hipLaunchKernelGGL((k_pass_bwd<RR, RB, WW, true>), dim3(grid), dim3(1 << WW), 0, st,     \
                         d_items, n_items, total, chunk, cplx ? 1 : 0);                        \
    else                                                                                       \
      hipLaunchKernelGGL((k_pass_bwd<RR, RB, WW, false>), dim3(grid), dim3(1 << WW), 0, st,    \
                         d_items, n_items, total, chunk, 0);                                   \
    return hipGetLastError();                                                                  \
  }
  QSV_FUSED_CASES(X, R)
  X(R, 4, 8)
  if constexpr (sizeof(R) == 4) { X(R, 4, 9) }
#undef X
  return hipErrorInvalidValue;
}

template hipError_t launch_fused_forward<double>(const PassItem*, int, int64_t, int64_t, int, int,
                                                 bool, int, hipStream_t);
template hipError_t launch_fused_forward<float>(const PassItem*, int, int64_t, int64_t, int, int,
                                                bool, int, hipStream_t);
template hipError_t launch_fused_backward<double>(const PassItem*, int, int64_t, int64_t, int,
                                                  int, bool, int, hipStream_t, bool);
template hipError_t launch_fused_backward<float>(const PassItem*, int, int64_t, int64_t, int, int,
                                                 bool, int, hipStream_t, bool);

}  // namespace qsv
