// Algorithm 1 for states of at most 6 qubits in one wave: amplitude j of psi, phi and lambda sits
// in lane j (lanes >= 2^n hold zeros, and every gate keeps them among themselves), and one wave
// runs the whole gradient of one circuit: the forward pass, the energy, the reverse sweep and the
// gradient entries. A launch of B workgroups of 64 threads runs B circuits side by side.
//
// The per-gate steps are those of Algorithm 1 (Sec. 2.3): the forward pass psi = U|in>, the
// application of H (X-mask groups: (P psi)_j = c (-1)^popcount((j^x)&z) psi_{j^x}), then for
// i = G..1: phi <- U_i^-1 phi, mu = dU_i/dtheta phi, the product Re <lambda|mu>, lambda <- U_i^dag
// lambda. Arithmetic is FP64 in both storage types (the state only passes through the storage
// type when |in> is read).
//
// A state this small leaves the sweep bound by the latency of its dependent steps, so the design
// keeps every step short:
//  - gate data is read 64 gates ahead, one gate per lane (kind and qubits packed in one word,
//    cos and sin of a rotation's half angle formed from theta), and broadcast with v_readlane
//    when the gate runs;
//  - rotations about X, Y, Z, CNOT and CZ have their own paths; the partner amplitude across a
//    qubit comes from a DPP lane permutation or a permlane swap (no LDS round trip), one code path
//    per qubit; other gates read their matrices from the gate records (scalar loads) and exchange
//    amplitudes with ds_bpermute;
//  - the products of kRows consecutive slots are staged in LDS, one row per slot, and each row
//    is then summed by one lane in lane order, so no product goes to memory per lane;
//  - the gradient entries (sums of a parameter's slots in sweep order) and the energy (lane parts
//    in lane order) are formed by the same wave at the end: one launch per gradient.
// The same steps serve the chunked sweep of one long circuit and Algorithm 2 (further below).
#include "qsv_device.h"
#include "sv_kernels.h"

namespace qsv {

namespace {

using C = cx<double>;

constexpr int kRows = 16;       // product slots staged in LDS before their rows are summed
constexpr int kRowStride = 65;  // doubles per row: 64 lanes and one word against bank conflicts

template <int N>
struct IQ {
  static constexpr int v = N;
};

// ---- lane exchanges ---------------------------------------------------------------------------

// any distance (generic gates): ds_bpermute
__device__ __forceinline__ C shfl_xor_c(C v, int mask) {
  return C{__shfl_xor(v.r, mask, 64), __shfl_xor(v.i, mask, 64)};
}

template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  // every lane reads a lane of the wave, so no lane keeps an old value
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
// the word of lane (lane ^ 2^Q). Distances 1 and 2: quad_perm [1,0,3,2] and [2,3,0,1].
// Distances 4 and 8: the lanes with the bit clear read 4 (8) lanes up (row_shl), those with the
// bit set 4 (8) lanes down (row_shr); each move writes only its banks of 4 lanes, and both read
// the source, so neither waits for the other. Distances 16 and 32: a permlane16 / permlane32
// swap of the word with itself leaves the partner row (half) in one of its two results.
template <int Q>
__device__ __forceinline__ int xor_word(int v, int lane) {
  if constexpr (Q == 0) {
    return dpp<0xb1>(v);
  } else if constexpr (Q == 1) {
    return dpp<0x4e>(v);
  } else if constexpr (Q == 2) {
    const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xf, 0x5, false);   // banks 0, 2
    return __builtin_amdgcn_update_dpp(up, v, 0x114, 0xf, 0xa, false);     // banks 1, 3
  } else if constexpr (Q == 3) {
    const int up = __builtin_amdgcn_mov_dpp(v, 0x108, 0xf, 0x3, false);   // banks 0, 1
    return __builtin_amdgcn_update_dpp(up, v, 0x118, 0xf, 0xc, false);     // banks 2, 3
  } else if constexpr (Q == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? (int)r[0] : (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? (int)r[0] : (int)r[1];
  }
}
template <int Q>
__device__ __forceinline__ double xor_double(double v, int lane) {
  return __hiloint2double(xor_word<Q>(__double2hiint(v), lane), xor_word<Q>(__double2loint(v), lane));
}
// amplitude of lane (lane ^ 2^Q)
template <int Q>
__device__ __forceinline__ C partner(C v, int lane) {
  return C{xor_double<Q>(v.r, lane), xor_double<Q>(v.i, lane)};
}
// f(IQ<q>) for a uniform q < 6
template <typename F>
__device__ __forceinline__ auto on_qubit(int q, F f) {
  switch (q) {
    case 0: return f(IQ<0>{});
    case 1: return f(IQ<1>{});
    case 2: return f(IQ<2>{});
    case 3: return f(IQ<3>{});
    case 4: return f(IQ<4>{});
    default: return f(IQ<5>{});
  }
}

// partners across a uniform qubit q of one state, or of two states at once
struct C2 {
  C a, b;
};
__device__ __forceinline__ C partner_of(C v, int q, int lane) {
  return on_qubit(q, [&](auto Q) { return partner<decltype(Q)::v>(v, lane); });
}
__device__ __forceinline__ C2 partners_of(C v, C w, int q, int lane) {
  return on_qubit(q, [&](auto Q) {
    constexpr int b = decltype(Q)::v;
    return C2{partner<b>(v, lane), partner<b>(w, lane)};
  });
}

__device__ __forceinline__ int rl(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ double rl(double v, int i) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), i),
                          __builtin_amdgcn_readlane(__double2loint(v), i));
}

// ---- gate data, one gate per lane -------------------------------------------------------------

// code = kind | q0 << 8 | q1 << 12; (c, s) = (cos, sin) of half the angle for RX, RY, RZ
// (RX = [[c, -is], [-is, c]], RY = [[c, -s], [s, c]], RZ = diag(c - is, c + is)), formed here
// from the angle as the gate records form them
struct LaneGate {
  int code;
  double c, s;
};
__device__ __forceinline__ void load_lane(const WaveJob& J, int base, int lane, LaneGate& d) {
  const int k = min(base + lane, J.n_gates - 1);
  const GateDesc g = J.gates[k];
  d.code = g.kind | (g.q0 << 8) | (g.q1 << 12);
  d.c = d.s = 0.0;
  if (g.kind == K_RX || g.kind == K_RY || g.kind == K_RZ) sincos(0.5 * J.theta[g.p[0]], &d.s, &d.c);
}

// ---- rotation, CNOT and CZ paths --------------------------------------------------------------

// Signs: sm = 0 on lanes whose bit of the rotation's qubit is 1 and the sign bit where it is 0;
// flip(x, sm) = x on the bit-1 lanes, -x on the bit-0 lanes.
__device__ __forceinline__ C flip(C v, int sm) {
  return C{__hiloint2double(__double2hiint(v.r) ^ sm, __double2loint(v.r)),
           __hiloint2double(__double2hiint(v.i) ^ sm, __double2loint(v.i))};
}
__device__ __forceinline__ int sign_mask(int lane, int q) { return (((lane >> q) & 1) ^ 1) << 31; }

// exp(-i t G/2) (sg = s) or its adjoint (sg = -s) on the lane's amplitude v:
//  Y: c v + sg f, f = flip(partner): RY = [[c, -s], [s, c]];
//  X: c v - i sg p, p = partner: RX = [[c, -is], [-is, c]];
//  Z: c v + i sg f, f = flip(v): RZ = diag(c - is, c + is).
__device__ __forceinline__ C rot_y(double c, double sg, C v, C f) {
  return C{c * v.r + sg * f.r, c * v.i + sg * f.i};
}
__device__ __forceinline__ C rot_x(double c, double sg, C v, C p) {
  return C{c * v.r + sg * p.i, c * v.i - sg * p.r};
}
__device__ __forceinline__ C rot_z(double c, double sg, C v, C f) {
  return C{c * v.r - sg * f.i, c * v.i + sg * f.r};
}
// Re <lambda|mu> for mu = dR/dt phi' = -(i/2) G phi (phi the state before un-applying R):
// Y: mu = f/2, f = flip(partner of phi); X: mu = -(i/2) p, p = partner of phi;
// Z: G phi = -flip(phi), so mu = (i/2) f, f = flip(phi)
__device__ __forceinline__ double prod_y(C lam, C f) { return 0.5 * (lam.r * f.r + lam.i * f.i); }
__device__ __forceinline__ double prod_x(C lam, C p) { return 0.5 * (lam.r * p.i - lam.i * p.r); }
__device__ __forceinline__ double prod_z(C lam, C f) { return 0.5 * (lam.i * f.r - lam.r * f.i); }
__device__ __forceinline__ C cz(C v, int q0, int q1, int lane) {
  const bool neg = (lane >> q0) & (lane >> q1) & 1;
  return sel(neg, C{-v.r, -v.i}, v);
}

// ---- generic gates: matrices from the record, ds_bpermute exchanges ---------------------------

__device__ __forceinline__ C mul(const double2 m, C a) {
  return C{m.x * a.r - m.y * a.i, m.x * a.i + m.y * a.r};
}
__device__ __forceinline__ C cmac(C acc, const double2 m, C a) {
  return C{acc.r + m.x * a.r - m.y * a.i, acc.i + m.x * a.i + m.y * a.r};
}
__device__ __forceinline__ double2 cj(double2 m) { return make_double2(m.x, -m.y); }
// A gate record read by a whole wave at one gate: the records are written by the launch before
// (they are constant while this kernel runs), so they are read through the constant address
// space, i.e. with scalar loads into uniform registers.
#define QSV_CONST __attribute__((address_space(4)))
using RecWords = const QSV_CONST double*;
__device__ __forceinline__ RecWords uniform_words(const GateRec* rec) {
  return (RecWords)(const void*)rec;
}
__device__ __forceinline__ double2 entry(RecWords w, int e) {
  return make_double2(w[2 * e], w[2 * e + 1]);
}

// One-qubit gate on qubit q: the lane's pair (a0, a1) in local order.
struct Pair {
  C a0, a1;
  bool hi;  // this lane holds the local index 1 amplitude
};
__device__ __forceinline__ Pair pair_of(C v, int q, int lane) {
  const C p = shfl_xor_c(v, 1 << q);
  const bool hi = (lane >> q) & 1;
  return Pair{sel(hi, p, v), sel(hi, v, p), hi};
}
__device__ __forceinline__ C row_apply(const double2 m[4], const Pair& P) {
  const C o0 = cmac(mul(m[0], P.a0), m[1], P.a1);
  const C o1 = cmac(mul(m[2], P.a0), m[3], P.a1);
  return sel(P.hi, o1, o0);
}

// Two-qubit gate on (q0, q1), local index 2 bit(q0) + bit(q1): the lane's four amplitudes in
// local order.
struct Quad {
  C a[4];
  int l;
};
// value k of (v0, v1, v2, v3) for a per-lane k < 4, as component selects (an indexed read of a
// register array would go through scratch memory)
__device__ __forceinline__ C pick4(int k, C v0, C v1, C v2, C v3) {
  const C lo = sel(k & 1, v1, v0), hi = sel(k & 1, v3, v2);
  return sel(k & 2, hi, lo);
}
__device__ __forceinline__ Quad quad_of(C v, int q0, int q1, int lane) {
  const int m1 = 1 << q1, m0 = 1 << q0;
  const C s1 = shfl_xor_c(v, m1), s2 = shfl_xor_c(v, m0), s3 = shfl_xor_c(v, m0 | m1);
  Quad Q;
  Q.l = 2 * ((lane >> q0) & 1) + ((lane >> q1) & 1);
  // a[k] sits at local index k = l ^ d, d the shuffle distance
#pragma unroll
  for (int k = 0; k < 4; ++k) Q.a[k] = pick4(k ^ Q.l, v, s1, s2, s3);
  return Q;
}
__device__ __forceinline__ C quad_apply(const double2 m[16], const Quad& Q) {
  C o[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    o[r] = mul(m[4 * r], Q.a[0]);
#pragma unroll
    for (int c = 1; c < 4; ++c) o[r] = cmac(o[r], m[4 * r + c], Q.a[c]);
  }
  return pick4(Q.l, o[0], o[1], o[2], o[3]);
}

// The record's 2x2 matrices: mode 0 = U, 1 = U^-1 (phi), 2 = U^dag (lambda), 3 + j =
// dU/dtheta_j (U at entries 0..3, dU_0 at 4..7, U^-1 of a non-unitary kind or dU_1 at 8..11,
// dU_2 at 12..15).
__device__ __forceinline__ void mat2(RecWords w, int kind, int mode, double2 m[4]) {
  if (mode == 1 && !kind_unitary(kind)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) m[e] = entry(w, 8 + e);
  } else if (mode == 1 || mode == 2) {
    m[0] = cj(entry(w, 0));
    m[1] = cj(entry(w, 2));
    m[2] = cj(entry(w, 1));
    m[3] = cj(entry(w, 3));
  } else {
    const int e0 = mode == 0 ? 0 : 4 * (mode - 2);
#pragma unroll
    for (int e = 0; e < 4; ++e) m[e] = entry(w, e0 + e);
  }
}
// 4x4: U at entries 0..15, dU at 16..31 (two-qubit kinds are unitary)
__device__ __forceinline__ void mat4(RecWords w, int mode, double2 m[16]) {
  if (mode == 1 || mode == 2) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) m[4 * r + c] = cj(entry(w, 4 * c + r));
  } else {
    const int e0 = mode == 0 ? 0 : 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) m[e] = entry(w, e0 + e);
  }
}
__device__ __forceinline__ C generic_apply(const GateRec* rec, int kind, int q0, int q1, int mode,
                                           C v, int lane) {
  const RecWords w = uniform_words(rec);
  if (kind_nqubits(kind) == 1) {
    double2 m[4];
    mat2(w, kind, mode, m);
    return row_apply(m, pair_of(v, q0, lane));
  }
  double2 m[16];
  mat4(w, mode, m);
  return quad_apply(m, quad_of(v, q0, q1, lane));
}

__device__ __forceinline__ double prod_re(C lam, C mu) { return lam.r * mu.r + lam.i * mu.i; }

// ---- one gate of each pass ----------------------------------------------------------------------

__device__ __forceinline__ C forward_gate(const WaveJob& J, const LaneGate& cur, int i, int k,
                                          C v, int lane, const int sm[6]) {
  const int code = rl(cur.code, i);
  const int kind = code & 31, q0 = (code >> 8) & 7, q1 = (code >> 12) & 7;
  if (kind == K_CZ) return cz(v, q0, q1, lane);
  if (kind == K_CNOT) {
    const C p = partner_of(v, q1, lane);
    return sel((lane >> q0) & 1, p, v);
  }
  if (kind == K_RY) {
    const double c = rl(cur.c, i), s = rl(cur.s, i);
    return on_qubit(q0, [&](auto Q) {
      constexpr int q = decltype(Q)::v;
      return rot_y(c, s, v, flip(partner<q>(v, lane), sm[q]));
    });
  }
  if (kind == K_RX) return rot_x(rl(cur.c, i), rl(cur.s, i), v, partner_of(v, q0, lane));
  if (kind == K_RZ) return rot_z(rl(cur.c, i), rl(cur.s, i), v, flip(v, sign_mask(lane, q0)));
  return generic_apply(J.recs + k, kind, q0, q1, 0, v, lane);
}

// Products of the reverse sweep: slot s goes to row s % kRows. A sweep (or a chunk of one)
// stages slots from s_begin on; when slot s starts a new group of kRows, the rows of the group
// before it are summed, one row per lane, in lane order.
struct Rows {
  double* rows;       // LDS, kRows * kRowStride
  double* slot_sum;   // global, one sum per slot
  int s_begin;        // first slot of this sweep
  int nl;             // lanes holding amplitudes (2^n)
};
__device__ __forceinline__ void flush_rows(const Rows& P, int first, int count, int lane) {
  __syncthreads();
  if (lane < count) {
    const double* row = P.rows + ((first + lane) & (kRows - 1)) * kRowStride;
    double t = 0;
    for (int l = 0; l < P.nl; ++l) t += row[l];
    P.slot_sum[first + lane] = t;
  }
  __syncthreads();
}
__device__ __forceinline__ void stage(const Rows& P, int slot, double v, int lane) {
  if ((slot & (kRows - 1)) == 0 && slot > P.s_begin) {
    const int first = max(slot - kRows, P.s_begin);
    flush_rows(P, first, slot - first, lane);
  }
  P.rows[(slot & (kRows - 1)) * kRowStride + lane] = v;
}
// the last group: slots [first, end)
__device__ __forceinline__ void flush_last(const Rows& P, int end, int lane) {
  if (end > P.s_begin) {
    const int first = max((end - 1) & ~(kRows - 1), P.s_begin);
    flush_rows(P, first, end - first, lane);
  }
}

// One step of the reverse sweep at gate k (entry i of the chunk's gate data): the product(s)
// of its parameters from phi and lambda, then phi <- U^-1 phi, lambda <- U^dag lambda. `slot`
// advances by the gate's parameter count.
__device__ __forceinline__ void backward_gate(const WaveJob& J, const LaneGate& cur, int i, int k,
                                              C& phi, C& lam, int& slot, const Rows& P, int lane,
                                              const int sm[6]) {
  const int code = rl(cur.code, i);
  const int kind = code & 31, q0 = (code >> 8) & 7, q1 = (code >> 12) & 7;
  if (kind == K_CZ) {
    phi = cz(phi, q0, q1, lane);
    lam = cz(lam, q0, q1, lane);
  } else if (kind == K_CNOT) {
    const C2 Pr = partners_of(phi, lam, q1, lane);
    const bool ctl = (lane >> q0) & 1;
    phi = sel(ctl, Pr.a, phi);
    lam = sel(ctl, Pr.b, lam);
  } else if (kind == K_RY) {
    const double c = rl(cur.c, i), s = rl(cur.s, i);
    const C2 Pr = on_qubit(q0, [&](auto Q) {
      constexpr int q = decltype(Q)::v;
      return C2{flip(partner<q>(phi, lane), sm[q]), flip(partner<q>(lam, lane), sm[q])};
    });
    stage(P, slot++, prod_y(lam, Pr.a), lane);
    phi = rot_y(c, -s, phi, Pr.a);
    lam = rot_y(c, -s, lam, Pr.b);
  } else if (kind == K_RX) {
    const double c = rl(cur.c, i), s = rl(cur.s, i);
    const C2 Pr = partners_of(phi, lam, q0, lane);
    stage(P, slot++, prod_x(lam, Pr.a), lane);
    phi = rot_x(c, -s, phi, Pr.a);
    lam = rot_x(c, -s, lam, Pr.b);
  } else if (kind == K_RZ) {
    const double c = rl(cur.c, i), s = rl(cur.s, i);
    const int m = sign_mask(lane, q0);
    const C fp = flip(phi, m), fl = flip(lam, m);
    stage(P, slot++, prod_z(lam, fp), lane);
    phi = rot_z(c, -s, phi, fp);
    lam = rot_z(c, -s, lam, fl);
  } else {
    const GateRec* rec = J.recs + k;
    const RecWords w = uniform_words(rec);
    const int np = kind_nparams(kind);
    if (np == 0) {
      phi = generic_apply(rec, kind, q0, q1, 1, phi, lane);
    } else if (kind_nqubits(kind) == 1) {
      // phi' = U^-1 phi for both local rows, mu_j = dU_j phi' (no second exchange)
      const Pair Pp = pair_of(phi, q0, lane);
      double2 ui[4];
      mat2(w, kind, 1, ui);
      const Pair F{cmac(mul(ui[0], Pp.a0), ui[1], Pp.a1), cmac(mul(ui[2], Pp.a0), ui[3], Pp.a1),
                   Pp.hi};
      phi = sel(F.hi, F.a1, F.a0);
      for (int j = 0; j < np; ++j) {
        double2 d[4];
        mat2(w, kind, 3 + j, d);
        stage(P, slot + j, prod_re(lam, row_apply(d, F)), lane);
      }
    } else {
      // two-qubit: f = U^dag (the lane's quad), phi = f at the lane's local index, mu = the
      // lane's row of dU f; matrix rows are read one at a time (uniform loads), so that the 32
      // entries of U and dU are never all live
      const Quad Q = quad_of(phi, q0, q1, lane);
      C f[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        __builtin_amdgcn_sched_barrier(0);
        C a{0, 0};
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) a = cmac(a, cj(entry(w, 4 * cc + r)), Q.a[cc]);
        f[r] = a;
      }
      phi = pick4(Q.l, f[0], f[1], f[2], f[3]);
      C mu{0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        __builtin_amdgcn_sched_barrier(0);
        C o{0, 0};
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) o = cmac(o, entry(w, 16 + 4 * r + cc), f[cc]);
        mu = sel(Q.l == r, o, mu);
      }
      stage(P, slot, prod_re(lam, mu), lane);
    }
    slot += np;
    lam = generic_apply(rec, kind, q0, q1, 2, lam, lane);
  }
}

// lambda = H psi (X-mask groups; lanes >= nl get 0) and E = <psi|lambda>, the lane parts summed in
// lane order through LDS (scratch: nl doubles)
__device__ __forceinline__ C apply_h(const WaveJob& J, C psi, int lane, double* scratch,
                                     double* energy) {
  const int nl = 1 << J.n;
  C lam{0, 0};
  for (int gi = 0; gi < J.n_groups; ++gi) {
    const PauliGroup Gp = J.groups[gi];
    const int x = (int)Gp.x;
    const C src = x ? shfl_xor_c(psi, x) : psi;
    double cr = 0, ci = 0;
    for (int t = Gp.t0; t < Gp.t1; ++t) {
      const PauliTerm T = J.terms[t];
      const bool neg = __popcll((uint64_t)(lane ^ x) & T.z) & 1;
      cr += neg ? -T.cre : T.cre;
      ci += neg ? -T.cim : T.cim;
    }
    lam = cmac(lam, make_double2(cr, ci), src);
  }
  if (lane >= nl) lam = C{0, 0};
  __syncthreads();
  scratch[lane] = lane < nl ? psi.r * lam.r + psi.i * lam.i : 0.0;
  __syncthreads();
  if (lane == 0 && energy) {
    double e = 0;
    for (int l = 0; l < nl; ++l) e += scratch[l];
    energy[0] = e;
  }
  __syncthreads();
  return lam;
}

// gradient entries: 2 Re of the sum of a parameter's slots, in sweep order (slot sums written by
// other lanes or waves: the caller makes them visible first). Eight parameters per lane at a
// time, so that their dependent loads (slot range, first slot, its sum) are in flight together.
__device__ __forceinline__ void gradient_entries(const WaveJob& J, int lane) {
  constexpr int U = 8;
  for (int p0 = lane; p0 < J.n_theta; p0 += 64 * U) {
    int b[U], e[U], o[U];
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + 64 * u;
      b[u] = p < J.n_theta ? J.param_ptr[p] : 0;
      e[u] = p < J.n_theta ? J.param_ptr[p + 1] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) o[u] = b[u] < e[u] ? J.occ[b[u]] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = o[u] >= 0 ? J.slot_sum[o[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      for (int k = b[u] + 1; k < e[u]; ++k) t[u] += J.slot_sum[J.occ[k]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (p0 + 64 * u < J.n_theta) J.grad[p0 + 64 * u] = 2.0 * t[u];
  }
}

template <typename R>
__device__ __forceinline__ C load_in(const WaveJob& J, int lane) {
  using V = typename Vec2<R>::T;
  if (lane >= (1 << J.n)) return C{0, 0};
  const cx<R> a = load<R>(static_cast<const V*>(J.in), (uint64_t)lane);
  return C{(double)a.r, (double)a.i};
}

__device__ __forceinline__ void sign_masks(int lane, int sm[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) sm[q] = sign_mask(lane, q);
}

}  // namespace

template <typename R, bool BATCH>
__global__ void __launch_bounds__(64) k_wave_adjoint(const WaveJob* __restrict__ jobs,
                                                     WaveJob single, const double* theta_base,
                                                     double* energy_base, double* grad_base) {
  __shared__ double rows[kRows * kRowStride];
  WaveJob J = BATCH ? jobs[blockIdx.x] : single;
  if (BATCH) {
    J.theta = theta_base;  // batch gate tables index the flat parameter vector
    J.energy = energy_base + blockIdx.x;
    J.grad = grad_base ? grad_base + J.grad_off : nullptr;
  }
  const int lane = threadIdx.x;
  const int G = J.n_gates;
  int sm[6];
  sign_masks(lane, sm);
  C psi = load_in<R>(J, lane);
  LaneGate cur{}, nxt{};
  // forward pass psi = U_G ... U_1 |in>, gate data one chunk of 64 gates ahead
  if (G > 0) load_lane(J, 0, lane, cur);
  for (int base = 0; base < G; base += 64) {
    if (base + 64 < G) load_lane(J, base + 64, lane, nxt);
    const int cnt = min(64, G - base);
    for (int i = 0; i < cnt; ++i) psi = forward_gate(J, cur, i, base + i, psi, lane, sm);
    cur = nxt;
  }
  C lam = apply_h(J, psi, lane, rows, J.energy);
  // reverse sweep; slots are numbered in sweep order, so the slot of the next product is the
  // count of products so far
  const Rows P{rows, J.slot_sum, 0, 1 << J.n};
  C phi = psi;
  int slot = 0;
  const int last = G > 0 ? ((G - 1) / 64) * 64 : 0;
  if (G > 0) load_lane(J, last, lane, cur);
  for (int base = last; base >= 0 && G > 0; base -= 64) {
    if (base > 0) load_lane(J, base - 64, lane, nxt);
    const int cnt = min(64, G - base);
    for (int i = cnt - 1; i >= 0; --i) backward_gate(J, cur, i, base + i, phi, lam, slot, P, lane, sm);
    cur = nxt;
  }
  flush_last(P, slot, lane);
  __threadfence();
  __syncthreads();
  gradient_entries(J, lane);
}

// ---- chunked sweep of one circuit ---------------------------------------------------------------
// Gates in chunks of 64 (chunk c: gates [64 c, 64 c + 64)); W_c = the product of chunk c's gates.
//  1. k_wave_chunk_ops: W_c for every chunk, in parallel: the chunk applied to the 2^n basis
//     states, 64 / 2^n of them per wave (lane = row + 2^n * column within the wave). W_c is stored
//     twice: A_c[j * N + r] = W_c[r][j] and B_c[j * N + r] = W_c[j][r], so that the products W v
//     (from A) and W^dag v (from B, conjugated) read each j's entries with consecutive lanes.
//  2. k_wave_chunk_chain (two waves): psi = W_C-1 ... W_0 |in>, lambda = H psi, E; then for
//     c = C-1 .. 0 it records (phi, lambda) at the end of chunk c and un-applies the chunk,
//     phi <- W_c^dag phi (wave 0), lambda <- W_c^dag lambda (wave 1) (every gate unitary).
//  3. k_wave_chunk_sweep: chunk c's steps of the reverse sweep from its recorded (phi, lambda),
//     for all chunks at once; its product slots start after those of the later chunks. The last
//     wave to finish forms the gradient entries.
// The steps within a chunk are those of the one-wave sweep; only the states at chunk boundaries
// come from the chunk operators instead of gate-by-gate updates.

template <typename R>
__global__ void __launch_bounds__(64) k_wave_chunk_ops(WaveJob J, WaveChunks K) {
  const int c = blockIdx.y;
  const int lane = threadIdx.x;
  const int n = J.n, N = 1 << n;
  const int r = lane & (N - 1);
  const int col = blockIdx.x * (64 >> n) + (lane >> n);
  int sm[6];
  sign_masks(lane, sm);
  C v{(col < N && r == col) ? 1.0 : 0.0, 0.0};
  LaneGate cur{};
  const int base = 64 * c, cnt = min(64, J.n_gates - base);
  load_lane(J, base, lane, cur);
  for (int i = 0; i < cnt; ++i) v = forward_gate(J, cur, i, base + i, v, lane, sm);
  if (col < N) {
    K.A[(size_t)c * N * N + (size_t)col * N + r] = make_double2(v.r, v.i);
    K.B[(size_t)c * N * N + (size_t)r * N + col] = make_double2(v.r, v.i);
  }
}

// v <- M v (adj = false, M = A_c) or W^dag v (adj = true, M = B_c) for the lane's row
// r = lane % N; m[t] = the lane's entries for columns j = h * JN + t, h = lane / N the lane's
// slice of the columns. v passes through LDS (vb, N entries); the slices' partial sums are
// added across lanes.
template <int NQ>
struct Mv {
  static constexpr int N = 1 << NQ;
  static constexpr int JN = N * N >= 64 ? N * N / 64 : 1;  // columns per lane
  static constexpr int SL = N / JN;                         // lanes per row
  static constexpr int LSL = NQ - (N * N >= 64 ? 2 * NQ - 6 : 0);  // log2(SL)
};
template <int NQ>
__device__ __forceinline__ void mv_load(const double2* M, int lane, double2 m[Mv<NQ>::JN]) {
  constexpr int N = Mv<NQ>::N, JN = Mv<NQ>::JN, SL = Mv<NQ>::SL;
  const int r = lane & (N - 1), h = lane >> NQ;
#pragma unroll
  for (int t = 0; t < JN; ++t) {
    const int j = (h < SL ? h : 0) * JN + t;
    m[t] = M[j * N + r];
  }
}
template <int NQ>
__device__ __forceinline__ C mv_apply(const double2 m[Mv<NQ>::JN], bool adj, C v, int lane,
                                      double2* vb) {
  constexpr int N = Mv<NQ>::N, JN = Mv<NQ>::JN, SL = Mv<NQ>::SL;
  const int h = lane >> NQ;
  __syncthreads();
  if (lane < N) vb[lane] = make_double2(v.r, v.i);
  __syncthreads();
  C a0{0, 0}, a1{0, 0};
  if (h < SL) {
#pragma unroll
    for (int t = 0; t < JN; ++t) {
      const double2 x = vb[h * JN + t];
      const double2 w = adj ? cj(m[t]) : m[t];
      C& a = (t & 1) ? a1 : a0;
      a = cmac(a, w, C{x.x, x.y});
    }
  }
  C acc{a0.r + a1.r, a0.i + a1.i};
#pragma unroll
  for (int b = NQ; b < NQ + Mv<NQ>::LSL; ++b) {
    C p;
    if (b == 0) p = partner<0>(acc, lane);
    else if (b == 1) p = partner<1>(acc, lane);
    else if (b == 2) p = partner<2>(acc, lane);
    else if (b == 3) p = partner<3>(acc, lane);
    else if (b == 4) p = partner<4>(acc, lane);
    else p = partner<5>(acc, lane);
    acc = C{acc.r + p.r, acc.i + p.i};
  }
  return acc;
}

// Two waves: both carry psi forward (the same steps, each in its own registers), then wave 0
// carries phi and wave 1 lambda back, each recording its state at the chunk boundaries.
template <typename R, int NQ>
__global__ void __launch_bounds__(128) k_wave_chunk_chain(WaveJob J, WaveChunks K) {
  constexpr int N = 1 << NQ, JN = Mv<NQ>::JN;
  __shared__ double2 vbuf[2][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2* vb = vbuf[wave];
  const int C_ = K.n_chunks;
  const size_t NN = (size_t)N * N;
  C psi = load_in<R>(J, lane);
  double2 mc[JN], mn[JN];
  mv_load<NQ>(K.A, lane, mc);
  for (int c = 0; c < C_; ++c) {
    if (c + 1 < C_) mv_load<NQ>(K.A + (c + 1) * NN, lane, mn);
    psi = mv_apply<NQ>(mc, false, psi, lane, vb);
#pragma unroll
    for (int t = 0; t < JN; ++t) mc[t] = mn[t];
  }
  if (lane >= N) psi = C{0, 0};
  C lam = apply_h(J, psi, lane, reinterpret_cast<double*>(vb), wave == 0 ? J.energy : nullptr);
  C v = wave == 0 ? psi : lam;  // phi (wave 0) or lambda (wave 1)
  double2* rec = wave == 0 ? K.phi : K.lam;
  mv_load<NQ>(K.B + (C_ - 1) * NN, lane, mc);
  for (int c = C_ - 1; c >= 0; --c) {
    if (lane < N) rec[(size_t)c * N + lane] = make_double2(v.r, v.i);
    if (c == 0) break;
    mv_load<NQ>(K.B + (c - 1) * NN, lane, mn);
    v = mv_apply<NQ>(mc, true, v, lane, vb);
#pragma unroll
    for (int t = 0; t < JN; ++t) mc[t] = mn[t];
  }
}

template <typename R>
__global__ void __launch_bounds__(64) k_wave_chunk_sweep(WaveJob J, WaveChunks K) {
  __shared__ double rows[kRows * kRowStride];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int N = 1 << J.n;
  int sm[6];
  sign_masks(lane, sm);
  C phi{0, 0}, lam{0, 0};
  if (lane < N) {
    const double2 a = K.phi[(size_t)c * N + lane], b = K.lam[(size_t)c * N + lane];
    phi = C{a.x, a.y};
    lam = C{b.x, b.y};
  }
  LaneGate cur{};
  const int base = 64 * c, cnt = min(64, J.n_gates - base);
  load_lane(J, base, lane, cur);
  int slot = K.slot0[c];
  const Rows P{rows, J.slot_sum, slot, N};
  for (int i = cnt - 1; i >= 0; --i) backward_gate(J, cur, i, base + i, phi, lam, slot, P, lane, sm);
  flush_last(P, slot, lane);
  // the last chunk to finish forms the gradient entries and re-arms the counter
  __threadfence();
  __syncthreads();
  __shared__ int ticket;
  if (lane == 0) ticket = atomicAdd(K.done, 1);
  __syncthreads();
  if (ticket == K.n_chunks - 1) {
    __threadfence();
    gradient_entries(J, lane);
    if (lane == 0) atomicExch(K.done, 0);
  }
}

template <typename R>
hipError_t launch_wave_adjoint(const WaveJob* d_jobs, int n_jobs, const WaveJob& single,
                               const double* theta_base, double* energy_base, double* grad_base,
                               hipStream_t st) {
  if (d_jobs)
    hipLaunchKernelGGL((k_wave_adjoint<R, true>), dim3(n_jobs), dim3(64), 0, st, d_jobs, single,
                       theta_base, energy_base, grad_base);
  else
    hipLaunchKernelGGL((k_wave_adjoint<R, false>), dim3(1), dim3(64), 0, st, d_jobs, single,
                       theta_base, energy_base, grad_base);
  return hipGetLastError();
}

// ---- Algorithm 2 (the reference scheme of Sec. 3) -------------------------------------------

template <typename R, bool BATCH>
__global__ void __launch_bounds__(64) k_wave_ref_lambda(const WaveJob* __restrict__ jobs,
                                                        WaveJob single, const double* theta_base,
                                                        double* energy_base) {
  __shared__ double scratch[64];
  WaveJob J = BATCH ? jobs[blockIdx.x] : single;
  if (BATCH) {
    J.theta = theta_base;  // batch gate tables index the flat parameter vector
    J.energy = energy_base + blockIdx.x;
  }
  const int lane = threadIdx.x;
  const int G = J.n_gates;
  int sm[6];
  sign_masks(lane, sm);
  C psi = load_in<R>(J, lane);
  LaneGate cur{}, nxt{};
  if (G > 0) load_lane(J, 0, lane, cur);
  for (int base = 0; base < G; base += 64) {
    if (base + 64 < G) load_lane(J, base + 64, lane, nxt);
    const int cnt = min(64, G - base);
    for (int i = 0; i < cnt; ++i) psi = forward_gate(J, cur, i, base + i, psi, lane, sm);
    cur = nxt;
  }
  const C lam = apply_h(J, psi, lane, scratch, J.energy);
  J.ref_lam[lane] = make_double2(lam.r, lam.i);
}

// mu = U_G .. U_k+1 dU_k/dtheta_j U_k-1 .. U_1 |in> for slot o = blockIdx.x (gate k, parameter j
// of the gate), then slot_sum[o] = Re <lambda|mu>
template <typename R, bool BATCH>
__global__ void __launch_bounds__(64) k_wave_ref_entry(const WaveJob* __restrict__ jobs,
                                                       WaveJob single, const double* theta_base) {
  __shared__ double scratch[64];
  WaveJob J = BATCH ? jobs[blockIdx.y] : single;
  if (BATCH) J.theta = theta_base;  // batch gate tables index the flat parameter vector
  const int o = blockIdx.x;
  if (o >= J.n_occ) return;
  const int kd = J.occ_gate[o] >> 2, jd = J.occ_gate[o] & 3;
  const int lane = threadIdx.x;
  const int G = J.n_gates;
  int sm[6];
  sign_masks(lane, sm);
  C v = load_in<R>(J, lane);
  LaneGate cur{}, nxt{};
  load_lane(J, 0, lane, cur);
  for (int base = 0; base < G; base += 64) {
    if (base + 64 < G) load_lane(J, base + 64, lane, nxt);
    const int cnt = min(64, G - base);
    for (int i = 0; i < cnt; ++i) {
      const int k = base + i;
      if (k == kd) {
        const int code = rl(cur.code, i);
        const int kind = code & 31, q0 = (code >> 8) & 7, q1 = (code >> 12) & 7;
        if (kind == K_RX || kind == K_RY || kind == K_RZ) {
          // dR/dt = -(s/2) 1 - i (c/2) G: a rotation's form with (c, s) -> (-s/2, c/2)
          const double c = -0.5 * rl(cur.s, i), s = 0.5 * rl(cur.c, i);
          if (kind == K_RZ) {
            v = rot_z(c, s, v, flip(v, sign_mask(lane, q0)));
          } else {
            const C p = partner_of(v, q0, lane);
            v = kind == K_RX ? rot_x(c, s, v, p) : rot_y(c, s, v, flip(p, sign_mask(lane, q0)));
          }
        } else {
          v = generic_apply(J.recs + k, kind, q0, q1, 3 + jd, v, lane);
        }
      } else {
        v = forward_gate(J, cur, i, k, v, lane, sm);
      }
    }
    cur = nxt;
  }
  const double2 l = J.ref_lam[lane];
  scratch[lane] = lane < (1 << J.n) ? l.x * v.r + l.y * v.i : 0.0;
  __syncthreads();
  if (lane == 0) {
    double t = 0;
    for (int q = 0; q < (1 << J.n); ++q) t += scratch[q];
    J.slot_sum[o] = t;
  }
}

template <bool BATCH>
__global__ void __launch_bounds__(64) k_wave_ref_grad(const WaveJob* __restrict__ jobs,
                                                      WaveJob single, double* grad_base) {
  WaveJob J = BATCH ? jobs[blockIdx.x] : single;
  if (BATCH) J.grad = grad_base ? grad_base + J.grad_off : nullptr;
  gradient_entries(J, threadIdx.x);
}

template <typename R>
hipError_t launch_wave_reference(const WaveJob* d_jobs, int n_jobs, int max_occ,
                                 const WaveJob& single, const double* theta_base,
                                 double* energy_base, double* grad_base, hipStream_t st) {
  if (d_jobs) {
    hipLaunchKernelGGL((k_wave_ref_lambda<R, true>), dim3(n_jobs), dim3(64), 0, st, d_jobs,
                       single, theta_base, energy_base);
    if (max_occ > 0)
      hipLaunchKernelGGL((k_wave_ref_entry<R, true>), dim3(max_occ, n_jobs), dim3(64), 0, st,
                         d_jobs, single, theta_base);
    hipLaunchKernelGGL((k_wave_ref_grad<true>), dim3(n_jobs), dim3(64), 0, st, d_jobs, single,
                       grad_base);
  } else {
    hipLaunchKernelGGL((k_wave_ref_lambda<R, false>), dim3(1), dim3(64), 0, st, d_jobs, single,
                       theta_base, energy_base);
    if (single.n_occ > 0)
      hipLaunchKernelGGL((k_wave_ref_entry<R, false>), dim3(single.n_occ, 1), dim3(64), 0, st,
                         d_jobs, single, theta_base);
    hipLaunchKernelGGL((k_wave_ref_grad<false>), dim3(1), dim3(64), 0, st, d_jobs, single,
                       grad_base);
  }
  return hipGetLastError();
}

template hipError_t launch_wave_reference<double>(const WaveJob*, int, int, const WaveJob&,
                                                  const double*, double*, double*, hipStream_t);
template hipError_t launch_wave_reference<float>(const WaveJob*, int, int, const WaveJob&,
                                                 const double*, double*, double*, hipStream_t);

template <typename R>
hipError_t launch_wave_chunked(const WaveJob& J, const WaveChunks& K, hipStream_t st) {
  const int n = J.n;
  if (n < 1 || n > kWaveChunkMaxQubits || K.n_chunks < 1) return hipErrorInvalidValue;
  const int per_wave = 64 >> n;
  const int waves = ((1 << n) + per_wave - 1) / per_wave;
  hipLaunchKernelGGL((k_wave_chunk_ops<R>), dim3(waves, K.n_chunks), dim3(64), 0, st, J, K);
  switch (n) {
    case 1: hipLaunchKernelGGL((k_wave_chunk_chain<R, 1>), dim3(1), dim3(128), 0, st, J, K); break;
    case 2: hipLaunchKernelGGL((k_wave_chunk_chain<R, 2>), dim3(1), dim3(128), 0, st, J, K); break;
    case 3: hipLaunchKernelGGL((k_wave_chunk_chain<R, 3>), dim3(1), dim3(128), 0, st, J, K); break;
    case 4: hipLaunchKernelGGL((k_wave_chunk_chain<R, 4>), dim3(1), dim3(128), 0, st, J, K); break;
    default: hipLaunchKernelGGL((k_wave_chunk_chain<R, 5>), dim3(1), dim3(128), 0, st, J, K); break;
  }
  hipLaunchKernelGGL((k_wave_chunk_sweep<R>), dim3(K.n_chunks), dim3(64), 0, st, J, K);
  return hipGetLastError();
}

template hipError_t launch_wave_chunked<double>(const WaveJob&, const WaveChunks&, hipStream_t);
template hipError_t launch_wave_chunked<float>(const WaveJob&, const WaveChunks&, hipStream_t);
template hipError_t launch_wave_adjoint<double>(const WaveJob*, int, const WaveJob&,
                                                const double*, double*, double*, hipStream_t);
template hipError_t launch_wave_adjoint<float>(const WaveJob*, int, const WaveJob&, const double*,
                                               double*, double*, hipStream_t);

}  // namespace qsv
