// Fusion scheduler (host code): partitions a gate sequence into fused passes (tile qubit sets) and
// each pass into register phases, preserving the order of the gates on every qubit.
//
// Both partitions use the same "blocked scan": walk the remaining gates in order; a gate is taken
// when all of its qubits are admissible and none of them is blocked, otherwise its qubits become
// blocked for the rest of the scan. Every taken gate therefore only follows gates it commutes with
// (disjoint qubits) or gates taken before it, so the executed order is a valid reordering.
#include <algorithm>
#include <cstring>
#include <string>

#include "fused.h"

namespace qsv {

static uint64_t qmask(const GateDesc& g) {
  uint64_t m = 1ull << g.q0;
  if (kind_nqubits(g.kind) == 2) m |= 1ull << g.q1;
  return m;
}

// Physical qubits that must be register bits for the gate (its non-diagonal targets).
static uint64_t regneed(const GateDesc& g) {
  switch (g.kind) {
    case K_RZ: case K_Z: case K_S: case K_T: case K_SDG: case K_PHASE: case K_CZ: case K_RZZ:
    case K_CRZ:
      return 0;
    case K_CNOT: case K_CRX: case K_CRY:
      return 1ull << g.q1;
    case K_RXX: case K_RYY:
      return (1ull << g.q0) | (1ull << g.q1);
    default:
      return 1ull << g.q0;
  }
}

static int popc(uint64_t x) { return __builtin_popcountll(x); }

// Gates taken by a blocked scan of `rem` with admissible qubits `allowed`, at most `max_slots`
// products (backward) and `max_ops` gates.
static void scan(const std::vector<int>& rem, const std::vector<GateDesc>& g, uint64_t allowed,
                 bool backward, int max_slots, int max_ops, std::vector<int>* taken, int* count) {
  uint64_t blocked = 0;
  int slots = 0, ops = 0, cnt = 0;
  for (int k : rem) {
    const uint64_t m = qmask(g[k]);
    const int np = backward ? kind_nparams(g[k].kind) : 0;
    if ((m & blocked) || (m & ~allowed) || slots + np > max_slots || ops + 1 > max_ops) {
      blocked |= m;
      continue;
    }
    slots += np;
    ++ops;
    ++cnt;
    if (taken) taken->push_back(k);
  }
  *count = cnt;
}

// Greedy tile growth along the gate order, starting from `seed`.
static uint64_t grow_tile(const std::vector<int>& rem, const std::vector<GateDesc>& g,
                          uint64_t seed, int t) {
  uint64_t T = seed, blocked = 0;
  for (int k : rem) {
    const uint64_t m = qmask(g[k]);
    if (m & blocked) {
      blocked |= m;
      continue;
    }
    if (popc(T | m) <= t) T |= m;
    else blocked |= m;
  }
  return T;
}

static uint64_t fill_tile(uint64_t T, int n, int t) {
  for (int q = 0; q < n && popc(T) < t; ++q) T |= 1ull << q;
  return T;
}

// Rotation macros. In a run of consecutive rotations about the same axis (RY, RX, or RZ) every
// op commutes with every other (and with the others' generators), so the run may execute in any
// order with the same products. When the run holds a rotation on each of the r register
// positions, the first such rotation per position is moved to the front of the run in position
// order and the first of them is flagged as a macro head: the kernel applies all r as one
// straight-line op (one dispatch). The other r - 1 records (the kernel reads only their cos/sin)
// are stored after the pass's executed ops, at the index the head's k1 names.
static int rotation_axis(const FusedOp& op) {
  if (op.flags & FOPF_DIAG) return 0;  // in a diagonal block
  if (op.type == FOP_RY) return 1;
  if (op.type == FOP_RX) return 2;
  if (op.type == FOP_RZ && (op.flags & FOPF_S0_REG)) return 3;
  if (op.type == FOP_RZ) return 4;  // RZ on a thread bit: commutes with the run, not a member
  return 0;
}

static bool is_diagonal(const FusedOp& op) {
  return op.type == FOP_RZ || op.type == FOP_CZ || op.type == FOP_DIAG1 || op.type == FOP_PDIAG1 ||
         op.type == FOP_DIAG2;
}

// Diagonal blocks. The diagonal gates of a run of consecutive diagonal gates commute, so the run
// may execute in any order with the same products. Its RZ gates on register bits and its CZ
// gates with both bits in registers are taken together (in run order, at most kMaxMacroRegBits
// RZ at a time) as one diagonal matrix on the thread's 2^r amplitudes when that saves arithmetic: per
// amplitude and state an RZ costs three FMAs (the shears), a CZ about one sign flip per two
// amplitudes, a block one complex product (four) plus the load of its entry. A head entry (gate
// index -1) precedes the block's members; the run's other diagonal gates follow the blocks.
// blocks_left and records_left bound the blocks of the pass (LDS tables) and its staged records.
static void form_diagonal_blocks(std::vector<std::pair<int, FusedOp>>& ops, bool backward,
                                 int& blocks_left, int& records_left) {
  std::vector<std::pair<int, FusedOp>> out;
  out.reserve(ops.size() + 8);
  size_t i = 0;
  while (i < ops.size()) {
    if (!is_diagonal(ops[i].second)) {
      out.push_back(ops[i++]);
      continue;
    }
    size_t j = i;
    while (j < ops.size() && is_diagonal(ops[j].second)) ++j;
    // members in run order, cut after every kMaxMacroRegBits-th RZ
    std::vector<std::vector<std::pair<int, FusedOp>>> groups(1);
    std::vector<std::pair<int, FusedOp>> rest;
    int nr = 0;
    for (size_t t = i; t < j; ++t) {
      const FusedOp& op = ops[t].second;
      const bool rz = op.type == FOP_RZ && (op.flags & FOPF_S0_REG);
      const bool cz = op.type == FOP_CZ && (op.flags & FOPF_S0_REG) && (op.flags & FOPF_S1_REG);
      if (!rz && !cz) {
        rest.push_back(ops[t]);
        continue;
      }
      if (rz && nr == kMaxMacroRegBits) {
        groups.emplace_back();
        nr = 0;
      }
      nr += rz;
      groups.back().push_back(ops[t]);
    }
    for (auto& grp : groups) {
      int g_rz = 0;
      for (auto& e : grp) g_rz += e.second.type == FOP_RZ;
      const int g_cz = (int)grp.size() - g_rz;
      if (6 * g_rz + g_cz >= 12 && blocks_left > 0 && records_left > 0) {
        FusedOp h;
        std::memset(&h, 0, sizeof h);
        h.type = FOP_RZ;
        h.flags = FOPF_DIAG;
        h.opc = (uint16_t)QSV_OPC(FOP_RZ, QSV_V_DIAG);
        h.s0 = (uint8_t)grp.size();
        h.np = (uint8_t)(backward ? g_rz : 0);
        h.ks1 = (uint8_t)(kMaxDiagBlocks - blocks_left);
        int m = 0;
        for (auto& e : grp)
          if (e.second.type == FOP_RZ) h.gate |= (int32_t)e.second.ks0 << (4 * m++);
        --blocks_left;
        --records_left;
        out.emplace_back(-1, h);
        for (auto& e : grp) {
          out.push_back(e);
          out.back().second.flags |= FOPF_DIAG;
        }
      } else {
        for (auto& e : grp) out.push_back(e);
      }
    }
    for (auto& e : rest) out.push_back(e);
    i = j;
  }
  ops.swap(out);
}

static int register_position(const FusedOp& op) {
  return op.type == FOP_RZ ? op.ks0 : op.k0;
}

static void form_rotation_macros(std::vector<std::pair<int, FusedOp>>& ops, int r) {
  size_t i = 0;
  while (i < ops.size()) {
    int axis = rotation_axis(ops[i].second);
    if (!axis) {
      ++i;
      continue;
    }
    const bool z = axis >= 3;
    size_t j = i;  // the run: same axis (RZ on any bit counts as one axis)
    while (j < ops.size()) {
      const int a = rotation_axis(ops[j].second);
      if (!a || (a >= 3) != z || (!z && a != axis)) break;
      ++j;
    }
    // as many macros as the run holds: each takes the earliest remaining rotation per position
    std::vector<std::pair<int, FusedOp>> out;
    std::vector<char> used(j - i, 0);
    while (r >= 2) {
      int pick[kMaxRegBits];
      for (int k = 0; k < r; ++k) pick[k] = -1;
      for (size_t t = i; t < j; ++t) {
        if (used[t - i] || rotation_axis(ops[t].second) == 4) continue;
        const int k = register_position(ops[t].second);
        if (pick[k] < 0) pick[k] = (int)t;
      }
      bool full = true;
      for (int k = 0; k < r; ++k) full = full && pick[k] >= 0;
      if (!full) break;
      for (int k = 0; k < r; ++k) {
        out.push_back(ops[pick[k]]);
        if (k == 0) out.back().second.flags |= FOPF_MACRO;
        used[pick[k] - i] = 1;
      }
    }
    for (size_t t = i; t < j; ++t)
      if (!used[t - i]) out.push_back(ops[t]);
    for (size_t t = i; t < j; ++t) ops[t] = out[t - i];
    i = j;
  }
}

bool build_schedule(int n, const std::vector<GateDesc>& gates, const std::vector<int>& seq,
                    const std::vector<int32_t>& slot_of_gate, bool backward, int t, int r, int w,
                    int run_qubits, Schedule& out, std::string* msg, bool macros,
                    const std::vector<PassPlan>* given) {
  out = Schedule();
  out.t = t;
  out.r = r;
  out.w = w;
  if (t != r + w || t > kMaxTileBits || r > kMaxRegBits || r < 1 || n < 1) {
    if (msg) *msg = "tile/register sizes do not fit the state";
    return false;
  }
  const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
  // a state smaller than the tile fills its low tile bits; the other tile bits are phantom
  // (their amplitudes are never loaded or stored and stay zero)
  const int tq = std::min(t, n);
  // low qubits always in the tile: contiguous runs of 2^c amplitudes per load
  const int c = std::min(run_qubits, std::min(w, n));
  const uint64_t low = (1ull << c) - 1;

  // candidate tiles for the gates `r`: greedy growth along the gate order (from the low qubits,
  // and from them plus the first gate's qubits), and windows along the qubit chain
  auto candidates = [&](const std::vector<int>& r) {
    std::vector<uint64_t> cs;
    auto add = [&](uint64_t T) {
      if (popc(T) == tq && std::find(cs.begin(), cs.end(), T) == cs.end()) cs.push_back(T);
    };
    add(fill_tile(grow_tile(r, gates, low, tq), n, tq));
    add(fill_tile(grow_tile(r, gates, low | qmask(gates[r[0]]), tq), n, tq));
    for (int a = c; a + (tq - c) <= n; ++a) add(((((1ull << (tq - c)) - 1) << a) | low) & all);
    return cs;
  };

  std::vector<int> rem(seq);
  size_t next_given = 0;
  while (given ? next_given < given->size() : !rem.empty()) {
    uint64_t bestT = 0;
    std::vector<int> taken;
    if (given) {  // the passes are given: tile and gates (in execution order)
      bestT = (*given)[next_given].tile;
      taken = (*given)[next_given].gates;
      ++next_given;
    } else {
      // ---- choose the tile: the candidate that takes the most gates in this pass and the best
      // next pass together (one pass of lookahead), ties to the larger first pass
      int best = -1, best_first = -1;
      for (uint64_t T : candidates(rem)) {
        std::vector<int> tk;
        int cnt = 0;
        scan(rem, gates, T, backward, kMaxSlotsPerPass, kMaxOpsPerPass, &tk, &cnt);
        if (cnt <= 0) continue;
        int next = 0;
        if (cnt < (int)rem.size()) {
          std::vector<char> in(gates.size(), 0);
          for (int k : tk) in[k] = 1;
          std::vector<int> rest;
          rest.reserve(rem.size() - tk.size());
          for (int k : rem)
            if (!in[k]) rest.push_back(k);
          for (uint64_t T2 : candidates(rest)) {
            int c2 = 0;
            scan(rest, gates, T2, backward, kMaxSlotsPerPass, kMaxOpsPerPass, nullptr, &c2);
            next = std::max(next, c2);
          }
        }
        if (cnt + next > best || (cnt + next == best && cnt > best_first)) {
          best = cnt + next;
          best_first = cnt;
          bestT = T;
        }
      }
      if (best <= 0) {
        if (msg) *msg = "a gate does not fit any tile";
        return false;
      }
      int cnt = 0;
      scan(rem, gates, bestT, backward, kMaxSlotsPerPass, kMaxOpsPerPass, &taken, &cnt);
    }

    PassDesc pd;
    std::memset(&pd, 0, sizeof pd);
    pd.nt = t;
    int tb_of[64];
    for (int q = 0; q < 64; ++q) tb_of[q] = -1;
    int s = 0, o = 0;
    for (int q = 0; q < n; ++q) {
      if ((bestT >> q) & 1) {
        tb_of[q] = s;
        pd.tile[s++] = (int8_t)q;
      } else {
        pd.outer[o++] = (int8_t)q;
        pd.outer_mask |= 1ull << q;
      }
    }
    while (s < t) pd.tile[s++] = -1;  // phantom tile bits
    pd.n_outer = o;
    pd.phase_begin = (int32_t)out.phases.size();
    pd.op_begin = (int32_t)out.ops.size();
    pd.slot_begin = (int32_t)out.slot_map.size();
    const int pass_id = (int32_t)out.passes.size();
    out.tile_mask.push_back(bestT);

    // ---- register phases inside the pass
    const uint32_t dmask = ((1u << t) - 1) & ~((1u << w) - 1);  // layout D register bits
    std::vector<int> prem(taken);
    std::vector<int> placed;
    int lslot = 0;
    int blocks_left = kMaxDiagBlocks, records_left = kMaxOpsPerPass - (int)taken.size();
    uint32_t prev_R = 0;  // register bits of the previous phase of the pass
    // rotation macros: the members after a head are stored past the executed ops of the pass
    std::vector<FusedOp> members;
    std::vector<std::pair<size_t, size_t>> heads;  // (op index, first member in `members`)
    // phases up to the staging limit; gates left over return to the remaining sequence (the
    // phase scan is itself a blocked scan, so they only follow gates they commute with)
    while (!prem.empty() && (int)out.phases.size() - pd.phase_begin < kMaxPhasesPerPass) {
      uint32_t R = 0;
      uint64_t blocked = 0;
      std::vector<int> ph;
      std::vector<int> left;
      // prefer the direct layout if the first gate that needs registers fits in it
      for (int k : prem) {
        const uint64_t m = qmask(gates[k]);
        if (m & blocked) {
          blocked |= m;
          left.push_back(k);
          continue;
        }
        uint32_t need = 0;
        for (uint64_t rn = regneed(gates[k]); rn; rn &= rn - 1) need |= 1u << tb_of[__builtin_ctzll(rn)];
        if (popc(R | need) <= r) {
          R |= need;
          ph.push_back(k);
        } else {
          blocked |= m;
          left.push_back(k);
        }
      }
      // complete the register set: direct-layout bits first, then the lowest free bits above
      // the contiguous runs (so that the phase can still load or store its tiles directly),
      // then any
      for (uint32_t d = dmask & ~R; d && popc(R) < r; d &= d - 1) R |= d & (~d + 1);
      for (int b = c; b < t && popc(R) < r; ++b) R |= 1u << b;
      for (int b = 0; b < t && popc(R) < r; ++b) R |= 1u << b;

      PhaseDesc P;
      std::memset(&P, 0, sizeof P);
      int regpos[kMaxTileBits];
      int kk = 0;
      for (int b = 0; b < t; ++b)
        if ((R >> b) & 1) {
          regpos[b] = kk;
          P.regbit[kk++] = (int8_t)b;
        } else {
          regpos[b] = -1;
        }
      const int phase_id = (int32_t)out.phases.size();
      uint64_t rphys = 0;
      for (int k2 = 0; k2 < r; ++k2)
        if (pd.tile[P.regbit[k2]] >= 0) rphys |= 1ull << pd.tile[P.regbit[k2]];
      out.reg_mask.push_back(rphys);
      std::vector<std::pair<int, FusedOp>> emitted;  // (gate, op) in execution order
      for (int k : ph) {
        const GateDesc& g = gates[k];
        FusedOp op;
        std::memset(&op, 0, sizeof op);
        op.gate = k;
        const int b0 = tb_of[g.q0], b1 = kind_nqubits(g.kind) == 2 ? tb_of[g.q1] : 0;
        const int np = backward ? kind_nparams(g.kind) : 0;
        op.np = (uint8_t)np;
        auto locate0 = [&](int b) {
          op.s0 = (uint8_t)b;
          if (regpos[b] >= 0) {
            op.flags |= FOPF_S0_REG;
            op.ks0 = (uint8_t)regpos[b];
          }
        };
        auto locate1 = [&](int b) {
          op.s1 = (uint8_t)b;
          if (regpos[b] >= 0) {
            op.flags |= FOPF_S1_REG;
            op.ks1 = (uint8_t)regpos[b];
          }
        };
        switch (g.kind) {
          case K_RY:
            op.type = FOP_RY; op.k0 = (uint8_t)regpos[b0];
            break;
          case K_RX:
            op.type = FOP_RX; op.k0 = (uint8_t)regpos[b0];
            break;
          case K_H: case K_X: case K_Y:
            op.type = FOP_DENSE1; op.k0 = (uint8_t)regpos[b0];
            break;
          case K_U3:
            op.type = FOP_PDENSE1; op.k0 = (uint8_t)regpos[b0];
            break;
          case K_NRX: case K_NRY: case K_NRZ:
            op.type = FOP_NDENSE1; op.k0 = (uint8_t)regpos[b0];
            break;
          case K_RZ:
            op.type = FOP_RZ; locate0(b0);
            break;
          case K_Z: case K_S: case K_T: case K_SDG:
            op.type = FOP_DIAG1; locate0(b0);
            break;
          case K_PHASE:
            op.type = FOP_PDIAG1; locate0(b0);
            break;
          case K_CNOT:
            op.type = FOP_CNOT; locate0(b0); op.k0 = (uint8_t)regpos[b1];
            break;
          case K_CZ:
            op.type = FOP_CZ; locate0(b0); locate1(b1);
            break;
          case K_CRX: case K_CRY:
            op.type = FOP_CDENSE1; locate0(b0); op.k0 = (uint8_t)regpos[b1];
            break;
          case K_CRZ: case K_RZZ:
            op.type = FOP_DIAG2; locate0(b0); locate1(b1);
            break;
          case K_RXX: case K_RYY:
            op.type = FOP_DENSE2; op.k0 = (uint8_t)regpos[b0]; op.k1 = (uint8_t)regpos[b1];
            break;
          default:
            if (msg) *msg = "unknown gate kind";
            return false;
        }
        const bool r0 = op.flags & FOPF_S0_REG, r1 = op.flags & FOPF_S1_REG;
        int v = 0;
        switch (op.type) {
          case FOP_RY: case FOP_RX: case FOP_DENSE1: v = op.k0; break;
          case FOP_RZ: case FOP_DIAG1: v = r0 ? op.ks0 : QSV_V_THREAD; break;
          case FOP_CNOT: v = r0 ? 8 * op.ks0 + op.k0 : QSV_V_CTL_THREAD + op.k0; break;
          case FOP_CZ:
            v = r0 && r1 ? 8 * op.ks0 + op.ks1 : r0 ? QSV_V_REG0 + op.ks0
                : r1 ? QSV_V_REG1 + op.ks1 : QSV_V_THREAD;
            break;
          default: v = 0; break;
        }
        op.opc = (uint16_t)QSV_OPC(op.type, v);
        if (op.type >= FOP_FIRST_GENERAL) pd.general = 1;
        emitted.emplace_back(k, op);
      }
      if (macros && r <= kMaxMacroRegBits) {
        form_diagonal_blocks(emitted, backward, blocks_left, records_left);
        form_rotation_macros(emitted, r);
        // reverse sweep: CNOTs with both bits in registers that open a phase entered by a
        // relayout permute the register indices; the relayout's reads take them (rperm) and they
        // are not executed (in the forward sweep few CNOTs open a phase, and the permuted reads
        // cost the forward pass more than they save)
        if (backward && out.phases.size() > (size_t)pd.phase_begin && R != prev_R) {
          size_t m = 0;
          while (m < emitted.size() && emitted[m].second.type == FOP_CNOT &&
                 (emitted[m].second.flags & FOPF_S0_REG))
            ++m;
          if (m > 0) {
            uint32_t q = 0;
            for (int k2 = 0; k2 < r; ++k2) {
              uint32_t v = 1u << k2;
              for (size_t j = m; j-- > 0;) {
                const FusedOp& c = emitted[j].second;
                v ^= ((v >> c.ks0) & 1u) << c.k0;
              }
              q |= v << (4 * k2);
            }
            P.rperm = (uint16_t)q;
            out.n_folded += (int)m;
            for (size_t j = 0; j < m; ++j) {
              placed.push_back(emitted[j].first);
              out.order.push_back(emitted[j].first);
              out.pass_of.push_back(pass_id);
              out.phase_of.push_back(phase_id);
            }
            emitted.erase(emitted.begin(), emitted.begin() + (long)m);
          }
        }
      }
      prev_R = R;
      int members_left = 0, block_left = 0;
      size_t block_head = 0;
      for (auto& e : emitted) {
        const int k = e.first;
        FusedOp& op = e.second;
        if (k < 0) {  // diagonal block head: its members follow
          heads.emplace_back(out.ops.size(), members.size());
          block_head = out.ops.size();
          out.ops.push_back(op);
          block_left = op.s0;
          // the RZ members take consecutive local slots from here (the CZ members take none)
          if (op.np) out.ops[block_head].lslot = (uint8_t)lslot;
          continue;
        }
        const int np = backward ? kind_nparams(gates[k].kind) : 0;
        if (np) {
          op.lslot = (uint8_t)lslot;
          for (int j = 0; j < np; ++j) out.slot_map.push_back(slot_of_gate[k] + j);
          lslot += np;
        }
        if (block_left > 0) {
          members.push_back(op);
          --block_left;
        } else if (op.flags & FOPF_MACRO) {  // products of all r positions, consecutive local slots
          op.np = (uint8_t)(backward ? r : 0);
          op.opc = (uint16_t)QSV_OPC(op.type, QSV_V_MACRO);
          heads.emplace_back(out.ops.size(), members.size());
          out.ops.push_back(op);
          members_left = r - 1;
        } else if (members_left > 0) {
          members.push_back(op);
          --members_left;
        } else {
          out.ops.push_back(op);
        }
        placed.push_back(k);
        out.order.push_back(k);
        out.pass_of.push_back(pass_id);
        out.phase_of.push_back(phase_id);
      }
      P.op_end = (int32_t)out.ops.size() - pd.op_begin;
      out.phases.push_back(P);
      prem.swap(left);
    }
    pd.phase_end = (int32_t)out.phases.size();
    // tiles move in the first / last phase's layout when it keeps the runs on the low lane bits
    if (tq == t && pd.phase_end > pd.phase_begin) {
      auto keeps_runs = [&](const PhaseDesc& P) {
        for (int k2 = 0; k2 < r; ++k2)
          if (P.regbit[k2] < c) return false;
        return true;
      };
      if (keeps_runs(out.phases[pd.phase_begin])) pd.io_flags |= PASS_LOAD_FIRST_PHASE;
      if (keeps_runs(out.phases[pd.phase_end - 1])) pd.io_flags |= PASS_STORE_LAST_PHASE;
    }
    pd.n_slots = lslot;
    pd.n_diag = (int8_t)(kMaxDiagBlocks - blocks_left);
    const size_t n_exec = out.ops.size() - pd.op_begin;
    for (const auto& h : heads) out.ops[h.first].k1 = (uint8_t)(n_exec + h.second);
    out.ops.insert(out.ops.end(), members.begin(), members.end());
    pd.n_ops = (int32_t)out.ops.size() - pd.op_begin;
    out.passes.push_back(pd);

    // drop the executed gates from the remaining sequence
    std::vector<char> done(gates.size(), 0);
    for (int k : placed) done[k] = 1;
    std::vector<int> nrem;
    nrem.reserve(rem.size());
    for (int k : rem)
      if (!done[k]) nrem.push_back(k);
    rem.swap(nrem);
  }
  return true;
}

bool build_forward_schedule(int n, const std::vector<GateDesc>& gates, int t, int r, int w,
                            int run_qubits, const Schedule& bwd, Schedule& out,
                            std::string* msg, bool macros) {
  const int G = (int)gates.size();
  std::vector<int> seq(G);
  for (int k = 0; k < G; ++k) seq[k] = k;
  const std::vector<int32_t> no_slots(G, -1);
  if (!build_schedule(n, gates, seq, no_slots, false, t, r, w, run_qubits, out, msg, macros))
    return false;
  // the reverse sweep's passes, last first, each in forward gate order: every pass is a set of
  // gates that are consecutive in a valid order of the reversed circuit, so the reversed list is
  // a valid order of the circuit
  std::vector<PassPlan> rev(bwd.passes.size());
  for (size_t i = 0; i < bwd.order.size(); ++i) rev[bwd.pass_of[i]].gates.push_back(bwd.order[i]);
  for (size_t p = 0; p < rev.size(); ++p) {
    std::sort(rev[p].gates.begin(), rev[p].gates.end());
    rev[p].tile = bwd.tile_mask[p];
  }
  std::reverse(rev.begin(), rev.end());
  Schedule alt;
  std::string m2;
  if (build_schedule(n, gates, seq, no_slots, false, t, r, w, run_qubits, alt, &m2, macros, &rev) &&
      alt.passes.size() < out.passes.size())
    out = std::move(alt);
  return true;
}

}  // namespace qsv
