// Fused passes: a run of gates applied to every tile of 2^t amplitudes in one HBM round trip.
//
// A pass names t "tile qubits"; a tile is the set of 2^t amplitudes that share the values of all
// other ("outer") qubits. Tile bit s stands for physical qubit tile[s] (ascending). A workgroup of
// 2^w threads holds a tile in registers, 2^r amplitudes per thread (t = r + w). In each "phase" r
// chosen tile bits are register bits (thread-private array index) and the other w bits come from
// the thread index. Gates whose non-diagonal targets are register bits run entirely in registers;
// diagonal gates and controls may sit on any tile bit. Between phases the tile is re-laid out
// through LDS. The direct layout D (thread bits = tile bits 0..w-1, register bits = w..t-1) is the
// one used for the coalesced loads and stores from HBM.
#pragma once

#include <vector>

#include "qsv_internal.h"

namespace qsv {

constexpr int kMaxTileBits = 14;
constexpr int kMaxRegBits = 5;
constexpr int kMaxSlotsPerPass = 128;   // two accumulator registers, one wave lane per slot
constexpr int kMaxOpsPerPass = 256;     // ops of a pass are staged in LDS
constexpr int kMaxPhasesPerPass = 64;

enum FusedOpType : uint8_t {
  // lean op set (every bit location compile-time in registers or constant per thread)
  FOP_RY = 0,       // exp(-i t Y/2) on register position k0
  FOP_RX = 1,       // exp(-i t X/2) on register position k0
  FOP_RZ = 2,       // exp(-i t Z/2) on tile bit s0
  FOP_CNOT = 3,     // control tile bit s0, target register position k0
  FOP_CZ = 4,       // tile bits s0, s1
  FOP_DENSE1 = 5,   // fixed 2x2 on register position k0 (no parameter)
  FOP_DIAG1 = 6,    // fixed diagonal 2x2 on tile bit s0 (no parameter)
  // general op set (parameterised matrices with explicit derivatives, controlled and two-qubit)
  FOP_PDENSE1 = 7,  // 2x2 with 1 or 3 parameters on register position k0 (U3)
  FOP_PDIAG1 = 8,   // diagonal 2x2 with a parameter on tile bit s0 (PHASE)
  FOP_CDENSE1 = 9,  // control tile bit s0, 2x2 block (rows/cols 2,3 of the 4x4) on register k0
  FOP_DIAG2 = 10,   // diagonal 4x4 on tile bits s0 (q0), s1 (q1)
  FOP_DENSE2 = 11,  // 4x4 on register positions k0 (q0), k1 (q1)
  FOP_NDENSE1 = 12, // non-unitary 2x2 with a parameter on register position k0: phi is un-done
                    // by the stored inverse, lambda by the adjoint
  FOP_FIRST_GENERAL = FOP_PDENSE1,
};

// A tile bit referenced by an op (control or diagonal bit) is either a register bit of the phase
// (flag set, register position in ks0/ks1) or a thread bit (its value is constant per thread).
enum : uint8_t { FOPF_S0_REG = 1, FOPF_S1_REG = 2, FOPF_MACRO = 4, FOPF_FLIP = 8, FOPF_DIAG = 16 };
// FOPF_FLIP is set when a pass is staged (never by the scheduler): a rotation whose half angle
// has a negative cosine runs as -1 times a rotation by the half angle minus pi (see OpStage).

// Rotation macros (see form_rotation_macros): a head flagged FOPF_MACRO, op code
// QSV_OPC(type, QSV_V_MACRO), stands for r rotations about one axis, one per register position
// (the head is position 0). The records of positions 1 .. r - 1 sit after the executed ops of the
// pass, from op index k1 of the pass on. The head's np counts the products of all r
// (consecutive local slots). Only for r <= kMaxMacroRegBits.
constexpr int kMaxMacroRegBits = 4;

// Diagonal blocks: consecutive diagonal gates of a phase whose bits are all register bits (RZ,
// and CZ with both bits in registers) commute and act as one diagonal matrix d on the thread's
// 2^r amplitudes. A head (type FOP_RZ, flag FOPF_DIAG, op code QSV_OPC(FOP_RZ, QSV_V_DIAG))
// stands for them: its s0 member records (the gates, in run order) sit after the executed ops
// of the pass from op index k1 on; np counts the RZ members (their products, consecutive local
// slots from lslot) and gate holds their register positions, four bits each. When the pass is
// staged, d is computed from the members into table ks1 of the pass (2^r complex entries).
// Products of the reverse sweep are taken once for the block: Z of a member and the other
// members commute, so Im <lambda|Z_k|phi> is the same at every point of the block.
// Only for r <= kMaxMacroRegBits; at most kMaxDiagBlocks blocks per pass.
constexpr int kMaxDiagBlocks = 24;

struct FusedOp {
  uint8_t type;
  uint8_t k0, k1;   // register positions of targets
  uint8_t s0, s1;   // tile bits (controls, diagonal bits)
  uint8_t np;       // products (derivative parameters) of this op in the reverse sweep
  uint8_t lslot;    // local slot of the first product
  uint8_t flags;    // FOPF_*
  uint8_t ks0, ks1; // register positions of s0 / s1 when they are register bits
  uint16_t opc;     // lean op code QSV_OPC(type, variant), see below
  int32_t gate;     // gate record index
};

// Op codes of the lean ops: type * 64 + variant, the variant naming the register positions:
//   RY, RX, DENSE1: k0;  RZ, DIAG1: ks0, or QSV_V_THREAD for a thread bit;
//   CNOT: 8 * ks0 + k0 (register control), QSV_V_CTL_THREAD + k0 (thread control);
//   CZ: 8 * ks0 + ks1 (both register bits), QSV_V_REG0 + ks0 (only s0 in registers),
//       QSV_V_REG1 + ks1 (only s1 in registers), QSV_V_THREAD (both thread bits).
#define QSV_OPC(T, V) ((T) * 64 + (V))
#define QSV_V_REG0 40
#define QSV_V_REG1 48
#define QSV_V_CTL_THREAD 48
#define QSV_V_THREAD 63
#define QSV_V_MACRO 32  // RX/RY/RZ: a rotation macro head
#define QSV_V_DIAG 36   // RZ: a diagonal block head

// Tiles of a pass are loaded in the first phase's layout (stored from the last phase's) instead
// of the direct layout when that phase keeps the contiguous runs on the low lane bits (none of
// its register bits is one of the low run qubits) and the pass has no phantom bits: the relayout
// after the loads (before the stores) is then skipped.
enum : uint8_t { PASS_LOAD_FIRST_PHASE = 1, PASS_STORE_LAST_PHASE = 2 };

struct PhaseDesc {
  int32_t op_end;                 // ops [previous op_end, op_end) of the pass
  int8_t regbit[kMaxRegBits];     // tile bit of each register position
  uint8_t pad;
  // 0, or (reverse sweep) the register-index map of CNOTs with both bits in registers that open
  // the phase, taken into the relayout before it: register ri reads the element of index Q(ri), Q linear
  // over GF(2) with Q(e_k) in bits 4k .. 4k + 3 (reg_qubits <= 4)
  uint16_t rperm;
};

struct PassDesc {
  uint64_t outer_mask;            // physical qubits outside the tile
  int32_t nt;                     // tile bits t
  int32_t n_outer;                // N - t
  int8_t tile[kMaxTileBits];      // physical qubit of tile bit s (ascending)
  uint8_t io_flags;               // PASS_LOAD_FIRST_PHASE | PASS_STORE_LAST_PHASE
  int8_t n_diag;                  // diagonal blocks (their tables are staged with the pass)
  int8_t outer[40];               // physical qubits outside the tile (ascending)
  int32_t phase_begin, phase_end; // into the phase table
  int32_t op_begin;               // into the op table (phase op_end values are relative)
  int32_t n_slots;                // products accumulated by this pass
  int32_t slot_begin;             // into the slot map (local slot -> global reduction slot)
  int32_t general;                // 1 if any op of the pass is of the general set
  int32_t n_ops;                  // ops of the pass
};

// One unit of work of a fused launch: one pass of one circuit over all of its tiles. A launch
// takes a table of items (several circuits of a batch, or one pass of one circuit) and splits the
// concatenated tiles into contiguous chunks, one per workgroup. Items are built on the host and
// hold device pointers only.
struct PassItem {
  PassDesc pd;          // the pass (a copy: one load gives the kernel its whole description)
  const PhaseDesc* phases;
  const FusedOp* ops;
  const GateRec* recs;
  const int32_t* slot_map;
  const void* src;      // forward: state read by the pass
  void* dst;            // forward: state written (may equal src); backward: phi
  void* lam;            // backward: lambda. Forward (reference gradient): if set, the item ends
                        // with Re <lam|state> per workgroup in partials[] instead of a store
  double2* partials;    // backward: this item's block of partials, [local slot][workgroup]
  int64_t tile_begin;   // first tile of the item in the launch's concatenated tile range
  int32_t n_outer;      // log2 of the item's tile count
  int32_t first_wg;     // first workgroup whose chunk reaches into the item
  int32_t nb;           // workgroups whose chunks reach into the item (partials stride)
  int32_t sub_op;       // forward, general instance: pass-local op applied as its derivative
                        // in parameter sub_param instead of its matrix (-1: none)
  int32_t sub_param;
  int32_t pad;
};

// An op as staged in LDS at the start of a pass: the op record and, for RX/RY/RZ, the shear
// factors of its rotation. Each such gate is a plane rotation by phi = t/2 of pairs of real
// components (RY: (re a0, re a1), (im a0, im a1); RX and RZ: real/imaginary pairs), applied in
// place as three shears x += alpha y, y += beta x, x += alpha y with alpha = -tan(phi/2) and
// beta = sin(phi). When cos(phi) < 0 the gate runs as -1 times the rotation by phi - pi
// (FOPF_FLIP set), which keeps |alpha|, |beta| <= 1; the sign is carried per tile and applied
// when the tile is stored (the products of the reverse sweep see it on phi and lambda alike).
struct alignas(16) OpStage {
  FusedOp op;
  double alpha, beta;
};

// A schedule of one gate sequence (forward order, or the reverse sweep) as host tables ready to
// be copied to the device.
struct Schedule {
  int t = 0, r = 0, w = 0;
  std::vector<PassDesc> passes;
  std::vector<PhaseDesc> phases;
  std::vector<FusedOp> ops;
  std::vector<int32_t> slot_map;
  // for inspection: gate order and pass/phase of each executed gate (order[i] is the gate of
  // ops[i] when the schedule has no rotation macros)
  std::vector<int32_t> order, pass_of, phase_of;
  std::vector<uint64_t> tile_mask, reg_mask;
  int n_folded = 0;  // CNOTs taken into a relayout (PhaseDesc::rperm) instead of executed
};

// Builds the schedule of `gates` taken in order `seq` (gate indices). slot_of_gate[k] is the first
// global reduction slot of gate k (or -1); it is only used when `backward` is set. Every tile
// holds qubits 0 .. run_qubits - 1 (see run_qubits_for). With `given`, the passes are not chosen
// but taken from that list (which must cover `seq` in a valid order). `macros`
// allows rotation macros (off for schedules whose ops are addressed one by one, as the
// derivative substitution of Algorithm 2 does). Returns false (with msg) if the gates cannot be
// scheduled with these sizes.
// A pass given in advance: its tile (physical-qubit mask) and gates in execution order.
struct PassPlan {
  uint64_t tile = 0;
  std::vector<int> gates;
};

bool build_schedule(int n, const std::vector<GateDesc>& gates, const std::vector<int>& seq,
                    const std::vector<int32_t>& slot_of_gate, bool backward, int t, int r, int w,
                    int run_qubits, Schedule& out, std::string* msg, bool macros = true,
                    const std::vector<PassPlan>* given = nullptr);

// The forward schedule: the scheduler's own, or the reverse sweep's passes taken last to first
// (each in forward gate order) if those are fewer.
bool build_forward_schedule(int n, const std::vector<GateDesc>& gates, int t, int r, int w,
                            int run_qubits, const Schedule& bwd, Schedule& out,
                            std::string* msg, bool macros = true);

// Lowest qubits every tile holds, so that loads and stores move contiguous runs: fewer forced
// qubits leave more tile bits to the scheduler (fewer passes), shorter runs use cache lines
// (128 bytes) less well. Complex128: 3 (8 amplitudes, one line; 2 measured slower at 20 and 30
// qubits). Complex64: 4 (16 amplitudes, one line) for states streamed from HBM, 3 (half a line)
// for states of up to 24 qubits (128 MB), which stay in the 256 MB Infinity Cache (20 qubits:
// 1.42 -> 1.37 ms per gradient; at 26 qubits half lines measured 3 % slower).
inline int run_qubits_for(bool c128, int n) { return c128 ? 3 : (n <= 24 ? 3 : 4); }

// Geometries (r, w) with a fused kernel instance whose amplitude registers do not spill (reverse
// sweep: two states per thread); the launchers in fused_kernels.hip instantiate exactly these.
inline bool fused_config_supported(int r, int w, bool c128) {
  if (w == 9) return r >= 2 && r <= (c128 ? 3 : 4);
  if (w == 8) return r >= 2 && r <= 4;
  if (w == 6) return r >= 2 && r <= 3;
  return false;
}

// Launch over `n_items` items whose tiles total `total`; workgroup w takes tiles
// [w * chunk, (w + 1) * chunk). `general` selects the kernel instance that also handles the
// general op set.
template <typename R>
hipError_t launch_fused_forward(const PassItem* d_items, int n_items, int64_t total, int64_t chunk,
                                int r, int w, bool general, int grid, hipStream_t st);

// cplx: complex entries <lambda|mu> (non-Hermitian operators); runs the general instance.
template <typename R>
hipError_t launch_fused_backward(const PassItem* d_items, int n_items, int64_t total,
                                 int64_t chunk, int r, int w, bool general, int grid,
                                 hipStream_t st, bool cplx = false);

}  // namespace qsv
