// Host-side planner: validates a gate stream and rewrites it into layers.
//
// The rewrite is exact in exact arithmetic (paper, Section "Semantics-
// Preserving Fusion"): only consecutive gates of one class are merged, gates
// are reordered only when they commute, and numeric collapse tests (identity,
// Hadamard, bit flip) use a tolerance of a few ulps on complex128 products so
// that a small rotation such as RZ(1e-6) is never dropped.
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "layout.h"
#include "qs.h"

namespace qs {

using cd = std::complex<double>;

struct Error {
  qs_status code;
  std::string msg;
};
[[noreturn]] void fail(qs_status code, const std::string& msg);

// Angle = c0 + sum_k coef_k * params[k]  (kept symbolic so that parameters can
// be re-bound without re-planning).
struct Angle {
  double c0 = 0.0;
  std::vector<std::pair<int32_t, double>> lin;  // sorted by parameter index
  bool is_const() const { return lin.empty(); }
  double eval(const std::vector<double>& p) const;
  Angle plus(const Angle& o) const;
  Angle scaled(double s) const;
  bool same(const Angle& o) const;  // bit-identical
};

// A validated gate with wires converted to state bit positions.
struct NGate {
  int32_t kind = 0;
  std::vector<int> bits;   // listed order (controls first, target last)
  uint32_t all_mask = 0;   // MCZ / MCP support
  Angle angle;
  std::vector<cd> mat;     // U, CU (2x2), UNITARY (2^k x 2^k)
  int32_t index = 0;       // position in the stream (first gate of a fused window)
  int32_t fused = 0;       // > 0: a dense window standing for this many consecutive gates
};

bool gate_is_diagonal(int kind);
int gate_arity(const qs_gate& g);
// Dense matrix of a gate (2^k x 2^k, row-major, first listed wire = most
// significant row bit; MCZ/MCP over their sorted support bits, highest bit
// first).  Angles evaluated with params.
std::vector<cd> gate_matrix(const NGate& g, const std::vector<double>& params);

// ---- layer IR -------------------------------------------------------------------
struct DiagTermIR {
  int32_t type;     // 0 BIT, 1 XOR pair, 2 AND pair, 3 ALL (k >= 3), 4 PARITY (k >= 3)
  uint32_t mask;
  Angle angle;
};
struct DiagGroupIR {
  Angle angle;
  std::vector<DiagTerm> terms;  // device count terms
  int32_t max_count = 0;
};
struct DiagIR {
  std::vector<DiagGroupIR> groups;
  Angle global;
  uint32_t support = 0;
  std::vector<DiagTermIR> raw;  // the merged terms the groups were built from
};

// One butterfly operation of a tile pass.
struct OpIR {
  int32_t kind;  // TileOpKind
  int32_t bit;   // state bit
  // OP_MAT / OP_DIAG: the single-qubit window on this wire, gates in stream
  // order (the op's matrix is their product).
  std::vector<int32_t> gates;
  bool fixed_h = false;  // OP_H produced by a basis change (no source gates)
  int32_t fixed_mat = -1;  // basis-change matrix id (0: H S^dagger, 1: S H)
  int32_t base = 0;        // OP_QFT / OP_QFT_INV: the register's lowest state bit
};

struct ItemIR {
  int32_t type;  // 0 op, 1 diag
  int32_t index; // into Plan::ops or Plan::diags
};

struct TilePassIR {
  int32_t L, a, h;           // tile bits [0, L) U [a, a+h)
  std::vector<ItemIR> items; // in execution order
  // built by finalize(): rounds and ops in device form (coef offsets are
  // relative to this pass's coefficient array)
  std::vector<TileRound> rounds;
  std::vector<TileOp> ops;
  std::vector<int32_t> op_src;   // OpIR index per device op (or -1 for QFT-only ops)
  std::vector<int32_t> diag_slots;  // DiagIR index per slot
  int32_t n_coef = 0;
  int32_t n_butterfly = 0;  // unscaled H / QFT butterflies in the pass
  double scale = 1.0;       // 2^(-n_butterfly/2), applied at the store
  bool inverse = false;     // ops are inverses of their sources (U^dagger, QFT^-1, conj diagonals)
};

struct Gf2IR {
  std::vector<uint32_t> rows;  // A rows: src bit r = parity(rows[r] & y)
  uint32_t cprime = 0;
  std::vector<int32_t> gates;  // source gates (for describe)
};

enum LayerKind : int32_t { L_DIAG = 0, L_TILE = 1, L_GF2 = 2, L_PLAIN = 3, L_DENSE = 4 };

// A dense k-qubit block (k = 4..6) for the matrix cores: the gate's matrix with
// row / column index bit u on the state bit bits[u] (ascending), and its
// conjugate transpose for the inverse plan.
struct DenseIR {
  int32_t gate = 0;          // index into Plan::gates
  std::vector<int> bits;     // ascending
  std::vector<cd> mat, mat_dagger;
};

struct LayerIR {
  int32_t kind;
  int32_t index;  // into diags / passes / gf2s / plain gate index (into Plan::gates)
  int32_t inverse = 0;  // L_DIAG / L_PLAIN: apply the inverse (conjugate / dagger)
};

struct PlanOptions {
  int mode = QS_FUSED;
  int max_tile_bits = 0;  // 0 = default by dtype at apply time
  int dense_k_max = 6;    // largest UNITARY gate run as a dense block (< 4: none)
  int window_k = 5;       // dense-window fusion: largest window (< 4: off)
  int coset_order = 0;    // tile passes' workgroup -> coset order: 0 by geometry,
                          // 1 XCD-blocked, 2 launch order
  int diag_low_bits = 0;  // high tile passes carrying diagonal layers: 0 default,
                          // -1 the group's low bits, k > 0 at most k low bits
  int balance_passes = 0; // >= 0: ops after a pass's last diagonal may move to
                          // the next tile pass to even out the two (-1: off)
};

struct PlanIR {
  int n = 0;
  size_t n_params = 0;
  PlanOptions opt;
  std::vector<NGate> gates;
  std::vector<DiagIR> diags;
  std::vector<OpIR> ops;
  std::vector<TilePassIR> passes;
  std::vector<Gf2IR> gf2s;
  std::vector<DenseIR> denses;
  std::vector<LayerIR> layers;
  int tile_bits = 13;  // tile size used to build the passes
  int low_bits = 0;    // L of high tiles (0: per group, tile_bits - h)
  int windows = 0;     // dense windows formed by window fusion (0: structured plan)
};

// Estimated cost of a plan in state passes (a dense block of 5 or 6 bits
// costs more than one pass: its arithmetic leaves the memory-bound regime).
double plan_cost(const PlanIR& P);
// Dense-window fusion of a gate stream: consecutive constant gates are
// collected into windows of at most kmax bits (open windows on disjoint bits,
// so reordering them is exact) and every window of two or more gates on two
// or more bits becomes one UNITARY gate, padded with identity bits to at least
// 4 bits.  Returns the number of windows formed.
int fuse_windows(int n, const std::vector<NGate>& in, int kmax, std::vector<NGate>& out);

// Optional observer of the planner's phases (the library installs one that
// opens and closes profiler ranges; none by default).
using PlanPhaseHook = void (*)(const char* phase, bool begin);
void set_plan_phase_hook(PlanPhaseHook hook);

// Validate + normalise the user's gates.
std::vector<NGate> normalise_gates(int n, const qs_gate* g, size_t count, size_t n_params);
// Build the plan.  tile_bits / low_bits fix the tile geometry.
PlanIR build_plan(int n, std::vector<NGate> gates, size_t n_params, const PlanOptions& opt,
                  int tile_bits, int low_bits);

// ---- numeric materialisation ----------------------------------------------------
// LUT of one diagonal layer (complex128) and per-pass coefficients.
struct DiagNumeric {
  std::vector<DiagTerm> terms;
  std::vector<DiagGroup> groups;
  std::vector<cd> lut;
  std::vector<double> theta;  // per group: its angle reduced to [-pi, pi]
  double global = 0.0;        // global phase angle, reduced
};
// x mod 2 pi in [-pi, pi], against 2 pi carried in two doubles.
double reduce_2pi(double x);
DiagNumeric diag_numeric(const DiagIR& d, const std::vector<double>& params, bool conj = false);
// A group whose count is a sum of distinct bit-pair mismatches (every term
// DT_SHIFT_XOR; bit j of a term's mask pairs state bits j and j + shift, a
// partner at or above bit n being a constant zero): per state bit p its real
// partners N_p and its number of pairs deg_p, so that setting a zero bit p of
// i changes the count by deg_p - 2 popcount(N_p & i).  ok = false otherwise.
struct PairNeighbours {
  bool ok = false;
  uint32_t mask[32] = {0};
  int32_t deg[32] = {0};
};
std::vector<PairNeighbours> pair_neighbours(const DiagNumeric& num, int n);
// Diagonal observable sum_t c_t Z-string_t as value(i) = global + sum_g angle_g
// count_g(i) (the groups' "angles" are the real weights -2 c).
DiagIR diag_observable(int n, const qs_pauli* terms, size_t n_terms);
std::vector<cd> pass_coefficients(const PlanIR& p, const TilePassIR& t, const std::vector<double>& params);
// Device form of a pass's rounds and coefficients (RX / RY refinements applied).
std::vector<cd> pass_coefficients_device(const PlanIR& p, const TilePassIR& t, const std::vector<double>& params,
                                         std::vector<TileRound>& rounds);
cd op_matrix_entry(const PlanIR& p, const OpIR& op, const std::vector<double>& params, int r, int c);
std::vector<cd> op_matrix(const PlanIR& p, const OpIR& op, const std::vector<double>& params);
Gf2Args gf2_args(int n, const Gf2IR& g, int c_bits);

std::string describe_json(const PlanIR& p, const std::vector<double>& params, bool bound);

// ---- adjoint support ------------------------------------------------------------
// The inverse plan: layers in reverse order, each replaced by its inverse.
PlanIR invert_plan(const PlanIR& p);
// Dagger of a gate's matrix.
std::vector<cd> dagger(const std::vector<cd>& M, int d);

// One parameter occurrence of a forward layer: dE/dparam += coef * 2 Re <lambda|K|phi>
// evaluated on the states before the layer.  kind 0: K is a 2x2 matrix on state
// bit `bit`; kind 1: K = i * count_g (diagonal group g of diag layer `diag`).
struct GradEntry {
  int32_t kind;
  int32_t bit;
  int32_t param;
  double coef;
  cd K[4];
  int32_t diag;
  int32_t group;
};
// Entries of every forward layer (index = forward layer).  Fails with
// QS_EUNSUPPORTED for parameters the adjoint sweep cannot isolate.
std::vector<std::vector<GradEntry>> grad_entries(const PlanIR& p, const std::vector<double>& params);

}  // namespace qs
