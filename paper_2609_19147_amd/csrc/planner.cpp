// Host planner: gate validation, structure detection, tile-pass scheduling and
// numeric tables.  See planner.h for the contract.  No HIP calls in this file:
// plans can be built and inspected without a GPU.
#include "planner.h"

#include <algorithm>
#include <iomanip>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <sstream>
#include <unordered_map>

namespace qs {

namespace {
PlanPhaseHook g_phase_hook = nullptr;

struct Phase {
  const char* name;
  explicit Phase(const char* n) : name(n) {
    if (g_phase_hook) g_phase_hook(name, true);
  }
  ~Phase() {
    if (g_phase_hook) g_phase_hook(name, false);
  }
};
}  // namespace

void set_plan_phase_hook(PlanPhaseHook hook) { g_phase_hook = hook; }


void fail(qs_status code, const std::string& msg) { throw Error{code, msg}; }

static const double kPi = 3.14159265358979323846;
// Collapse tolerance on complex128 window products (a few ulps): identity,
// Hadamard and bit-flip recognition never swallows a real small rotation.
static const double kCollapseTol = 8.0 * 1.1102230246251565e-16;

// ---------------------------------------------------------------- Angle
double Angle::eval(const std::vector<double>& p) const {
  double v = c0;
  for (auto& t : lin) v += t.second * p[t.first];
  return v;
}
Angle Angle::plus(const Angle& o) const {
  Angle r;
  r.c0 = c0 + o.c0;
  std::map<int32_t, double> m;
  for (auto& t : lin) m[t.first] += t.second;
  for (auto& t : o.lin) m[t.first] += t.second;
  for (auto& t : m)
    if (t.second != 0.0) r.lin.push_back(t);
  return r;
}
Angle Angle::scaled(double s) const {
  Angle r;
  r.c0 = c0 * s;
  for (auto& t : lin) r.lin.push_back({t.first, t.second * s});
  return r;
}
bool Angle::same(const Angle& o) const {
  if (std::memcmp(&c0, &o.c0, sizeof(double)) != 0) return false;
  if (lin.size() != o.lin.size()) return false;
  for (size_t i = 0; i < lin.size(); ++i)
    if (lin[i].first != o.lin[i].first || std::memcmp(&lin[i].second, &o.lin[i].second, 8) != 0)
      return false;
  return true;
}

// ---------------------------------------------------------------- gates
bool gate_is_diagonal(int k) {
  switch (k) {
    case QS_GATE_I: case QS_GATE_Z: case QS_GATE_S: case QS_GATE_SDG: case QS_GATE_T:
    case QS_GATE_TDG: case QS_GATE_RZ: case QS_GATE_P: case QS_GATE_CZ: case QS_GATE_CPHASE:
    case QS_GATE_RZZ: case QS_GATE_MCZ: case QS_GATE_MCP:
      return true;
    default:
      return false;
  }
}

static bool kind_has_angle(int k) {
  switch (k) {
    case QS_GATE_RX: case QS_GATE_RY: case QS_GATE_RZ: case QS_GATE_P: case QS_GATE_CPHASE:
    case QS_GATE_RZZ: case QS_GATE_RXX: case QS_GATE_RYY: case QS_GATE_MCP:
      return true;
    default:
      return false;
  }
}

int gate_arity(const qs_gate& g) {
  switch (g.kind) {
    case QS_GATE_I: case QS_GATE_H: case QS_GATE_X: case QS_GATE_Y: case QS_GATE_Z:
    case QS_GATE_S: case QS_GATE_SDG: case QS_GATE_T: case QS_GATE_TDG: case QS_GATE_SX:
    case QS_GATE_RX: case QS_GATE_RY: case QS_GATE_RZ: case QS_GATE_P: case QS_GATE_U:
      return 1;
    case QS_GATE_CNOT: case QS_GATE_CZ: case QS_GATE_CPHASE: case QS_GATE_SWAP:
    case QS_GATE_RZZ: case QS_GATE_RXX: case QS_GATE_RYY: case QS_GATE_CU:
      return 2;
    case QS_GATE_MCZ: case QS_GATE_MCP:
      return 0;  // from mask
    case QS_GATE_UNITARY:
      return -1;  // from nw
    default:
      return -2;
  }
}

std::vector<NGate> normalise_gates(int n, const qs_gate* g, size_t count, size_t n_params) {
  const Phase ph("qs.plan.normalise");
  if (n < 1 || n > QS_MAX_QUBITS) fail(QS_EINVAL, "qubit count out of range");
  if (count > 0 && !g) fail(QS_EINVAL, "gate array is NULL");
  std::vector<NGate> out;
  out.reserve(count);
  for (size_t i = 0; i < count; ++i) {
    const qs_gate& q = g[i];
    char where[64];
    std::snprintf(where, sizeof where, "gate %zu: ", i);
    int ar = gate_arity(q);
    if (ar == -2) fail(QS_EINVAL, std::string(where) + "unknown kind");
    NGate ng;
    ng.kind = q.kind;
    ng.index = (int32_t)i;
    std::vector<int> wires;
    if (ar == 0) {
      if (q.mask == 0 || (n < 64 && (q.mask >> n) != 0))
        fail(QS_EINVAL, std::string(where) + "multi-controlled mask empty or out of range");
      for (int w = 0; w < n; ++w)
        if ((q.mask >> w) & 1) wires.push_back(w);
    } else {
      int k = ar == -1 ? q.nw : ar;
      if (ar == -1 && (k < 1 || k > QS_MAX_GATE_WIRES))
        fail(QS_EINVAL, std::string(where) + "UNITARY wire count out of range");
      if (q.nw != k) fail(QS_EINVAL, std::string(where) + "wire count does not match kind");
      for (int j = 0; j < k; ++j) wires.push_back(q.wires[j]);
    }
    std::set<int> seen;
    for (int w : wires) {
      if (w < 0 || w >= n) fail(QS_EINVAL, std::string(where) + "wire out of range");
      if (!seen.insert(w).second) fail(QS_EINVAL, std::string(where) + "duplicate wire");
      ng.bits.push_back(n - 1 - w);
    }
    if (ar == 0)
      for (int b : ng.bits) ng.all_mask |= 1u << b;
    if (q.param >= 0) {
      if (!kind_has_angle(q.kind)) fail(QS_EINVAL, std::string(where) + "parameter on a fixed gate");
      if ((size_t)q.param >= n_params) fail(QS_EINVAL, std::string(where) + "parameter index out of range");
      ng.angle.c0 = q.theta;
      if (q.scale != 0.0) ng.angle.lin.push_back({q.param, q.scale});
    } else if (q.param < -1) {
      fail(QS_EINVAL, std::string(where) + "negative parameter index");
    } else {
      ng.angle.c0 = q.theta;
    }
    if (!std::isfinite(q.theta) || (q.param >= 0 && !std::isfinite(q.scale)))
      fail(QS_EINVAL, std::string(where) + "non-finite angle");
    if (q.kind == QS_GATE_U || q.kind == QS_GATE_CU || q.kind == QS_GATE_UNITARY) {
      if (!q.mat) fail(QS_EINVAL, std::string(where) + "matrix missing");
      int d = q.kind == QS_GATE_UNITARY ? (1 << q.nw) : 2;
      ng.mat.resize((size_t)d * d);
      for (int e = 0; e < d * d; ++e) {
        double re = q.mat[2 * e], im = q.mat[2 * e + 1];
        if (!std::isfinite(re) || !std::isfinite(im))
          fail(QS_EINVAL, std::string(where) + "non-finite matrix entry");
        ng.mat[e] = cd(re, im);
      }
    }
    out.push_back(std::move(ng));
  }
  return out;
}

static std::vector<cd> m2(cd a, cd b, cd c, cd d) { return {a, b, c, d}; }

std::vector<cd> gate_matrix(const NGate& g, const std::vector<double>& params) {
  const cd I(0, 1);
  double t = g.angle.eval(params);
  double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
  const double r = 1.0 / std::sqrt(2.0);
  switch (g.kind) {
    case QS_GATE_I: return m2(1, 0, 0, 1);
    case QS_GATE_H: return m2(r, r, r, -r);
    case QS_GATE_X: return m2(0, 1, 1, 0);
    case QS_GATE_Y: return m2(0, -I, I, 0);
    case QS_GATE_Z: return m2(1, 0, 0, -1);
    case QS_GATE_S: return m2(1, 0, 0, I);
    case QS_GATE_SDG: return m2(1, 0, 0, -I);
    case QS_GATE_T: return m2(1, 0, 0, std::polar(1.0, kPi / 4));
    case QS_GATE_TDG: return m2(1, 0, 0, std::polar(1.0, -kPi / 4));
    case QS_GATE_SX: return m2(cd(0.5, 0.5), cd(0.5, -0.5), cd(0.5, -0.5), cd(0.5, 0.5));
    case QS_GATE_RX: return m2(c, -I * s, -I * s, c);
    case QS_GATE_RY: return m2(c, -s, s, c);
    case QS_GATE_RZ: return m2(cd(c, -s), 0, 0, cd(c, s));
    case QS_GATE_P: return m2(1, 0, 0, std::polar(1.0, t));
    case QS_GATE_U: return g.mat;
    default: break;
  }
  int k = (int)g.bits.size();
  int d = 1 << k;
  std::vector<cd> M((size_t)d * d, cd(0, 0));
  auto id = [&]() { for (int i = 0; i < d; ++i) M[(size_t)i * d + i] = 1; };
  switch (g.kind) {
    case QS_GATE_CNOT: id(); M[10] = 0; M[15] = 0; M[11] = 1; M[14] = 1; break;
    case QS_GATE_CZ: id(); M[15] = -1; break;
    case QS_GATE_CPHASE: id(); M[15] = std::polar(1.0, t); break;
    case QS_GATE_SWAP: M[0] = 1; M[6] = 1; M[9] = 1; M[15] = 1; break;
    case QS_GATE_RZZ:
      M[0] = cd(c, -s); M[5] = cd(c, s); M[10] = cd(c, s); M[15] = cd(c, -s); break;
    case QS_GATE_RXX:
      id(); for (int i = 0; i < 4; ++i) M[i * 4 + i] = c;
      M[3] = M[6] = M[9] = M[12] = -I * s; break;
    case QS_GATE_RYY:
      id(); for (int i = 0; i < 4; ++i) M[i * 4 + i] = c;
      M[3] = I * s; M[12] = I * s; M[6] = -I * s; M[9] = -I * s; break;
    case QS_GATE_CU:
      id(); M[10] = g.mat[0]; M[11] = g.mat[1]; M[14] = g.mat[2]; M[15] = g.mat[3]; break;
    case QS_GATE_MCZ: id(); M[(size_t)d * d - 1] = -1; break;
    case QS_GATE_MCP: id(); M[(size_t)d * d - 1] = std::polar(1.0, t); break;
    case QS_GATE_UNITARY: return g.mat;
    default: fail(QS_EINVAL, "no matrix for gate kind");
  }
  return M;
}

// 2x2 helpers
static std::vector<cd> mul2(const std::vector<cd>& A, const std::vector<cd>& B) {
  return {A[0] * B[0] + A[1] * B[2], A[0] * B[1] + A[1] * B[3],
          A[2] * B[0] + A[3] * B[2], A[2] * B[1] + A[3] * B[3]};
}
static bool near2(const std::vector<cd>& A, cd a, cd b, cd c, cd d) {
  cd ref[4] = {a, b, c, d};
  for (int i = 0; i < 4; ++i)
    if (std::abs(A[i] - ref[i]) > kCollapseTol) return false;
  return true;
}

// ---------------------------------------------------------------- diagonal terms
// Terms of one diagonal gate: phase(i) = exp(i (global + sum angle_t f_t(i))).
static void diag_terms_of(const NGate& g, std::vector<DiagTermIR>& terms, Angle& global) {
  auto bitm = [&](int j) { return 1u << g.bits[j]; };
  Angle a = g.angle;
  switch (g.kind) {
    case QS_GATE_I: return;
    case QS_GATE_Z: terms.push_back({0, bitm(0), Angle{kPi, {}}}); return;
    case QS_GATE_S: terms.push_back({0, bitm(0), Angle{kPi / 2, {}}}); return;
    case QS_GATE_SDG: terms.push_back({0, bitm(0), Angle{-kPi / 2, {}}}); return;
    case QS_GATE_T: terms.push_back({0, bitm(0), Angle{kPi / 4, {}}}); return;
    case QS_GATE_TDG: terms.push_back({0, bitm(0), Angle{-kPi / 4, {}}}); return;
    case QS_GATE_P: terms.push_back({0, bitm(0), a}); return;
    case QS_GATE_RZ:  // exp(-i t/2) |0>, exp(+i t/2) |1>
      global = global.plus(a.scaled(-0.5));
      terms.push_back({0, bitm(0), a});
      return;
    case QS_GATE_CZ: terms.push_back({2, bitm(0) | bitm(1), Angle{kPi, {}}}); return;
    case QS_GATE_CPHASE: terms.push_back({2, bitm(0) | bitm(1), a}); return;
    case QS_GATE_RZZ:  // exp(-i t/2) on equal bits, exp(+i t/2) on different bits
      global = global.plus(a.scaled(-0.5));
      terms.push_back({1, bitm(0) | bitm(1), a});
      return;
    case QS_GATE_MCZ:
    case QS_GATE_MCP: {
      Angle aa = g.kind == QS_GATE_MCZ ? Angle{kPi, {}} : a;
      int pc = __builtin_popcount(g.all_mask);
      terms.push_back({pc == 1 ? 0 : pc == 2 ? 2 : 3, g.all_mask, aa});
      return;
    }
    default: fail(QS_EINVAL, "not a diagonal gate");
  }
}

static DiagIR build_diag(const std::vector<DiagTermIR>& raw, const Angle& global) {
  // merge identical (type, mask) terms
  std::vector<DiagTermIR> terms;
  for (auto& t : raw) {
    bool merged = false;
    for (auto& u : terms)
      if (u.type == t.type && u.mask == t.mask) { u.angle = u.angle.plus(t.angle); merged = true; break; }
    if (!merged) terms.push_back(t);
  }
  DiagIR d;
  d.global = global;
  d.raw = terms;
  for (auto& t : terms) d.support |= t.mask;
  // group by bit-identical symbolic angle, skipping exact zeros
  std::vector<std::vector<const DiagTermIR*>> groups;
  std::vector<Angle> gang;
  for (auto& t : terms) {
    if (t.angle.is_const() && t.angle.c0 == 0.0) continue;
    size_t gi = 0;
    for (; gi < gang.size(); ++gi)
      if (gang[gi].same(t.angle)) break;
    if (gi == gang.size()) { gang.push_back(t.angle); groups.emplace_back(); }
    groups[gi].push_back(&t);
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    DiagGroupIR G;
    G.angle = gang[gi];
    uint32_t bits = 0;
    std::map<std::pair<int, int>, uint32_t> shifted;  // (form, shift) -> lower-bit mask
    for (auto* t : groups[gi]) {
      int pc = __builtin_popcount(t->mask);
      if (t->type == 0) {
        bits |= t->mask;
        G.max_count += 1;
      } else if ((t->type == 1 || t->type == 2) && pc == 2) {
        int lo = __builtin_ctz(t->mask);
        int hi = 31 - __builtin_clz(t->mask);
        shifted[{t->type == 1 ? DT_SHIFT_XOR : DT_SHIFT_AND, hi - lo}] |= 1u << lo;
        G.max_count += 1;
      } else if (t->type == 1 || t->type == 4) {
        G.terms.push_back({DT_PARITY, 0, t->mask, 0});
        G.max_count += 1;
      } else {
        G.terms.push_back({DT_ALL, 0, t->mask, 0});
        G.max_count += 1;
      }
    }
    if (bits) G.terms.insert(G.terms.begin(), DiagTerm{DT_BITS, 0, bits, 0});
    for (auto& s : shifted) G.terms.push_back({s.first.first, s.first.second, s.second, 0});
    d.groups.push_back(std::move(G));
  }
  return d;
}

DiagIR diag_observable(int n, const qs_pauli* terms, size_t n_terms) {
  // c (-1)^{parity(i & z)} = c - 2 c parity(i & z): count terms weighted -2c
  std::vector<DiagTermIR> raw;
  Angle gl;
  for (size_t t = 0; t < n_terms; ++t) {
    const qs_pauli& P = terms[t];
    if (P.x_mask) fail(QS_EINVAL, "diagonal observable with an X or Y factor");
    if (!std::isfinite(P.coeff)) fail(QS_EINVAL, "non-finite coefficient");
    if (n < 64 && (P.z_mask >> n)) fail(QS_EINVAL, "Pauli mask out of range");
    uint32_t z = 0;
    for (int q = 0; q < n; ++q)
      if ((P.z_mask >> q) & 1) z |= 1u << (n - 1 - q);
    gl.c0 += P.coeff;
    int pc = __builtin_popcount(z);
    if (pc == 0) continue;
    raw.push_back({pc == 1 ? 0 : pc == 2 ? 1 : 4, z, Angle{-2.0 * P.coeff, {}}});
  }
  return build_diag(raw, gl);
}

// exp(i c th) with the product c th carried as hi + lo (lo = the rounding error
// of the FP64 product, exact by FMA); the library's sin / cos reduce hi
// exactly, so large angles (e.g. phase ladders up to ~1e7 rad) lose nothing
// to a reduction against an FP64 approximation of 2 pi.
static cd cis_product(double th, int c) {
  const double hi = th * (double)c;
  const double lo = std::fma(th, (double)c, -hi);
  return std::polar(1.0, hi) * cd(std::cos(lo), std::sin(lo));
}

double reduce_2pi(double x) {
  const double hi = 6.283185307179586, lo = 2.4492935982947064e-16;  // 2 pi = hi + lo
  const double k = std::nearbyint(x / hi);
  return std::fma(-k, lo, std::fma(-k, hi, x));
}

DiagNumeric diag_numeric(const DiagIR& d, const std::vector<double>& params, bool conj) {
  DiagNumeric out;
  double gl = d.global.eval(params);
  cd gph = std::polar(1.0, gl);
  out.global = reduce_2pi(conj ? -gl : gl);
  if (d.groups.empty()) {
    out.groups.push_back({0, 0, 0, 1});
    out.lut.push_back(conj ? std::conj(gph) : gph);
    out.theta.push_back(0.0);
    return out;
  }
  for (size_t gi = 0; gi < d.groups.size(); ++gi) {
    const DiagGroupIR& G = d.groups[gi];
    DiagGroup dg;
    dg.term_begin = (int32_t)out.terms.size();
    for (auto& t : G.terms) out.terms.push_back(t);
    dg.term_end = (int32_t)out.terms.size();
    dg.lut_begin = (int32_t)out.lut.size();
    dg.lut_len = G.max_count + 1;
    double th = G.angle.eval(params);
    out.theta.push_back(reduce_2pi(conj ? -th : th));
    for (int c = 0; c <= G.max_count; ++c) {
      cd v = cis_product(th, c);
      if (gi == 0) v *= gph;
      out.lut.push_back(conj ? std::conj(v) : v);
    }
    out.groups.push_back(dg);
  }
  return out;
}

// ---------------------------------------------------------------- GF(2) maps
// Row r of A: src bit r = parity(rows[r] & y).
static void gf2_push_gate(Gf2IR& G, const NGate& g) {
  // src map <- g o src map (gates are replayed in reverse order)
  auto& A = G.rows;
  if (g.kind == QS_GATE_X) {
    G.cprime ^= 1u << g.bits[0];
  } else if (g.kind == QS_GATE_CNOT) {
    int c = g.bits[0], t = g.bits[1];
    A[t] ^= A[c];
    G.cprime ^= ((G.cprime >> c) & 1u) << t;
  } else if (g.kind == QS_GATE_SWAP) {
    int a = g.bits[0], b = g.bits[1];
    std::swap(A[a], A[b]);
    uint32_t d = ((G.cprime >> a) ^ (G.cprime >> b)) & 1u;
    G.cprime ^= (d << a) | (d << b);
  } else {
    fail(QS_EINVAL, "not a permutation gate");
  }
}

static Gf2IR build_gf2(int n, const std::vector<NGate>& gates, const std::vector<int>& idx) {
  Gf2IR G;
  G.rows.resize(n);
  for (int r = 0; r < n; ++r) G.rows[r] = 1u << r;
  for (auto it = idx.rbegin(); it != idx.rend(); ++it) gf2_push_gate(G, gates[*it]);
  G.gates = idx;
  return G;
}

// Compose: first apply F (out1[y] = in[A_F y ^ c_F]) then S (out2[y] = out1[A_S y ^ c_S])
// => out2[y] = in[A_F (A_S y ^ c_S) ^ c_F].
static Gf2IR compose_gf2(int n, const Gf2IR& F, const Gf2IR& S) {
  auto apply = [&](const std::vector<uint32_t>& rows, uint32_t v) {
    uint32_t r = 0;
    for (int b = 0; b < n; ++b) r |= (uint32_t)(__builtin_popcount(rows[b] & v) & 1) << b;
    return r;
  };
  Gf2IR R;
  R.rows.assign(n, 0);
  // column j of A_F A_S = A_F (A_S e_j)
  for (int j = 0; j < n; ++j) {
    uint32_t col = apply(F.rows, apply(S.rows, 1u << j));
    for (int b = 0; b < n; ++b)
      if ((col >> b) & 1) R.rows[b] |= 1u << j;
  }
  R.cprime = apply(F.rows, S.cprime) ^ F.cprime;
  R.gates = F.gates;
  R.gates.insert(R.gates.end(), S.gates.begin(), S.gates.end());
  return R;
}

static uint32_t gf2_apply_rows(int n, const std::vector<uint32_t>& rows, uint32_t v) {
  uint32_t r = 0;
  for (int b = 0; b < n; ++b) r |= (uint32_t)(__builtin_popcount(rows[b] & v) & 1) << b;
  return r;
}

// Reduced basis helper: insert v; returns true if v was independent.
struct Gf2Basis {
  uint32_t piv[32] = {0};  // piv[b]: basis vector with leading bit b
  int dim = 0;
  uint32_t reduce(uint32_t v) const {
    for (int b = 31; b >= 0; --b)
      if (((v >> b) & 1) && piv[b]) v ^= piv[b];
    return v;
  }
  bool insert(uint32_t v) {
    v = reduce(v);
    if (!v) return false;
    piv[31 - __builtin_clz(v)] = v;
    ++dim;
    return true;
  }
};

Gf2Args gf2_args(int n, const Gf2IR& g, int c_bits) {
  Gf2Args a;
  std::memset(&a, 0, sizeof a);
  int c = std::min(c_bits, n / 2);
  if (c < 1) c = 1;
  if (c > n) c = n;
  int d = std::min(2 * c, n);
  a.n = n;
  a.c = c;
  a.d = d;
  a.cprime = g.cprime;
  for (int j = 0; j < n; ++j) {
    uint32_t col = 0;
    for (int b = 0; b < n; ++b)
      if ((g.rows[b] >> j) & 1) col |= 1u << b;
    a.acol[j] = col;
  }
  // M = A^{-1}: M e_j is the y with A y = e_j; solve through an index table
  // of the columns (Gaussian elimination with combination tracking).
  std::vector<uint32_t> Mcol(n, 0);
  {
    // rows of the augmented system [A | I] reduced on columns of A
    std::vector<uint32_t> colv(a.acol, a.acol + n);  // A e_j
    std::vector<uint32_t> comb(n);
    for (int j = 0; j < n; ++j) comb[j] = 1u << j;
    // eliminate to obtain combinations whose image is e_b
    std::vector<int> used(n, 0);
    for (int b = 0; b < n; ++b) {
      int pivot = -1;
      for (int j = 0; j < n; ++j)
        if (!used[j] && ((colv[j] >> b) & 1)) { pivot = j; break; }
      if (pivot < 0) fail(QS_EINVAL, "permutation block is not invertible");
      used[pivot] = 1;
      for (int j = 0; j < n; ++j)
        if (j != pivot && ((colv[j] >> b) & 1)) { colv[j] ^= colv[pivot]; comb[j] ^= comb[pivot]; }
    }
    for (int j = 0; j < n; ++j) {
      int b = __builtin_ctz(colv[j]);
      Mcol[b] = comb[j];  // A * comb[j] = e_b (as a combination of unit vectors)
    }
  }
  // tile subspace V = span(e_0..e_{c-1}, M e_0..M e_{c-1}) padded to dimension d
  Gf2Basis V;
  std::vector<uint32_t> vb;  // destination basis v_0..v_{d-1}
  for (int j = 0; j < c; ++j) { V.insert(1u << j); vb.push_back(1u << j); }
  for (int j = 0; j < c && V.dim < d; ++j)
    if (V.insert(Mcol[j])) vb.push_back(Mcol[j]);
  for (int b = c; b < n && V.dim < d; ++b)
    if (V.insert(1u << b)) vb.push_back(1u << b);
  // source basis u_0..u_{d-1}: u_j = M e_j for j < c, completed from vb
  Gf2Basis U;
  std::vector<uint32_t> ub;
  for (int j = 0; j < c; ++j) { U.insert(Mcol[j]); ub.push_back(Mcol[j]); }
  for (auto v : vb)
    if ((int)ub.size() < d && U.insert(v)) ub.push_back(v);
  if ((int)ub.size() != d || (int)vb.size() != d) fail(QS_EINVAL, "internal: tile basis");
  // coordinates in the v basis
  std::unordered_map<uint32_t, uint32_t> coord;
  for (uint32_t t = 0; t < (1u << d); ++t) {
    uint32_t y = 0;
    for (int j = 0; j < d; ++j)
      if ((t >> j) & 1) y ^= vb[j];
    coord[y] = t;
  }
  std::vector<uint32_t> ucoord(d);
  for (int j = 0; j < d; ++j) ucoord[j] = coord.at(ub[j]);
  int hi = d - c;
  for (uint32_t s = 0; s < (1u << c); ++s) {
    uint32_t t = 0;
    for (int j = 0; j < c; ++j)
      if ((s >> j) & 1) t ^= ucoord[j];
    a.t_lo[s] = t;
  }
  for (uint32_t s = 0; s < (1u << hi); ++s) {
    uint32_t t = 0, x = 0, y = 0;
    for (int j = 0; j < hi; ++j)
      if ((s >> j) & 1) {
        t ^= ucoord[c + j];
        x ^= gf2_apply_rows(n, g.rows, ub[c + j]);
        y ^= vb[c + j];
      }
    a.t_hi[s] = t;
    a.au_hi[s] = x;
    a.v_hi[s] = y;
  }
  // LDS swizzle: a linear h on the high tile coordinate with t_lo ^ h(t_hi)
  // injective over the 2^c low source coordinates, so the scattered writes of
  // 2^c consecutive lanes hit distinct banks (reads of consecutive t stay
  // conflict-free because the XOR permutes within aligned blocks of 2^c)
  {
    const uint32_t lo_mask = (1u << c) - 1;
    auto injective = [&](const uint32_t* hcol) {
      uint64_t seen = 0;
      for (uint32_t s = 0; s < (1u << c); ++s) {
        uint32_t t = a.t_lo[s];
        uint32_t th = t >> c, h = 0;
        for (int j = 0; j < hi; ++j)
          if ((th >> j) & 1) h ^= hcol[j];
        uint32_t v = (t ^ h) & lo_mask;
        if ((seen >> v) & 1) return false;
        seen |= 1ull << v;
      }
      return true;
    };
    uint32_t hcol[32] = {0};
    bool ok = injective(hcol);
    uint64_t rng = 0x9e3779b97f4a7c15ull ^ (uint64_t)g.cprime;
    for (int tries = 0; !ok && tries < 4096; ++tries) {
      for (int j = 0; j < hi; ++j) {
        rng ^= rng << 13;
        rng ^= rng >> 7;
        rng ^= rng << 17;
        hcol[j] = (uint32_t)rng & lo_mask;
      }
      ok = injective(hcol);
    }
    if (!ok) std::memset(hcol, 0, sizeof hcol);  // keep the (conflicting) identity layout
    for (uint32_t v = 0; v < (1u << hi); ++v) {
      uint32_t h = 0;
      for (int j = 0; j < hi; ++j)
        if ((v >> j) & 1) h ^= hcol[j];
      a.hx[v] = h;
    }
  }
  // complement: unit vectors independent of V
  Gf2Basis C = V;
  int nf = 0;
  for (int b = 0; b < n; ++b)
    if (C.insert(1u << b)) a.free_bits[nf++] = (uint32_t)b;
  a.n_free = nf;
  if (nf != n - d) fail(QS_EINVAL, "internal: coset complement");
  return a;
}

// ---------------------------------------------------------------- plan building
// ---------------------------------------------------------------- dense windows
// Gates that cannot change the fused operator of a window: constant angle and
// no more bits than the window may hold.
static bool window_fusable(const NGate& g, int kmax) {
  if (!g.angle.is_const()) return false;
  return (int)g.bits.size() <= kmax;
}

static uint32_t gate_mask(const NGate& g) {
  uint32_t m = 0;
  for (int b : g.bits) m |= 1u << b;
  return m;
}

// U <- E(g) U, where E(g) is gate g on its bits inside a window whose matrix
// index bit u holds state bit asc[u].
static void window_apply(std::vector<cd>& U, const std::vector<int>& asc, const NGate& g) {
  const std::vector<double> none;
  const std::vector<cd> M = gate_matrix(g, none);
  const int k = (int)asc.size(), K = 1 << k;
  const int a = (int)g.bits.size(), A = 1 << a;
  std::vector<int> lb(a);  // window bit of gate-matrix bit t (gate wire j is matrix bit a-1-j)
  uint32_t gm = 0;
  for (int j = 0; j < a; ++j) {
    const int u = (int)(std::find(asc.begin(), asc.end(), g.bits[j]) - asc.begin());
    lb[a - 1 - j] = u;
    gm |= 1u << u;
  }
  std::vector<int> ex(A, 0);
  for (int t = 0; t < A; ++t)
    for (int v = 0; v < a; ++v)
      if ((t >> v) & 1) ex[t] |= 1 << lb[v];
  std::vector<cd> out((size_t)K * K);
  for (int r0 = 0; r0 < K; ++r0) {
    if (r0 & (int)gm) continue;
    for (int c = 0; c < K; ++c)
      for (int s = 0; s < A; ++s) {
        cd acc = 0;
        for (int t = 0; t < A; ++t) acc += M[(size_t)s * A + t] * U[(size_t)(r0 | ex[t]) * K + c];
        out[(size_t)(r0 | ex[s]) * K + c] = acc;
      }
  }
  U.swap(out);
}

int fuse_windows(int n, const std::vector<NGate>& in, int kmax, std::vector<NGate>& out) {
  struct Win {
    uint32_t mask;
    std::vector<int> gates;
  };
  std::vector<Win> open;
  int formed = 0;
  out.clear();
  auto emit = [&](Win& w) {
    if (w.gates.size() < 2 || __builtin_popcount(w.mask) < 2) {
      for (int gi : w.gates) out.push_back(in[gi]);
      return;
    }
    uint32_t m = w.mask;
    for (int b = 0; b < n && __builtin_popcount(m) < 4; ++b) m |= 1u << b;  // identity padding
    std::vector<int> asc;
    for (int b = 0; b < n; ++b)
      if ((m >> b) & 1) asc.push_back(b);
    const int k = (int)asc.size(), K = 1 << k;
    std::vector<cd> U((size_t)K * K, cd(0, 0));
    for (int i = 0; i < K; ++i) U[(size_t)i * K + i] = 1;
    for (int gi : w.gates) window_apply(U, asc, in[gi]);
    NGate g;
    g.kind = QS_GATE_UNITARY;
    g.bits.assign(asc.rbegin(), asc.rend());  // first listed bit = most significant matrix bit
    g.mat = std::move(U);
    g.index = in[w.gates.front()].index;
    g.fused = (int32_t)w.gates.size();
    out.push_back(std::move(g));
    ++formed;
  };
  for (size_t i = 0; i < in.size(); ++i) {
    const NGate& g = in[i];
    const uint32_t gm = gate_mask(g);
    std::vector<size_t> hit;
    for (size_t w = 0; w < open.size(); ++w)
      if (open[w].mask & gm) hit.push_back(w);
    if (!window_fusable(g, kmax)) {
      // close every window it touches, keep the others open (they commute with g)
      for (size_t w : hit) emit(open[w]);
      for (size_t j = hit.size(); j-- > 0;) open.erase(open.begin() + (long)hit[j]);
      out.push_back(g);
      continue;
    }
    // Windows on disjoint bits commute, so the touched windows can be
    // concatenated and g appended.  When they do not all fit, the smallest
    // ones are merged while they fit and the rest are emitted first.
    std::vector<size_t> order = hit;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
      return __builtin_popcount(open[x].mask) < __builtin_popcount(open[y].mask);
    });
    Win W{gm, {}};
    std::vector<char> take(open.size(), 0);
    for (size_t w : order)
      if (__builtin_popcount(W.mask | open[w].mask) <= kmax) {
        W.mask |= open[w].mask;
        take[w] = 1;
      }
    for (size_t w : hit)
      if (!take[w]) emit(open[w]);
    for (size_t w : hit)
      if (take[w]) W.gates.insert(W.gates.end(), open[w].gates.begin(), open[w].gates.end());
    W.gates.push_back((int)i);
    for (size_t j = hit.size(); j-- > 0;) open.erase(open.begin() + (long)hit[j]);
    open.push_back(std::move(W));
  }
  for (Win& w : open) emit(w);
  return formed;
}

double plan_cost(const PlanIR& P) {
  double c = 0.0;
  for (const LayerIR& L : P.layers) {
    if (L.kind == L_DENSE) {
      const int k = (int)P.denses[L.index].bits.size();
      c += k <= 4 ? 1.0 : k == 5 ? 1.2 : 2.0;
    } else if (L.kind == L_PLAIN) {
      const int k = (int)P.gates[L.index].bits.size();
      c += k <= 2 ? 1.0 : (double)(1 << (k - 2));
    } else {
      c += 1.0;
    }
  }
  return c;
}

namespace {

// Low bits kept by high tile passes with diagonal layers unless the plan
// options say otherwise (-1: as many as the pass's group has).
constexpr int kDefaultDiagLowBits = 6;

struct Sched {
  int n;
  int L;                                // least low bits of a high tile
  std::vector<std::array<int, 3>> grp;  // (L, a, h)
  std::vector<uint32_t> gmask;
};

Sched make_groups(int n, int tile_bits, int low_bits) {
  Sched s;
  s.n = n;
  s.L = low_bits > 0 ? low_bits : 4;
  if (n <= tile_bits) {
    s.grp.push_back({n, n, 0});
    s.gmask.push_back(n >= 32 ? 0xffffffffu : ((1u << n) - 1));
    return s;
  }
  int m0 = tile_bits;
  s.grp.push_back({m0, m0, 0});
  s.gmask.push_back((1u << m0) - 1);
  int rest = n - m0;
  // low_bits > 0: every high tile holds the lowest low_bits state bits;
  // low_bits == 0: a group of h high bits fills its tile with the lowest
  // tile_bits - h state bits (at least 4), i.e. longer contiguous runs per HBM
  // access (2^L amplitudes) at the price of larger tiles
  const int Lmin = low_bits > 0 ? low_bits : 4;
  int hmax = tile_bits - Lmin;
  int ng = (rest + hmax - 1) / hmax;
  int a = m0;
  for (int k = 0; k < ng; ++k) {
    int h = rest / ng + (k < rest % ng ? 1 : 0);
    const int L = low_bits > 0 ? low_bits : tile_bits - h;
    s.grp.push_back({L, a, h});
    uint32_t m = (1u << L) - 1;
    for (int b = a; b < a + h; ++b) m |= 1u << b;
    s.gmask.push_back(m);
    a += h;
  }
  return s;
}

// The gate's matrix (first listed wire = most significant index bit) re-indexed
// so that index bit u sits on the u-th smallest target bit.
DenseIR make_dense(const NGate& g, int32_t gi) {
  DenseIR D;
  D.gate = gi;
  const int k = (int)g.bits.size();
  D.bits = g.bits;
  std::sort(D.bits.begin(), D.bits.end());
  std::vector<int> gate_bit(k);  // index bit of the gate's matrix holding D.bits[u]
  for (int u = 0; u < k; ++u)
    for (int j = 0; j < k; ++j)
      if (g.bits[j] == D.bits[u]) gate_bit[u] = k - 1 - j;
  const int K = 1 << k;
  std::vector<int> perm(K);
  for (int r = 0; r < K; ++r) {
    int q = 0;
    for (int u = 0; u < k; ++u)
      if ((r >> u) & 1) q |= 1 << gate_bit[u];
    perm[r] = q;
  }
  D.mat.resize((size_t)K * K);
  D.mat_dagger.resize((size_t)K * K);
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) {
      D.mat[(size_t)r * K + c] = g.mat[(size_t)perm[r] * K + perm[c]];
      D.mat_dagger[(size_t)c * K + r] = std::conj(D.mat[(size_t)r * K + c]);
    }
  return D;
}

struct Item {
  ItemIR ir;
  uint32_t W = 0, R = 0;
};

class Builder {
 public:
  Builder(PlanIR& P, int tile_bits, int low_bits)
      : P(P), n(P.n), sched(make_groups(P.n, tile_bits, low_bits)), window(P.n) {}

  void run() {
    const auto& G = P.gates;
    size_t i = 0;
    while (i < G.size()) {
      const NGate& g = G[i];
      size_t used = 0;
      int base = 0;
      if (g.kind == QS_GATE_H && (used = qft_stage_len(i, &base)) > 0) {
        close_open();
        OpIR op{OP_QFT, g.bits[0], {}, false, -1};
        op.base = base;
        add_op_item(op);
        last_qft_bit = g.bits[0];
        last_qft_base = base;
        i += used;
        continue;
      }
      if (g.kind == QS_GATE_CPHASE && (used = qft_inv_stage_len(i, &base)) > 0) {
        // inverse QFT stage: the controlled-phase ladder undone, then H
        close_open();
        OpIR op{OP_QFT_INV, P.gates[i + used - 1].bits[0], {}, false, -1};
        op.base = base;
        add_op_item(op);
        last_qft_bit = -1;
        i += used;
        continue;
      }
      last_qft_bit = -1;
      int k = g.kind;
      if (k == QS_GATE_I) { ++i; continue; }
      bool one = g.bits.size() == 1 && k != QS_GATE_MCZ && k != QS_GATE_MCP;
      if (k == QS_GATE_X && open == PERM) {
        perm.push_back((int)i);
      } else if (one && gate_is_diagonal(k)) {
        if (open == DIAG) diag.push_back((int)i);
        else { open_block(WINDOW); window[g.bits[0]].push_back((int)i); }
      } else if (one) {
        open_block(WINDOW);
        window[g.bits[0]].push_back((int)i);
      } else if (gate_is_diagonal(k)) {
        open_block(DIAG);
        diag.push_back((int)i);
      } else if (k == QS_GATE_CNOT || k == QS_GATE_SWAP) {
        open_block(PERM);
        perm.push_back((int)i);
      } else if (k == QS_GATE_RXX) {
        open_block(XX);
        pp.push_back((int)i);
      } else if (k == QS_GATE_RYY) {
        open_block(YY);
        pp.push_back((int)i);
      } else if (k == QS_GATE_UNITARY && (int)g.bits.size() >= 4 && (int)g.bits.size() <= P.opt.dense_k_max &&
                 n - (int)g.bits.size() >= 4) {
        close_open();
        barrier({L_DENSE, (int32_t)P.denses.size()});
        P.denses.push_back(make_dense(g, (int32_t)i));
      } else {
        close_open();
        barrier({L_PLAIN, (int32_t)i});
      }
      ++i;
    }
    close_open();
    flush_segment();
  }

 private:
  enum Open { NONE, DIAG, WINDOW, PERM, XX, YY };
  PlanIR& P;
  int n;
  Sched sched;
  Open open = NONE;
  std::vector<int> diag, perm, pp;
  std::vector<std::vector<int>> window;
  std::vector<Item> seg;
  int last_qft_bit = -1, last_qft_base = 0;
  // the closing basis change of the last XX / YY run: the segment size right
  // after it, its bits and its family
  size_t pp_tail_end = (size_t)-1;
  uint32_t pp_tail_inv = 0;
  bool pp_tail_yy = false;

  // Number of gates of a QFT stage starting at gate i, or 0: H on bit p
  // followed by CPHASE(pi / 2^(p-b)) on (b, p) for every b in [r0, p), in any
  // order (a register whose lowest bit is r0, *base).  A lone H right after the
  // stage on bit p + 1 of a register based at p is that register's last stage.
  size_t qft_stage_len(size_t i, int* base) const {
    const auto& G = P.gates;
    const int p = G[i].bits[0];
    uint32_t seen = 0;
    size_t j = i + 1;
    for (; j < G.size(); ++j) {
      const NGate& c = G[j];
      if (c.kind != QS_GATE_CPHASE || !c.angle.is_const()) break;
      const int a = c.bits[0], b = c.bits[1];
      const int other = a == p ? b : b == p ? a : -1;
      if (other < 0 || other >= p || ((seen >> other) & 1)) break;
      if (c.angle.c0 != std::ldexp(kPi, -(p - other))) break;
      seen |= 1u << other;
    }
    const int k = (int)(j - i - 1);
    if (k == 0) {
      *base = p;
      return last_qft_bit == p + 1 && last_qft_base == p ? 1 : 0;
    }
    const int r0 = p - k;
    if (seen != (((1u << p) - 1u) & ~((1u << r0) - 1u))) return 0;
    *base = r0;
    return (size_t)k + 1;
  }

  // Number of gates of an inverse QFT stage starting at gate i, or 0:
  // CPHASE(-pi / 2^(p-b)) on (b, p) for every b in [r0, p), in any order, then
  // H on bit p (*base = r0).
  size_t qft_inv_stage_len(size_t i, int* base) const {
    const auto& G = P.gates;
    const NGate& g0 = G[i];
    if (g0.bits.size() != 2) return 0;
    const int p = std::max(g0.bits[0], g0.bits[1]);
    uint32_t seen = 0;
    size_t j = i;
    for (; j < G.size(); ++j) {
      const NGate& c = G[j];
      if (c.kind != QS_GATE_CPHASE || !c.angle.is_const()) break;
      const int a = c.bits[0], b = c.bits[1];
      const int other = a == p ? b : b == p ? a : -1;
      if (other < 0 || other >= p || ((seen >> other) & 1)) break;
      if (c.angle.c0 != -std::ldexp(kPi, -(p - other))) break;
      seen |= 1u << other;
    }
    const int k = (int)(j - i);
    if (k == 0 || j >= G.size() || G[j].kind != QS_GATE_H || G[j].bits[0] != p) return 0;
    const int r0 = p - k;
    if (seen != (((1u << p) - 1u) & ~((1u << r0) - 1u))) return 0;
    *base = r0;
    return (size_t)k + 1;
  }

  void open_block(Open o) {
    if (open != o) close_open();
    open = o;
  }

  void close_open() {
    switch (open) {
      case DIAG: close_diag(); break;
      case WINDOW: close_window(); break;
      case PERM: close_perm(); break;
      case XX: case YY: close_pp(); break;
      default: break;
    }
    open = NONE;
  }

  void close_diag() {
    std::vector<DiagTermIR> raw;
    Angle gl;
    for (int gi : diag) diag_terms_of(P.gates[gi], raw, gl);
    diag.clear();
    DiagIR d = build_diag(raw, gl);
    if (d.groups.empty() && d.global.is_const() && d.global.c0 == 0.0) return;
    add_diag_item(std::move(d));
  }

  void add_diag_item(DiagIR d) {
    // a diagonal layer right after another one (no op in between) multiplies
    // into it: one table lookup pass instead of two
    if (!seg.empty() && seg.back().ir.type == 1) {
      DiagIR& prev = P.diags[seg.back().ir.index];
      std::vector<DiagTermIR> raw = prev.raw;
      raw.insert(raw.end(), d.raw.begin(), d.raw.end());
      prev = build_diag(raw, prev.global.plus(d.global));
      seg.back().R = prev.support;
      return;
    }
    Item it;
    it.ir = {1, (int32_t)P.diags.size()};
    it.R = d.support;
    P.diags.push_back(std::move(d));
    seg.push_back(it);
  }

  void add_op_item(OpIR op) {
    Item it;
    it.ir = {0, (int32_t)P.ops.size()};
    it.W = 1u << op.bit;
    if (op.kind == OP_QFT || op.kind == OP_QFT_INV) it.R = ((1u << op.bit) - 1u) & ~((1u << op.base) - 1u);
    P.ops.push_back(std::move(op));
    seg.push_back(it);
  }

  void close_window() {
    std::vector<double> none;
    bool all_x = true, any = false;
    uint32_t xmask = 0;
    std::vector<std::pair<int, std::vector<cd>>> prods;
    for (int b = 0; b < n; ++b) {
      auto& w = window[b];
      if (w.empty()) continue;
      bool fixed = true;
      for (int gi : w) fixed = fixed && P.gates[gi].angle.is_const();
      if (!fixed) { all_x = false; any = true; continue; }
      std::vector<cd> U = gate_matrix(P.gates[w[0]], none);
      for (size_t j = 1; j < w.size(); ++j) U = mul2(gate_matrix(P.gates[w[j]], none), U);
      if (near2(U, 1, 0, 0, 1)) { w.clear(); continue; }
      any = true;
      if (near2(U, 0, 1, 1, 0)) xmask |= 1u << b;
      else all_x = false;
    }
    if (!any) return;
    if (all_x && xmask) {
      std::vector<int> gl;
      for (int b = 0; b < n; ++b) { for (int gi : window[b]) gl.push_back(gi); window[b].clear(); }
      Gf2IR G;
      G.rows.resize(n);
      for (int r = 0; r < n; ++r) G.rows[r] = 1u << r;
      G.cprime = xmask;
      G.gates = gl;
      barrier_gf2(std::move(G));
      return;
    }
    for (int b = 0; b < n; ++b) {
      auto& w = window[b];
      if (w.empty()) continue;
      bool fixed = true, diagonal = true;
      for (int gi : w) {
        fixed = fixed && P.gates[gi].angle.is_const();
        diagonal = diagonal && gate_is_diagonal(P.gates[gi].kind);
      }
      OpIR op{OP_MAT, b, w, false, -1};
      if (diagonal) op.kind = OP_DIAG;
      else if (fixed) {
        std::vector<cd> U = gate_matrix(P.gates[w[0]], none);
        for (size_t j = 1; j < w.size(); ++j) U = mul2(gate_matrix(P.gates[w[j]], none), U);
        const double r = 1.0 / std::sqrt(2.0);
        if (near2(U, r, r, r, -r)) op.kind = OP_H;
      }
      add_op_item(std::move(op));
      w.clear();
    }
  }

  void close_perm() {
    Gf2IR G = build_gf2(n, P.gates, perm);
    perm.clear();
    barrier_gf2(std::move(G));
  }

  void close_pp() {
    // same-family run: basis change on the involved bits, ZZ-type diagonal, basis change back
    bool yy = open == YY;
    uint32_t inv = 0;
    std::vector<DiagTermIR> raw;
    Angle gl;
    for (int gi : pp) {
      const NGate& g = P.gates[gi];
      inv |= (1u << g.bits[0]) | (1u << g.bits[1]);
      NGate z = g;
      z.kind = QS_GATE_RZZ;
      diag_terms_of(z, raw, gl);
    }
    pp.clear();
    // Opening basis change.  When the previous run of the other family closed
    // on the same bits with nothing in between, its closing change and this
    // opening one multiply into one 2x2 per bit (one op instead of two).
    if (pp_tail_end == seg.size() && pp_tail_inv == inv && pp_tail_yy != yy) {
      for (size_t k = seg.size() - (size_t)__builtin_popcount(inv); k < seg.size(); ++k) {
        OpIR& op = P.ops[seg[k].ir.index];
        op.kind = OP_MAT;
        op.fixed_h = true;
        op.fixed_mat = yy ? 2 : 3;
      }
    } else {
      for (int b = 0; b < n; ++b)
        if ((inv >> b) & 1) add_op_item(OpIR{yy ? OP_MAT : OP_H, b, {}, true, yy ? 0 : -1});
    }
    add_diag_item(build_diag(raw, gl));
    for (int b = 0; b < n; ++b)
      if ((inv >> b) & 1) add_op_item(OpIR{yy ? OP_MAT : OP_H, b, {}, true, yy ? 1 : -1});
    pp_tail_end = seg.size();
    pp_tail_inv = inv;
    pp_tail_yy = yy;
  }

  void barrier_gf2(Gf2IR G) {
    // merge with an immediately preceding permutation layer
    if (seg.empty() && !P.layers.empty() && P.layers.back().kind == L_GF2) {
      Gf2IR& F = P.gf2s[P.layers.back().index];
      F = compose_gf2(n, F, G);
      return;
    }
    // a lone X / CNOT / SWAP moves half the state in place on the per-gate
    // kernel; a gather moves all of it
    if (G.gates.size() == 1) {
      barrier({L_PLAIN, (int32_t)G.gates[0]});
      return;
    }
    barrier({L_GF2, (int32_t)P.gf2s.size()});
    P.gf2s.push_back(std::move(G));
  }

  void barrier(LayerIR L) {
    flush_segment();
    P.layers.push_back(L);
  }

  // ---- tile-pass scheduling of one segment ------------------------------------
  // A Hadamard butterfly (an H, or a QFT stage whose twiddle bits [base, p)
  // are empty) followed by another on the same bit, with no item touching the
  // bit in between, is the identity: both are dropped (exactly; the pass
  // scale counts the remaining butterflies).
  bool plain_butterfly(const Item& it) const {
    if (it.ir.type != 0) return false;
    const OpIR& op = P.ops[it.ir.index];
    if (op.kind == OP_H) return op.fixed_mat < 0;
    return (op.kind == OP_QFT || op.kind == OP_QFT_INV) && op.base == op.bit;
  }

  void cancel_butterfly_pairs() {
    std::vector<char> dead(seg.size(), 0);
    for (size_t i = 0; i < seg.size(); ++i) {
      if (dead[i] || !plain_butterfly(seg[i])) continue;
      const uint32_t b = seg[i].W;
      for (size_t j = i + 1; j < seg.size(); ++j) {
        if (dead[j] || !((seg[j].W | seg[j].R) & b)) continue;
        if (plain_butterfly(seg[j]) && seg[j].W == b) dead[i] = dead[j] = 1;
        break;
      }
    }
    size_t k = 0;
    for (size_t i = 0; i < seg.size(); ++i)
      if (!dead[i]) seg[k++] = seg[i];
    seg.resize(k);
  }

  void flush_segment() {
    cancel_butterfly_pairs();
    if (seg.empty()) return;
    size_t N = seg.size();
    std::vector<std::vector<int>> deps(N);
    for (size_t j = 0; j < N; ++j)
      for (size_t i = 0; i < j; ++i) {
        bool conflict = (seg[i].W & (seg[j].W | seg[j].R)) || (seg[j].W & seg[i].R);
        if (conflict) deps[j].push_back((int)i);
      }
    std::vector<char> done(N, 0);
    size_t remaining = N;
    while (remaining) {
      int best = -1, best_ops = -1;
      std::vector<int> best_list;
      for (size_t g = 0; g < sched.grp.size(); ++g) {
        std::vector<int> list;
        int ops = scan(g, deps, done, list);
        if (ops > best_ops) { best_ops = ops; best = (int)g; best_list = list; }
      }
      if (best_ops <= 0) {
        // only diagonal layers are ready: run them as standalone passes
        for (int idx : best_list) {
          P.layers.push_back({L_DIAG, seg[idx].ir.index});
          done[idx] = 1;
          --remaining;
        }
        if (best_list.empty()) fail(QS_EINVAL, "internal: scheduler made no progress");
        continue;
      }
      TilePassIR T;
      T.L = sched.grp[best][0];
      T.a = sched.grp[best][1];
      T.h = sched.grp[best][2];
      // diag_low_bits = k > 0: a high pass with diagonal layers keeps only k
      // low bits (smaller tiles, more of them per compute unit, shorter HBM
      // runs); ops on the bits given up wait for a later pass.
      const int dl = P.opt.diag_low_bits == 0 ? kDefaultDiagLowBits : P.opt.diag_low_bits;
      bool has_diag = false;
      for (int idx : best_list) has_diag = has_diag || seg[idx].ir.type == 1;
      if (dl > 0 && has_diag && T.h > 0 && T.L > dl) {
        const uint32_t small = ((1u << dl) - 1u) | (((1u << T.h) - 1u) << T.a);
        std::vector<int> list;
        scan_mask(small, deps, done, list);
        bool diag_kept = false;
        for (int idx : list) diag_kept = diag_kept || seg[idx].ir.type == 1;
        if (diag_kept) {
          T.L = dl;
          best_list = list;
        }
      }
      for (int idx : best_list) {
        T.items.push_back(seg[idx].ir);
        done[idx] = 1;
        --remaining;
      }
      P.layers.push_back({L_TILE, (int32_t)P.passes.size()});
      P.passes.push_back(std::move(T));
    }
    seg.clear();
  }

  int scan(size_t g, const std::vector<std::vector<int>>& deps, const std::vector<char>& done,
           std::vector<int>& list) {
    return scan_mask(sched.gmask[g], deps, done, list);
  }

  // Every ready item in stream order whose written bits lie in the tile mask
  // (at most kMaxDiagSlots diagonal layers); returns the number of ops taken.
  int scan_mask(uint32_t gmask, const std::vector<std::vector<int>>& deps, const std::vector<char>& done,
                std::vector<int>& list) {
    std::vector<char> taken(seg.size(), 0);
    int ops = 0, ndiag = 0;
    for (size_t j = 0; j < seg.size(); ++j) {
      if (done[j]) continue;
      bool ok = true;
      for (int d : deps[j])
        if (!done[d] && !taken[d]) { ok = false; break; }
      if (!ok) continue;
      if (seg[j].ir.type == 0) {
        if ((seg[j].W & ~gmask) != 0) continue;
        ++ops;
      } else {
        if (ndiag == kMaxDiagSlots) continue;
        ++ndiag;
      }
      taken[j] = 1;
      list.push_back((int)j);
    }
    return ops;
  }
};

int tile_pos(const TilePassIR& T, int sb) {
  if (sb < T.L) return sb;
  if (sb >= T.a && sb < T.a + T.h) return T.L + (sb - T.a);
  return -1;
}
int tile_state_bit(const TilePassIR& T, int tb) { return tb < T.L ? tb : T.a + (tb - T.L); }

// Conflict test between two tile ops (same rule as the pass scheduler): an op
// writes its bit; a QFT stage on bit p also reads every bit below p.
bool ops_conflict(const OpIR& a, const OpIR& b) {
  uint32_t Wa = 1u << a.bit, Wb = 1u << b.bit;
  const bool qa = a.kind == OP_QFT || a.kind == OP_QFT_INV, qb = b.kind == OP_QFT || b.kind == OP_QFT_INV;
  uint32_t Ra = qa ? ((1u << a.bit) - 1u) & ~((1u << a.base) - 1u) : 0;
  uint32_t Rb = qb ? ((1u << b.bit) - 1u) & ~((1u << b.base) - 1u) : 0;
  return (Wa & (Wb | Rb)) || (Wb & Ra);
}

uint32_t lds_off(uint32_t pos) { return pos + ((pos >> 5) << 1); }

// Pattern of a round's op list (see TileRoundType).  RT_MAT4 may be refined to
// the RX / RY forms when the plan's numbers are bound.
int32_t classify_round(const PlanIR& P, const TilePassIR& T, const TileRound& r) {
  (void)P;
  const int n = r.op_end - r.op_begin;
  auto op = [&](int k) -> const TileOp& { return T.ops[r.op_begin + k]; };
  auto is = [&](int k, int kind, int rbit) { return op(k).kind == kind && op(k).rbit == rbit; };
  if (n == 4 && is(0, OP_QFT, 3) && is(1, OP_QFT, 2) && is(2, OP_QFT, 1) && is(3, OP_QFT, 0)) return RT_QFT4;
  if (n == 8 && is(0, OP_QFT, 3) && is(1, OP_QFT, 2) && is(2, OP_QFT, 1) && is(3, OP_QFT, 0)) {
    uint32_t hb = 0;
    for (int k = 4; k < 8; ++k)
      if (op(k).kind == OP_H) hb |= 1u << op(k).rbit;
    if (hb == 15u) return RT_QFT4_H4;
  }
  if (n == 1 && (op(0).kind == OP_QFT || op(0).kind == OP_QFT_INV)) return RT_QFT1;
  if (n == 2 && op(0).kind == OP_QFT && op(1).kind == OP_H && op(0).rbit == op(1).rbit) return RT_QH1;
  if (n == 1 && (op(0).kind == OP_MAT || op(0).kind == OP_DIAG || op(0).kind == OP_H)) return RT_OP1;
  if (n > 4) return RT_GENERIC;
  uint32_t seen = 0;
  bool all_h = true;
  for (int k = 0; k < n; ++k) {
    const TileOp& o = op(k);
    if (o.kind != OP_MAT && o.kind != OP_DIAG && o.kind != OP_H) return RT_GENERIC;
    if ((seen >> o.rbit) & 1) return RT_GENERIC;
    seen |= 1u << o.rbit;
    all_h = all_h && o.kind == OP_H;
  }
  if (all_h && n == 4) return RT_H4;
  return RT_MAT4;
}

void finalize_pass(const PlanIR& P, TilePassIR& T) {
  const int RB = kRoundBits;
  int m = T.L + T.h;
  T.rounds.clear();
  T.ops.clear();
  T.op_src.clear();
  T.diag_slots.clear();
  T.n_coef = 0;
  T.n_butterfly = 0;
  int pending_diag = -1;
  auto emit_round = [&](std::vector<int> bits, const std::vector<int>& ops) {
    TileRound r;
    std::memset(&r, 0, sizeof r);
    r.qoff = -1;
    for (int tb = 0; (int)bits.size() < RB && tb < m; ++tb)
      if (std::find(bits.begin(), bits.end(), tb) == bits.end()) bits.push_back(tb);
    std::sort(bits.begin(), bits.end());
    for (int k = 0; k < RB; ++k) r.tbit[k] = bits[k];
    for (int j = 0; j < (1 << RB); ++j) {
      uint32_t o = 0;
      for (int k = 0; k < RB; ++k)
        if ((j >> k) & 1) o |= 1u << bits[k];
      r.loff[j] = lds_off(o);
    }
    r.op_begin = (int32_t)T.ops.size();
    int prev_qft_bit = -1, prev_qft_base = -1;
    for (int oi : ops) {
      const OpIR& o = P.ops[oi];
      TileOp op;
      std::memset(&op, 0, sizeof op);
      op.kind = o.kind;
      op.sbit = o.bit;
      op.base = o.base;
      int tb = tile_pos(T, o.bit);
      op.rbit = (int32_t)(std::find(bits.begin(), bits.end(), tb) - bits.begin());
      op.coef = T.n_coef;
      op.slot = -1;
      if (o.kind == OP_MAT) T.n_coef += 4;
      else if (o.kind == OP_DIAG) T.n_coef += 2;
      else if (o.kind == OP_QFT || o.kind == OP_QFT_INV) T.n_coef += 1 << op.rbit;
      if (o.kind == OP_QFT) {
        // exp(i pi low_p / 2^p) = (exp(i pi low_{p+1} / 2^{p+1}))^2 when bit p is a
        // round bit (zero in the group base) and both stages read the bits from
        // the same base (low_q = the group bits in [base, q)): the round then
        // evaluates its first stage's twiddle and squares it for the next (at
        // most three squarings in a row, each doubling the phase's relative
        // rounding error).  Stages with different bases (an approximate QFT,
        // two QFTs on adjacent registers) evaluate their own.
        op.square = (prev_qft_bit == o.bit + 1 && prev_qft_base == o.base) ? 1 : 0;
        prev_qft_bit = o.bit;
        prev_qft_base = o.base;
      }
      if (o.kind == OP_H || o.kind == OP_QFT || o.kind == OP_QFT_INV) T.n_butterfly += 1;
      T.ops.push_back(op);
      T.op_src.push_back(oi);
    }
    r.op_end = (int32_t)T.ops.size();
    r.diag = pending_diag;
    r.diag_conj = 0;
    r.type = classify_round(P, T, r);
    pending_diag = -1;
    if (r.type != RT_GENERIC) {
      if (r.type == RT_MAT4) {
        r.coef4 = T.n_coef;
        T.n_coef += 16;
      }
      T.rounds.push_back(r);
      return;
    }
    // split: consecutive single-qubit ops on distinct register bits form one
    // RT_MAT4 round; every QFT stage becomes an RT_QFT1 round
    int k = r.op_begin;
    bool first = true;
    while (k < r.op_end) {
      TileRound q = r;
      q.diag = first ? r.diag : -1;
      first = false;
      q.op_begin = k;
      if (T.ops[k].kind == OP_QFT || T.ops[k].kind == OP_QFT_INV) {
        q.op_end = k + 1;
        q.type = RT_QFT1;
        q.coef4 = -1;
        T.ops[k].square = 0;  // the stage it would square now sits in another round
        if (T.ops[k].kind == OP_QFT && k + 1 < r.op_end && T.ops[k + 1].kind == OP_H &&
            T.ops[k + 1].rbit == T.ops[k].rbit) {
          q.op_end = k + 2;
          q.type = RT_QH1;
        }
      } else {
        uint32_t seen = 0;
        int e = k;
        while (e < r.op_end && T.ops[e].kind != OP_QFT && T.ops[e].kind != OP_QFT_INV &&
               !((seen >> T.ops[e].rbit) & 1)) {
          seen |= 1u << T.ops[e].rbit;
          ++e;
        }
        q.op_end = e;
        if (e - k == 1) {
          q.type = RT_OP1;
          q.coef4 = -1;
        } else {
          q.type = RT_MAT4;
          q.coef4 = T.n_coef;
          T.n_coef += 16;
        }
      }
      k = q.op_end;
      T.rounds.push_back(q);
    }
  };
  // Ops between two diagonal items are packed into rounds greedily: each
  // round takes, in stream order, every op whose conflicting predecessors are
  // done and whose bit fits in the round's four register bits.
  auto pack = [&](const std::vector<int>& seg_ops) {
    size_t N = seg_ops.size();
    std::vector<char> done(N, 0);
    size_t left = N;
    while (left) {
      std::vector<int> bits, ops;
      bool progress = true;
      while (progress) {
        progress = false;
        for (size_t j = 0; j < N; ++j) {
          if (done[j]) continue;
          const OpIR& o = P.ops[seg_ops[j]];
          bool ready = true;
          for (size_t i = 0; i < j && ready; ++i)
            if (!done[i] && ops_conflict(P.ops[seg_ops[i]], o)) ready = false;
          if (!ready) continue;
          int tb = tile_pos(T, o.bit);
          if (tb < 0) fail(QS_EINVAL, "internal: op outside its tile");
          bool have = std::find(bits.begin(), bits.end(), tb) != bits.end();
          if (!have && (int)bits.size() == RB) continue;
          if (!have) bits.push_back(tb);
          ops.push_back(seg_ops[j]);
          done[j] = 1;
          --left;
          progress = true;
        }
      }
      emit_round(bits, ops);
    }
  };
  std::vector<int> seg_ops;
  for (auto& it : T.items) {
    if (it.type == 1) {
      if (!seg_ops.empty()) pack(seg_ops);
      seg_ops.clear();
      if (pending_diag >= 0) emit_round({}, {});  // two diagonals in a row
      pending_diag = (int)T.diag_slots.size();
      T.diag_slots.push_back(it.index);
      continue;
    }
    seg_ops.push_back(it.index);
  }
  if (!seg_ops.empty()) pack(seg_ops);
  if (pending_diag >= 0) emit_round({}, {});
  T.scale = std::pow(0.5, 0.5 * T.n_butterfly);
}

// Read / write masks of a pass item (the scheduler's conflict rule): an op
// writes its bit, a QFT stage also reads the bits below it down to its
// register base, a diagonal reads its support.
void item_masks(const PlanIR& P, const ItemIR& it, uint32_t& W, uint32_t& R) {
  if (it.type == 1) {
    W = 0;
    R = P.diags[it.index].support;
    return;
  }
  const OpIR& o = P.ops[it.index];
  W = 1u << o.bit;
  R = (o.kind == OP_QFT || o.kind == OP_QFT_INV) ? ((1u << o.bit) - 1u) & ~((1u << o.base) - 1u) : 0u;
}

// Vector-ALU work of a finalized pass per group of 16 amplitudes, in units of
// one register bit's 2x2 butterflies (64 lane operations): a four-bit round of
// 2x2 matrices or rotations about 4.5, a one-op round 1.5, a diagonal round 3,
// the tile's load and store 1.5.
double pass_work(const TilePassIR& T) {
  double w = 1.5;
  for (const TileRound& r : T.rounds) {
    if (r.op_end > r.op_begin) {
      if (r.type == RT_OP1 || r.type == RT_QFT1 || r.type == RT_QH1) w += 1.5;
      else if (r.type == RT_H4) w += 2.5;
      else w += 4.5;
    }
    if (r.diag >= 0) w += 3.0;
  }
  return w;
}

// A pass with diagonal layers followed by another tile pass: single-qubit ops
// after the pass's last diagonal, on bits that the next tile also holds,
// commute past the rest of the pass when nothing after them in it touches
// their bits, and may then run at the start of the next pass instead.  The
// pass carrying the diagonal is the one whose arithmetic approaches the
// memory time, so ops move (lowest bits first, as many as lower the larger
// of the two passes' work) when that evens out the pair.
void rebalance_diag_passes(PlanIR& P) {
  for (size_t li = 0; li + 1 < P.layers.size(); ++li) {
    if (P.layers[li].kind != L_TILE || P.layers[li + 1].kind != L_TILE) continue;
    TilePassIR& A = P.passes[P.layers[li].index];
    TilePassIR& B = P.passes[P.layers[li + 1].index];
    int last = -1;
    for (size_t k = 0; k < A.items.size(); ++k)
      if (A.items[k].type == 1) last = (int)k;
    if (last < 0) continue;
    std::vector<int> cand;  // candidate bits, ascending
    for (size_t k = last + 1; k < A.items.size(); ++k) {
      const OpIR& o = P.ops[A.items[k].index];
      if (o.kind == OP_QFT || o.kind == OP_QFT_INV || tile_pos(B, o.bit) < 0) continue;
      if (std::find(cand.begin(), cand.end(), o.bit) == cand.end()) cand.push_back(o.bit);
    }
    if (cand.empty()) continue;
    std::sort(cand.begin(), cand.end());
    auto split = [&](uint32_t S, TilePassIR& A2, TilePassIR& B2) -> bool {
      A2 = A;
      B2 = B;
      A2.items.assign(A.items.begin(), A.items.begin() + last + 1);
      std::vector<ItemIR> moved;
      for (size_t k = last + 1; k < A.items.size(); ++k) {
        const ItemIR& it = A.items[k];
        const OpIR& o = P.ops[it.index];
        const bool mv = (S >> o.bit) & 1u && o.kind != OP_QFT && o.kind != OP_QFT_INV;
        if (!mv) {
          A2.items.push_back(it);
          continue;
        }
        // every later item that stays must commute with it
        uint32_t W, R;
        item_masks(P, it, W, R);
        for (size_t k2 = k + 1; k2 < A.items.size(); ++k2) {
          const OpIR& o2 = P.ops[A.items[k2].index];
          if ((S >> o2.bit) & 1u && o2.kind != OP_QFT && o2.kind != OP_QFT_INV) continue;
          uint32_t W2, R2;
          item_masks(P, A.items[k2], W2, R2);
          if ((W & (W2 | R2)) || (W2 & R)) return false;
        }
        moved.push_back(it);
      }
      B2.items = moved;
      B2.items.insert(B2.items.end(), B.items.begin(), B.items.end());
      finalize_pass(P, A2);
      finalize_pass(P, B2);
      return true;
    };
    TilePassIR A0 = A, B0 = B;
    finalize_pass(P, A0);
    finalize_pass(P, B0);
    double best = std::max(pass_work(A0), pass_work(B0));
    uint32_t bestS = 0;
    uint32_t S = 0;
    for (int b : cand) {
      S |= 1u << b;
      TilePassIR A2, B2;
      if (!split(S, A2, B2)) continue;
      const double w = std::max(pass_work(A2), pass_work(B2));
      if (w < best - 1e-9) {
        best = w;
        bestS = S;
      }
    }
    if (bestS) {
      TilePassIR A2, B2;
      split(bestS, A2, B2);
      A.items = A2.items;
      B.items = B2.items;
    }
  }
}

}  // namespace

std::vector<PairNeighbours> pair_neighbours(const DiagNumeric& num, int n) {
  std::vector<PairNeighbours> out(num.groups.size());
  for (size_t g = 0; g < num.groups.size(); ++g) {
    PairNeighbours& P = out[g];
    bool ok = true;
    std::vector<uint64_t> seen;  // pair (lo, hi) as lo * 64 + hi, hi = 63 for a constant partner
    for (int t = num.groups[g].term_begin; t < num.groups[g].term_end && ok; ++t) {
      const DiagTerm& D = num.terms[t];
      if (D.form != DT_SHIFT_XOR || D.shift <= 0) {
        ok = false;
        break;
      }
      for (int j = 0; j < 32 && j < n; ++j) {
        if (!((D.mask >> j) & 1u)) continue;
        const int q = j + D.shift;
        const bool real = q < n;
        const uint64_t key = (uint64_t)j * 64 + (real ? q : 63);
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) {
          ok = false;
          break;
        }
        seen.push_back(key);
        P.deg[j] += 1;
        if (real) {
          P.deg[q] += 1;
          P.mask[j] |= 1u << q;
          P.mask[q] |= 1u << j;
        }
      }
    }
    if (!ok) P = PairNeighbours{};
    P.ok = ok;
  }
  return out;
}

// A structured plan of a gate list (no window fusion).
static PlanIR structured_plan(int n, std::vector<NGate> gates, size_t n_params, const PlanOptions& opt,
                              int tile_bits, int low_bits, int windows) {
  PlanIR P;
  P.n = n;
  P.n_params = n_params;
  P.opt = opt;
  P.gates = std::move(gates);
  P.tile_bits = tile_bits;
  P.low_bits = low_bits;
  P.windows = windows;
  {
    const Phase ph("qs.plan.schedule");
    Builder B(P, tile_bits, low_bits);
    B.run();
  }
  if (opt.balance_passes >= 0) {
    const Phase ph("qs.plan.balance");
    rebalance_diag_passes(P);
  }
  const Phase ph("qs.plan.rounds");
  for (auto& T : P.passes) finalize_pass(P, T);
  return P;
}

PlanIR build_plan(int n, std::vector<NGate> gates, size_t n_params, const PlanOptions& opt,
                  int tile_bits, int low_bits) {
  if (opt.mode == QS_PLAIN || n < kRoundBits) {
    PlanIR P;
    P.n = n;
    P.n_params = n_params;
    P.opt = opt;
    P.gates = std::move(gates);
    P.tile_bits = tile_bits;
    P.low_bits = low_bits;
    for (size_t i = 0; i < P.gates.size(); ++i) P.layers.push_back({L_PLAIN, (int32_t)i});
    return P;
  }
  const Phase ph("qs.plan.build");
  PlanIR best = structured_plan(n, gates, n_params, opt, tile_bits, low_bits, 0);
  // Generic matrix fusion of decomposed blocks (Section "Limitations and
  // Future Work"): candidates with dense windows over the whole stream and
  // chunk by chunk (each chunk of consecutive gates keeps its windows only
  // when they need fewer passes there), kept when cheaper than the
  // structured plan.
  const int kw = std::min(std::min(opt.window_k, opt.dense_k_max), std::min(n - 4, QS_MAX_GATE_WIRES));
  if (kw < 4) return best;
  double best_cost = plan_cost(best);
  const Phase phw("qs.plan.windows");
  std::vector<NGate> fused;
  const int formed = fuse_windows(n, gates, kw, fused);
  if (formed == 0) return best;
  PlanIR W = structured_plan(n, std::move(fused), n_params, opt, tile_bits, low_bits, formed);
  const double w_cost = plan_cost(W);
  constexpr size_t kChunk = 96;
  if (gates.size() > kChunk) {
    std::vector<NGate> mixed;
    int mixed_windows = 0;
    bool any_struct = false, any_win = false;
    for (size_t c0 = 0; c0 < gates.size(); c0 += kChunk) {
      std::vector<NGate> chunk(gates.begin() + c0, gates.begin() + std::min(gates.size(), c0 + kChunk));
      std::vector<NGate> fc;
      const int f = fuse_windows(n, chunk, kw, fc);
      bool use_win = false;
      if (f > 0) {
        const double cs = plan_cost(structured_plan(n, chunk, n_params, opt, tile_bits, low_bits, 0));
        const double cw = plan_cost(structured_plan(n, fc, n_params, opt, tile_bits, low_bits, f));
        use_win = cw < cs;
      }
      if (use_win) {
        mixed.insert(mixed.end(), fc.begin(), fc.end());
        mixed_windows += f;
        any_win = true;
      } else {
        mixed.insert(mixed.end(), chunk.begin(), chunk.end());
        any_struct = true;
      }
    }
    if (any_win && any_struct) {
      PlanIR M = structured_plan(n, std::move(mixed), n_params, opt, tile_bits, low_bits, mixed_windows);
      const double m_cost = plan_cost(M);
      if (m_cost < best_cost && m_cost < w_cost) return M;
    }
  }
  if (w_cost < best_cost) return W;
  return best;
}

// ---------------------------------------------------------------- numerics
std::vector<cd> op_matrix(const PlanIR& P, const OpIR& op, const std::vector<double>& params) {
  const double r = 1.0 / std::sqrt(2.0);
  const cd I(0, 1);
  if (op.fixed_h) {
    if (op.fixed_mat == 0) return {r, -I * r, r, I * r};   // H S^dagger
    if (op.fixed_mat == 1) return {r, r, I * r, -I * r};   // S H
    // closing change of one family times the opening change of the other
    if (op.fixed_mat == 2) return mul2({r, -I * r, r, I * r}, {r, r, r, -r});   // (H S^dagger) H
    if (op.fixed_mat == 3) return mul2({r, r, r, -r}, {r, r, I * r, -I * r});   // H (S H)
    return {r, r, r, -r};
  }
  if (op.kind == OP_H) return {r, r, r, -r};
  std::vector<cd> U = gate_matrix(P.gates[op.gates[0]], params);
  for (size_t j = 1; j < op.gates.size(); ++j) U = mul2(gate_matrix(P.gates[op.gates[j]], params), U);
  return U;
}

std::vector<cd> pass_coefficients(const PlanIR& P, const TilePassIR& T, const std::vector<double>& params) {
  std::vector<cd> coef((size_t)T.n_coef);
  auto opm = [&](int k) {
    std::vector<cd> U = op_matrix(P, P.ops[T.op_src[k]], params);
    return T.inverse ? dagger(U, 2) : U;
  };
  for (const TileRound& r : T.rounds) {
    if (r.type != RT_MAT4) continue;
    for (int b = 0; b < 4; ++b) {
      coef[r.coef4 + 4 * b] = 1.0;
      coef[r.coef4 + 4 * b + 3] = 1.0;
    }
    for (int k = r.op_begin; k < r.op_end; ++k) {
      const TileOp& op = T.ops[k];
      std::vector<cd> U;
      if (op.kind == OP_H) U = {1.0, 1.0, 1.0, -1.0};  // unscaled butterfly
      else U = opm(k);
      if (op.kind == OP_DIAG) U = {U[0], 0.0, 0.0, U[3]};
      for (int e = 0; e < 4; ++e) coef[r.coef4 + 4 * op.rbit + e] = U[e];
    }
  }
  for (size_t k = 0; k < T.ops.size(); ++k) {
    const TileOp& op = T.ops[k];
    if (T.op_src[k] < 0) continue;
    if (op.kind == OP_MAT) {
      auto U = opm((int)k);
      for (int e = 0; e < 4; ++e) coef[op.coef + e] = U[e];
    } else if (op.kind == OP_DIAG) {
      auto U = opm((int)k);
      coef[op.coef] = U[0];
      coef[op.coef + 1] = U[3];
    } else if (op.kind == OP_QFT || op.kind == OP_QFT_INV) {
      // intra-round twiddles: register bits below the op's bit
      const TileRound* R = nullptr;
      for (auto& r : T.rounds)
        if ((int)k >= r.op_begin && (int)k < r.op_end) R = &r;
      int s = op.rbit, p = op.sbit;
      for (int kk = 0; kk < (1 << s); ++kk) {
        double frac = 0.0;  // sum bit_t(kk) 2^(sb_t - p), exact in FP64
        for (int t = 0; t < s; ++t) {
          const int sb = tile_state_bit(T, R->tbit[t]);
          if (((kk >> t) & 1) && sb >= op.base) frac += std::ldexp(1.0, sb - p);
        }
        coef[op.coef + kk] = std::polar(1.0, kPi * frac);
      }
    }
  }
  return coef;
}

std::vector<TileRound> pass_rounds(const PlanIR& P, const TilePassIR& T, const std::vector<cd>& coef) {
  (void)P;
  std::vector<TileRound> rounds = T.rounds;
  for (TileRound& r : rounds) {
    if (r.type != RT_MAT4) continue;
    bool rx = true, ry = true;
    for (int b = 0; b < 4; ++b) {
      const cd* U = &coef[r.coef4 + 4 * b];
      rx = rx && U[0] == U[3] && U[0].imag() == 0.0 && U[1] == U[2] && U[1].real() == 0.0;
      ry = ry && U[0] == U[3] && U[0].imag() == 0.0 && U[1] == -U[2] && U[1].imag() == 0.0 && U[2].imag() == 0.0;
    }
    if (rx) r.type = RT_MAT4_RX;
    else if (ry) r.type = RT_MAT4_RY;
  }
  return rounds;
}

// Device coefficient array: RX / RY rounds store (a, b) per register bit at
// coef4 + r instead of the full matrices.
std::vector<cd> pass_coefficients_device(const PlanIR& P, const TilePassIR& T, const std::vector<double>& params,
                                         std::vector<TileRound>& rounds) {
  std::vector<cd> coef = pass_coefficients(P, T, params);
  rounds = pass_rounds(P, T, coef);
  for (const TileRound& r : rounds) {
    if (r.type == RT_MAT4_RX) {
      for (int b = 0; b < 4; ++b) {
        const cd* U = &coef[r.coef4 + 4 * b];
        coef[r.coef4 + b] = cd(U[0].real(), -U[1].imag());
      }
    } else if (r.type == RT_MAT4_RY) {
      for (int b = 0; b < 4; ++b) {
        const cd* U = &coef[r.coef4 + 4 * b];
        coef[r.coef4 + b] = cd(U[0].real(), U[2].real());
      }
    }
  }
  return coef;
}

// ---------------------------------------------------------------- adjoint support
std::vector<cd> dagger(const std::vector<cd>& M, int d) {
  std::vector<cd> R((size_t)d * d);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) R[(size_t)r * d + c] = std::conj(M[(size_t)c * d + r]);
  return R;
}

static TilePassIR invert_pass(const PlanIR& P, const TilePassIR& F) {
  TilePassIR T;
  T.L = F.L;
  T.a = F.a;
  T.h = F.h;
  T.inverse = true;
  T.diag_slots = F.diag_slots;
  T.n_butterfly = F.n_butterfly;
  T.scale = F.scale;
  int carry_diag = -1;  // a forward round's diagonal, undone after its inverted ops
  auto push_round = [&](const TileRound& src, std::vector<int> fwd_ops, int diag_before) {
    TileRound r = src;
    r.op_begin = (int32_t)T.ops.size();
    for (auto it = fwd_ops.rbegin(); it != fwd_ops.rend(); ++it) {
      TileOp op = F.ops[*it];
      if (op.kind == OP_QFT) op.kind = OP_QFT_INV;
      else if (op.kind == OP_QFT_INV) op.kind = OP_QFT;
      op.square = 0;
      op.coef = T.n_coef;
      if (op.kind == OP_MAT) T.n_coef += 4;
      else if (op.kind == OP_DIAG) T.n_coef += 2;
      else if (op.kind == OP_QFT_INV || op.kind == OP_QFT) T.n_coef += 1 << op.rbit;
      T.ops.push_back(op);
      T.op_src.push_back(F.op_src[*it]);
    }
    r.op_end = (int32_t)T.ops.size();
    r.diag = diag_before;
    r.diag_conj = 1;
    r.type = classify_round(P, T, r);
    r.coef4 = -1;
    if (r.type == RT_GENERIC) {
      // split, as in finalize_pass
      int k = r.op_begin;
      bool first = true;
      while (k < r.op_end) {
        TileRound q = r;
        q.diag = first ? r.diag : -1;
        first = false;
        q.op_begin = k;
        if (T.ops[k].kind == OP_QFT_INV || T.ops[k].kind == OP_QFT) {
          q.op_end = k + 1;
          q.type = RT_QFT1;
        } else {
          uint32_t seen = 0;
          int e = k;
          while (e < r.op_end && T.ops[e].kind != OP_QFT_INV && T.ops[e].kind != OP_QFT &&
                 !((seen >> T.ops[e].rbit) & 1)) {
            seen |= 1u << T.ops[e].rbit;
            ++e;
          }
          q.op_end = e;
          if (e - k == 1) {
            q.type = RT_OP1;
          } else {
            q.type = RT_MAT4;
            q.coef4 = T.n_coef;
            T.n_coef += 16;
          }
        }
        k = q.op_end;
        T.rounds.push_back(q);
      }
      return;
    }
    if (r.type == RT_MAT4) {
      r.coef4 = T.n_coef;
      T.n_coef += 16;
    }
    T.rounds.push_back(r);
  };
  for (auto it = F.rounds.rbegin(); it != F.rounds.rend(); ++it) {
    std::vector<int> ops;
    for (int k = it->op_begin; k < it->op_end; ++k) ops.push_back(k);
    push_round(*it, ops, carry_diag);
    carry_diag = it->diag;
  }
  if (carry_diag >= 0) push_round(F.rounds.front(), {}, carry_diag);
  return T;
}

static Gf2IR invert_gf2(int n, const Gf2IR& G) {
  // forward: out[y] = in[A y ^ c'];  inverse: out[x] = in[M x ^ M c'], M = A^{-1}
  std::vector<uint32_t> aug(n);  // rows of [A | I]
  std::vector<uint32_t> A = G.rows, inv(n);
  for (int r = 0; r < n; ++r) inv[r] = 1u << r;
  for (int c = 0; c < n; ++c) {
    int piv = -1;
    for (int r = c; r < n; ++r)
      if ((A[r] >> c) & 1) { piv = r; break; }
    if (piv < 0) fail(QS_EINVAL, "permutation block is not invertible");
    std::swap(A[c], A[piv]);
    std::swap(inv[c], inv[piv]);
    for (int r = 0; r < n; ++r)
      if (r != c && ((A[r] >> c) & 1)) { A[r] ^= A[c]; inv[r] ^= inv[c]; }
  }
  Gf2IR R;
  R.rows = inv;
  uint32_t c2 = 0;
  for (int r = 0; r < n; ++r) c2 |= (uint32_t)(__builtin_popcount(inv[r] & G.cprime) & 1) << r;
  R.cprime = c2;
  R.gates = G.gates;
  return R;
}

PlanIR invert_plan(const PlanIR& F) {
  PlanIR P;
  P.n = F.n;
  P.n_params = F.n_params;
  P.opt = F.opt;
  P.gates = F.gates;
  P.diags = F.diags;
  P.denses = F.denses;
  P.ops = F.ops;
  P.tile_bits = F.tile_bits;
  P.low_bits = F.low_bits;
  P.windows = F.windows;
  for (auto it = F.layers.rbegin(); it != F.layers.rend(); ++it) {
    LayerIR L = *it;
    if (L.kind == L_TILE) {
      L.index = (int32_t)P.passes.size();
      P.passes.push_back(invert_pass(F, F.passes[it->index]));
    } else if (L.kind == L_GF2) {
      L.index = (int32_t)P.gf2s.size();
      P.gf2s.push_back(invert_gf2(F.n, F.gf2s[it->index]));
    } else {
      L.inverse = 1;
    }
    P.layers.push_back(L);
  }
  return P;
}

// u^dagger du/dangle for the rotation kinds (angle derivative, before `scale`)
static std::vector<cd> gen_of(int kind) {
  const cd mi(0, -0.5);
  switch (kind) {
    case QS_GATE_RX: return {0, mi, mi, 0};
    case QS_GATE_RY: return {0, -0.5, 0.5, 0};  // -(i/2) Y
    case QS_GATE_RZ: return {mi, 0, 0, -mi};
    case QS_GATE_P: return {0, 0, 0, cd(0, 1)};
    default: fail(QS_EUNSUPPORTED, "adjoint gradient for this parametrised gate kind");
  }
}

std::vector<std::vector<GradEntry>> grad_entries(const PlanIR& P, const std::vector<double>& params) {
  std::vector<std::vector<GradEntry>> out(P.layers.size());
  for (size_t li = 0; li < P.layers.size(); ++li) {
    const LayerIR& L = P.layers[li];
    if (L.kind == L_PLAIN) {
      if (!P.gates[L.index].angle.is_const()) fail(QS_EUNSUPPORTED, "parameter on a gate run by the plain path");
      continue;
    }
    if (L.kind == L_GF2 || L.kind == L_DENSE) continue;
    if (L.kind == L_DIAG) {
      const DiagIR& D = P.diags[L.index];
      for (size_t g = 0; g < D.groups.size(); ++g)
        for (auto& t : D.groups[g].angle.lin)
          out[li].push_back({1, -1, t.first, t.second, {0, 0, 0, 0}, L.index, (int32_t)g});
      continue;
    }
    const TilePassIR& T = P.passes[L.index];
    // device op order of the pass, with the diagonal slots in between
    std::vector<std::pair<int, int>> seq;  // (0, op) or (1, slot)
    for (const TileRound& r : T.rounds) {
      if (r.diag >= 0) seq.push_back({1, r.diag});
      for (int k = r.op_begin; k < r.op_end; ++k) seq.push_back({0, k});
    }
    for (size_t pos = 0; pos < seq.size(); ++pos) {
      if (seq[pos].first == 1) {
        const DiagIR& D = P.diags[T.diag_slots[seq[pos].second]];
        bool has = false;
        for (auto& G : D.groups) has = has || !G.angle.is_const();
        if (has) fail(QS_EUNSUPPORTED, "parametrised diagonal fused inside a tile pass");
        continue;
      }
      const int k = seq[pos].second;
      const TileOp& op = T.ops[k];
      if (T.op_src[k] < 0) continue;
      const OpIR& o = P.ops[T.op_src[k]];
      bool param = false;
      for (int gi : o.gates) param = param || !P.gates[gi].angle.is_const();
      if (!param) continue;
      // every earlier op of the pass must commute with an operator on this bit
      for (size_t q = 0; q < pos; ++q) {
        bool clash = false;
        if (seq[q].first == 1) {
          clash = (P.diags[T.diag_slots[seq[q].second]].support >> op.sbit) & 1;
        } else {
          const TileOp& e = T.ops[seq[q].second];
          clash = e.sbit == op.sbit || ((e.kind == OP_QFT || e.kind == OP_QFT_INV) && e.sbit > op.sbit);
        }
        if (clash) fail(QS_EUNSUPPORTED, "parametrised window follows a non-commuting op in its pass");
      }
      std::vector<cd> V = {1, 0, 0, 1};  // product of the window's gates before gate m
      for (size_t m = 0; m < o.gates.size(); ++m) {
        const NGate& g = P.gates[o.gates[m]];
        if (!g.angle.is_const()) {
          std::vector<cd> G = gen_of(g.kind);
          std::vector<cd> K = mul2(dagger(V, 2), mul2(G, V));
          for (auto& t : g.angle.lin) {
            GradEntry e{0, op.sbit, t.first, t.second, {K[0], K[1], K[2], K[3]}, -1, -1};
            out[li].push_back(e);
          }
        }
        V = mul2(gate_matrix(g, params), V);
      }
    }
  }
  return out;
}

// ---------------------------------------------------------------- describe
static void jnum(std::ostringstream& o, double v) {
  char b[40];
  std::snprintf(b, sizeof b, "%.17g", v);
  o << b;
}
static void jc(std::ostringstream& o, cd v) {
  o << "[";
  jnum(o, v.real());
  o << ",";
  jnum(o, v.imag());
  o << "]";
}

static void describe_diag(std::ostringstream& o, const DiagIR& d, const std::vector<double>& params, bool bound) {
  o << "{\"support\":" << d.support << ",\"groups\":[";
  for (size_t g = 0; g < d.groups.size(); ++g) {
    if (g) o << ",";
    o << "{\"terms\":[";
    for (size_t t = 0; t < d.groups[g].terms.size(); ++t) {
      auto& tt = d.groups[g].terms[t];
      if (t) o << ",";
      o << "[" << tt.form << "," << tt.shift << "," << tt.mask << "]";
    }
    o << "],\"max_count\":" << d.groups[g].max_count << "}";
  }
  o << "]";
  if (bound) {
    DiagNumeric num = diag_numeric(d, params);
    o << ",\"lut\":[";
    for (size_t i = 0; i < num.lut.size(); ++i) { if (i) o << ","; jc(o, num.lut[i]); }
    o << "],\"lut_groups\":[";
    for (size_t i = 0; i < num.groups.size(); ++i) {
      if (i) o << ",";
      o << "[" << num.groups[i].term_begin << "," << num.groups[i].term_end << ","
        << num.groups[i].lut_begin << "," << num.groups[i].lut_len << "]";
    }
    o << "],\"lut_terms\":[";
    for (size_t i = 0; i < num.terms.size(); ++i) {
      if (i) o << ",";
      o << "[" << num.terms[i].form << "," << num.terms[i].shift << "," << num.terms[i].mask << "]";
    }
    o << "]";
  }
  o << "}";
}

std::string describe_json(const PlanIR& P, const std::vector<double>& params, bool bound) {
  std::ostringstream o;
  o << "{\"n\":" << P.n << ",\"n_params\":" << P.n_params << ",\"mode\":"
    << (P.opt.mode == QS_PLAIN ? "\"plain\"" : "\"fused\"") << ",\"tile_bits\":" << P.tile_bits
    << ",\"bound\":" << (bound ? "true" : "false") << ",\"windows\":" << P.windows << ",\"layers\":[";
  for (size_t li = 0; li < P.layers.size(); ++li) {
    if (li) o << ",";
    const LayerIR& L = P.layers[li];
    if (L.kind == L_DIAG) {
      o << "{\"kind\":\"diag\",\"inverse\":" << L.inverse << ",\"diag\":";
      describe_diag(o, P.diags[L.index], params, bound);
      o << "}";
    } else if (L.kind == L_GF2) {
      const Gf2IR& G = P.gf2s[L.index];
      o << "{\"kind\":\"gf2\",\"rows\":[";
      for (size_t r = 0; r < G.rows.size(); ++r) { if (r) o << ","; o << G.rows[r]; }
      o << "],\"cprime\":" << G.cprime << ",\"n_gates\":" << G.gates.size() << "}";
    } else if (L.kind == L_DENSE) {
      const DenseIR& D = P.denses[L.index];
      o << "{\"kind\":\"dense\",\"inverse\":" << L.inverse << ",\"gate\":" << P.gates[D.gate].index
        << ",\"window\":" << P.gates[D.gate].fused << ",\"bits\":[";
      for (size_t b = 0; b < D.bits.size(); ++b) { if (b) o << ","; o << D.bits[b]; }
      o << "],\"mat\":[";
      const std::vector<cd>& M = L.inverse ? D.mat_dagger : D.mat;
      o << std::setprecision(17);
      for (size_t e = 0; e < M.size(); ++e) {
        if (e) o << ",";
        o << "[" << M[e].real() << "," << M[e].imag() << "]";
      }
      o << "]}";
    } else if (L.kind == L_PLAIN) {
      const NGate& g = P.gates[L.index];
      o << "{\"kind\":\"plain\",\"inverse\":" << L.inverse << ",\"gate\":" << g.index
        << ",\"gate_kind\":" << g.kind << ",\"bits\":[";
      for (size_t b = 0; b < g.bits.size(); ++b) { if (b) o << ","; o << g.bits[b]; }
      o << "]}";
    } else {
      const TilePassIR& T = P.passes[L.index];
      o << "{\"kind\":\"tile\",\"inverse\":" << (T.inverse ? 1 : 0) << ",\"L\":" << T.L << ",\"a\":" << T.a
        << ",\"h\":" << T.h << ",\"rounds\":[";
      for (size_t r = 0; r < T.rounds.size(); ++r) {
        auto& R = T.rounds[r];
        if (r) o << ",";
        o << "{\"tbits\":[" << R.tbit[0] << "," << R.tbit[1] << "," << R.tbit[2] << "," << R.tbit[3]
          << "],\"diag\":" << R.diag << ",\"type\":" << R.type << ",\"ops\":[" << R.op_begin << "," << R.op_end
          << "]}";
      }
      o << "],\"ops\":[";
      std::vector<cd> coef;
      if (bound) coef = pass_coefficients(P, T, params);
      for (size_t k = 0; k < T.ops.size(); ++k) {
        auto& op = T.ops[k];
        if (k) o << ",";
        o << "{\"kind\":" << op.kind << ",\"bit\":" << op.sbit << ",\"rbit\":" << op.rbit
          << ",\"square\":" << op.square << ",\"base\":" << op.base;
        if (bound) {
          int nc = op.kind == OP_MAT ? 4 : op.kind == OP_DIAG ? 2
                   : (op.kind == OP_QFT || op.kind == OP_QFT_INV) ? (1 << op.rbit) : 0;
          o << ",\"coef\":[";
          for (int e = 0; e < nc; ++e) { if (e) o << ","; jc(o, coef[op.coef + e]); }
          o << "]";
        }
        o << "}";
      }
      o << "],\"diags\":[";
      for (size_t s = 0; s < T.diag_slots.size(); ++s) {
        if (s) o << ",";
        describe_diag(o, P.diags[T.diag_slots[s]], params, bound);
      }
      o << "]}";
    }
  }
  o << "]}";
  return o.str();
}

}  // namespace qs
