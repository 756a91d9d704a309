// Layer execution, plan device tables and reduction drivers.
#include "runtime.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

namespace qs {

namespace {

struct Blob {
  std::vector<unsigned char> bytes;
  template <class T>
  size_t put(const std::vector<T>& v) {
    size_t off = (bytes.size() + 15) & ~size_t(15);
    bytes.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

template <class R>
std::vector<cplx<R>> cast(const std::vector<cd>& v) {
  std::vector<cplx<R>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = {(R)v[i].real(), (R)v[i].imag()};
  return o;
}

// Diagonal rounds of layers with at least this many groups (all quadratic)
// evaluate the total phase angle instead of one table lookup per group.
constexpr int kAngleModeGroups = 3;

// Pair coefficients of a diagonal round.  Over the round's four register bits
// (state bits g_0..g_3) a group's count is a polynomial of degree <= 2 when all
// its terms are BITS, SHIFT_XOR or SHIFT_AND: x XOR y = x + y - 2xy and
// x AND y = xy for a bond on two register bits, linear or constant otherwise.
// The kernel then evaluates the count at the group's base index and at the
// four single-bit flips, and adds q_kl for every pair of set register bits.
// Row per group (kPairRowWords 32-bit words): {quadratic flag, q01, q02, q03,
// q12, q13, q23, pair flag, deg_0..deg_3, N_0..N_3}.  With the pair flag set
// (a sum of distinct bit-pair mismatches) the kernel obtains the four flipped
// counts from the base count as base + deg_k - 2 popcount(N_k & base) instead
// of evaluating every term four more times.  Whole words keep every field a
// scalar load in the kernel.
void round_pair_table(const DiagNumeric& num, const std::vector<PairNeighbours>& pn, const int g[4],
                      std::vector<int32_t>& out) {
  static const int pk[6] = {0, 0, 0, 1, 1, 2}, pl[6] = {1, 2, 3, 2, 3, 3};
  for (size_t gi = 0; gi < num.groups.size(); ++gi) {
    const DiagGroup& G = num.groups[gi];
    int32_t row[kPairRowWords] = {1, 0};
    int q[6] = {0, 0, 0, 0, 0, 0};
    for (int t = G.term_begin; t < G.term_end; ++t) {
      const DiagTerm& T = num.terms[t];
      if (T.form == DT_BITS) continue;
      if (T.form != DT_SHIFT_XOR && T.form != DT_SHIFT_AND) {
        row[0] = 0;
        break;
      }
      for (int e = 0; e < 6; ++e) {
        const int lo = std::min(g[pk[e]], g[pl[e]]), hi = std::max(g[pk[e]], g[pl[e]]);
        if (hi - lo == T.shift && ((T.mask >> lo) & 1u)) q[e] += T.form == DT_SHIFT_XOR ? -2 : 1;
      }
    }
    for (int e = 0; e < 6; ++e) row[1 + e] = q[e];
    if (row[0] != 0 && pn[gi].ok) {
      row[7] = 1;
      for (int k = 0; k < 4; ++k) {
        row[8 + k] = pn[gi].deg[g[k]];
        std::memcpy(row + 12 + k, &pn[gi].mask[g[k]], 4);
      }
    }
    out.insert(out.end(), row, row + kPairRowWords);
  }
}

// A 2x2 matrix M = lambda V (V unitary, lambda > 0) as lambda c D2 T(t) D1
// with T(t) = [[1, -t], [t, 1]], D1 = diag(1, p1) and D2 = diag(q0, q1) unit
// phases, c = |V11| and t real: V11 = c q1 p1, V10 = c t q1, V00 = c q0 and
// V01 = -c t q0 p1.  p1 = 1 when V10 / V11 is real (t keeps its sign), else
// the phase that makes t = |V10 / V11|.  A D1 that is not all ones takes
// D2's common phase q0 (then D2 = diag(1, q1 / q0)), so that rounds of one
// kind of rotation pair (RZ after RY, or RY after RZ) need one table only.
// False when M is not a scaled unitary or |t| > 8 (the bound of the
// factored rotations).
struct ZyzFactor {
  cd p0 = 1.0, p1 = 1.0, q0 = 1.0, q1 = 1.0;
  double t = 0.0, scale = 1.0;
};
static bool zyz_factor(const cd* M, ZyzFactor& f) {
  const double lam = std::sqrt(std::abs(M[0] * M[3] - M[1] * M[2]));
  if (!(lam > 0.0)) return false;
  const cd V[4] = {M[0] / lam, M[1] / lam, M[2] / lam, M[3] / lam};
  // unitarity: unit columns, orthogonal
  if (std::fabs(std::norm(V[0]) + std::norm(V[2]) - 1.0) > 1e-10 ||
      std::fabs(std::norm(V[1]) + std::norm(V[3]) - 1.0) > 1e-10 ||
      std::abs(std::conj(V[0]) * V[1] + std::conj(V[2]) * V[3]) > 1e-10)
    return false;
  const double c = std::abs(V[3]);
  if (!(c > 0.0)) return false;
  const cd r = V[2] / V[3];
  if (std::abs(r) > 8.0) return false;
  if (std::fabs(r.imag()) <= 1e-15 * std::abs(r)) {
    f.p1 = 1.0;
    f.t = r.real();
  } else {
    f.p1 = std::abs(r) / r;
    f.t = std::abs(r);
  }
  f.q1 = V[3] / (c * f.p1);
  f.q0 = V[0] / c;
  f.q0 /= std::abs(f.q0);
  f.q1 /= std::abs(f.q1);
  f.p1 /= std::abs(f.p1);
  if (std::abs(-c * f.t * f.q0 * f.p1 - V[1]) > 1e-10) return false;
  if (std::abs(f.p1 - 1.0) > 1e-15) {
    f.p0 = f.q0;
    f.p1 *= f.q0;
    f.q1 /= f.q0;
    f.q0 = 1.0;
  }
  f.scale = lam * c;
  return true;
}

// The rotations and 2x2 unitaries a tile pass applies, rounded to float in
// round order with the plan's running norm compensation (fround.h); the
// entries were first rounded one by one (phases to unit modulus).
template <class R>
void round_pass_unitaries(const TilePassIR& T, const std::vector<TileRound>& rounds, const std::vector<cd>& coef,
                          std::vector<cplx<R>>& cr, NormAcc& acc) {
  auto mat2 = [&](int off) {
    if (off < 0 || (size_t)off + 4 > coef.size()) return;
    cplx<float> f[4];
    fround_unitary2(&coef[off], f, acc);
    for (int e = 0; e < 4; ++e) cr[off + e] = {(R)f[e].re, (R)f[e].im};
  };
  for (const TileRound& r : rounds) {
    if (r.type == RT_MAT4) {
      for (int bb = 0; bb < 4; ++bb) mat2(r.coef4 + 4 * bb);
    } else if (r.type == RT_MAT4_RX || r.type == RT_MAT4_RY || r.type == RT_DIAG_PAIR_RX) {
      for (int bb = 0; bb < 4; ++bb) {
        const cplx<float> f = fround_pair(coef[r.coef4 + bb], acc);
        cr[r.coef4 + bb] = {(R)f.re, (R)f.im};
      }
    } else if (r.type == RT_MAT4_RXF || r.type == RT_MAT4_RYF || r.type == RT_DIAG_PAIR_RXF ||
               r.type == RT_ZYZ4 || r.type == RT_YZ4 || r.type == RT_ZY4) {
      continue;  // factored rotations: their norm is in the pass scale
    } else {
      for (int k = r.op_begin; k < r.op_end; ++k) {
        const TileOp& op = T.ops[k];
        if (op.kind == OP_MAT) {
          mat2(op.coef);
        } else if (op.kind == OP_DIAG) {
          const cd D[4] = {coef[op.coef], 0.0, 0.0, coef[op.coef + 1]};
          cplx<float> f[4];
          fround_unitary2(D, f, acc);
          cr[op.coef] = {(R)f[0].re, (R)f[0].im};
          cr[op.coef + 1] = {(R)f[3].re, (R)f[3].im};
        }
      }
    }
  }
}

template <class R>
void build_blob(const qs_plan& p, PlanDev& d, Blob& b) {
  const PlanIR& P = p.ir;
  NormAcc acc;
  d.diag_terms.assign(P.diags.size(), 0);
  d.diag_groups.assign(P.diags.size(), 0);
  d.diag_lut.assign(P.diags.size(), 0);
  d.diag_ngroups.assign(P.diags.size(), 0);
  d.diag_theta.assign(P.diags.size(), 0);
  d.diag_global.assign(P.diags.size(), 0.0);
  std::vector<DiagNumeric> nums;
  std::vector<std::vector<PairNeighbours>> pns;
  for (size_t i = 0; i < P.diags.size(); ++i) {
    DiagNumeric num = diag_numeric(P.diags[i], p.params);
    pns.push_back(pair_neighbours(num, P.n));
    d.diag_terms[i] = b.put(num.terms);
    d.diag_groups[i] = b.put(num.groups);
    d.diag_lut[i] = b.put(round_entries<R>(num.lut));
    d.diag_ngroups[i] = (int)num.groups.size();
    d.diag_theta[i] = b.put(num.theta);
    d.diag_global[i] = num.global;
    nums.push_back(std::move(num));
  }
  d.pass_rounds.assign(P.passes.size(), 0);
  d.pass_ops.assign(P.passes.size(), 0);
  d.pass_coef.assign(P.passes.size(), 0);
  d.pass_diag.assign(P.passes.size(), 0);
  d.pass_qtab.assign(P.passes.size(), 0);
  d.pass_nrounds.assign(P.passes.size(), 0);
  d.pass_scale.assign(P.passes.size(), 1.0);
  for (size_t i = 0; i < P.passes.size(); ++i) {
    const TilePassIR& T = P.passes[i];
    std::vector<TileRound> planned, rounds;
    std::vector<cd> coef = pass_coefficients_device(P, T, p.params, planned);
    // A round's diagonal runs as a round of its own over the same register
    // bits (RT_DIAG), so that the butterfly rounds' code carries no phase
    // evaluation; a one-group layer in the pair-mismatch form has its own
    // round (RT_DIAG_PAIR), fused with a following rotation round into one
    // (RT_DIAG_PAIR_RX).
    std::vector<int32_t> qtab;
    for (TileRound r : planned) {
      r.qoff = -1;
      r.qcoef = -1;
      if (r.diag < 0) {
        rounds.push_back(r);
        continue;
      }
      int g[4];
      for (int k = 0; k < 4; ++k) g[k] = r.tbit[k] < T.L ? r.tbit[k] : r.tbit[k] - T.L + T.a;
      const DiagNumeric& num = nums[T.diag_slots[r.diag]];
      TileRound dr = r;
      dr.op_end = dr.op_begin;
      dr.coef4 = -1;
      dr.type = RT_DIAG;
      dr.qoff = (int32_t)qtab.size();
      round_pair_table(num, pns[T.diag_slots[r.diag]], g, qtab);
      const int32_t* row0 = qtab.data() + dr.qoff;
      if (num.groups.size() == 1 && row0[0] && row0[7]) {
        if (r.type == RT_MAT4_RX) {
          r.type = RT_DIAG_PAIR_RX;
          r.qoff = dr.qoff;
          rounds.push_back(r);
          continue;
        }
        dr.type = RT_DIAG_PAIR;
      } else {
        // angle mode for layers with many groups, all quadratic: the six pair
        // phases exp(i sum_g theta_g q_g,kl) join the pass's coefficients
        bool all_quad = num.groups.size() >= (size_t)kAngleModeGroups;
        for (size_t gi = 0; gi < num.groups.size(); ++gi)
          all_quad = all_quad && qtab[dr.qoff + kPairRowWords * gi] != 0;
        if (all_quad) {
          dr.qcoef = (int32_t)coef.size();
          for (int e = 0; e < 6; ++e) {
            double Q = 0.0;
            for (size_t gi = 0; gi < num.groups.size(); ++gi)
              Q += num.theta[gi] * qtab[dr.qoff + kPairRowWords * gi + 1 + e];
            coef.push_back(std::polar(1.0, Q));
          }
        }
      }
      rounds.push_back(dr);
      r.diag = -1;
      rounds.push_back(r);
    }
    d.pass_nrounds[i] = (uint32_t)rounds.size();
    // Rotation rounds (RX / RY, alone or after a pair diagonal) whose four
    // matrices all have |b| <= 8 |a| run factored: [[a, -i b], [-i b, a]] =
    // a [[1, -i t], [-i t, 1]] with t = b / a (RY alike), one multiply-add
    // per output component in the kernel, the factors a joining the pass
    // scale applied at the store.  With t rounded to the state's precision
    // the factor is taken as a sqrt((1 + t^2) / (1 + t'^2)), which keeps a
    // unitary rotation unitary for the rounded t'.  The bound on |t| keeps the
    // unnormalised amplitudes of a pass far from overflow.
    double pscale = T.scale;
    std::vector<int32_t> rot_coef;  // coefficient indices in factored form
    for (TileRound& r : rounds) {
      if (r.type != RT_MAT4_RX && r.type != RT_MAT4_RY && r.type != RT_DIAG_PAIR_RX) continue;
      bool ok = true;
      for (int bb = 0; bb < 4; ++bb) {
        const cd e = coef[r.coef4 + bb];
        ok = ok && e.real() != 0.0 && std::fabs(e.imag()) <= 8.0 * std::fabs(e.real());
      }
      if (!ok) continue;
      r.type = r.type == RT_MAT4_RX ? RT_MAT4_RXF : (r.type == RT_MAT4_RY ? RT_MAT4_RYF : RT_DIAG_PAIR_RXF);
      for (int bb = 0; bb < 4; ++bb) {
        cd& e = coef[r.coef4 + bb];
        rot_coef.push_back(r.coef4 + bb);
        const double t = e.imag() / e.real();
        const double tr = sizeof(R) == sizeof(float) ? (double)(float)t : t;
        pscale *= e.real() * std::sqrt((1.0 + t * t) / (1.0 + tr * tr));
        e = cd(tr, 0.0);
      }
    }
    // General single-qubit rounds (RT_MAT4) whose matrices all factor as
    // D2 T D1 (zyz_factor): two 16-entry phase tables (one when the other is
    // all ones) and four factored real rotations, whose factors join the
    // pass scale with the same unitarity correction as above.
    for (TileRound& r : rounds) {
      if (r.type != RT_MAT4) continue;
      ZyzFactor f[4];
      bool ok = true;
      for (int bb = 0; bb < 4 && ok; ++bb) ok = zyz_factor(&coef[r.coef4 + 4 * bb], f[bb]);
      if (!ok) continue;
      bool d1 = false, d2 = false;
      for (int bb = 0; bb < 4; ++bb) {
        d1 = d1 || std::abs(f[bb].p0 - 1.0) > 1e-15 || std::abs(f[bb].p1 - 1.0) > 1e-15;
        d2 = d2 || std::abs(f[bb].q0 - 1.0) > 1e-15 || std::abs(f[bb].q1 - 1.0) > 1e-15;
      }
      const int32_t off = (int32_t)coef.size();
      auto table = [&](bool first) {
        for (int j = 0; j < 16; ++j) {
          cd v = 1.0;
          for (int bb = 0; bb < 4; ++bb)
            v *= first ? ((j >> bb) & 1 ? f[bb].p1 : f[bb].p0) : ((j >> bb) & 1 ? f[bb].q1 : f[bb].q0);
          coef.push_back(v / std::abs(v));
        }
      };
      if (d1) table(true);
      if (d2 || !d1) table(false);
      for (int bb = 0; bb < 4; ++bb) {
        const double t = f[bb].t;
        const double tr = sizeof(R) == sizeof(float) ? (double)(float)t : t;
        pscale *= f[bb].scale * std::sqrt((1.0 + t * t) / (1.0 + tr * tr));
        rot_coef.push_back((int32_t)coef.size());
        coef.push_back(cd(tr, 0.0));
      }
      r.coef4 = off;
      r.type = d1 && d2 ? RT_ZYZ4 : (d1 ? RT_ZY4 : RT_YZ4);
    }
    // QFT rounds over consecutive qubits: the upper half of each stage's
    // intra-round factors is i times the lower half (RT_QFT4S, RT_QFT4S_H4)
    for (TileRound& r : rounds) {
      if (r.type != RT_QFT4 && r.type != RT_QFT4_H4) continue;
      bool sym = true;
      for (int st = r.op_begin; st < r.op_end && sym; ++st) {
        const TileOp& op = T.ops[st];
        const int h = (1 << op.rbit) / 2;
        for (int k = 0; k < h && sym; ++k)
          sym = std::abs(coef[op.coef + k] * cd(0.0, 1.0) - coef[op.coef + k + h]) <= 1e-14;
      }
      if (sym) r.type = r.type == RT_QFT4 ? RT_QFT4S : RT_QFT4S_H4;
    }
    if (!qtab.empty()) d.pass_qtab[i] = b.put(qtab);
    d.pass_rounds[i] = b.put(rounds);
    d.pass_ops[i] = b.put(T.ops);
    std::vector<cplx<R>> cr = round_entries<R>(coef);
    if (sizeof(R) == sizeof(float)) round_pass_unitaries(T, rounds, coef, cr, acc);
    for (int32_t k : rot_coef) cr[k] = {(R)coef[k].real(), (R)coef[k].imag()};
    if (sizeof(R) == sizeof(float)) pscale = fround_scale(pscale, acc);
    d.pass_scale[i] = pscale;
    d.pass_coef[i] = b.put(cr);
    // slot descriptors hold device addresses: filled in once the blob has one
    if (!T.diag_slots.empty()) d.pass_diag[i] = b.put(std::vector<DiagDev>(T.diag_slots.size()));
  }
  d.dense_mat.assign(P.denses.size(), 0);
  d.dense_mat_dagger.assign(P.denses.size(), 0);
  for (size_t i = 0; i < P.denses.size(); ++i) {
    d.dense_mat[i] = b.put(cast<R>(P.denses[i].mat));
    d.dense_mat_dagger[i] = b.put(cast<R>(P.denses[i].mat_dagger));
  }
  b.put(std::vector<double>(2, 0.0));  // never zero bytes
}

DiagDev diag_dev(const PlanDev& d, const char* base, int i, bool conj) {
  DiagDev D{};
  D.terms = (const DiagTerm*)(base + d.diag_terms[i]);
  D.groups = (const DiagGroup*)(base + d.diag_groups[i]);
  D.lut = base + d.diag_lut[i];
  D.n_groups = d.diag_ngroups[i];
  D.conj = conj ? 1 : 0;
  D.theta = (const double*)(base + d.diag_theta[i]);
  D.global = d.diag_global[i];
  return D;
}

// The per-pass diagonal slot arrays, pointing into the blob at device address base.
void fill_slots(const PlanIR& P, const PlanDev& d, const char* base, Blob& b) {
  for (size_t i = 0; i < P.passes.size(); ++i) {
    const TilePassIR& T = P.passes[i];
    for (size_t k = 0; k < T.diag_slots.size(); ++k) {
      const DiagDev D = diag_dev(d, base, T.diag_slots[k], T.inverse != 0);
      std::memcpy(b.bytes.data() + d.pass_diag[i] + k * sizeof(DiagDev), &D, sizeof D);
    }
  }
}

}  // namespace

}  // namespace qs

using namespace qs;

const PlanDev& qs_plan::device_for(qs_dtype dt) {
  PlanDev& d = dev[dt];
  if (gf2.size() != ir.gf2s.size()) {
    gf2.clear();
    for (auto& g : ir.gf2s) gf2.push_back(gf2_args(ir.n, g, kGf2MaxC));
  }
  if (d.valid) return d;
  const Range range("qs.plan.tables");
  Blob b;
  if (dt == QS_C64) build_blob<float>(*this, d, b);
  else build_blob<double>(*this, d, b);
  if (d.blob && d.bytes != b.bytes.size()) {
    hipFree(d.blob);
    d.blob = nullptr;
  }
  if (!d.blob) check_hip(hipMalloc(&d.blob, b.bytes.size()), "hipMalloc(plan tables)");
  d.bytes = b.bytes.size();
  fill_slots(ir, d, (const char*)d.blob, b);
  check_hip(hipMemcpy(d.blob, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice), "hipMemcpy(plan tables)");
  d.valid = true;
  return d;
}

qs_plan& qs_plan::inverse() {
  if (!inv) {
    inv = new qs_plan();
    inv->ir = invert_plan(ir);
    inv_version = version + 1;  // force a parameter copy below
  }
  if (inv_version != version) {
    inv->params = params;
    inv->bound = bound;
    inv->version += 1;
    inv->refresh_device();
    inv_version = version;
  }
  return *inv;
}

namespace {

// The library's stream for table uploads on the current device (default
// priority, non-blocking: it never waits for the null stream).
hipStream_t upload_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) fail(QS_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev]) check_hip(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking), "hipStreamCreateWithFlags");
  return streams[dev];
}

qs_plan::TableUser& user_of(std::vector<qs_plan::TableUser>& users, hipStream_t s) {
  for (auto& u : users)
    if (u.stream == s && !u.external) return u;
  qs_plan::TableUser u;
  u.stream = s;
  check_hip(hipEventCreateWithFlags(&u.done, hipEventDisableTiming), "hipEventCreateWithFlags");
  users.push_back(u);
  return users.back();
}

}  // namespace

const PlanDev& qs_plan::acquire(qs_dtype dt, hipStream_t s) {
  const PlanDev& d = device_for(dt);
  TableUser& u = user_of(users[dt], s);
  if (u.seen < uploads[dt]) {
    check_hip(hipStreamWaitEvent(s, ready[dt], 0), "hipStreamWaitEvent");
    u.seen = uploads[dt];
  }
  return d;
}

void qs_plan::release(qs_dtype dt, hipStream_t s) {
  check_hip(hipEventRecord(user_of(users[dt], s).done, s), "hipEventRecord");
}

void qs_plan::add_external_user(qs_dtype dt, hipStream_t s, hipEvent_t done, qs_batch* b) {
  device_for(dt);
  for (auto& u : users[dt])
    if (u.external && u.done == done) return;
  TableUser u;
  u.stream = s;
  u.done = done;
  u.external = true;
  u.batch = b;
  u.seen = uploads[dt];  // the batch waits when it (re)reads the tables
  users[dt].push_back(u);
}

void qs_plan::sync_external_user(qs_dtype dt, hipEvent_t done, hipStream_t s) {
  for (auto& u : users[dt])
    if (u.external && u.done == done) {
      if (u.seen < uploads[dt]) {
        check_hip(hipStreamWaitEvent(s, ready[dt], 0), "hipStreamWaitEvent");
        u.seen = uploads[dt];
      }
      return;
    }
}

void qs_plan::remove_external_user(qs_dtype dt, hipEvent_t done) {
  auto& v = users[dt];
  for (size_t k = 0; k < v.size(); ++k)
    if (v[k].external && v[k].done == done) {
      v.erase(v.begin() + (long)k);
      return;
    }
}

void qs_plan::refresh_device() {
  const Range range("qs.plan.update");
  for (int k = 0; k < 2; ++k) {
    PlanDev& d = dev[k];
    if (!d.blob) continue;
    PlanDev nd;
    Blob b;
    if (k == QS_C64) build_blob<float>(*this, nd, b);
    else build_blob<double>(*this, nd, b);
    if (b.bytes.size() != d.bytes) {
      // a different table size (never for a parameter update of one plan):
      // wait for the readers, then rebuild in place of the old tables
      for (auto& u : users[k]) check_hip(hipEventSynchronize(u.done), "hipEventSynchronize");
      d.valid = false;
      device_for((qs_dtype)k);
      continue;
    }
    fill_slots(ir, nd, (const char*)d.blob, b);
    // the staging buffer is free once the previous upload has run
    if (uploads[k]) check_hip(hipEventSynchronize(ready[k]), "hipEventSynchronize");
    if (staging_cap[k] < b.bytes.size()) {
      if (staging[k]) check_hip(hipHostFree(staging[k]), "hipHostFree");
      staging[k] = nullptr;
      staging_cap[k] = 0;
      check_hip(hipHostMalloc(&staging[k], b.bytes.size(), hipHostMallocDefault), "hipHostMalloc(plan tables)");
      staging_cap[k] = b.bytes.size();
    }
    if (!ready[k]) check_hip(hipEventCreateWithFlags(&ready[k], hipEventDisableTiming), "hipEventCreateWithFlags");
    std::memcpy(staging[k], b.bytes.data(), b.bytes.size());
    const hipStream_t up = upload_stream();
    for (auto& u : users[k]) check_hip(hipStreamWaitEvent(up, u.done, 0), "hipStreamWaitEvent");
    check_hip(hipMemcpyAsync(d.blob, staging[k], b.bytes.size(), hipMemcpyHostToDevice, up), "hipMemcpyAsync(plan tables)");
    check_hip(hipEventRecord(ready[k], up), "hipEventRecord");
    uploads[k] += 1;
    // host-side kernel arguments (offsets are unchanged; scales follow the parameters)
    nd.blob = d.blob;
    nd.bytes = d.bytes;
    nd.valid = true;
    d = std::move(nd);
  }
}

namespace qs {

namespace {

// Coset order of a tile pass (TileKArgs::order).  By geometry: measured at
// 30 qubits, contiguous tiles stream fastest XCD-blocked, tiles over high
// bits with runs of 2^5 amplitudes or more in launch order (neighbouring
// cosets of all XCDs share DRAM rows), shorter runs XCD-blocked again.
uint32_t tile_order(int opt, int L, int a) {
  if (opt == 1) return 0;
  if (opt == 2) return 1;
  return (L == a || L <= 4) ? 0u : 1u;
}

}  // namespace

template <class R>
TileKArgs<R> tile_args(qs_state& s, qs_plan& p, int pass) {
  const PlanDev& d = p.device_for(s.dtype);
  const char* base = (const char*)d.blob;
  const PlanIR& P = p.ir;
  const TilePassIR& T = P.passes[pass];
  if (T.L + T.h > (s.dtype == QS_C64 ? 14 : 13)) fail(QS_EINVAL, "tile too large for this dtype");
  TileKArgs<R> A;
  std::memset(&A, 0, sizeof A);
  A.psi = (cplx<R>*)s.cur_ptr();
  A.rounds = (const TileRound*)(base + d.pass_rounds[pass]);
  A.ops = (const TileOp*)(base + d.pass_ops[pass]);
  A.coef = (const cplx<R>*)(base + d.pass_coef[pass]);
  A.diag = d.pass_diag[pass] ? (const DiagDev*)(base + d.pass_diag[pass]) : nullptr;
  A.qtab = (const int32_t*)(base + d.pass_qtab[pass]);
  A.L = T.L;
  A.a = T.a;
  A.h = T.h;
  A.m = T.L + T.h;
  A.order = tile_order(P.opt.coset_order, T.L, T.a);
  A.n_rounds = d.pass_nrounds[pass];
  A.n = s.n;
  A.scale = d.pass_scale[pass];
  return A;
}
template TileKArgs<float> tile_args<float>(qs_state&, qs_plan&, int);
template TileKArgs<double> tile_args<double>(qs_state&, qs_plan&, int);

namespace {

template <class R>
void apply_layers_t(qs_state& s, qs_plan& p, size_t first, size_t last, double* norm_last = nullptr) {
  const PlanDev& d = p.device_for(s.dtype);
  const char* base = (const char*)d.blob;
  const PlanIR& P = p.ir;
  for (size_t li = first; li < last; ++li) {
    const LayerIR& L = P.layers[li];
    switch (L.kind) {
      case L_DIAG:
        launch_diag<R>((cplx<R>*)s.cur_ptr(), s.n, diag_dev(d, base, L.index, L.inverse != 0), s.stream);
        break;
      case L_TILE: {
        TileKArgs<R> A = tile_args<R>(s, p, L.index);
        A.norm_part = li + 1 == last ? norm_last : nullptr;
        launch_tile<R>(A, s.stream);
        break;
      }
      case L_GF2: {
        s.ensure_other();
        launch_gf2<R>((const cplx<R>*)s.buf[s.cur], (cplx<R>*)s.buf[1 - s.cur], p.gf2[L.index], s.stream,
                      li + 1 == last ? norm_last : nullptr);
        s.cur = 1 - s.cur;
        break;
      }
      case L_DENSE: {
        const DenseIR& D = P.denses[L.index];
        const cplx<R>* U = (const cplx<R>*)(base + (L.inverse ? d.dense_mat_dagger[L.index] : d.dense_mat[L.index]));
        if (!launch_dense<R>((cplx<R>*)s.cur_ptr(), s.n, (int)D.bits.size(), D.bits.data(), U, s.stream)) {
          // the per-gate k-qubit kernel, with the first listed bit most significant
          std::vector<int> desc(D.bits.rbegin(), D.bits.rend());
          launch_matk<R>((cplx<R>*)s.cur_ptr(), s.n, (int)desc.size(), desc.data(), U, s.stream);
        }
        break;
      }
      case L_PLAIN:
        apply_plain_gate(s, P.gates[L.index], p.params, L.inverse != 0);
        break;
      default:
        fail(QS_EINVAL, "internal: unknown layer kind");
    }
  }
}

template <class R>
void plain_t(qs_state& s, const NGate& g, const std::vector<double>& params, bool inverse) {
  cplx<R>* psi = (cplx<R>*)s.cur_ptr();
  const int n = s.n;
  std::vector<cd> M = gate_matrix(g, params);
  if (inverse) M = dagger(M, 1 << (int)g.bits.size());
  std::vector<cplx<R>> m = round_gate<R>(M, 1 << (int)g.bits.size(), s.plain_acc);
  const auto& b = g.bits;
  switch (g.kind) {
    case QS_GATE_I:
      return;
    case QS_GATE_X:
      launch_flip<R>(psi, n, b[0], s.stream);
      return;
    case QS_GATE_Z: case QS_GATE_S: case QS_GATE_SDG: case QS_GATE_T: case QS_GATE_TDG: case QS_GATE_P:
      launch_phase_mask<R>(psi, n, 1u << b[0], m[3], s.stream);
      return;
    case QS_GATE_RZ:
      launch_diag1<R>(psi, n, b[0], m[0], m[3], s.stream);
      return;
    case QS_GATE_CNOT:
      launch_cflip<R>(psi, n, b[0], b[1], s.stream);
      return;
    case QS_GATE_CZ: case QS_GATE_CPHASE:
      launch_phase_mask<R>(psi, n, (1u << b[0]) | (1u << b[1]), m[15], s.stream);
      return;
    case QS_GATE_MCZ: case QS_GATE_MCP:
      launch_phase_mask<R>(psi, n, g.all_mask, m.back(), s.stream);
      return;
    case QS_GATE_SWAP:
      launch_swap<R>(psi, n, b[0], b[1], s.stream);
      return;
    case QS_GATE_RZZ:
      launch_parity_phase<R>(psi, n, (1u << b[0]) | (1u << b[1]), m[0], m[5], s.stream);
      return;
    case QS_GATE_CU: {
      const cplx<R> u[4] = {m[10], m[11], m[14], m[15]};  // target block of the controlled matrix
      launch_cmat1<R>(psi, n, b[0], b[1], u, s.stream);
      return;
    }
    default:
      break;
  }
  if (b.size() == 1) {
    launch_mat1<R>(psi, n, b[0], m.data(), s.stream);
  } else if (b.size() == 2) {
    launch_mat2<R>(psi, n, b[0], b[1], m.data(), s.stream);
  } else {
    if (!s.matbuf) check_hip(hipMalloc(&s.matbuf, 64 * 64 * sizeof(cplx<double>)), "hipMalloc");
    check_hip(hipMemcpyAsync(s.matbuf, m.data(), m.size() * sizeof(cplx<R>), hipMemcpyHostToDevice, s.stream),
              "hipMemcpyAsync");
    launch_matk<R>(psi, n, (int)b.size(), b.data(), (const cplx<R>*)s.matbuf, s.stream);
    s.sync();  // the staging buffer is reused by the next dense gate
  }
}

template <class Ra, class Rb>
std::complex<double> overlap_t(qs_state& a, qs_state& b) {
  a.ensure_red();
  launch_overlap<Ra, Rb>((const cplx<Ra>*)a.cur_ptr(), (const cplx<Rb>*)b.cur_ptr(), 1ull << a.n, a.red_partials,
                         a.red_out, a.stream);
  double o[2];
  check_hip(hipMemcpyAsync(o, a.red_out, sizeof o, hipMemcpyDeviceToHost, a.stream), "hipMemcpyAsync");
  a.sync();
  return {o[0], o[1]};
}

template <class Ra, class Rb>
double distance_t(qs_state& a, qs_state& b, double ar, double ai, double bs) {
  a.ensure_red();
  launch_distance2<Ra, Rb>((const cplx<Ra>*)a.cur_ptr(), (const cplx<Rb>*)b.cur_ptr(), 1ull << a.n, ar, ai, bs,
                           a.red_partials, a.red_out, a.stream);
  double o;
  check_hip(hipMemcpyAsync(&o, a.red_out, sizeof o, hipMemcpyDeviceToHost, a.stream), "hipMemcpyAsync");
  a.sync();
  return o;
}

}  // namespace

void apply_layers(qs_state& s, qs_plan& p, size_t first, size_t last, bool track) {
  const Range range("qs.apply");
  s.plain_acc = NormAcc{};  // plain layers' rounding compensation restarts with every call
  if (track) {
    // nothing is recorded into a stream that is being captured
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    check_hip(hipStreamIsCapturing(s.stream, &cs), "hipStreamIsCapturing");
    track = cs == hipStreamCaptureStatusNone;
  }
  if (track) p.acquire(s.dtype, s.stream);
  if (s.dtype == QS_C64) apply_layers_t<float>(s, p, first, last);
  else apply_layers_t<double>(s, p, first, last);
  if (track) p.release(s.dtype, s.stream);
}

void apply_plain_gate(qs_state& s, const NGate& g, const std::vector<double>& params, bool inverse) {
  if (s.dtype == QS_C64) plain_t<float>(s, g, params, inverse);
  else plain_t<double>(s, g, params, inverse);
}

void prof_suspend(bool on);

uint64_t new_plan_uid() {
  static std::atomic<uint64_t> next{1};
  return next.fetch_add(1);
}

void free_graphs(qs_state& s) {
  for (auto& e : s.graphs)
    if (e.exec) hipGraphExecDestroy(e.exec);
  s.graphs.clear();
  if (s.capture_stream) hipStreamDestroy(s.capture_stream);
  s.capture_stream = nullptr;
}

void apply_graph(qs_state& s, qs_plan& p) {
  const PlanIR& P = p.ir;
  bool gather = false;
  for (const LayerIR& L : P.layers) {
    if (L.kind == L_PLAIN && P.gates[L.index].bits.size() > 2) {
      apply_layers(s, p, 0, P.layers.size());  // its matrix is staged from the host per call
      return;
    }
    gather = gather || L.kind == L_GF2;
  }
  if (P.layers.empty()) return;
  if (gather) s.ensure_other();
  p.acquire(s.dtype, s.stream);
  PlanGraphEntry* hit = nullptr;
  for (auto& e : s.graphs)
    if (e.plan_uid == p.uid && e.version == p.version && e.cur0 == s.cur) hit = &e;
  if (!hit) {
    // record on a private stream (the state's stream may be the null stream,
    // which cannot capture; nothing runs during capture), then launch on the
    // state's stream; keep at most 8 graphs per state
    if (!s.capture_stream)
      check_hip(hipStreamCreateWithFlags(&s.capture_stream, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    const int cur0 = s.cur;
    const hipStream_t user = s.stream;
    hipGraph_t g = nullptr;
    prof_suspend(true);
    s.stream = s.capture_stream;
    check_hip(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      apply_layers(s, p, 0, P.layers.size(), false);
    } catch (...) {
      hipGraph_t gg = nullptr;
      hipStreamEndCapture(s.stream, &gg);
      if (gg) hipGraphDestroy(gg);
      s.stream = user;
      prof_suspend(false);
      s.cur = cur0;
      throw;
    }
    const hipError_t ec = hipStreamEndCapture(s.stream, &g);
    s.stream = user;
    prof_suspend(false);
    PlanGraphEntry e;
    e.plan_uid = p.uid;
    e.version = p.version;
    e.cur0 = cur0;
    e.cur1 = s.cur;
    s.cur = cur0;
    check_hip(ec, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    check_hip(ei, "hipGraphInstantiate");
    if (s.graphs.size() >= 8) {
      hipGraphExecDestroy(s.graphs.front().exec);
      s.graphs.erase(s.graphs.begin());
    }
    s.graphs.push_back(e);
    hit = &s.graphs.back();
  }
  prof_begin("plan_graph", s.stream);
  check_hip(hipGraphLaunch(hit->exec, s.stream), "hipGraphLaunch");
  prof_end(s.stream);
  p.release(s.dtype, s.stream);
  s.cur = hit->cur1;
}

double apply_norm2(qs_state& s, qs_plan& p) {
  const size_t L = p.ir.layers.size();
  uint64_t tiles = 0;
  if (L > 0) {
    const LayerIR& last = p.ir.layers.back();
    if (last.kind == L_TILE) {
      const TilePassIR& T = p.ir.passes[last.index];
      tiles = 1ull << (s.n - (T.L + T.h));
    } else if (last.kind == L_GF2) {
      p.device_for(s.dtype);
      tiles = gf2_norm_slots(p.gf2[last.index]);
    }
  }
  if (tiles == 0 || tiles > (1ull << 24)) {
    apply_layers(s, p, 0, L);
    return state_norm2(s);
  }
  s.ensure_red();
  s.ensure_norm(tiles);
  p.acquire(s.dtype, s.stream);
  if (s.dtype == QS_C64) apply_layers_t<float>(s, p, 0, L, s.norm_part);
  else apply_layers_t<double>(s, p, 0, L, s.norm_part);
  p.release(s.dtype, s.stream);
  launch_fold_partials(s.norm_part, tiles, s.red_partials, s.red_out, s.stream);
  double o;
  check_hip(hipMemcpyAsync(&o, s.red_out, sizeof o, hipMemcpyDeviceToHost, s.stream), "hipMemcpyAsync");
  s.sync();
  return o;
}

double state_norm2(qs_state& s) {
  s.ensure_red();
  if (s.dtype == QS_C64)
    launch_norm2<float>((const cplx<float>*)s.cur_ptr(), 1ull << s.n, s.red_partials, s.red_out, s.stream);
  else
    launch_norm2<double>((const cplx<double>*)s.cur_ptr(), 1ull << s.n, s.red_partials, s.red_out, s.stream);
  double o;
  check_hip(hipMemcpyAsync(&o, s.red_out, sizeof o, hipMemcpyDeviceToHost, s.stream), "hipMemcpyAsync");
  s.sync();
  return o;
}

std::complex<double> state_overlap(qs_state& a, qs_state& b) {
  if (a.stream != b.stream) b.sync();
  if (a.dtype == QS_C64 && b.dtype == QS_C64) return overlap_t<float, float>(a, b);
  if (a.dtype == QS_C64) return overlap_t<float, double>(a, b);
  if (b.dtype == QS_C64) return overlap_t<double, float>(a, b);
  return overlap_t<double, double>(a, b);
}

double state_infidelity(qs_state& a, qs_state& b) {
  const double na = state_norm2(a), nb = state_norm2(b);
  if (!(na > 0) || !(nb > 0)) fail(QS_EINVAL, "zero state");
  const std::complex<double> ov = state_overlap(a, b);
  const double ph = std::arg(ov);
  const double ar = std::cos(ph) / std::sqrt(na), ai = std::sin(ph) / std::sqrt(na), bs = 1.0 / std::sqrt(nb);
  if (a.stream != b.stream) b.sync();
  double D;
  if (a.dtype == QS_C64 && b.dtype == QS_C64) D = distance_t<float, float>(a, b, ar, ai, bs);
  else if (a.dtype == QS_C64) D = distance_t<float, double>(a, b, ar, ai, bs);
  else if (b.dtype == QS_C64) D = distance_t<double, float>(a, b, ar, ai, bs);
  else D = distance_t<double, double>(a, b, ar, ai, bs);
  return std::max(0.0, D * (1.0 - D / 4.0));
}

std::vector<double> state_expect(qs_state& s, const qs_pauli* terms, size_t n_terms) {
  const int n = s.n;
  std::vector<double> out(n_terms, 0.0);
  std::map<uint32_t, std::vector<size_t>> by_x;
  std::vector<uint32_t> zb(n_terms);
  std::vector<int> ny(n_terms);
  for (size_t t = 0; t < n_terms; ++t) {
    const qs_pauli& P = terms[t];
    if (!std::isfinite(P.coeff)) fail(QS_EINVAL, "non-finite Pauli coefficient");
    if (n < 64 && ((P.x_mask >> n) || (P.z_mask >> n))) fail(QS_EINVAL, "Pauli mask out of range");
    uint32_t x = 0, z = 0;
    for (int q = 0; q < n; ++q) {
      if ((P.x_mask >> q) & 1) x |= 1u << (n - 1 - q);
      if ((P.z_mask >> q) & 1) z |= 1u << (n - 1 - q);
    }
    zb[t] = z;
    ny[t] = __builtin_popcount(x & z) & 3;
    by_x[x].push_back(t);
  }
  s.ensure_red();
  for (auto& kv : by_x) {
    const auto& idx = kv.second;
    for (size_t c0 = 0; c0 < idx.size(); c0 += kMaxTermsPerLaunch) {
      int nt = (int)std::min<size_t>(kMaxTermsPerLaunch, idx.size() - c0);
      uint32_t zz[kMaxTermsPerLaunch];
      int yy[kMaxTermsPerLaunch];
      for (int k = 0; k < nt; ++k) {
        zz[k] = zb[idx[c0 + k]];
        yy[k] = ny[idx[c0 + k]];
      }
      if (kv.first == 0) {
        if (s.dtype == QS_C64)
          launch_expect_z<float>((const cplx<float>*)s.cur_ptr(), n, zz, nt, s.red_partials, s.red_out, s.stream);
        else
          launch_expect_z<double>((const cplx<double>*)s.cur_ptr(), n, zz, nt, s.red_partials, s.red_out, s.stream);
      } else {
        if (s.dtype == QS_C64)
          launch_expect_x<float>((const cplx<float>*)s.cur_ptr(), n, kv.first, zz, yy, nt, s.red_partials, s.red_out,
                                 s.stream);
        else
          launch_expect_x<double>((const cplx<double>*)s.cur_ptr(), n, kv.first, zz, yy, nt, s.red_partials,
                                  s.red_out, s.stream);
      }
      double o[kMaxTermsPerLaunch];
      check_hip(hipMemcpyAsync(o, s.red_out, sizeof o, hipMemcpyDeviceToHost, s.stream), "hipMemcpyAsync");
      s.sync();
      for (int k = 0; k < nt; ++k) out[idx[c0 + k]] = terms[idx[c0 + k]].coeff * o[k];
    }
  }
  return out;
}

}  // namespace qs
