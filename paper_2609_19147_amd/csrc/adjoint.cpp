// Adjoint-method gradients of E = <psi_L|H|psi_L> for a parametrised plan.
//
// Forward: psi_L = U_L ... U_1 psi_0 (the fused layers).  Backward: phi = psi_L,
// lambda = H psi_L; for l = L..1 both states are un-applied through the inverse
// of layer l, after which every parameter occurrence of that layer contributes
// 2 Re <lambda|K|phi> with K = U_l^dagger dU_l/dtheta restricted to its wire
// (tile-pass windows: a 2x2 operator; diagonal layers: i * count of the
// parameter's group).  All reductions are FP64.  A tile pass is undone on both
// states by one fused kernel that also sums the layer's cross densities from
// the two tiles in LDS (4 S of traffic per layer); layers whose two tiles do
// not fit in LDS take two passes and a separate cross-density read (6 S).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>

#include "runtime.h"

using namespace qs;

namespace {

// Both LDS tiles of the fused adjoint pass (the tile kernels' dynamic LDS limit).
constexpr size_t kDualLdsBytes = 144 * 1024;

// Work state k of psi (same n, dtype, device and stream), made on first use
// and kept with psi; its contents are overwritten by each sweep.
qs_state& work_state(qs_state& psi, int k) {
  std::unique_ptr<qs_state>& w = psi.work[k];
  if (!w) {
    auto s = std::make_unique<qs_state>();
    s->n = psi.n;
    s->dtype = psi.dtype;
    s->device = psi.device;
    s->stream = psi.stream;
    s->buf[0] = alloc_amplitudes(s->state_bytes(), "adjoint work state");
    s->owned[0] = true;
    w = std::move(s);
  }
  w->stream = psi.stream;
  return *w;
}

template <class R>
void copy_state(qs_state& dst, qs_state& src) {
  launch_convert<R, R>((cplx<R>*)dst.cur_ptr(), (const cplx<R>*)src.cur_ptr(), 1ull << src.n, dst.stream);
}

template <class R>
void run_adjoint(qs_state& psi, qs_plan& p, const qs_pauli* terms, size_t n_terms, double* energy, double* grad) {
  const PlanIR& P = p.ir;
  const int n = psi.n;
  // host-side validation of every parameter occurrence first (no device work on failure)
  std::vector<std::vector<GradEntry>> entries = grad_entries(P, p.params);
  qs_plan& inv = p.inverse();
  const TableUse use_fwd(p, psi.dtype, psi.stream), use_inv(inv, psi.dtype, psi.stream);
  const size_t L = P.layers.size();
  // Pauli terms -> bit masks, sorted by x, complex coefficient c * i^{#Y}
  struct T3 {
    uint32_t x, z;
    double cr, ci;
  };
  std::vector<T3> ts;
  for (size_t t = 0; t < n_terms; ++t) {
    const qs_pauli& Q = terms[t];
    if (!std::isfinite(Q.coeff)) fail(QS_EINVAL, "non-finite Pauli coefficient");
    if (n < 64 && ((Q.x_mask >> n) || (Q.z_mask >> n))) fail(QS_EINVAL, "Pauli mask out of range");
    uint32_t x = 0, z = 0;
    for (int q = 0; q < n; ++q) {
      if ((Q.x_mask >> q) & 1) x |= 1u << (n - 1 - q);
      if ((Q.z_mask >> q) & 1) z |= 1u << (n - 1 - q);
    }
    const int ny = __builtin_popcount(x & z) & 3;
    const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
    ts.push_back({x, z, Q.coeff * re[ny], Q.coeff * im[ny]});
  }
  std::stable_sort(ts.begin(), ts.end(), [](const T3& a, const T3& b) { return a.x < b.x; });

  const Range range("qs.adjoint");
  // forward
  apply_layers(psi, p, 0, L, false);
  qs_state& phi = work_state(psi, 0);
  qs_state& lam = work_state(psi, 1);
  copy_state<R>(phi, psi);
  {
    // groups of one X mask; within a group each term's sign (-1)^{popcount(j & z)}
    // is 1 - 2 count(j): constants join c0, Z and ZZ terms of equal coefficient
    // share one count (disjoint masks), longer Z strings count their parity
    std::vector<PauliGroup> groups;
    std::vector<PauliCount> counts;
    for (size_t t0 = 0; t0 < ts.size();) {
      size_t t1 = t0;
      while (t1 < ts.size() && ts[t1].x == ts[t0].x) ++t1;
      PauliGroup G{};
      G.x = ts[t0].x;
      G.k0 = (int32_t)counts.size();
      for (size_t t = t0; t < t1; ++t) {
        const T3& T = ts[t];
        G.c0re += T.cr;
        G.c0im += T.ci;
        if (T.z == 0) continue;
        const int nz = __builtin_popcount(T.z);
        int32_t form = DT_PARITY;
        uint32_t shift = 0, mask = T.z;
        if (nz == 1) {
          form = DT_BITS;
        } else if (nz == 2) {
          const int lo = __builtin_ctz(T.z), hi = 31 - __builtin_clz(T.z);
          form = DT_SHIFT_XOR;
          shift = (uint32_t)(hi - lo);
          mask = 1u << lo;
        }
        const double wre = -2.0 * T.cr, wim = -2.0 * T.ci;
        bool merged = false;
        if (form != DT_PARITY)
          for (size_t k = (size_t)G.k0; k < counts.size() && !merged; ++k) {
            PauliCount& K = counts[k];
            if (K.form == form && K.shift == shift && K.wre == wre && K.wim == wim && !(K.mask & mask)) {
              K.mask |= mask;
              merged = true;
            }
          }
        if (!merged) counts.push_back(PauliCount{form, shift, mask, 0, wre, wim});
      }
      G.nk = (int32_t)counts.size() - G.k0;
      groups.push_back(G);
      t0 = t1;
    }
    const size_t gbytes = std::max<size_t>(groups.size(), 1) * sizeof(PauliGroup);
    const size_t kbytes = std::max<size_t>(counts.size(), 1) * sizeof(PauliCount);
    void* dterms = psi.ensure_work_buf(gbytes + kbytes);
    PauliGroup* dg = (PauliGroup*)dterms;
    PauliCount* dk = (PauliCount*)((char*)dterms + gbytes);
    if (!groups.empty())
      check_hip(hipMemcpyAsync(dg, groups.data(), groups.size() * sizeof(PauliGroup), hipMemcpyHostToDevice,
                               psi.stream),
                "hipMemcpyAsync");
    if (!counts.empty())
      check_hip(hipMemcpyAsync(dk, counts.data(), counts.size() * sizeof(PauliCount), hipMemcpyHostToDevice,
                               psi.stream),
                "hipMemcpyAsync");
    launch_pauli_apply<R>((const cplx<R>*)phi.cur_ptr(), (cplx<R>*)lam.cur_ptr(), n, dg, (int)groups.size(), dk,
                          psi.stream);
    psi.sync();
  }
  *energy = state_overlap(phi, lam).real();

  // backward: every reduction writes its own slot of one device array, read
  // back once after the sweep (no host round trip per layer)
  std::vector<double> g(p.ir.n_params, 0.0);
  phi.ensure_red();
  const PlanDev& d = p.device_for(psi.dtype);
  // per forward layer: the cross densities of all of a tile layer's parameter
  // bits in one read of phi and lambda (the layer's tile geometry), else one
  // reduction per bit; diagonal-layer parameters one reduction per group
  std::vector<RhoTileArgs> tile_rho(L);
  std::vector<RhoTileArgs> dual_rho(L);             // fused: bits as positions in the inverse pass's tile
  std::vector<char> dual(L, 0);
  std::vector<double> rho_scale(L, 1.0);            // fused: staged tiles are unnormalised
  std::vector<std::map<int, size_t>> rho_slot(L);   // bit -> offset of its 8 sums
  std::vector<std::vector<int>> single_bits(L);     // bits reduced one at a time
  std::vector<std::map<std::pair<int, int>, size_t>> diag_slot(L);  // (diag, group) -> offset
  std::vector<size_t> tile_slot(L, 0);
  size_t n_res = 0, rho_partials = 0;
  for (size_t fl = 0; fl < L; ++fl) {
    const LayerIR& FL = p.ir.layers[fl];
    std::vector<int> bits;
    for (const GradEntry& e : entries[fl]) {
      if (e.kind == 0) {
        if (std::find(bits.begin(), bits.end(), e.bit) == bits.end()) bits.push_back(e.bit);
      } else if (!diag_slot[fl].count({e.diag, e.group})) {
        diag_slot[fl][{e.diag, e.group}] = n_res++;
      }
    }
    const LayerIR& IL = inv.ir.layers[L - 1 - fl];
    if (IL.kind == L_TILE && bits.size() <= 32) {
      const TilePassIR& T = inv.ir.passes[IL.index];
      const uint32_t m = (uint32_t)(T.L + T.h), M = 1u << m;
      bool ok = 2 * sizeof(cplx<R>) * (M + ((M >> 5) << 1)) <= kDualLdsBytes && m <= (sizeof(R) == 4 ? 14u : 13u);
      RhoTileArgs A{};
      A.L = (uint32_t)T.L;
      A.a = (uint32_t)T.a;
      A.h = (uint32_t)T.h;
      A.m = m;
      for (int b : bits) {
        const int pos = b < T.L ? b : (b >= T.a && b < T.a + T.h ? T.L + b - T.a : -1);
        if (pos < 0) ok = false;
        else A.tbit[A.nbits++] = (uint32_t)pos;
      }
      if (ok) {
        dual[fl] = 1;
        dual_rho[fl] = A;
        const double sc = inv.device_for(psi.dtype).pass_scale[IL.index];
        rho_scale[fl] = sc * sc;
        tile_slot[fl] = n_res;
        for (size_t k = 0; k < bits.size(); ++k) rho_slot[fl][bits[k]] = n_res + 8 * k;
        n_res += 8 * bits.size();
        rho_partials = std::max(rho_partials, rho_tile_partials(n, A));
        continue;
      }
    }
    if (bits.empty()) continue;
    bool tiled = false;
    if (FL.kind == L_TILE && bits.size() <= 32) {
      const TilePassIR& T = p.ir.passes[FL.index];
      // the pass's tile bits, with the low run [0, L) cut to the requested low
      // bits (at least 5: 256-byte runs, and a tile of at least 2^7): smaller
      // tiles let several workgroups share a CU
      int lo_needed = 0;
      for (int b : bits)
        if (b < T.L) lo_needed = std::max(lo_needed, b + 1);
      int Lr = std::min(T.L, std::max(lo_needed, 5));
      while (Lr < T.L && Lr + T.h < 7) ++Lr;
      RhoTileArgs A{};
      A.L = (uint32_t)Lr;
      A.a = (uint32_t)T.a;
      A.h = (uint32_t)T.h;
      A.m = (uint32_t)(Lr + T.h);
      tiled = Lr >= 1 && rho_tile_fits(A.m, sizeof(R));
      for (int b : bits) {
        const int pos = b < Lr ? b : (b >= T.a && b < T.a + T.h ? Lr + b - T.a : -1);
        if (pos < 0) tiled = false;
        else A.tbit[A.nbits++] = (uint32_t)pos;
      }
      if (tiled) {
        tile_rho[fl] = A;
        tile_slot[fl] = n_res;
        for (size_t k = 0; k < bits.size(); ++k) rho_slot[fl][bits[k]] = n_res + 8 * k;
        n_res += 8 * bits.size();
        rho_partials = std::max(rho_partials, rho_tile_partials(n, A));
      }
    }
    if (!tiled) {
      for (int b : bits) {
        rho_slot[fl][b] = n_res;
        n_res += 8;
      }
      single_bits[fl] = bits;
    }
  }
  // (the forward sweep has finished with the scratch area: psi was synchronised)
  void* buf = n_res ? psi.ensure_work_buf((rho_partials + n_res) * sizeof(double)) : nullptr;
  double* part = (double*)buf;
  double* res = part + rho_partials;
  for (size_t j = 0; j < L; ++j) {
    const size_t fl = L - 1 - j;  // forward layer being undone
    if (dual[fl]) {
      const TileKArgs<R> A = tile_args<R>(phi, inv, inv.ir.layers[j].index);
      if (!launch_tile_dual<R>(A, (cplx<R>*)lam.cur_ptr(), dual_rho[fl], part, res + tile_slot[fl], psi.stream))
        fail(QS_EDEVICE, "internal: fused adjoint pass rejected its tiles");
    } else {
      apply_layers(phi, inv, j, j + 1, false);
      apply_layers(lam, inv, j, j + 1, false);
    }
    const cplx<R>* ph = (const cplx<R>*)phi.cur_ptr();
    const cplx<R>* la = (const cplx<R>*)lam.cur_ptr();
    if (tile_rho[fl].nbits) launch_rho_tile<R>(ph, la, n, tile_rho[fl], part, res + tile_slot[fl], psi.stream);
    for (int b : single_bits[fl])
      launch_pair_rho<R>(ph, la, n, b, phi.red_partials, res + rho_slot[fl][b], psi.stream);
    for (const auto& kv : diag_slot[fl]) {
      const char* base = (const char*)d.blob;
      const int di = kv.first.first;
      DiagDev D{};
      D.terms = (const DiagTerm*)(base + d.diag_terms[di]);
      D.groups = (const DiagGroup*)(base + d.diag_groups[di]);
      D.lut = base + d.diag_lut[di];
      D.n_groups = d.diag_ngroups[di];
      D.conj = 0;
      launch_diag_grad<R>(ph, la, n, D, kv.first.second, 1, phi.red_partials, res + kv.second, psi.stream);
    }
  }
  std::vector<double> r(n_res);
  if (n_res)
    check_hip(hipMemcpyAsync(r.data(), res, n_res * sizeof(double), hipMemcpyDeviceToHost, psi.stream),
              "hipMemcpyAsync");
  psi.sync();
  for (size_t fl = 0; fl < L; ++fl)
    for (const GradEntry& e : entries[fl]) {
      if (e.kind == 0) {
        const double* q = r.data() + rho_slot[fl].at(e.bit);
        cd acc = 0;
        for (int k = 0; k < 4; ++k) acc += e.K[k] * cd(q[2 * k], q[2 * k + 1]);
        g[e.param] += e.coef * 2.0 * rho_scale[fl] * acc.real();
      } else {
        g[e.param] += e.coef * (-2.0) * r[diag_slot[fl].at({e.diag, e.group})];
      }
    }
  std::copy(g.begin(), g.end(), grad);
}

}  // namespace

extern "C" qs_status qs_adjoint_grad(qs_state* psi, const qs_plan* cp, const qs_pauli* terms, size_t n_terms,
                                     double* energy, double* grad, size_t n_params) {
  try {
    if (!psi || !cp || !energy) fail(QS_EINVAL, "NULL argument");
    if (n_terms && !terms) fail(QS_EINVAL, "terms is NULL");
    qs_plan& p = const_cast<qs_plan&>(*cp);
    if (p.ir.n != psi->n) fail(QS_EINVAL, "plan and state qubit counts differ");
    if (!p.bound) fail(QS_EINVAL, "plan parameters are not bound");
    if (n_params != p.ir.n_params) fail(QS_EINVAL, "gradient length does not match the plan");
    if (n_params && !grad) fail(QS_EINVAL, "grad is NULL");
    if (psi->dtype == QS_C64) run_adjoint<float>(*psi, p, terms, n_terms, energy, grad);
    else run_adjoint<double>(*psi, p, terms, n_terms, energy, grad);
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return QS_ENOMEM;
  }
}
