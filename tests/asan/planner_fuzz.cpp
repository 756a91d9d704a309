// Host-only ASan/UBSan driver of the planner (built by
// tests/test_planner_sanitizers.py): random gate streams through
// normalisation, planning (several option sets), description, inversion,
// gradient bookkeeping, GF(2) kernel arguments and numeric tables.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>
#include "planner.h"
using namespace qs;

static std::vector<double> rand_unitary_flat(std::mt19937_64& r, int d) {
  // not unitary in general: the planner only multiplies matrices
  std::normal_distribution<double> N;
  std::vector<double> m(2 * d * d);
  for (auto& x : m) x = N(r);
  return m;
}

int main(int argc, char** argv) {
  int iters = argc > 1 ? atoi(argv[1]) : 300;
  std::mt19937_64 rng(12345);
  size_t ok = 0, errs = 0;
  for (int it = 0; it < iters; ++it) {
    const int n = 1 + (int)(rng() % 32);
    const int ng = (int)(rng() % 120);
    const size_t n_params = rng() % 4;
    std::vector<qs_gate> gs(ng);
    std::vector<std::vector<double>> mats(ng);
    for (int i = 0; i < ng; ++i) {
      qs_gate& g = gs[i];
      std::memset(&g, 0, sizeof g);
      g.kind = (int)(rng() % QS_GATE_KIND_COUNT);
      g.param = -1;
      g.theta = std::uniform_real_distribution<double>(-10, 10)(rng);
      g.scale = 1.0;
      int ar = gate_arity(g);
      if (ar == -2) continue;
      int k = ar == -1 ? 1 + (int)(rng() % std::min(n, 6)) : ar;
      if (ar == 0) {
        int c = 1 + (int)(rng() % std::min(n, 5));
        uint64_t mask = 0;
        while (__builtin_popcountll(mask) < c) mask |= 1ull << (rng() % n);
        g.mask = mask;
        g.nw = 0;
      } else {
        if (k > n) { g.kind = QS_GATE_H; k = 1; }
        g.nw = k;
        std::vector<int> w;
        while ((int)w.size() < k) {
          int x = (int)(rng() % n);
          bool dup = false;
          for (int y : w) dup = dup || y == x;
          if (!dup) w.push_back(x);
        }
        for (int j = 0; j < k; ++j) g.wires[j] = w[j];
      }
      if (g.kind == QS_GATE_U || g.kind == QS_GATE_CU) { mats[i] = rand_unitary_flat(rng, 2); g.mat = mats[i].data(); }
      if (g.kind == QS_GATE_UNITARY) { mats[i] = rand_unitary_flat(rng, 1 << g.nw); g.mat = mats[i].data(); }
      if (n_params && (rng() % 3 == 0) && (g.kind == QS_GATE_RX || g.kind == QS_GATE_RY || g.kind == QS_GATE_RZ ||
                                          g.kind == QS_GATE_P || g.kind == QS_GATE_RZZ || g.kind == QS_GATE_CPHASE)) {
        g.param = (int)(rng() % n_params);
        g.scale = 0.5;
      }
    }
    std::vector<double> params(n_params);
    for (auto& p : params) p = std::uniform_real_distribution<double>(-3, 3)(rng);
    try {
      auto G = normalise_gates(n, gs.data(), gs.size(), n_params);
      for (int variant = 0; variant < 4; ++variant) {
        PlanOptions o;
        o.window_k = variant == 1 ? -1 : (variant == 2 ? 4 : (variant == 3 ? 6 : 5));
        int tb = 5 + (int)(rng() % 10);
        int low = variant == 2 ? 4 : 0;
        PlanIR P = build_plan(n, G, n_params, o, tb, low);
        std::string js = describe_json(P, params, true);
        PlanIR I = invert_plan(P);
        std::string js2 = describe_json(I, params, true);
        for (auto& T : P.passes) {
          std::vector<TileRound> rounds;
          auto coef = pass_coefficients_device(P, T, params, rounds);
          (void)coef;
        }
        for (auto& g2 : P.gf2s) { Gf2Args a = gf2_args(n, g2, 5); (void)a; }
        for (auto& d : P.diags) { auto num = diag_numeric(d, params); (void)num; }
        if (n_params) { try { auto ge = grad_entries(P, params); (void)ge; } catch (const Error&) {} }
        ok += js.size() > 0 && js2.size() > 0;
      }
    } catch (const Error& e) {
      ++errs;
    }
  }
  std::printf("plans ok: %zu, rejected streams: %zu\n", ok, errs);
  return 0;
}
