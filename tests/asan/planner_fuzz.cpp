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
  size_t ok = 0, errs = 0, nbr_checks = 0;
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
        for (auto& d : P.diags) {
          auto num = diag_numeric(d, params);
          // neighbour masks of pair-mismatch groups against direct counts:
          // setting zero bits p (and q) of i moves the count by deg - 2|N & i|
          // (and -2 more when p, q are a pair)
          auto pn = pair_neighbours(num, n);
          for (size_t g = 0; g < pn.size(); ++g) {
            if (!pn[g].ok) continue;
            auto count = [&](uint32_t i) {
              int c = 0;
              for (int t = num.groups[g].term_begin; t < num.groups[g].term_end; ++t)
                c += __builtin_popcount((i ^ (i >> num.terms[t].shift)) & num.terms[t].mask);
              return c;
            };
            const uint32_t full = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
            for (int trial = 0; trial < 8; ++trial) {
              const int bp = (int)(rng() % n), bq = (int)(rng() % n);
              const uint32_t i = (uint32_t)rng() & full & ~(1u << bp) & ~(1u << bq);
              const int dp = pn[g].deg[bp] - 2 * __builtin_popcount(pn[g].mask[bp] & i);
              const int dq = pn[g].deg[bq] - 2 * __builtin_popcount(pn[g].mask[bq] & i);
              const int pair = bp != bq && ((pn[g].mask[bp] >> bq) & 1u) ? -2 : 0;
              const int want1 = count(i | (1u << bp)) - count(i);
              const int want2 = bp != bq ? count(i | (1u << bp) | (1u << bq)) - count(i) : want1;
              if (want1 != dp || want2 != (bp != bq ? dp + dq + pair : dp)) {
                std::printf("pair neighbours disagree: n=%d group=%zu bits %d %d\n", n, g, bp, bq);
                return 1;
              }
              ++nbr_checks;
            }
          }
        }
        if (n_params) { try { auto ge = grad_entries(P, params); (void)ge; } catch (const Error&) {} }
        ok += js.size() > 0 && js2.size() > 0;
      }
    } catch (const Error& e) {
      ++errs;
    }
  }
  std::printf("plans ok: %zu, rejected streams: %zu, pair-neighbour checks: %zu\n", ok, errs, nbr_checks);
  return 0;
}
