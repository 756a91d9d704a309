// Rounding of unit-modulus coefficients and 2x2 unitaries to float that keeps
// them as close to unit modulus / unitary as float allows (host only).
//
// Round-to-nearest of a phase (c, s) = (cos x, sin x) gives c^2 + s^2 = 1 + d
// with |d| up to ~1.2e-7.  A layer that applies the same rotation to every
// qubit then scales the norm by about (1 + d)^n: a systematic drift that the
// expectation values of a complex64 state inherit (at 24 qubits and four
// mixer layers, ~1e-5 relative).  Among the floats within one ulp of each
// rounded component, the pair minimising |c^2 + s^2 - 1| is chosen instead
// (lookup-table phases); rotations and 2x2 unitaries of a plan additionally
// cancel their deviations against each other (NormAcc below).  A 2x2 unitary
// is treated through its Gram matrix U^dagger U (coordinate descent over its
// eight real parts, each held within two ulp of its nearest float).
// Components that are exactly zero stay zero.  Double precision needs none of
// this (the cast is exact).
#pragma once
#include <cmath>
#include <complex>
#include <cstddef>
#include <vector>

#include "dev.h"

namespace qs {

inline float fround_step(float x, int k) {
  for (; k > 0; --k) x = std::nextafter(x, INFINITY);
  for (; k < 0; ++k) x = std::nextafter(x, -INFINITY);
  return x;
}

// True when |v| = 1 to within rounding of its double computation.
inline bool fround_is_phase(std::complex<double> v) { return std::fabs(std::norm(v) - 1.0) < 1e-12; }

inline bool fround_exact(double x);

inline cplx<float> fround_phase(std::complex<double> v) {
  const float r0 = (float)v.real(), i0 = (float)v.imag();
  cplx<float> best = {r0, i0};
  double best_e = INFINITY, best_d = INFINITY;
  for (int a = -1; a <= 1; ++a) {
    if (a && fround_exact(v.real())) continue;
    const float r = fround_step(r0, a);
    for (int b = -1; b <= 1; ++b) {
      if (b && fround_exact(v.imag())) continue;
      const float i = fround_step(i0, b);
      // r*r and i*i are exact in double; their sum is rounded once
      const double e = std::fabs((double)r * r + (double)i * i - 1.0);
      const double d = std::norm(std::complex<double>(r, i) - v);
      if (e < best_e || (e == best_e && d < best_d)) {
        best_e = e;
        best_d = d;
        best = {r, i};
      }
    }
  }
  return best;
}

// Norm compensation across a plan.  A rotation pair (c, s) as the tile
// rounds use it (RX: [[c, -i s], [-i s, c]], RY: [[c, -s], [s, c]]) scales
// every state's norm by exactly c^2 + s^2 = 1 + d; a 2x2 U scales it by
// 1 + t on average, t = the mean deviation of its column norms.  Those
// factors multiply along the plan, so the rounding of each successive
// rotation (candidates within two ulp of each rounded component) is chosen to
// bring the running sum of deviations back towards zero: the plan's total
// norm factor then stays within about one step of 1 instead of growing with
// the number of rotations (a QAOA mixer applies the same angle to every qubit,
// so plain rounding would add n equal deviations per layer).
struct NormAcc {
  double sum = 0.0;
};

// Components that float holds exactly (0, +-1, +-1/2, ...) are kept as they are.
inline bool fround_exact(double x) { return (double)(float)x == x; }

inline cplx<float> fround_pair(std::complex<double> v, NormAcc& acc) {
  const float r0 = (float)v.real(), i0 = (float)v.imag();
  if (!fround_is_phase(v)) return {r0, i0};
  cplx<float> best = {r0, i0};
  double best_e = INFINITY, best_d = INFINITY, best_dev = 0.0;
  for (int a = -2; a <= 2; ++a) {
    if (a && fround_exact(v.real())) continue;
    const float r = fround_step(r0, a);
    for (int b = -2; b <= 2; ++b) {
      if (b && fround_exact(v.imag())) continue;
      const float i = fround_step(i0, b);
      const double dev = (double)r * r + (double)i * i - 1.0;
      const double e = std::fabs(acc.sum + dev);
      const double d = std::norm(std::complex<double>(r, i) - v);
      if (e < best_e || (e == best_e && d < best_d)) {
        best_e = e;
        best_d = d;
        best_dev = dev;
        best = {r, i};
      }
    }
  }
  acc.sum += best_dev;
  return best;
}

// Deviation of U^dagger U from the identity (U row-major 2x2, entries
// interleaved re, im as floats widened to double): the squared off-diagonal
// and column-norm difference, plus the squared running norm factor after U.
inline double fround_gram_error(const float* u, double acc, double* trace_dev) {
  const std::complex<double> a(u[0], u[1]), b(u[2], u[3]), c(u[4], u[5]), d(u[6], u[7]);
  const double n0 = std::norm(a) + std::norm(c) - 1.0, n1 = std::norm(b) + std::norm(d) - 1.0;
  const std::complex<double> o = std::conj(a) * b + std::conj(c) * d;
  const double t = 0.5 * (n0 + n1), h = 0.5 * (n0 - n1);
  *trace_dev = t;
  return (acc + t) * (acc + t) + h * h + 2.0 * std::norm(o);
}

// U must be unitary (in double) to take part: anything else (the unscaled
// Hadamard butterfly of a tile round, say) is rounded to nearest and leaves
// acc alone.
inline bool fround_is_unitary2(const std::complex<double>* U) {
  const double n0 = std::norm(U[0]) + std::norm(U[2]) - 1.0, n1 = std::norm(U[1]) + std::norm(U[3]) - 1.0;
  const std::complex<double> o = std::conj(U[0]) * U[1] + std::conj(U[2]) * U[3];
  return std::fabs(n0) < 1e-12 && std::fabs(n1) < 1e-12 && std::abs(o) < 1e-12;
}

inline void fround_unitary2(const std::complex<double>* U, cplx<float>* out, NormAcc& acc) {
  float v[8], v0[8];
  bool fixed[8];
  for (int e = 0; e < 4; ++e) {
    v0[2 * e] = v[2 * e] = (float)U[e].real();
    v0[2 * e + 1] = v[2 * e + 1] = (float)U[e].imag();
    fixed[2 * e] = fround_exact(U[e].real());
    fixed[2 * e + 1] = fround_exact(U[e].imag());
  }
  if (!fround_is_unitary2(U)) {
    for (int e = 0; e < 4; ++e) out[e] = {v[2 * e], v[2 * e + 1]};
    return;
  }
  double t = 0.0;
  double err = fround_gram_error(v, acc.sum, &t);
  int off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int sweep = 0; sweep < 8 && err > 0.0; ++sweep) {
    bool moved = false;
    for (int k = 0; k < 8; ++k) {
      if (fixed[k]) continue;
      for (int step = -1; step <= 1; step += 2) {
        const int o = off[k] + step;
        if (o < -2 || o > 2) continue;
        const float keep = v[k];
        v[k] = fround_step(v0[k], o);
        double tt;
        const double e = fround_gram_error(v, acc.sum, &tt);
        if (e < err) {
          err = e;
          off[k] = o;
          moved = true;
        } else {
          v[k] = keep;
        }
      }
    }
    if (!moved) break;
  }
  fround_gram_error(v, acc.sum, &t);
  acc.sum += t;
  for (int e = 0; e < 4; ++e) out[e] = {v[2 * e], v[2 * e + 1]};
}

// Entries in device precision: unit-modulus ones as fround_phase, anything
// else to nearest.
// A tile pass's store scale in float: among the floats within two ulp of the
// nearest, the one whose norm factor (f / x)^2 best cancels the running
// deviation (the scale carries the normalisation of factored rotations and
// of unscaled butterflies, so its rounding acts like a rotation's).
inline double fround_scale(double x, NormAcc& acc) {
  if (fround_exact(x)) return x;
  const float f0 = (float)x;
  double best = f0, best_e = INFINITY, best_dev = 0.0;
  for (int k = -2; k <= 2; ++k) {
    const double f = fround_step(f0, k);
    const double dev = (f / x) * (f / x) - 1.0;
    const double e = std::fabs(acc.sum + dev);
    if (e < best_e) {
      best_e = e;
      best = f;
      best_dev = dev;
    }
  }
  acc.sum += best_dev;
  return best;
}

template <class R>
std::vector<cplx<R>> round_entries(const std::vector<std::complex<double>>& v) {
  std::vector<cplx<R>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    if (sizeof(R) == sizeof(float) && fround_is_phase(v[i])) {
      const cplx<float> f = fround_phase(v[i]);
      o[i] = {(R)f.re, (R)f.im};
    } else {
      o[i] = {(R)v[i].real(), (R)v[i].imag()};
    }
  }
  return o;
}

// A gate matrix (dim x dim, row-major) in device precision: 2x2 unitaries and
// unit-modulus entries (diagonal gates) as above, anything else to nearest.
// A 2x2 takes part in the running compensation acc (the per-gate path keeps
// one per state).
template <class R>
std::vector<cplx<R>> round_gate(const std::vector<std::complex<double>>& M, int dim, NormAcc& acc);

template <>
inline std::vector<cplx<double>> round_gate<double>(const std::vector<std::complex<double>>& M, int, NormAcc&) {
  std::vector<cplx<double>> o(M.size());
  for (size_t i = 0; i < M.size(); ++i) o[i] = {M[i].real(), M[i].imag()};
  return o;
}

template <>
inline std::vector<cplx<float>> round_gate<float>(const std::vector<std::complex<double>>& M, int dim,
                                                  NormAcc& acc) {
  std::vector<cplx<float>> o(M.size());
  if (dim == 2 && M.size() == 4) {
    fround_unitary2(M.data(), o.data(), acc);
    return o;
  }
  bool diag = (size_t)dim * dim == M.size();
  for (int r = 0; r < dim && diag; ++r)
    for (int c = 0; c < dim && diag; ++c) diag = r == c ? fround_is_phase(M[r * dim + r]) : M[r * dim + c] == 0.0;
  if (diag) {
    // a diagonal unitary scales the norm by 1 + (mean deviation of its
    // entries) on average: its entries are chosen in turn to cancel acc
    double run = acc.sum * dim;
    for (int r = 0; r < dim; ++r) {
      NormAcc part{run};
      o[r * dim + r] = fround_pair(M[r * dim + r], part);
      run = part.sum;
    }
    acc.sum = run / dim;
    return o;
  }
  for (size_t i = 0; i < M.size(); ++i)
    o[i] = fround_is_phase(M[i]) ? fround_phase(M[i]) : cplx<float>{(float)M[i].real(), (float)M[i].imag()};
  return o;
}

}  // namespace qs
