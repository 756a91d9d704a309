// Device-side helpers: complex amplitudes, index bit manipulation and the
// diagonal phase evaluator shared by the streaming diagonal kernel and the
// tile passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace qs {

template <class R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};
// Two consecutive amplitudes: one 16-byte (complex64) / 32-byte (complex128) access.
template <class R>
struct alignas(4 * sizeof(R)) cplx2 {
  cplx<R> a, b;
};

// Streaming (non-temporal) global accesses: state passes touch every byte
// once, so they should not displace reusable lines from the caches.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ cplx2<float> ld_nt(const cplx2<float>* p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return {{v.x, v.y}, {v.z, v.w}};
}
__device__ __forceinline__ cplx2<double> ld_nt(const cplx2<double>* p) {
  const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  const nt_d2 b = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p) + 1);
  return {{a.x, a.y}, {b.x, b.y}};
}
__device__ __forceinline__ void st_nt(cplx2<float>* p, const cplx2<float>& v) {
  const nt_f4 w = {v.a.re, v.a.im, v.b.re, v.b.im};
  __builtin_nontemporal_store(w, reinterpret_cast<nt_f4*>(p));
}
__device__ __forceinline__ void st_nt(cplx2<double>* p, const cplx2<double>& v) {
  const nt_d2 a = {v.a.re, v.a.im}, b = {v.b.re, v.b.im};
  __builtin_nontemporal_store(a, reinterpret_cast<nt_d2*>(p));
  __builtin_nontemporal_store(b, reinterpret_cast<nt_d2*>(p) + 1);
}
__device__ __forceinline__ cplx<float> ld_nt(const cplx<float>* p) {
  const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
  return {v.x, v.y};
}
__device__ __forceinline__ cplx<double> ld_nt(const cplx<double>* p) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return {v.x, v.y};
}
__device__ __forceinline__ void st_nt(cplx<float>* p, const cplx<float>& v) {
  const nt_f2 w = {v.re, v.im};
  __builtin_nontemporal_store(w, reinterpret_cast<nt_f2*>(p));
}
__device__ __forceinline__ void st_nt(cplx<double>* p, const cplx<double>& v) {
  const nt_d2 w = {v.re, v.im};
  __builtin_nontemporal_store(w, reinterpret_cast<nt_d2*>(p));
}

// Read-only per-launch tables (round and op descriptors, coefficients, count
// terms) are read through constant-address-space pointers: the compiler then
// treats them as invariant and uses scalar loads for uniform addresses, which
// it cannot prove safe for global pointers across the workgroup barriers of a
// tile pass.  Fields are read one by one (a struct cannot be copied out of
// that address space).
#define QS_CONST __attribute__((address_space(4)))
template <class T>
using cptr = const QS_CONST T*;
template <class T>
__device__ __forceinline__ cptr<T> to_const(const T* p) {
  return (cptr<T>)p;
}
template <class R>
__device__ __forceinline__ cplx<R> ldc(cptr<cplx<R>> p, int k) {
  return {p[k].re, p[k].im};
}

template <class R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <class R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.re, -a.im}; }

// Insert a zero bit at position b of x.
__device__ __forceinline__ uint32_t insert0(uint32_t x, uint32_t b) {
  uint32_t lo = x & ((1u << b) - 1u);
  return ((x >> b) << (b + 1)) | lo;
}
__device__ __forceinline__ uint64_t insert0_64(uint64_t x, uint32_t b) {
  uint64_t lo = x & ((1ull << b) - 1ull);
  return ((x >> b) << (b + 1)) | lo;
}

__device__ __forceinline__ int popc(uint32_t x) { return __builtin_popcount(x); }

// exp(i pi x) for x = num / 2^p (num < 2^p): the argument is formed exactly
// up to the conversion of num, then sincospi of the device math library.
__device__ __forceinline__ cplx<float> cispi_frac(uint32_t num, int p) {
  float x = ldexpf((float)num, -p);
  float s, c;
  sincospif(x, &s, &c);
  return {c, s};
}
__device__ __forceinline__ cplx<double> cispi_frac_d(uint32_t num, int p) {
  double x = ldexp((double)num, -p);
  double s, c;
  sincospi(x, &s, &c);
  return {c, s};
}
template <class R>
__device__ __forceinline__ cplx<R> cispi(uint32_t num, int p);
template <>
__device__ __forceinline__ cplx<float> cispi<float>(uint32_t num, int p) { return cispi_frac(num, p); }
template <>
__device__ __forceinline__ cplx<double> cispi<double>(uint32_t num, int p) { return cispi_frac_d(num, p); }

// Diagonal phase of basis index i: prod_g LUT_g[count_g(i)].
struct DiagDev {
  const DiagTerm* terms;
  const DiagGroup* groups;
  const void* lut;      // cplx<R>
  int32_t n_groups;
  int32_t conj;
  const double* theta;  // per group: its angle reduced to (-pi, pi] (angle mode)
  double global;        // the layer's global phase angle, reduced (angle mode)
};

template <class R>
__device__ __forceinline__ int diag_count(uint32_t i, const DiagTerm* __restrict__ terms, int tb, int te) {
  int cnt = 0;
  for (int t = tb; t < te; ++t) {
    const DiagTerm T = terms[t];
    switch (T.form) {
      case DT_BITS: cnt += popc(i & T.mask); break;
      case DT_SHIFT_XOR: cnt += popc((i ^ (i >> T.shift)) & T.mask); break;
      case DT_SHIFT_AND: cnt += popc((i & (i >> T.shift)) & T.mask); break;
      case DT_PARITY: cnt += popc(i & T.mask) & 1; break;
      default: cnt += (i & T.mask) == T.mask ? 1 : 0; break;
    }
  }
  return cnt;
}

template <class R>
__device__ __forceinline__ cplx<R> diag_phase(uint32_t i, const DiagDev& D) {
  const cplx<R>* __restrict__ lut = (const cplx<R>*)D.lut;
  cplx<R> ph = {R(1), R(0)};
  for (int g = 0; g < D.n_groups; ++g) {
    const DiagGroup G = D.groups[g];
    int cnt = diag_count<R>(i, D.terms, G.term_begin, G.term_end);
    cplx<R> v = lut[G.lut_begin + cnt];
    ph = g == 0 ? v : cmul(ph, v);
  }
  if (D.conj) ph.im = -ph.im;
  return ph;
}

// Counts of NJ basis indices i0 | off[j] of one group at once.  i0 has every
// bit of every off[j] clear and off[] is the same across the workgroup, so
// each term is read once and its count splits into a part of i0, evaluated
// once, and a part of off[j]:
//   BITS       popc(i0 & m) + popc(off & m)
//   SHIFT_XOR  popc(((i0 ^ i0 >> s) & m) ^ ((off ^ off >> s) & m))   (xor is linear)
//   SHIFT_AND  popc(v & (v >> s) & m) with v = i0 | off
//   PARITY     parity(i0 & m) ^ parity(off & m)
//   ALL        ((i0 | off) & m) == m
template <int NJ>
__device__ __forceinline__ void diag_counts(uint32_t i0, const uint32_t (&off)[NJ], const DiagTerm* terms_, int tb,
                                            int te, int (&cnt)[NJ]) {
  const cptr<DiagTerm> terms = to_const(terms_);
#pragma unroll
  for (int j = 0; j < NJ; ++j) cnt[j] = 0;
  for (int t = tb; t < te; ++t) {
    const uint32_t m = terms[t].mask;
    const int s = terms[t].shift;
    switch (terms[t].form) {
      case DT_BITS: {
        const int c0 = popc(i0 & m);
#pragma unroll
        for (int j = 0; j < NJ; ++j) cnt[j] += c0 + popc(off[j] & m);
        break;
      }
      case DT_SHIFT_XOR: {
        const uint32_t y = (i0 ^ (i0 >> s)) & m;
#pragma unroll
        for (int j = 0; j < NJ; ++j) cnt[j] += popc(y ^ ((off[j] ^ (off[j] >> s)) & m));
        break;
      }
      case DT_SHIFT_AND: {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const uint32_t v = i0 | off[j];
          cnt[j] += popc(v & (v >> s) & m);
        }
        break;
      }
      case DT_PARITY: {
        const int p0 = popc(i0 & m) & 1;
#pragma unroll
        for (int j = 0; j < NJ; ++j) cnt[j] += p0 ^ (popc(off[j] & m) & 1);
        break;
      }
      default: {
#pragma unroll
        for (int j = 0; j < NJ; ++j) cnt[j] += ((i0 | off[j]) & m) == m ? 1 : 0;
        break;
      }
    }
  }
}

// a[j] *= phase(i0 | off[j]) for NJ amplitudes (same conditions as diag_counts).
template <class R, int NJ>
__device__ __forceinline__ void diag_apply(cplx<R>* a, uint32_t i0, const uint32_t (&off)[NJ], const DiagDev& D) {
  const cplx<R>* __restrict__ lut = (const cplx<R>*)D.lut;
  const cptr<DiagGroup> groups = to_const(D.groups);
  for (int g = 0; g < D.n_groups; ++g) {
    const int lb = groups[g].lut_begin;
    int cnt[NJ];
    diag_counts<NJ>(i0, off, D.terms, groups[g].term_begin, groups[g].term_end, cnt);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      cplx<R> v = lut[lb + cnt[j]];
      if (D.conj) v.im = -v.im;
      a[j] = cmul(a[j], v);
    }
  }
}

// a[j] *= exp(i (global + sum_g theta_g count_g(i0 | off[j]))): the layer's
// total angle per amplitude in FP64, then one sincos (for layers of many
// groups this replaces a table multiply per group).
template <class R, int NJ>
__device__ __forceinline__ void diag_apply_total_angle(cplx<R>* a, uint32_t i0, const uint32_t (&off)[NJ],
                                                       const DiagDev& D);

// exp(i x) for an FP64 angle: reduced to [-pi, pi] against 2 pi split in two
// doubles, then sin / cos in the state's precision.
__device__ __forceinline__ double reduce_2pi(double x) {
  const double k = rint(x * 0.15915494309189535);
  x = fma(-k, 6.283185307179586, x);
  return fma(-k, 2.4492935982947064e-16, x);
}
template <class R>
__device__ __forceinline__ cplx<R> cis_reduced(double x);
template <>
__device__ __forceinline__ cplx<float> cis_reduced<float>(double x) {
  float s, c;
  sincosf((float)reduce_2pi(x), &s, &c);
  return {c, s};
}
template <>
__device__ __forceinline__ cplx<double> cis_reduced<double>(double x) {
  double s, c;
  sincos(reduce_2pi(x), &s, &c);
  return {c, s};
}

template <class R, int NJ>
__device__ __forceinline__ void diag_apply_total_angle(cplx<R>* a, uint32_t i0, const uint32_t (&off)[NJ],
                                                       const DiagDev& D) {
  const cptr<DiagGroup> groups = to_const(D.groups);
  const cptr<double> theta = to_const(D.theta);
  double ang[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) ang[j] = D.global;
  for (int g = 0; g < D.n_groups; ++g) {
    int cnt[NJ];
    diag_counts<NJ>(i0, off, D.terms, groups[g].term_begin, groups[g].term_end, cnt);
    const double th = theta[g];
#pragma unroll
    for (int j = 0; j < NJ; ++j) ang[j] = fma(th, (double)cnt[j], ang[j]);
  }
  const double sg = D.conj ? -1.0 : 1.0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) a[j] = cmul(a[j], cis_reduced<R>(sg * ang[j]));
}

// Angle mode: every group quadratic in the round's bits, so the total phase
// angle sum_g theta_g count_g over the 16 amplitudes is A0 + sum_k x_k D_k +
// sum_{k<l} x_k x_l Q_kl; A0 and D_k come from 5 evaluations per group in
// FP64, exp(i Q_kl) are host constants (qp[0..5] for pairs 01 02 03 12 13 23).
template <class R>
__device__ __forceinline__ void diag_apply_angles(cplx<R>* a, uint32_t i0, uint32_t b0, uint32_t b1, uint32_t b2,
                                                  uint32_t b3, const DiagDev& D, const cplx<R>* qp_) {
  const cptr<DiagGroup> groups = to_const(D.groups);
  const cptr<double> theta = to_const(D.theta);
  const cptr<cplx<R>> qp = to_const(qp_);
  const uint32_t off5[5] = {0u, b0, b1, b2, b3};
  double A0 = D.global, Dk[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = 0; g < D.n_groups; ++g) {
    int c5[5];
    diag_counts<5>(i0, off5, D.terms, groups[g].term_begin, groups[g].term_end, c5);
    const double th = theta[g];
    A0 = fma(th, (double)c5[0], A0);
#pragma unroll
    for (int k = 0; k < 4; ++k) Dk[k] = fma(th, (double)(c5[k + 1] - c5[0]), Dk[k]);
  }
  const double sg = D.conj ? -1.0 : 1.0;
  cplx<R> e[4], ph[16];
  ph[0] = cis_reduced<R>(sg * A0);
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k] = cis_reduced<R>(sg * Dk[k]);
  cplx<R> q[4][4];
  {
    const int pk[6] = {0, 0, 0, 1, 1, 2}, pl[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const cplx<R> v = ldc(qp, t);
      q[pk[t]][pl[t]] = D.conj ? cconj(v) : v;
    }
  }
  // ph[j] = ph[j without its top bit t] e_t prod_{k in rest} exp(i Q_kt)
#pragma unroll
  for (int j = 1; j < 16; ++j) {
    const int t = j >= 8 ? 3 : j >= 4 ? 2 : j >= 2 ? 1 : 0;
    const int rest = j & ~(1 << t);
    cplx<R> v = cmul(ph[rest], e[t]);
#pragma unroll
    for (int k = 0; k < t; ++k)
      if ((rest >> k) & 1) v = cmul(v, q[k][t]);
    ph[j] = v;
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) a[j] = cmul(a[j], ph[j]);
}

// Lookup-table mode of a diagonal round: a[j] *= prod_g LUT_g[count_g(i0 |
// off_j)] (times the conjugates with kConj), off_j the subset j of the round's
// register bits b[0..3].  A group whose pair-table row (qt, kPairRowWords
// words per group) marks it quadratic gets its 16 counts from the count at i0,
// the four single-bit changes d_k and the pair coefficients:
//   count(j) = count(j without its top bit t) + d_t + sum_{k < t, k in j} q_kt,
// one add per amplitude since the q sums are uniform; other groups evaluate all
// 16 indices.  Table entries are read at 32-bit byte offsets from the group's
// first entry.
template <class R, bool kConj>
__device__ __forceinline__ void diag_lut_round(cplx<R>* a, uint32_t i0, const uint32_t (&b)[4], const DiagDev& D,
                                               cptr<int32_t> qt) {
  const cptr<DiagGroup> groups = to_const(D.groups);
  const cptr<DiagTerm> terms = to_const(D.terms);
  for (int g = 0; g < D.n_groups; ++g) {
    const cptr<int32_t> row = qt + kPairRowWords * g;
    const char* lut = reinterpret_cast<const char*>(D.lut) + sizeof(cplx<R>) * (size_t)groups[g].lut_begin;
    int cnt[16];
    if (row[0]) {
      int c0, d[4];
      if (row[7]) {
        // distinct bit-pair mismatches: deg_k - 2 popcount(N_k & i0) per bit
        c0 = 0;
        for (int t = groups[g].term_begin; t < groups[g].term_end; ++t)
          c0 += popc((i0 ^ (i0 >> terms[t].shift)) & terms[t].mask);
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = row[8 + k] - 2 * popc(i0 & (uint32_t)row[12 + k]);
      } else {
        const uint32_t off5[5] = {0u, b[0], b[1], b[2], b[3]};
        int c5[5];
        diag_counts<5>(i0, off5, D.terms, groups[g].term_begin, groups[g].term_end, c5);
        c0 = c5[0];
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = c5[k + 1] - c5[0];
      }
      // q[k][t] for k < t: pairs 01 02 03 12 13 23 at row[1..6]
      const int q01 = row[1], q02 = row[2], q03 = row[3], q12 = row[4], q13 = row[5], q23 = row[6];
      cnt[0] = c0;
#pragma unroll
      for (int j = 1; j < 16; ++j) {
        const int t = j >= 8 ? 3 : j >= 4 ? 2 : j >= 2 ? 1 : 0;
        const int rest = j & ~(1 << t);
        int qs = 0;
        if (t == 1) qs = (rest & 1) ? q01 : 0;
        if (t == 2) qs = ((rest & 1) ? q02 : 0) + ((rest & 2) ? q12 : 0);
        if (t == 3) qs = ((rest & 1) ? q03 : 0) + ((rest & 2) ? q13 : 0) + ((rest & 4) ? q23 : 0);
        cnt[j] = cnt[rest] + (d[t] + qs);
      }
    } else {
      uint32_t off[16];
#pragma unroll
      for (int j = 0; j < 16; ++j)
        off[j] = ((j & 1) ? b[0] : 0u) | ((j & 2) ? b[1] : 0u) | ((j & 4) ? b[2] : 0u) | ((j & 8) ? b[3] : 0u);
      diag_counts<16>(i0, off, D.terms, groups[g].term_begin, groups[g].term_end, cnt);
    }
    // entries fetched eight at a time, all eight loads issued before the
    // first use (the scheduler would otherwise wait on each load in turn to
    // save registers)
#pragma unroll
    for (int j0 = 0; j0 < 16; j0 += 8) {
      cplx<R> v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        v[k] = *reinterpret_cast<const cplx<R>*>(lut + (uint32_t)cnt[j0 + k] * (uint32_t)sizeof(cplx<R>));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 8; ++k) a[j0 + k] = kConj ? cmulc(a[j0 + k], v[k]) : cmul(a[j0 + k], v[k]);
    }
  }
}

// A one-group layer whose count is a sum of distinct bit-pair mismatches (the
// row's quadratic and pair flags set): the lookup-table round without loops
// over groups or branches on the row, for the pair row of the round's bits.
template <class R, bool kConj>
__device__ __forceinline__ void diag_pair_round(cplx<R>* a, uint32_t i0, const DiagDev& D, cptr<int32_t> row) {
  const cptr<DiagGroup> groups = to_const(D.groups);
  const cptr<DiagTerm> terms = to_const(D.terms);
  const char* lut = reinterpret_cast<const char*>(D.lut) + sizeof(cplx<R>) * (size_t)groups[0].lut_begin;
  int c0 = 0;
  for (int t = groups[0].term_begin; t < groups[0].term_end; ++t)
    c0 += popc((i0 ^ (i0 >> terms[t].shift)) & terms[t].mask);
  int d[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) d[k] = row[8 + k] - 2 * popc(i0 & (uint32_t)row[12 + k]);
  const int q01 = row[1], q02 = row[2], q03 = row[3], q12 = row[4], q13 = row[5], q23 = row[6];
  int cnt[16];
  cnt[0] = c0;
#pragma unroll
  for (int j = 1; j < 16; ++j) {
    const int t = j >= 8 ? 3 : j >= 4 ? 2 : j >= 2 ? 1 : 0;
    const int rest = j & ~(1 << t);
    int qs = 0;
    if (t == 1) qs = (rest & 1) ? q01 : 0;
    if (t == 2) qs = ((rest & 1) ? q02 : 0) + ((rest & 2) ? q12 : 0);
    if (t == 3) qs = ((rest & 1) ? q03 : 0) + ((rest & 2) ? q13 : 0) + ((rest & 4) ? q23 : 0);
    cnt[j] = cnt[rest] + (d[t] + qs);
  }
#pragma unroll
  for (int j0 = 0; j0 < 16; j0 += 8) {
    cplx<R> v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      v[k] = *reinterpret_cast<const cplx<R>*>(lut + (uint32_t)cnt[j0 + k] * (uint32_t)sizeof(cplx<R>));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[j0 + k] = kConj ? cmulc(a[j0 + k], v[k]) : cmul(a[j0 + k], v[k]);
  }
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup w on XCD w mod 8).
// Virtual block (w mod 8) G/8 + w/8 gives each XCD a contiguous range of the
// G blocks, so the work one XCD has in flight is contiguous in memory.  A
// bijection of [0, G) when G is a multiple of 8 (identity otherwise).
__device__ __forceinline__ uint32_t xcd_block(uint32_t w, uint32_t grid) {
  return (grid & 7u) == 0u ? (w & 7u) * (grid >> 3) + (w >> 3) : w;
}

// |a|^2 in FP64.
template <class R>
__device__ __forceinline__ double abs2_d(const cplx<R>& a) {
  const double x = (double)a.re, y = (double)a.im;
  return x * x + y * y;
}

// Wavefront sum of one FP64 value per lane in a fixed butterfly order (every
// lane receives the total).
__device__ __forceinline__ double wave_sum_fixed(double x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Workgroup sum of one FP64 value per thread in a fixed order (butterflies
// within each wavefront, then the wavefronts in order); thread 0 receives
// the total.  Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum_fixed(double x) {
  __shared__ double wsum[16];
  x = wave_sum_fixed(x);
  if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (uint32_t k = 0; k < (blockDim.x >> 6); ++k) t += wsum[k];
  return t;
}

}  // namespace qs
