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
  const void* lut;  // cplx<R>
  int32_t n_groups;
  int32_t conj;
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

}  // namespace qs
