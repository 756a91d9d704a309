// FP64 reductions over a state: norms, overlaps, distances and Pauli
// expectations.  Every amplitude is upcast to FP64; each thread keeps a
// Neumaier (compensated) sum per output, the workgroup folds its threads'
// sums pairwise, and a one-block kernel folds the workgroup partials in a
// fixed order, so results are bitwise repeatable for a given size.
#include "kernels.h"

namespace qs {

namespace {

constexpr int kThreads = 256;

struct Acc {
  double s, c;
};

__device__ __forceinline__ void nadd(Acc& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ Acc ncombine(Acc a, const Acc& b) {
  nadd(a, b.s);
  a.c += b.c;
  return a;
}

template <int NV, class F>
__global__ void __launch_bounds__(kThreads) reduce_kernel(F f, uint64_t count, double* __restrict__ partials) {
  Acc acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = {0.0, 0.0};
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < count; t += (uint64_t)gridDim.x * kThreads)
    f(t, acc);
  __shared__ Acc red[NV][kThreads];
#pragma unroll
  for (int v = 0; v < NV; ++v) red[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) {
#pragma unroll
      for (int v = 0; v < NV; ++v) red[v][threadIdx.x] = ncombine(red[v][threadIdx.x], red[v][threadIdx.x + stride]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      partials[(blockIdx.x * NV + v) * 2] = red[v][0].s;
      partials[(blockIdx.x * NV + v) * 2 + 1] = red[v][0].c;
    }
  }
}

template <int NV>
__global__ void finalize_kernel(const double* __restrict__ partials, int nblocks, double* __restrict__ out) {
  const int v = threadIdx.x;
  if (v >= NV) return;
  Acc a = {0.0, 0.0};
  for (int b = 0; b < nblocks; ++b) a = ncombine(a, Acc{partials[(b * NV + v) * 2], partials[(b * NV + v) * 2 + 1]});
  out[v] = a.s + a.c;
}

template <class R>
__device__ __forceinline__ double abs2d(cplx<R> a) {
  const double x = (double)a.re, y = (double)a.im;
  return x * x + y * y;
}

template <class R>
struct NormF {
  const cplx2<R>* psi;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const cplx2<R> v = psi[t];
    nadd(acc[0], abs2d(v.a) + abs2d(v.b));
  }
};

template <class Ra, class Rb>
struct OverlapF {
  const cplx<Ra>* a;
  const cplx<Rb>* b;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const double ar = a[t].re, ai = a[t].im, br = b[t].re, bi = b[t].im;
    nadd(acc[0], ar * br + ai * bi);
    nadd(acc[1], ar * bi - ai * br);
  }
};

template <class Ra, class Rb>
struct DistanceF {
  const cplx<Ra>* a;
  const cplx<Rb>* b;
  double ar, ai, bs;  // || bs * b - (ar + i ai) * a ||^2
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const double xr = a[t].re, xi = a[t].im;
    const double dr = bs * (double)b[t].re - (ar * xr - ai * xi);
    const double di = bs * (double)b[t].im - (ar * xi + ai * xr);
    nadd(acc[0], dr * dr + di * di);
  }
};

struct Masks8 {
  uint32_t z[kMaxTermsPerLaunch];
  int32_t ny[kMaxTermsPerLaunch];
};

template <class R>
struct ExpectZF {
  const cplx2<R>* psi;
  Masks8 M;
  int nt;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const cplx2<R> v = psi[t];
    const double p0 = abs2d(v.a), p1 = abs2d(v.b);
    const uint32_t i = (uint32_t)(2 * t);
#pragma unroll
    for (int k = 0; k < kMaxTermsPerLaunch; ++k) {
      if (k >= nt) break;
      const double s0 = (popc(i & M.z[k]) & 1) ? -p0 : p0;
      const double s1 = (popc((i + 1) & M.z[k]) & 1) ? -p1 : p1;
      nadd(acc[k], s0 + s1);
    }
  }
};

template <class R>
struct ExpectXF {
  const cplx<R>* psi;
  Masks8 M;
  int nt;
  uint32_t x, h;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const uint32_t i = insert0((uint32_t)t, h), j = i ^ x;
    const cplx<R> a = psi[i], b = psi[j];
    // q = conj(a) b
    const double qr = (double)a.re * b.re + (double)a.im * b.im;
    const double qi = (double)a.re * b.im - (double)a.im * b.re;
#pragma unroll
    for (int k = 0; k < kMaxTermsPerLaunch; ++k) {
      if (k >= nt) break;
      const double si = (popc(i & M.z[k]) & 1) ? -1.0 : 1.0;
      const double sj = (popc(j & M.z[k]) & 1) ? -1.0 : 1.0;
      const double ur = (sj + si) * qr, ui = (sj - si) * qi;
      double v;
      switch (M.ny[k] & 3) {
        case 0: v = ur; break;
        case 1: v = -ui; break;
        case 2: v = -ur; break;
        default: v = ui; break;
      }
      nadd(acc[k], v);
    }
  }
};

inline int nblocks_for(uint64_t count) {
  uint64_t b = (count + kThreads - 1) / kThreads;
  if (b > (uint64_t)kRedBlocks) b = kRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

template <int NV, class F>
void run_reduce(const char* name, F f, uint64_t count, double* partials, double* out, hipStream_t s) {
  const int nb = nblocks_for(count);
  QS_LAUNCH(name, s, (reduce_kernel<NV, F>), dim3(nb), dim3(kThreads), 0, s, f, count, partials);
  QS_LAUNCH("reduce_finalize", s, finalize_kernel<NV>, dim3(1), dim3(64), 0, s, partials, nb, out);
}

}  // namespace

template <class R>
void launch_norm2(const cplx<R>* psi, uint64_t N, double* partials, double* out, hipStream_t s) {
  run_reduce<1>("reduce_norm2", NormF<R>{reinterpret_cast<const cplx2<R>*>(psi)}, N / 2, partials, out, s);
}

template <class Ra, class Rb>
void launch_overlap(const cplx<Ra>* a, const cplx<Rb>* b, uint64_t N, double* partials, double* out, hipStream_t s) {
  run_reduce<2>("reduce_overlap", OverlapF<Ra, Rb>{a, b}, N, partials, out, s);
}

template <class Ra, class Rb>
void launch_distance2(const cplx<Ra>* a, const cplx<Rb>* b, uint64_t N, double ar, double ai, double bs,
                      double* partials, double* out, hipStream_t s) {
  run_reduce<1>("reduce_distance2", DistanceF<Ra, Rb>{a, b, ar, ai, bs}, N, partials, out, s);
}

template <class R>
void launch_expect_z(const cplx<R>* psi, int n, const uint32_t* z, int nt, double* partials, double* out,
                     hipStream_t s) {
  Masks8 M{};
  for (int k = 0; k < nt; ++k) M.z[k] = z[k];
  ExpectZF<R> f{reinterpret_cast<const cplx2<R>*>(psi), M, nt};
  run_reduce<kMaxTermsPerLaunch>("reduce_expect_z", f, (1ull << n) / 2, partials, out, s);
}

template <class R>
void launch_expect_x(const cplx<R>* psi, int n, uint32_t x, const uint32_t* z, const int* ny, int nt,
                     double* partials, double* out, hipStream_t s) {
  Masks8 M{};
  for (int k = 0; k < nt; ++k) {
    M.z[k] = z[k];
    M.ny[k] = ny[k];
  }
  const uint32_t h = 31 - __builtin_clz(x);
  ExpectXF<R> f{psi, M, nt, x, h};
  run_reduce<kMaxTermsPerLaunch>("reduce_expect_x", f, (1ull << n) / 2, partials, out, s);
}

template void launch_norm2<float>(const cplx<float>*, uint64_t, double*, double*, hipStream_t);
template void launch_norm2<double>(const cplx<double>*, uint64_t, double*, double*, hipStream_t);
#define INST2(A, B)                                                                                            \
  template void launch_overlap<A, B>(const cplx<A>*, const cplx<B>*, uint64_t, double*, double*, hipStream_t); \
  template void launch_distance2<A, B>(const cplx<A>*, const cplx<B>*, uint64_t, double, double, double,       \
                                       double*, double*, hipStream_t);
INST2(float, float)
INST2(float, double)
INST2(double, float)
INST2(double, double)
template void launch_expect_z<float>(const cplx<float>*, int, const uint32_t*, int, double*, double*, hipStream_t);
template void launch_expect_z<double>(const cplx<double>*, int, const uint32_t*, int, double*, double*, hipStream_t);
template void launch_expect_x<float>(const cplx<float>*, int, uint32_t, const uint32_t*, const int*, int, double*,
                                     double*, hipStream_t);
template void launch_expect_x<double>(const cplx<double>*, int, uint32_t, const uint32_t*, const int*, int, double*,
                                      double*, hipStream_t);

}  // namespace qs
