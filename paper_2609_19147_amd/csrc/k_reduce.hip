// FP64 reductions over a state: norms, overlaps, distances and Pauli
// expectations.  Every amplitude is upcast to FP64; each thread keeps a
// Neumaier (compensated) sum per output, the workgroup folds its threads'
// sums pairwise, and a second kernel (one workgroup per output) folds the
// workgroup partials in a fixed order, so results are bitwise repeatable for
// a given size.
#include "kernels.h"
#include "rho.h"

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
  for (uint64_t t = xcd_block(blockIdx.x, gridDim.x) * (uint64_t)kThreads + threadIdx.x; t < count;
       t += (uint64_t)gridDim.x * kThreads)
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

// Fold of a block's per-thread sums in a fixed pairwise order (every thread
// of the block must call it).
__device__ __forceinline__ Acc block_fold(Acc a, Acc* red) {
  red[threadIdx.x] = a;
  __syncthreads();
  for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) red[threadIdx.x] = ncombine(red[threadIdx.x], red[threadIdx.x + stride]);
    __syncthreads();
  }
  return red[0];
}

// One workgroup per output: thread x folds partials x, x + kThreads, ... in
// order, then the workgroup folds its threads pairwise.
template <int NV>
__global__ void __launch_bounds__(kThreads) finalize_kernel(const double* __restrict__ partials, int nblocks,
                                                            double* __restrict__ out) {
  const int v = blockIdx.x;
  Acc a = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kThreads)
    a = ncombine(a, Acc{partials[(b * NV + v) * 2], partials[(b * NV + v) * 2 + 1]});
  __shared__ Acc red[kThreads];
  a = block_fold(a, red);
  if (threadIdx.x == 0) out[v] = a.s + a.c;
}


template <class R>
struct NormF {
  const cplx2<R>* psi;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const cplx2<R> v = psi[t];
    nadd(acc[0], abs2_d(v.a) + abs2_d(v.b));
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
    const double p0 = abs2_d(v.a), p1 = abs2_d(v.b);
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

template <class R>
struct PairRhoF {
  const cplx<R>* phi;
  const cplx<R>* lam;
  uint32_t b;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const uint32_t i0 = insert0((uint32_t)t, b), i1 = i0 | (1u << b);
    const cplx<R> p0 = phi[i0], p1 = phi[i1], l0 = lam[i0], l1 = lam[i1];
    const double p0r = p0.re, p0i = p0.im, p1r = p1.re, p1i = p1.im;
    const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
    // conj(l_r) * p_c
    nadd(acc[0], l0r * p0r + l0i * p0i);
    nadd(acc[1], l0r * p0i - l0i * p0r);
    nadd(acc[2], l0r * p1r + l0i * p1i);
    nadd(acc[3], l0r * p1i - l0i * p1r);
    nadd(acc[4], l1r * p0r + l1i * p0i);
    nadd(acc[5], l1r * p0i - l1i * p0r);
    nadd(acc[6], l1r * p1r + l1i * p1i);
    nadd(acc[7], l1r * p1i - l1i * p1r);
  }
};

template <class R>
struct DiagGradF {
  const cplx<R>* phi;
  const cplx<R>* lam;
  DiagDev D;
  int g0, ng;
  __device__ void operator()(uint64_t t, Acc* acc) const {
    const uint32_t i = (uint32_t)t;
    const cplx<R> p = phi[i], l = lam[i];
    const double im = (double)l.re * p.im - (double)l.im * p.re;  // Im(conj(l) p)
#pragma unroll
    for (int k = 0; k < kMaxTermsPerLaunch; ++k) {
      if (k >= ng) break;
      const DiagGroup G = D.groups[g0 + k];
      nadd(acc[k], im * (double)diag_count<R>(i, D.terms, G.term_begin, G.term_end));
    }
  }
};

// Batched diagonal observable: block b covers chunk (b & (2^cs - 1)) of
// instance (b >> cs); each chunk is 2^ls consecutive amplitudes.
template <class R>
__global__ void __launch_bounds__(kThreads) batch_obs_kernel(const ObsDev* __restrict__ obs, uint32_t cs, uint32_t ls,
                                                             double* __restrict__ partials) {
  const ObsDev& O = obs[blockIdx.x >> cs];
  const cplx2<R>* __restrict__ psi = (const cplx2<R>*)O.psi;
  const uint32_t base = (blockIdx.x & ((1u << cs) - 1u)) << ls;
  const uint32_t len = 1u << ls;
  constexpr int K = 4;  // pairs per thread per step
  Acc acc = {0.0, 0.0};
  if (len >= 2u * K * kThreads) {
    // thread x owns amplitudes 2x | (j & 1) | (j >> 1) 2 kThreads of each step
    uint32_t off[2 * K];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) off[j] = (uint32_t)(j & 1) | (uint32_t)(j >> 1) * (2u * kThreads);
    for (uint32_t c = 0; c < len; c += 2u * K * kThreads) {
      const uint32_t i0 = base + c + 2u * threadIdx.x;
      double p[2 * K], v[2 * K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const cplx2<R> x = psi[(i0 >> 1) + k * kThreads];
        p[2 * k] = abs2_d(x.a);
        p[2 * k + 1] = abs2_d(x.b);
      }
#pragma unroll
      for (int j = 0; j < 2 * K; ++j) v[j] = O.c0;
      for (int g = 0; g < O.n_groups; ++g) {
        const DiagGroup G = O.groups[g];
        int cnt[2 * K];
        const int32_t* nb = O.nbr + g * kObsNbrStride;
        if (nb[64]) {
          // a sum of distinct pair mismatches, quadratic in the flipped bits
          // 0, 9, 10 of the eight points (zero in i0): the count at i0, then
          // per flipped bit deg - 2 popcount(N & i0), and -2 per flipped pair
          int c0 = 0;
          for (int t = G.term_begin; t < G.term_end; ++t) {
            const uint32_t m = (uint32_t)O.terms[t].mask;
            const int s = O.terms[t].shift;
            c0 += popc((i0 ^ (i0 >> s)) & m);
          }
          static_assert(2 * kThreads == 512, "the eight points flip state bits 0, 9 and 10");
          constexpr int kb[3] = {0, 9, 10};
          int d[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) d[k] = nb[32 + kb[k]] - 2 * popc(i0 & (uint32_t)nb[kb[k]]);
          const int q01 = -2 * (int)(((uint32_t)nb[0] >> 9) & 1u), q02 = -2 * (int)(((uint32_t)nb[0] >> 10) & 1u);
          const int q12 = -2 * (int)(((uint32_t)nb[9] >> 10) & 1u);
#pragma unroll
          for (int j = 0; j < 2 * K; ++j) {
            const int f0 = j & 1, f1 = (j >> 1) & 1, f2 = (j >> 2) & 1;
            cnt[j] = c0 + f0 * d[0] + f1 * d[1] + f2 * d[2] + f0 * f1 * q01 + f0 * f2 * q02 + f1 * f2 * q12;
          }
        } else {
          diag_counts<2 * K>(i0, off, O.terms, G.term_begin, G.term_end, cnt);
        }
        const double w = O.w[g];
#pragma unroll
        for (int j = 0; j < 2 * K; ++j) v[j] += w * (double)cnt[j];
      }
#pragma unroll
      for (int j = 0; j < 2 * K; ++j) nadd(acc, p[j] * v[j]);
    }
  } else {
    const uint32_t off[2] = {0u, 1u};
    for (uint32_t t = threadIdx.x; t < len / 2; t += kThreads) {
      const uint32_t i0 = base + 2u * t;
      const cplx2<R> x = psi[i0 >> 1];
      const double p[2] = {abs2_d(x.a), abs2_d(x.b)};
      double v[2] = {O.c0, O.c0};
      for (int g = 0; g < O.n_groups; ++g) {
        const DiagGroup G = O.groups[g];
        int cnt[2];
        diag_counts<2>(i0, off, O.terms, G.term_begin, G.term_end, cnt);
        v[0] += O.w[g] * (double)cnt[0];
        v[1] += O.w[g] * (double)cnt[1];
      }
      nadd(acc, p[0] * v[0]);
      nadd(acc, p[1] * v[1]);
    }
  }
  __shared__ Acc red[kThreads];
  acc = block_fold(acc, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = acc.s;
    partials[2 * blockIdx.x + 1] = acc.c;
  }
}

// One workgroup per instance folds its 2^cs chunk partials.
__global__ void __launch_bounds__(kThreads) batch_obs_finalize(const double* __restrict__ partials, uint32_t cs,
                                                               double* __restrict__ out) {
  const uint32_t inst = blockIdx.x;
  Acc a = {0.0, 0.0};
  for (uint32_t c = threadIdx.x; c < (1u << cs); c += kThreads) {
    const uint32_t b = (inst << cs) + c;
    a = ncombine(a, Acc{partials[2 * b], partials[2 * b + 1]});
  }
  __shared__ Acc red[kThreads];
  a = block_fold(a, red);
  if (threadIdx.x == 0) out[inst] = a.s + a.c;
}

inline void batch_obs_shape(uint32_t n, uint32_t* cs, uint32_t* ls) {
  *ls = n < 14 ? n : 14;
  *cs = n - *ls;
}

inline int nblocks_for(uint64_t count) {
  uint64_t b = (count + kThreads - 1) / kThreads;
  if (b > (uint64_t)kRedBlocks) b = kRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

// Block b sums the partials [b chunk, (b + 1) chunk) with its threads
// strided (compensated), then pairwise (a fixed order throughout).
__global__ void __launch_bounds__(kThreads) fold_kernel(const double* __restrict__ partials, uint64_t count,
                                                        uint64_t chunk, double* __restrict__ out) {
  const uint64_t b0 = blockIdx.x * chunk, b1 = b0 + chunk < count ? b0 + chunk : count;
  Acc a = {0.0, 0.0};
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += kThreads) nadd(a, partials[i]);
  __shared__ Acc red[kThreads];
  a = block_fold(a, red);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = a.s;
    out[2 * blockIdx.x + 1] = a.c;
  }
}

template <int NV, class F>
void run_reduce(const char* name, F f, uint64_t count, double* partials, double* out, hipStream_t s) {
  const int nb = nblocks_for(count);
  QS_LAUNCH(name, s, (reduce_kernel<NV, F>), dim3(nb), dim3(kThreads), 0, s, f, count, partials);
  QS_LAUNCH("reduce_finalize", s, finalize_kernel<NV>, dim3(NV), dim3(kThreads), 0, s, partials, nb, out);
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

template <class R>
void launch_pair_rho(const cplx<R>* phi, const cplx<R>* lam, int n, int b, double* partials, double* out,
                     hipStream_t s) {
  run_reduce<8>("reduce_pair_rho", PairRhoF<R>{phi, lam, (uint32_t)b}, (1ull << n) / 2, partials, out, s);
}
template <class R>
void launch_diag_grad(const cplx<R>* phi, const cplx<R>* lam, int n, const DiagDev& D, int g0, int ng,
                      double* partials, double* out, hipStream_t s) {
  run_reduce<kMaxTermsPerLaunch>("reduce_diag_grad", DiagGradF<R>{phi, lam, D, g0, ng}, 1ull << n, partials, out, s);
}
template void launch_pair_rho<float>(const cplx<float>*, const cplx<float>*, int, int, double*, double*, hipStream_t);
template void launch_pair_rho<double>(const cplx<double>*, const cplx<double>*, int, int, double*, double*,
                                      hipStream_t);
template void launch_diag_grad<float>(const cplx<float>*, const cplx<float>*, int, const DiagDev&, int, int, double*,
                                      double*, hipStream_t);
template void launch_diag_grad<double>(const cplx<double>*, const cplx<double>*, int, const DiagDev&, int, int,
                                       double*, double*, hipStream_t);

// ---- cross densities of several bits at once (adjoint sweep) ---------------
namespace {
using namespace rho;

// One workgroup per coset of the tile bits [0, L) U [a, a + h): phi and lambda
// tiles staged in LDS, then the requested tile bits in chunks of four
// (complex64) or three (complex128), each
// giving per bit the eight sums rho_b[r][c] = sum conj(lam_r) phi_c over the
// tile's pairs along b.  Sums inside a thread run in the state's precision
// (eight pair terms per group), the folds across lanes, wavefronts (fixed
// order) and tiles (compensated, rho_finalize) in FP64.  Partials are stored
// value-major: partials[(8 bi + v) ntiles + tile].
template <class R>
__global__ void __launch_bounds__(kRhoMaxThreads) rho_tile_kernel(const cplx<R>* __restrict__ phi,
                                                                  const cplx<R>* __restrict__ lam, RhoTileArgs A,
                                                                  double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[kRhoMaxWaves][32];
  const uint32_t M = 1u << A.m;
  cplx<R>* P = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* Q = P + rho_lds_off(M);
  const uint32_t ntiles = gridDim.x;
  const uint32_t tile = xcd_block(blockIdx.x, ntiles);
  const uint32_t nlo = A.a - A.L, top = A.a + A.h;
  const uint32_t base = ((tile & ((1u << nlo) - 1u)) << A.L) | (top >= 32 ? 0u : ((tile >> nlo) << top));
  const uint32_t lmask = (1u << A.L) - 1u;
  const uint32_t stride = 2u * blockDim.x;
  // every thread's 16-byte accesses of both tiles in flight at once (up to
  // eight per state: 2^13 complex64 amplitudes over 512 threads)
  constexpr int kLd = 8;
  for (uint32_t p0 = 2u * threadIdx.x; p0 < M; p0 += kLd * stride) {
    cplx2<R> vf[kLd], vl[kLd];
#pragma unroll
    for (int k = 0; k < kLd; ++k) {
      const uint32_t pos = p0 + k * stride;
      if (pos < M) {
        const uint32_t g = base | (pos & lmask) | ((pos >> A.L) << A.a);
        vf[k] = ld_nt(reinterpret_cast<const cplx2<R>*>(phi + g));
        vl[k] = ld_nt(reinterpret_cast<const cplx2<R>*>(lam + g));
      }
    }
#pragma unroll
    for (int k = 0; k < kLd; ++k) {
      const uint32_t pos = p0 + k * stride;
      if (pos < M) {
        *reinterpret_cast<cplx2<R>*>(P + rho_lds_off(pos)) = vf[k];
        *reinterpret_cast<cplx2<R>*>(Q + rho_lds_off(pos)) = vl[k];
      }
    }
  }
  __syncthreads();
  accumulate_tile<R>(P, Q, M, A, red, partials, tile, ntiles);
}

// out[o] = sum over tiles t of partials[o * ntiles + t], compensated, fixed order.
__global__ void __launch_bounds__(kThreads) rho_finalize(const double* __restrict__ partials, uint32_t ntiles,
                                                         double* __restrict__ out) {
  const uint32_t o = blockIdx.x;
  const double* row = partials + (size_t)o * ntiles;
  Acc a = {0.0, 0.0};
  // eight loads in flight, added in the same order as one at a time (the
  // zeros past the end add nothing)
  for (uint32_t t0 = threadIdx.x; t0 < ntiles; t0 += 8 * kThreads) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t t = t0 + k * kThreads;
      v[k] = t < ntiles ? row[t] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) nadd(a, v[k]);
  }
  __shared__ Acc red[kThreads];
  a = block_fold(a, red);
  if (threadIdx.x == 0) out[o] = a.s + a.c;
}

}  // namespace

size_t rho_tile_partials(int n, const RhoTileArgs& A) { return ((size_t)1 << (n - A.m)) * A.nbits * 8; }

void launch_rho_finalize(const double* partials, uint32_t ntiles, uint32_t nvals, double* out, hipStream_t s) {
  QS_LAUNCH("reduce_rho_finalize", s, rho_finalize, dim3(nvals), dim3(kThreads), 0, s, partials, ntiles, out);
}

bool rho_tile_fits(uint32_t m, size_t amp_bytes) {
  const uint32_t M = 1u << m;
  // both tiles plus the kernel's 2 KiB of static LDS within the CU's 160 KiB
  return m >= 7 && 2 * amp_bytes * (M + ((M >> 5) << 1)) + 2048 <= 160 * 1024;
}

template <class R>
bool launch_rho_tile(const cplx<R>* phi, const cplx<R>* lam, int n, const RhoTileArgs& A, double* partials,
                     double* out, hipStream_t s) {
  constexpr size_t kMaxDynamic = 158 * 1024;
  const uint32_t M = 1u << A.m;
  const size_t lds = 2 * sizeof(cplx<R>) * (M + ((M >> 5) << 1));
  if (!rho_tile_fits(A.m, sizeof(cplx<R>)) || A.nbits == 0 || A.nbits > 32) return false;
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)rho_tile_kernel<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMaxDynamic) != hipSuccess) {
      (void)hipGetLastError();  // the caller falls back to the per-bit path
      return false;
    }
    attr_set = true;
  }
  const uint32_t ntiles = 1u << (n - A.m);
  QS_LAUNCH("reduce_rho_tile", s, rho_tile_kernel<R>, dim3(ntiles), dim3(rho_threads(A.m)), lds, s, phi, lam, A,
            partials);
  QS_LAUNCH("reduce_rho_finalize", s, rho_finalize, dim3(A.nbits * 8), dim3(kThreads), 0, s, partials, ntiles, out);
  return true;
}
template bool launch_rho_tile<float>(const cplx<float>*, const cplx<float>*, int, const RhoTileArgs&, double*, double*,
                                     hipStream_t);
template bool launch_rho_tile<double>(const cplx<double>*, const cplx<double>*, int, const RhoTileArgs&, double*,
                                      double*, hipStream_t);

size_t batch_observable_partials(uint32_t count, uint32_t n) {
  uint32_t cs, ls;
  batch_obs_shape(n, &cs, &ls);
  return 2ull * ((size_t)count << cs);
}

template <class R>
void launch_batch_observable(const ObsDev* obs_dev, uint32_t count, uint32_t n, double* partials, double* out,
                             hipStream_t s) {
  uint32_t cs, ls;
  batch_obs_shape(n, &cs, &ls);
  QS_LAUNCH("batch_observable", s, batch_obs_kernel<R>, dim3(count << cs), dim3(kThreads), 0, s, obs_dev, cs, ls,
            partials);
  QS_LAUNCH("batch_observable_finalize", s, batch_obs_finalize, dim3(count), dim3(kThreads), 0, s, partials, cs,
            out);
}
template void launch_batch_observable<float>(const ObsDev*, uint32_t, uint32_t, double*, double*, hipStream_t);
template void launch_batch_observable<double>(const ObsDev*, uint32_t, uint32_t, double*, double*, hipStream_t);

void launch_fold_partials(const double* partials, uint64_t count, double* scratch, double* out, hipStream_t s) {
  uint64_t nb = (count + kThreads - 1) / kThreads;
  if (nb > (uint64_t)kRedBlocks) nb = kRedBlocks;
  if (nb < 1) nb = 1;
  const uint64_t chunk = (count + nb - 1) / nb;
  QS_LAUNCH("fold_partials", s, fold_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, partials, count, chunk,
            scratch);
  QS_LAUNCH("reduce_finalize", s, finalize_kernel<1>, dim3(1), dim3(kThreads), 0, s, scratch, (int)nb, out);
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
