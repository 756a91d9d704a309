// Streaming kernels: state initialisation, dtype conversion, amplitude
// gathers, the stand-alone diagonal phase-LUT layer and the GF(2) affine
// permutation gather.
#include "kernels.h"

namespace qs {

namespace {

constexpr int kThreads = 256;
constexpr unsigned kGf2Batch = 2;  // cosets whose loads a gather workgroup issues together
constexpr int kDiagPairsPerThread = 8;
constexpr int kDiagAngleGroups = 4;  // from this many groups: total angle, one sincos per amplitude

inline unsigned grid_for(uint64_t work, int per_block) {
  uint64_t b = (work + per_block - 1) / per_block;
  const uint64_t cap = 256ull * 8 * 16;  // enough resident waves on 256 CUs
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

template <class R>
__global__ void fill_basis_kernel(cplx<R>* psi, uint64_t N, uint64_t index) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    psi[i] = {i == index ? R(1) : R(0), R(0)};
}

template <class R>
__global__ void fill_uniform_kernel(cplx<R>* psi, uint64_t N, R v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    psi[i] = {v, R(0)};
}

template <class Rd, class Rs>
__global__ void convert_kernel(cplx<Rd>* dst, const cplx<Rs>* src, uint64_t N) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = {(Rd)src[i].re, (Rd)src[i].im};
}

// Same-dtype copy: 16-byte accesses, four in flight per thread, one pass.
template <class R>
__global__ void __launch_bounds__(kThreads) copy_kernel(cplx2<R>* __restrict__ dst, const cplx2<R>* __restrict__ src,
                                                        uint64_t npairs) {
  const uint64_t step = (uint64_t)gridDim.x * kThreads;
  uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x;
  for (; i + 3 * step < npairs; i += 4 * step) {
    cplx2<R> v0 = ld_nt(src + i), v1 = ld_nt(src + i + step), v2 = ld_nt(src + i + 2 * step),
             v3 = ld_nt(src + i + 3 * step);
    st_nt(dst + i, v0);
    st_nt(dst + i + step, v1);
    st_nt(dst + i + 2 * step, v2);
    st_nt(dst + i + 3 * step, v3);
  }
  for (; i < npairs; i += step) dst[i] = src[i];
}

__global__ void __launch_bounds__(kThreads) copy1_kernel(cplx<double>* __restrict__ dst,
                                                         const cplx<double>* __restrict__ src, uint64_t n) {
  const uint64_t step = (uint64_t)gridDim.x * kThreads;
  uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x;
  for (; i + 3 * step < n; i += 4 * step) {
    const cplx<double> v0 = ld_nt(src + i), v1 = ld_nt(src + i + step), v2 = ld_nt(src + i + 2 * step),
                       v3 = ld_nt(src + i + 3 * step);
    st_nt(dst + i, v0);
    st_nt(dst + i + step, v1);
    st_nt(dst + i + 2 * step, v2);
    st_nt(dst + i + 3 * step, v3);
  }
  for (; i < n; i += step) dst[i] = src[i];
}

template <class R>
__global__ void gather_kernel(const cplx<R>* psi, const uint64_t* idx, cplx<R>* out, uint64_t count) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = psi[idx[i]];
}

// One diagonal layer in place: psi_i *= prod_g LUT_g[count_g(i)].  Two
// amplitudes per 16-byte access; the phase tables are small and stay cached.
template <class R>
__global__ void __launch_bounds__(kThreads) diag_kernel(cplx<R>* psi, uint64_t npairs, DiagDev D) {
  cplx2<R>* __restrict__ p2 = reinterpret_cast<cplx2<R>*>(psi);
  constexpr int K = kDiagPairsPerThread;
  const uint64_t nchunks = npairs / (kThreads * K);
  if constexpr (sizeof(R) == 8) {
    if (nchunks > 0) {
      // complex128: one 16-byte amplitude per lane and access; thread x owns
      // amplitudes x + j kThreads of each chunk of 2 K kThreads
      uint32_t off[2 * K];
#pragma unroll
      for (int j = 0; j < 2 * K; ++j) off[j] = (uint32_t)j * kThreads;
      for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint64_t a0 = c * (uint64_t)(2 * K * kThreads) + threadIdx.x;
        cplx<R> a[2 * K];
#pragma unroll
        for (int j = 0; j < 2 * K; ++j) a[j] = ld_nt(psi + a0 + (uint64_t)j * kThreads);
        if (D.n_groups >= kDiagAngleGroups) diag_apply_total_angle<R, 2 * K>(a, (uint32_t)a0, off, D);
        else diag_apply<R, 2 * K>(a, (uint32_t)a0, off, D);
#pragma unroll
        for (int j = 0; j < 2 * K; ++j) st_nt(psi + a0 + (uint64_t)j * kThreads, a[j]);
      }
      return;
    }
  }
  if (nchunks > 0) {
    // chunks of K * kThreads pairs: thread x owns pairs x + k kThreads, i.e.
    // amplitudes 2x | (j & 1) | (j >> 1) 2 kThreads of the chunk
    uint32_t off[2 * K];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) off[j] = (uint32_t)(j & 1) | (uint32_t)(j >> 1) * (2u * kThreads);
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
      const uint64_t t0 = c * (uint64_t)(kThreads * K) + threadIdx.x;
      cplx<R> a[2 * K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const cplx2<R> v = ld_nt(p2 + t0 + k * kThreads);
        a[2 * k] = v.a;
        a[2 * k + 1] = v.b;
      }
      if (D.n_groups >= kDiagAngleGroups) diag_apply_total_angle<R, 2 * K>(a, (uint32_t)(2 * t0), off, D);
      else diag_apply<R, 2 * K>(a, (uint32_t)(2 * t0), off, D);
#pragma unroll
      for (int k = 0; k < K; ++k) st_nt(p2 + t0 + k * kThreads, cplx2<R>{a[2 * k], a[2 * k + 1]});
    }
  } else {
    const uint32_t off[2] = {0u, 1u};
    for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < npairs; t += (uint64_t)gridDim.x * kThreads) {
      const cplx2<R> v = ld_nt(p2 + t);
      cplx<R> a[2] = {v.a, v.b};
      diag_apply<R, 2>(a, (uint32_t)(2 * t), off, D);
      st_nt(p2 + t, cplx2<R>{a[0], a[1]});
    }
  }
}

// GF(2) affine gather out[y] = in[A y ^ c'] over coset tiles of dimension d.
// Reads: x = x0 ^ s_lo ^ AU[s_hi] (aligned runs of 2^c); the element lands at
// tile coordinate t = TL[s_lo] ^ TH[s_hi].  Writes: y = y0 ^ t_lo ^ VH[t_hi]
// (aligned runs of 2^c).
// Representative y0 of coset c (its bits on the free positions) and its
// source x0 = A y0 ^ c'.
__device__ __forceinline__ void gf2_coset_rep(const Gf2Args& A, uint32_t c, uint32_t& y0, uint32_t& x0) {
  y0 = 0;
  for (uint32_t j = 0; j < A.n_free; ++j) y0 |= ((c >> j) & 1u) << A.free_bits[j];
  x0 = A.cprime;
  for (uint32_t j = 0; j < A.n; ++j)
    if ((y0 >> j) & 1u) x0 ^= A.acol[j];
}

// LDS tile of a gather: complex64 elements interleaved (one 8-byte word
// each, the swizzle keeps 2^c lanes on distinct words); complex128 elements
// as a real and an imaginary plane of 8-byte words, so the same swizzle
// applies to each plane.
template <class R>
struct GfTile {
  R* base;
  uint32_t D;
  __device__ __forceinline__ void put(uint32_t i, const cplx<R>& v) const {
    if constexpr (sizeof(R) == 4) {
      reinterpret_cast<cplx<R>*>(base)[i] = v;
    } else {
      base[i] = v.re;
      base[D + i] = v.im;
    }
  }
  __device__ __forceinline__ cplx<R> get(uint32_t i) const {
    if constexpr (sizeof(R) == 4) return reinterpret_cast<const cplx<R>*>(base)[i];
    else return cplx<R>{base[i], base[D + i]};
  }
};

template <class R, int kB>
__global__ void __launch_bounds__(kThreads) gf2_kernel(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out,
                                                       Gf2Args A, double* __restrict__ norm_part, uint32_t per) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  __shared__ uint32_t tl[1 << kGf2MaxC], th[1 << kGf2MaxC], au[1 << kGf2MaxC], vh[1 << kGf2MaxC],
      hx[1 << kGf2MaxC];
  const uint32_t nlo = 1u << A.c;
  const uint32_t nhi = 1u << (A.d - A.c);
  for (uint32_t k = threadIdx.x; k < nlo; k += kThreads) tl[k] = A.t_lo[k];
  for (uint32_t k = threadIdx.x; k < nhi; k += kThreads) {
    th[k] = A.t_hi[k];
    au[k] = A.au_hi[k];
    vh[k] = A.v_hi[k];
    hx[k] = A.hx[k];
  }
  __syncthreads();
  const uint32_t D = 1u << A.d;
  const uint32_t lomask = nlo - 1u;
  if constexpr (sizeof(R) == 8) {
    if (D == kThreads * 4) {
      // complex128 full tiles: one 16-byte element per lane and access
      // (source and destination runs are XOR-permuted aligned blocks of 2^c
      // elements, so consecutive lanes stay inside aligned blocks); kB cosets'
      // loads in flight, as below
      for (uint32_t q = 0; q < per; q += kB) {
        uint32_t y0[kB];
        cplx<R> w[kB][4];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
          uint32_t x0;
          gf2_coset_rep(A, blockIdx.x * per + q + b, y0[b], x0);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t s = threadIdx.x + kThreads * k;
            w[b][k] = ld_nt(in + (x0 ^ (s & lomask) ^ au[s >> A.c]));
          }
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
          const GfTile<R> Tb{reinterpret_cast<R*>(T + b * D), D};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t s = threadIdx.x + kThreads * k;
            const uint32_t t = tl[s & lomask] ^ th[s >> A.c];
            Tb.put(t ^ hx[t >> A.c], w[b][k]);
          }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < kB; ++b) {
          const GfTile<R> Tb{reinterpret_cast<R*>(T + b * D), D};
          cplx<R> v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t t = threadIdx.x + kThreads * k;
            v[k] = Tb.get(t ^ hx[t >> A.c]);
            st_nt(out + (y0[b] ^ (t & lomask) ^ vh[t >> A.c]), v[k]);
          }
          if (norm_part != nullptr) {
            const double tn = wave_sum_fixed(abs2_d(v[0]) + abs2_d(v[1]) + abs2_d(v[2]) + abs2_d(v[3]));
            if ((threadIdx.x & 63u) == 0) norm_part[4 * (size_t)(blockIdx.x * per + q + b) + (threadIdx.x >> 6)] = tn;
          }
        }
        __syncthreads();  // the next cosets rewrite the tiles
      }
      return;
    }
  }
  if (D == kThreads * 4) {
    // full tiles, `per` consecutive cosets per workgroup (the tables above are
    // loaded once), kB of them at a time in kB tiles of LDS: 2 kB 16-byte
    // loads in flight per thread, then 2 kB stores
    for (uint32_t q = 0; q < per; q += kB) {
      uint32_t y0[kB];
      cplx2<R> w[kB][2];
      uint32_t xa[kB][2];
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        uint32_t x0;
        gf2_coset_rep(A, blockIdx.x * per + q + b, y0[b], x0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t s = 2u * (threadIdx.x + kThreads * k);
          xa[b][k] = x0 ^ (s & lomask) ^ au[s >> A.c];
          w[b][k] = ld_nt(reinterpret_cast<const cplx2<R>*>(in + (xa[b][k] & ~1u)));
        }
      }
      // 16-byte accesses: source and destination runs are aligned blocks of
      // 2^c elements (c >= 1) XOR-permuted, so elements 2i, 2i + 1 of a run
      // share one aligned pair; `f` says whether the pair is swapped
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const GfTile<R> Tb{reinterpret_cast<R*>(T + b * D), D};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t s = 2u * (threadIdx.x + kThreads * k);
          const uint32_t slo = s & lomask, shi = s >> A.c;
          const uint32_t f = xa[b][k] & 1u;  // w.a holds source coordinate slo ^ f
          const uint32_t ta = tl[slo ^ f] ^ th[shi], tb = tl[slo ^ f ^ 1u] ^ th[shi];
          Tb.put(ta ^ hx[ta >> A.c], w[b][k].a);
          Tb.put(tb ^ hx[tb >> A.c], w[b][k].b);
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < kB; ++b) {
        const GfTile<R> Tb{reinterpret_cast<R*>(T + b * D), D};
        cplx<R> v[4];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t tt = 2u * (threadIdx.x + kThreads * k);
          const uint32_t ya = y0[b] ^ (tt & lomask) ^ vh[tt >> A.c];
          const uint32_t f = ya & 1u;  // the even destination takes tile coordinate tt ^ f
          const uint32_t te = tt ^ f, to = tt ^ f ^ 1u;
          v[2 * k] = Tb.get(te ^ hx[te >> A.c]);
          v[2 * k + 1] = Tb.get(to ^ hx[to >> A.c]);
          st_nt(reinterpret_cast<cplx2<R>*>(out + (ya & ~1u)), cplx2<R>{v[2 * k], v[2 * k + 1]});
        }
        if (norm_part != nullptr) {
          // the layer's norm, fused: each wavefront's FP64 sum of |psi|^2 over
          // what it stored (no workgroup barrier)
          const double tn = wave_sum_fixed(abs2_d(v[0]) + abs2_d(v[1]) + abs2_d(v[2]) + abs2_d(v[3]));
          if ((threadIdx.x & 63u) == 0) norm_part[4 * (size_t)(blockIdx.x * per + q + b) + (threadIdx.x >> 6)] = tn;
        }
      }
      __syncthreads();  // the next cosets rewrite the tiles
    }
    return;
  }
  // partial tiles (d < 10): one coset per workgroup
  const uint32_t coset = blockIdx.x;
  uint32_t y0, x0;
  gf2_coset_rep(A, coset, y0, x0);
  for (uint32_t s = threadIdx.x; s < D; s += kThreads) {
    const uint32_t slo = s & lomask, shi = s >> A.c;
    const uint32_t x = x0 ^ slo ^ au[shi];
    const uint32_t tk = tl[slo] ^ th[shi];
    GfTile<R>{reinterpret_cast<R*>(T), D}.put(tk ^ hx[tk >> A.c], in[x]);
  }
  __syncthreads();
  double nacc = 0.0;
  for (uint32_t t = threadIdx.x; t < D; t += kThreads) {
    const uint32_t y = y0 ^ (t & lomask) ^ vh[t >> A.c];
    const cplx<R> v = GfTile<R>{reinterpret_cast<R*>(T), D}.get(t ^ hx[t >> A.c]);
    out[y] = v;
    nacc += abs2_d(v);
  }
  if (norm_part != nullptr) {
    const double t = wave_sum_fixed(nacc);
    if ((threadIdx.x & 63u) == 0) norm_part[4 * (size_t)coset + (threadIdx.x >> 6)] = t;
  }
}

// out_i = sum over groups g of (c0_g + sum_k w_k count_k(j)) psi_j, j = i ^ x_g.
// A thread takes the amplitude pair (i, i ^ 1): for every group both sources
// j and j ^ 1 are one 16-byte load (swapped when x_g flips bit 0).
template <class R>
__device__ __forceinline__ void pauli_coef(cptr<PauliGroup> G, cptr<PauliCount> K, int g, uint32_t j, double& cr,
                                           double& ci) {
  cr = G[g].c0re;
  ci = G[g].c0im;
  const int k1 = G[g].k0 + G[g].nk;
  for (int k = G[g].k0; k < k1; ++k) {
    const int form = K[k].form;
    const uint32_t m = K[k].mask;
    int c;
    if (form == DT_SHIFT_XOR)
      c = popc((j ^ (j >> K[k].shift)) & m);
    else if (form == DT_PARITY)
      c = popc(j & m) & 1;
    else
      c = popc(j & m);
    cr = fma(K[k].wre, (double)c, cr);
    ci = fma(K[k].wim, (double)c, ci);
  }
}
template <class R>
__global__ void __launch_bounds__(kThreads) pauli_apply_kernel(const cplx<R>* __restrict__ psi,
                                                               cplx<R>* __restrict__ out, uint64_t N,
                                                               const PauliGroup* groups, int ng,
                                                               const PauliCount* counts) {
  const cptr<PauliGroup> G = to_const(groups);
  const cptr<PauliCount> K = to_const(counts);
  for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; 2 * t < N; t += (uint64_t)gridDim.x * kThreads) {
    const uint32_t i = 2u * (uint32_t)t;  // and i + 1
    double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
    for (int g = 0; g < ng; ++g) {
      const uint32_t x = G[g].x;
      const uint32_t j0 = i ^ x;  // source of i; i + 1 reads j0 ^ 1
      const cplx2<R> v = *reinterpret_cast<const cplx2<R>*>(psi + (j0 & ~1u));
      const cplx<R> s0 = (x & 1u) ? v.b : v.a, s1 = (x & 1u) ? v.a : v.b;
      double cr, ci;
      pauli_coef<R>(G, K, g, j0, cr, ci);
      a0r = fma(cr, (double)s0.re, fma(-ci, (double)s0.im, a0r));
      a0i = fma(cr, (double)s0.im, fma(ci, (double)s0.re, a0i));
      pauli_coef<R>(G, K, g, j0 ^ 1u, cr, ci);
      a1r = fma(cr, (double)s1.re, fma(-ci, (double)s1.im, a1r));
      a1i = fma(cr, (double)s1.im, fma(ci, (double)s1.re, a1i));
    }
    *reinterpret_cast<cplx2<R>*>(out + i) = cplx2<R>{{(R)a0r, (R)a0i}, {(R)a1r, (R)a1i}};
  }
}

}  // namespace

template <class R>
void launch_pauli_apply(const cplx<R>* psi, cplx<R>* out, int n, const PauliGroup* groups, int n_groups,
                        const PauliCount* counts, hipStream_t s) {
  const uint64_t N = 1ull << n;
  QS_LAUNCH("pauli_apply", s, pauli_apply_kernel<R>, dim3(grid_for(N / 2, kThreads)), dim3(kThreads), 0, s, psi, out,
            N, groups, n_groups, counts);
}
template void launch_pauli_apply<float>(const cplx<float>*, cplx<float>*, int, const PauliGroup*, int,
                                        const PauliCount*, hipStream_t);
template void launch_pauli_apply<double>(const cplx<double>*, cplx<double>*, int, const PauliGroup*, int,
                                         const PauliCount*, hipStream_t);

template <class R>
void launch_fill_basis(cplx<R>* psi, uint64_t N, uint64_t index, hipStream_t s) {
  QS_LAUNCH("fill_basis", s, fill_basis_kernel<R>, dim3(grid_for(N, kThreads * 4)), dim3(kThreads), 0, s, psi, N,
            index);
}
template <class R>
void launch_fill_uniform(cplx<R>* psi, uint64_t N, double v, hipStream_t s) {
  QS_LAUNCH("fill_uniform", s, fill_uniform_kernel<R>, dim3(grid_for(N, kThreads * 4)), dim3(kThreads), 0, s, psi,
            N, (R)v);
}
template <class Rd, class Rs>
void launch_convert(cplx<Rd>* dst, const cplx<Rs>* src, uint64_t N, hipStream_t s) {
  if (sizeof(Rd) == 8 && sizeof(Rs) == 8) {
    // complex128: one 16-byte amplitude per lane and access
    QS_LAUNCH("copy", s, copy1_kernel, dim3((unsigned)std::min<uint64_t>((N + kThreads * 4 - 1) / (kThreads * 4), 1u << 30)),
              dim3(kThreads), 0, s, reinterpret_cast<cplx<double>*>(dst), reinterpret_cast<const cplx<double>*>(src), N);
    return;
  }
  if (sizeof(Rd) == sizeof(Rs) && N >= 2) {
    const uint64_t npairs = N / 2;
    // one block per 4 kThreads pairs (no grid cap): every thread issues its
    // four loads once, which streams faster than a grid-stride loop here
    const uint64_t blocks = (npairs + kThreads * 4 - 1) / (kThreads * 4);
    QS_LAUNCH("copy", s, copy_kernel<Rd>, dim3((unsigned)(blocks < (1u << 30) ? blocks : (1u << 30))), dim3(kThreads), 0, s,
              reinterpret_cast<cplx2<Rd>*>(dst), reinterpret_cast<const cplx2<Rd>*>(src), npairs);
    return;
  }
  QS_LAUNCH("convert", s, (convert_kernel<Rd, Rs>), dim3(grid_for(N, kThreads * 4)), dim3(kThreads), 0, s, dst, src,
            N);
}
template <class R>
void launch_gather(const cplx<R>* psi, const uint64_t* idx, cplx<R>* out, uint64_t count, hipStream_t s) {
  QS_LAUNCH("gather", s, gather_kernel<R>, dim3(grid_for(count, kThreads)), dim3(kThreads), 0, s, psi, idx, out,
            count);
}
template <class R>
void launch_diag(cplx<R>* psi, int n, const DiagDev& D, hipStream_t s) {
  const uint64_t npairs = (1ull << n) / 2;
  QS_LAUNCH("diag_lut", s, diag_kernel<R>, dim3(grid_for(npairs, kThreads * kDiagPairsPerThread)), dim3(kThreads), 0,
            s, psi, npairs,
            D);
}
template <class R>
void launch_gf2(const cplx<R>* in, cplx<R>* out, const Gf2Args& A, hipStream_t s, double* norm_part) {
  const unsigned n_cosets = 1u << (A.n - A.d);
  // full tiles: four cosets per workgroup once there are plenty of them, the
  // loads of kGf2Batch of them issued together
  const bool full = (1u << A.d) == kThreads * 4u;
  const unsigned per = (full && n_cosets >= 8192u) ? 4u : 1u;
  if (per % kGf2Batch == 0) {
    QS_LAUNCH("gf2_gather", s, (gf2_kernel<R, kGf2Batch>), dim3(n_cosets / per), dim3(kThreads),
              (sizeof(cplx<R>) << A.d) * kGf2Batch, s, in, out, A, norm_part, per);
  } else {
    QS_LAUNCH("gf2_gather", s, (gf2_kernel<R, 1>), dim3(n_cosets / per), dim3(kThreads), sizeof(cplx<R>) << A.d, s, in,
              out, A, norm_part, per);
  }
}

#define INST(R)                                                                              \
  template void launch_fill_basis<R>(cplx<R>*, uint64_t, uint64_t, hipStream_t);            \
  template void launch_fill_uniform<R>(cplx<R>*, uint64_t, double, hipStream_t);            \
  template void launch_gather<R>(const cplx<R>*, const uint64_t*, cplx<R>*, uint64_t, hipStream_t); \
  template void launch_diag<R>(cplx<R>*, int, const DiagDev&, hipStream_t);                 \
  template void launch_gf2<R>(const cplx<R>*, cplx<R>*, const Gf2Args&, hipStream_t, double*);
INST(float)
INST(double)
template void launch_convert<float, double>(cplx<float>*, const cplx<double>*, uint64_t, hipStream_t);
template void launch_convert<double, float>(cplx<double>*, const cplx<float>*, uint64_t, hipStream_t);
template void launch_convert<float, float>(cplx<float>*, const cplx<float>*, uint64_t, hipStream_t);
template void launch_convert<double, double>(cplx<double>*, const cplx<double>*, uint64_t, hipStream_t);

}  // namespace qs
