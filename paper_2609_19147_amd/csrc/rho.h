// Cross densities of a tile pair in LDS (adjoint sweep): for requested tile
// bits b, the eight sums rho_b[r][c] = sum conj(lam_r) phi_c over the tile's
// pairs along b (re and im of rho00, rho01, rho10, rho11).  Shared by the
// standalone cross-density kernel and the fused adjoint tile pass.
#pragma once
#include "kernels.h"

namespace qs {
namespace rho {


constexpr int kRhoMaxThreads = 512;
constexpr int kRhoMaxWaves = kRhoMaxThreads / 64;

__device__ __forceinline__ uint32_t rho_lds_off(uint32_t pos) { return pos + ((pos >> 5) << 1); }

inline uint32_t rho_threads(uint32_t m) {
  const uint32_t t = (1u << m) >> 4;
  return t < 64 ? 64 : (t > (uint32_t)kRhoMaxThreads ? (uint32_t)kRhoMaxThreads : t);
}

// Register bits of a chunk: 2^4 complex64 or 2^3 complex128 amplitudes of
// each state per group.
template <class R>
constexpr int rho_chunk_bits() { return sizeof(R) == 4 ? 4 : 3; }

// The sums of one chunk of up to kB requested tile bits.  Register index bit
// k holds tile bit t[k] (the kReq requested bits first, then spare tile bits
// that only enumerate amplitudes); a thread takes whole groups of 2^kB
// amplitudes of both tiles into registers and adds, per requested bit, the
// eight sums over the group's pairs along that bit.
template <class R, int kReq>
__device__ __forceinline__ void rho_chunk(const cplx<R>* P, const cplx<R>* Q, uint32_t M, const uint32_t* t,
                                          double* out32) {
  constexpr int kB = rho_chunk_bits<R>(), kN = 1 << kB;
  static_assert(kReq >= 1 && kReq <= kB, "a chunk holds at most kB requested bits");
  uint32_t ts[kB];
#pragma unroll
  for (int k = 0; k < kB; ++k) ts[k] = t[k];
  // ascending, for inserting the zero bits of a group's base position
#pragma unroll
  for (int i = 1; i < kB; ++i)
#pragma unroll
    for (int j = kB - 1; j >= i; --j)
      if (ts[j - 1] > ts[j]) {
        const uint32_t x = ts[j - 1];
        ts[j - 1] = ts[j];
        ts[j] = x;
      }
  uint32_t loff[kN];
#pragma unroll
  for (int j = 0; j < kN; ++j) {
    uint32_t o = 0;
#pragma unroll
    for (int k = 0; k < kB; ++k)
      if ((j >> k) & 1) o |= 1u << t[k];
    loff[j] = rho_lds_off(o);
  }
  R acc[kReq][8];
#pragma unroll
  for (int k = 0; k < kReq; ++k)
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[k][v] = R(0);
  for (uint32_t g = threadIdx.x; g < (M >> kB); g += blockDim.x) {
    uint32_t gpos = g;
#pragma unroll
    for (int k = 0; k < kB; ++k) gpos = insert0(gpos, ts[k]);
    const cplx<R>* Pg = P + rho_lds_off(gpos);
    const cplx<R>* Qg = Q + rho_lds_off(gpos);
    cplx<R> f[kN], l[kN];
#pragma unroll
    for (int j = 0; j < kN; ++j) {
      f[j] = Pg[loff[j]];
      l[j] = Qg[loff[j]];
    }
    if constexpr (kReq == 4 && kN == 16) {
      // diagonal sums of all four bits from the 16 products conj(l_j) f_j and
      // one tree of partial sums (p1: over bit 0, p2: bits 0-1, p3: bits 0-2):
      // the sum over j with bit k clear is p3[0] (k = 3), p2[0] + p2[2],
      // p1[0] + p1[2] + p1[4] + p1[6], and the even j (k = 0); the sum with
      // bit k set is the total minus it
      auto prod = [&](int j) {
        return cplx<R>{(R)fma(l[j].re, f[j].re, l[j].im * f[j].im), (R)fma(l[j].re, f[j].im, -l[j].im * f[j].re)};
      };
      cplx<R> p1[8], p2[4], p3[2], even = {R(0), R(0)};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const cplx<R> c0 = prod(2 * j), c1 = prod(2 * j + 1);
        even = cadd(even, c0);
        p1[j] = cadd(c0, c1);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) p2[j] = cadd(p1[2 * j], p1[2 * j + 1]);
      p3[0] = cadd(p2[0], p2[1]);
      p3[1] = cadd(p2[2], p2[3]);
      const cplx<R> tot = cadd(p3[0], p3[1]);
      const cplx<R> s0[4] = {even, cadd(cadd(p1[0], p1[2]), cadd(p1[4], p1[6])), cadd(p2[0], p2[2]), p3[0]};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc[k][0] += s0[k].re;
        acc[k][1] += s0[k].im;
        acc[k][6] += tot.re - s0[k].re;
        acc[k][7] += tot.im - s0[k].im;
      }
      // the cross terms pair by pair, two multiply-adds per sum and pair
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          if ((j >> k) & 1) continue;
          const int j1 = j | (1 << k);
          const cplx<R> f0 = f[j], f1 = f[j1], l0 = l[j], l1 = l[j1];
          acc[k][2] = fma(l0.re, f1.re, fma(l0.im, f1.im, acc[k][2]));
          acc[k][3] = fma(l0.re, f1.im, fma(-l0.im, f1.re, acc[k][3]));
          acc[k][4] = fma(l1.re, f0.re, fma(l1.im, f0.im, acc[k][4]));
          acc[k][5] = fma(l1.re, f0.im, fma(-l1.im, f0.re, acc[k][5]));
        }
    } else {
#pragma unroll
      for (int k = 0; k < kReq; ++k)
#pragma unroll
        for (int j = 0; j < kN; ++j) {
          if ((j >> k) & 1) continue;
          const int j1 = j | (1 << k);
          const cplx<R> f0 = f[j], f1 = f[j1], l0 = l[j], l1 = l[j1];
          // two multiply-adds per sum and pair
          acc[k][0] = fma(l0.re, f0.re, fma(l0.im, f0.im, acc[k][0]));
          acc[k][1] = fma(l0.re, f0.im, fma(-l0.im, f0.re, acc[k][1]));
          acc[k][2] = fma(l0.re, f1.re, fma(l0.im, f1.im, acc[k][2]));
          acc[k][3] = fma(l0.re, f1.im, fma(-l0.im, f1.re, acc[k][3]));
          acc[k][4] = fma(l1.re, f0.re, fma(l1.im, f0.im, acc[k][4]));
          acc[k][5] = fma(l1.re, f0.im, fma(-l1.im, f0.re, acc[k][5]));
          acc[k][6] = fma(l1.re, f1.re, fma(l1.im, f1.im, acc[k][6]));
          acc[k][7] = fma(l1.re, f1.im, fma(-l1.im, f1.re, acc[k][7]));
        }
    }
  }
  // sums over the wavefront by recursive halving (fixed order): each exchange
  // at lane distance d hands half of a lane's values to its partner, so the
  // exchanges of one step are independent of each other
  const uint32_t lane = threadIdx.x & 63u;
  if constexpr (sizeof(R) == 4) {
    // all 8 kReq values together (padded to 32): three steps in FP32 (sums
    // of 8 lanes), then FP64; lane pair (2v, 2v + 1) ends with value v
    float y[32];
#pragma unroll
    for (int v = 0; v < 32; ++v) y[v] = v < 8 * kReq ? acc[v >> 3][v & 7] : 0.0f;
#pragma unroll
    for (int st = 0; st < 3; ++st) {
      const int d = 32 >> st, half = 16 >> st;
      const bool up = (lane & (uint32_t)d) != 0;
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const float send = up ? y[i] : y[i + half];
        const float keep = up ? y[i + half] : y[i];
        y[i] = keep + __shfl_xor(send, d, 64);
      }
    }
    double x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = (double)y[i];
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int d = 4 >> st, half = 2 >> st;
      const bool up = (lane & (uint32_t)d) != 0;
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const double send = up ? x[i] : x[i + half];
        const double keep = up ? x[i + half] : x[i];
        x[i] = keep + __shfl_xor(send, d, 64);
      }
    }
    x[0] += __shfl_xor(x[0], 1, 64);
    if ((lane & 1u) == 0 && (lane >> 1) < 8u * kReq) out32[lane >> 1] = x[0];
  } else {
    // per bit in FP64: after three exchanges lane l holds value l >> 3 summed
    // over the lanes that differ in bits 3..5, three more add the rest
#pragma unroll
    for (int k = 0; k < kReq; ++k) {
      double x[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) x[v] = (double)acc[k][v];
#pragma unroll
      for (int st = 0; st < 3; ++st) {
        const int d = 32 >> st, half = 4 >> st;
        const bool up = (lane & (uint32_t)d) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
          const double send = up ? x[i] : x[i + half];
          const double keep = up ? x[i + half] : x[i];
          x[i] = keep + __shfl_xor(send, d, 64);
        }
      }
#pragma unroll
      for (int d = 4; d > 0; d >>= 1) x[0] += __shfl_xor(x[0], d, 64);
      if ((lane & 7u) == 0) out32[8 * k + (lane >> 3)] = x[0];
    }
  }
}

// Every requested bit's eight sums over tiles P (phi) and Q (lambda) of 2^m
// amplitudes, in chunks of rho_chunk_bits; partials value-major:
// partials[(8 bi + v) ntiles + tile].  All threads of the block take part
// (barriers inside); red holds kRhoMaxWaves x 32 doubles of shared memory.
template <class R>
__device__ __forceinline__ void accumulate_tile(const cplx<R>* P, const cplx<R>* Q, uint32_t M, const RhoTileArgs& A,
                                                double (*red)[32], double* __restrict__ partials, uint32_t tile,
                                                uint32_t ntiles) {
  const uint32_t wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  constexpr uint32_t kB = rho_chunk_bits<R>();
  for (uint32_t c0 = 0; c0 < A.nbits; c0 += kB) {
    const int req = (int)min(kB, A.nbits - c0);
    uint32_t t[4];
    for (int k = 0; k < req; ++k) t[k] = A.tbit[c0 + k];
    // spare bits: the lowest tile bits not requested in this chunk
    for (uint32_t b = 0, k = (uint32_t)req; k < kB; ++b) {
      bool used = false;
      for (int i = 0; i < req; ++i) used |= t[i] == b;
      if (!used) t[k++] = b;
    }
    switch (req) {
      case 1: rho_chunk<R, 1>(P, Q, M, t, red[wave]); break;
      case 2: rho_chunk<R, 2>(P, Q, M, t, red[wave]); break;
      case 3: rho_chunk<R, 3>(P, Q, M, t, red[wave]); break;
      default: rho_chunk<R, kB>(P, Q, M, t, red[wave]); break;
    }
    __syncthreads();
    if (threadIdx.x < 8u * (uint32_t)req) {
      double sum = 0.0;
      for (uint32_t w = 0; w < nwaves; ++w) sum += red[w][threadIdx.x];
      partials[((size_t)(8 * c0) + threadIdx.x) * ntiles + tile] = sum;
    }
    __syncthreads();
  }
}

}  // namespace rho
}  // namespace qs
