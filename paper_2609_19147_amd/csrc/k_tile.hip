// Tile passes: multi-qubit butterflies staged through LDS.
//
// One workgroup owns one coset of the tile bits [0, L) U [a, a+h): it loads
// the coset's 2^m amplitudes (m = L + h) with 16-byte accesses -- runs of 2^L
// consecutive amplitudes, so every access is coalesced -- into LDS, runs the
// pass's rounds and stores the tile back in place.  A round moves, per
// thread, the 2^4 amplitudes that differ in the round's four tile bits into
// registers, multiplies them by a diagonal layer's phase if the round carries
// one, applies the round's single-bit operations and writes them back.
//
// Operations (paper, Section "Kernel Taxonomy"): per-wire 2x2 products of a
// single-qubit window (tensor-product layers), Hadamard butterflies (Walsh
// layers), and QFT stages -- the Hadamard butterfly of bit p followed by the
// stage's whole controlled-phase ladder as one twiddle exp(i pi low / 2^p),
// low = index mod 2^p.  The twiddle splits into a per-register-group factor
// (bits outside the round, one sincospi per group) times a host-built
// intra-round factor.
#include "kernels.h"

namespace qs {

namespace {

constexpr int RB = kRoundBits;
constexpr int RN = 1 << RB;
constexpr int kMaxThreads = 512;
constexpr int kChunk = 8;  // 16-byte accesses in flight per thread

// LDS element of tile position pos (two pad elements every 32).
__device__ __forceinline__ uint32_t lds_off(uint32_t pos) { return pos + ((pos >> 5) << 1); }

struct Ctx {
  uint32_t base;  // coset bits (tile bits zero)
  uint32_t L, a;
  __device__ __forceinline__ uint32_t dep(uint32_t pos) const {
    return (pos & ((1u << L) - 1u)) | ((pos >> L) << a);
  }
};

template <int S, class R>
__device__ __forceinline__ void op_mat(cplx<R>* a, const cplx<R>* __restrict__ u) {
  const cplx<R> u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = cadd(cmul(u00, x), cmul(u01, y));
    a[j | (1 << S)] = cadd(cmul(u10, x), cmul(u11, y));
  }
}

template <int S, class R>
__device__ __forceinline__ void op_diag(cplx<R>* a, const cplx<R>* __restrict__ u) {
  const cplx<R> d0 = u[0], d1 = u[1];
#pragma unroll
  for (int j = 0; j < RN; ++j) a[j] = cmul((j & (1 << S)) ? d1 : d0, a[j]);
}

// Unscaled Hadamard butterfly (the pass applies 2^(-k/2) at the store).
template <int S, class R>
__device__ __forceinline__ void op_h(cplx<R>* a) {
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = cadd(x, y);
    a[j | (1 << S)] = csub(x, y);
  }
}

// Unscaled QFT stage on register bit S: a1' = (a0 - a1) * w * E[k], with w the
// group twiddle (bits outside the round) and E[k] the intra-round factor of
// the register bits below S.
template <int S, class R>
__device__ __forceinline__ void op_qft(cplx<R>* a, cplx<R> w, const cplx<R>* __restrict__ E, bool inverse) {
  // pairs (j, j | 2^S) with j = k + hi * 2^(S+1): the twiddle depends on k only
#pragma unroll
  for (int k = 0; k < (1 << S); ++k) {
    const cplx<R> tw = k == 0 ? w : cmul(w, E[k]);
#pragma unroll
    for (int hi = 0; hi < (RN >> (S + 1)); ++hi) {
      const int j = k + (hi << (S + 1));
      const cplx<R> x = a[j], y = a[j | (1 << S)];
      if (!inverse) {
        a[j] = cadd(x, y);
        a[j | (1 << S)] = cmul(csub(x, y), tw);
      } else {
        const cplx<R> yt = cmulc(y, tw);
        a[j] = cadd(x, yt);
        a[j | (1 << S)] = csub(x, yt);
      }
    }
  }
}

// ---- straight-line round patterns -------------------------------------------
template <class R>
__device__ __forceinline__ cplx<R> qft_w(const TileOp& op, uint32_t gglobal, cplx<R> wprev) {
  if (op.square) return cmul(wprev, wprev);
  const int p = op.sbit;
  const uint32_t low = p == 0 ? 0u : (gglobal & ((1u << p) - 1u));
  return cispi<R>(low, p);
}

template <class R>
__device__ __forceinline__ void round_qft4(cplx<R>* a, const TileOp* __restrict__ ops, const cplx<R>* __restrict__ coef,
                                           uint32_t gglobal) {
  const TileOp o3 = ops[0], o2 = ops[1], o1 = ops[2], o0 = ops[3];
  cplx<R> w = qft_w<R>(o3, gglobal, cplx<R>{R(1), R(0)});
  op_qft<3>(a, w, coef + o3.coef, false);
  w = qft_w<R>(o2, gglobal, w);
  op_qft<2>(a, w, coef + o2.coef, false);
  w = qft_w<R>(o1, gglobal, w);
  op_qft<1>(a, w, coef + o1.coef, false);
  w = qft_w<R>(o0, gglobal, w);
  op_qft<0>(a, w, coef + o0.coef, false);
}

template <class R>
__device__ __forceinline__ void round_h4(cplx<R>* a) {
  op_h<3>(a);
  op_h<2>(a);
  op_h<1>(a);
  op_h<0>(a);
}

template <class R>
__device__ __forceinline__ void round_mat4(cplx<R>* a, const cplx<R>* __restrict__ c) {
  op_mat<0>(a, c);
  op_mat<1>(a, c + 4);
  op_mat<2>(a, c + 8);
  op_mat<3>(a, c + 12);
}

// [[x, -i y], [-i y, x]] with real (x, y) = c[S]: 2 real multiply-adds per output component.
template <int S, class R>
__device__ __forceinline__ void op_rx(cplx<R>* a, cplx<R> c) {
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = {c.re * x.re + c.im * y.im, c.re * x.im - c.im * y.re};
    a[j | (1 << S)] = {c.re * y.re + c.im * x.im, c.re * y.im - c.im * x.re};
  }
}
// [[x, -y], [y, x]] with real (x, y) = c[S].
template <int S, class R>
__device__ __forceinline__ void op_ry(cplx<R>* a, cplx<R> c) {
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = {c.re * x.re - c.im * y.re, c.re * x.im - c.im * y.im};
    a[j | (1 << S)] = {c.im * x.re + c.re * y.re, c.im * x.im + c.re * y.im};
  }
}

template <class R>
__global__ void __launch_bounds__(kMaxThreads) tile_kernel(TileKArgs<R> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  const uint32_t M = 1u << A.m;
  const uint32_t nthr = blockDim.x;
  const uint32_t coset = blockIdx.x;
  Ctx C;
  C.L = A.L;
  C.a = A.a;
  const uint32_t nlo = A.a - A.L;  // coset bits placed at [L, a)
  const uint32_t top = A.a + A.h;  // first coset bit above the high tile range
  C.base = ((coset & ((1u << nlo) - 1u)) << A.L) | (top >= 32 ? 0u : ((coset >> nlo) << top));
  cplx<R>* __restrict__ psi = A.psi;

  // ---- load: pairs (pos, pos+1) are adjacent in memory (tile bit 0 = state bit 0).
  // Tiles of >= 1024 amplitudes give every thread a multiple of kChunk pairs,
  // so the batch of loads is issued without per-element guards.
  const uint32_t stride = 2 * nthr;
  if (M >= stride * kChunk) {
    for (uint32_t p0 = 2 * threadIdx.x; p0 < M; p0 += stride * kChunk) {
      cplx2<R> v[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k)
        v[k] = ld_nt(reinterpret_cast<const cplx2<R>*>(psi + (C.base | C.dep(p0 + stride * k))));
#pragma unroll
      for (int k = 0; k < kChunk; ++k) *reinterpret_cast<cplx2<R>*>(T + lds_off(p0 + stride * k)) = v[k];
    }
  } else {
    for (uint32_t pos = 2 * threadIdx.x; pos < M; pos += stride)
      *reinterpret_cast<cplx2<R>*>(T + lds_off(pos)) = ld_nt(reinterpret_cast<const cplx2<R>*>(psi + (C.base | C.dep(pos))));
  }
  __syncthreads();

  // ---- rounds
  const uint32_t ngroups = M >> RB;
  for (uint32_t r = 0; r < A.n_rounds; ++r) {
    const TileRound& R_ = A.rounds[r];
    const int t0 = R_.tbit[0], t1 = R_.tbit[1], t2 = R_.tbit[2], t3 = R_.tbit[3];
    for (uint32_t g = threadIdx.x; g < ngroups; g += nthr) {
      uint32_t gpos = g;
      gpos = insert0(gpos, t0);
      gpos = insert0(gpos, t1);
      gpos = insert0(gpos, t2);
      gpos = insert0(gpos, t3);
      cplx<R>* Tg = T + lds_off(gpos);
      cplx<R> a[RN];
#pragma unroll
      for (int j = 0; j < RN; ++j) a[j] = Tg[R_.loff[j]];
      if (R_.diag >= 0) {
        const DiagDev& D = A.diag[R_.diag];
        const uint32_t b0 = 1u << t0, b1 = 1u << t1, b2 = 1u << t2, b3 = 1u << t3;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
          const uint32_t off = ((j & 1) ? b0 : 0u) | ((j & 2) ? b1 : 0u) | ((j & 4) ? b2 : 0u) | ((j & 8) ? b3 : 0u);
          a[j] = cmul(a[j], diag_phase<R>(C.base | C.dep(gpos | off), D));
        }
      }
      const uint32_t gglobal = C.base | C.dep(gpos);
      // every case writes its registers back itself, so nothing is live
      // across the join of the switch
      switch (R_.type) {
        case RT_QFT4:
          round_qft4<R>(a, A.ops + R_.op_begin, A.coef, gglobal);
          break;
        case RT_QFT4_H4:
          round_qft4<R>(a, A.ops + R_.op_begin, A.coef, gglobal);
          round_h4<R>(a);
          break;
        case RT_H4:
          round_h4<R>(a);
          break;
        case RT_MAT4:
          round_mat4<R>(a, A.coef + R_.coef4);
          break;
        case RT_MAT4_RX: {
          const cplx<R>* c = A.coef + R_.coef4;
          op_rx<0>(a, c[0]);
          op_rx<1>(a, c[1]);
          op_rx<2>(a, c[2]);
          op_rx<3>(a, c[3]);
          break;
        }
        case RT_MAT4_RY: {
          const cplx<R>* c = A.coef + R_.coef4;
          op_ry<0>(a, c[0]);
          op_ry<1>(a, c[1]);
          op_ry<2>(a, c[2]);
          op_ry<3>(a, c[3]);
          break;
        }
        case RT_OP1: {
          const TileOp op = A.ops[R_.op_begin];
          const cplx<R>* c = A.coef + op.coef;
          if (op.kind == OP_H) {
            switch (op.rbit) {
              case 0: op_h<0>(a); break;
              case 1: op_h<1>(a); break;
              case 2: op_h<2>(a); break;
              default: op_h<3>(a); break;
            }
          } else if (op.kind == OP_DIAG) {
            switch (op.rbit) {
              case 0: op_diag<0>(a, c); break;
              case 1: op_diag<1>(a, c); break;
              case 2: op_diag<2>(a, c); break;
              default: op_diag<3>(a, c); break;
            }
          } else {
            switch (op.rbit) {
              case 0: op_mat<0>(a, c); break;
              case 1: op_mat<1>(a, c); break;
              case 2: op_mat<2>(a, c); break;
              default: op_mat<3>(a, c); break;
            }
          }
          break;
        }
        case RT_QH1: {
          const TileOp op = A.ops[R_.op_begin];
          const int p = op.sbit;
          const cplx<R> w = cispi<R>(p == 0 ? 0u : (gglobal & ((1u << p) - 1u)), p);
          const cplx<R>* E = A.coef + op.coef;
          switch (op.rbit) {
            case 0: op_qft<0>(a, w, E, false); op_h<0>(a); break;
            case 1: op_qft<1>(a, w, E, false); op_h<1>(a); break;
            case 2: op_qft<2>(a, w, E, false); op_h<2>(a); break;
            default: op_qft<3>(a, w, E, false); op_h<3>(a); break;
          }
          break;
        }
        default: {  // RT_QFT1
          const TileOp op = A.ops[R_.op_begin];
          const int p = op.sbit;  // a lone stage always evaluates its twiddle
          const cplx<R> w = cispi<R>(p == 0 ? 0u : (gglobal & ((1u << p) - 1u)), p);
          const bool inv = op.kind == OP_QFT_INV;
          const cplx<R>* E = A.coef + op.coef;
          switch (op.rbit) {
            case 0: op_qft<0>(a, w, E, inv); break;
            case 1: op_qft<1>(a, w, E, inv); break;
            case 2: op_qft<2>(a, w, E, inv); break;
            default: op_qft<3>(a, w, E, inv); break;
          }
          break;
        }
      }
#pragma unroll
      for (int j = 0; j < RN; ++j) Tg[R_.loff[j]] = a[j];
    }
    __syncthreads();
  }

  // ---- store, with the pass's butterfly normalisation
  const R sc = (R)A.scale;
  const bool do_scale = A.scale != 1.0;
  if (M >= stride * kChunk) {
    for (uint32_t p0 = 2 * threadIdx.x; p0 < M; p0 += stride * kChunk) {
      cplx2<R> v[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) v[k] = *reinterpret_cast<const cplx2<R>*>(T + lds_off(p0 + stride * k));
      if (do_scale) {
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
          v[k].a = cscale(v[k].a, sc);
          v[k].b = cscale(v[k].b, sc);
        }
      }
#pragma unroll
      for (int k = 0; k < kChunk; ++k)
        st_nt(reinterpret_cast<cplx2<R>*>(psi + (C.base | C.dep(p0 + stride * k))), v[k]);
    }
  } else {
    for (uint32_t pos = 2 * threadIdx.x; pos < M; pos += stride) {
      cplx2<R> v = *reinterpret_cast<const cplx2<R>*>(T + lds_off(pos));
      if (do_scale) {
        v.a = cscale(v.a, sc);
        v.b = cscale(v.b, sc);
      }
      st_nt(reinterpret_cast<cplx2<R>*>(psi + (C.base | C.dep(pos))), v);
    }
  }
}

}  // namespace

template <class R>
void launch_tile(const TileKArgs<R>& A, hipStream_t s) {
  static bool attr_set = false;
  const uint32_t M = 1u << A.m;
  const size_t lds = sizeof(cplx<R>) * (M + ((M >> 5) << 1));
  if (!attr_set) {
    hipFuncSetAttribute((const void*)tile_kernel<R>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  // one thread per register group of a round, between 64 and 512 threads
  uint32_t threads = M >> RB;
  threads = threads < 64 ? 64 : (threads > (uint32_t)kMaxThreads ? (uint32_t)kMaxThreads : threads);
  const uint32_t n_cosets = 1u << (A.n - A.m);
  QS_LAUNCH("tile_pass", s, tile_kernel<R>, dim3(n_cosets), dim3(threads), lds, s, A);
}

template void launch_tile<float>(const TileKArgs<float>&, hipStream_t);
template void launch_tile<double>(const TileKArgs<double>&, hipStream_t);

}  // namespace qs
