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
constexpr int kThreads = 256;
constexpr int kChunk = 8;  // 16-byte accesses in flight per thread

__device__ __forceinline__ uint32_t sw(uint32_t pos) { return pos ^ ((pos >> 4) & 15u); }

template <class R>
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

template <int S, class R>
__device__ __forceinline__ void op_h(cplx<R>* a) {
  const R r = R(0.70710678118654752440);
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = cscale(cadd(x, y), r);
    a[j | (1 << S)] = cscale(csub(x, y), r);
  }
}

template <int S, class R>
__device__ __forceinline__ void op_qft(cplx<R>* a, cplx<R> w, const cplx<R>* __restrict__ E, bool inverse) {
  const R r = R(0.70710678118654752440);
  cplx<R> tw[1 << S];
  tw[0] = w;
#pragma unroll
  for (int k = 1; k < (1 << S); ++k) tw[k] = cmul(w, E[k]);
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const int k = j & ((1 << S) - 1);
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    if (!inverse) {
      a[j] = cscale(cadd(x, y), r);
      a[j | (1 << S)] = cmul(cscale(csub(x, y), r), tw[k]);
    } else {
      const cplx<R> yt = cmulc(y, tw[k]);
      a[j] = cscale(cadd(x, yt), r);
      a[j | (1 << S)] = cscale(csub(x, yt), r);
    }
  }
}

template <class R>
__device__ __forceinline__ void apply_op(cplx<R>* a, const TileOp& op, const cplx<R>* __restrict__ coef,
                                         uint32_t gglobal) {
  const cplx<R>* c = coef + op.coef;
  switch (op.kind) {
    case OP_MAT:
      switch (op.rbit) {
        case 0: op_mat<0>(a, c); break;
        case 1: op_mat<1>(a, c); break;
        case 2: op_mat<2>(a, c); break;
        default: op_mat<3>(a, c); break;
      }
      break;
    case OP_DIAG:
      switch (op.rbit) {
        case 0: op_diag<0>(a, c); break;
        case 1: op_diag<1>(a, c); break;
        case 2: op_diag<2>(a, c); break;
        default: op_diag<3>(a, c); break;
      }
      break;
    case OP_H:
      switch (op.rbit) {
        case 0: op_h<0>(a); break;
        case 1: op_h<1>(a); break;
        case 2: op_h<2>(a); break;
        default: op_h<3>(a); break;
      }
      break;
    case OP_QFT:
    case OP_QFT_INV: {
      const int p = op.sbit;
      const uint32_t low = p == 0 ? 0u : (gglobal & ((1u << p) - 1u));
      const cplx<R> w = cispi<R>(low, p);
      const bool inv = op.kind == OP_QFT_INV;
      switch (op.rbit) {
        case 0: op_qft<0>(a, w, c, inv); break;
        case 1: op_qft<1>(a, w, c, inv); break;
        case 2: op_qft<2>(a, w, c, inv); break;
        default: op_qft<3>(a, w, c, inv); break;
      }
      break;
    }
    default:
      break;
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) tile_kernel(TileKArgs<R> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  const uint32_t M = 1u << A.m;
  const uint32_t coset = blockIdx.x;
  Ctx<R> C;
  C.L = A.L;
  C.a = A.a;
  const uint32_t nlo = A.a - A.L;  // coset bits placed at [L, a)
  const uint32_t top = A.a + A.h;  // first coset bit above the high tile range
  C.base = ((coset & ((1u << nlo) - 1u)) << A.L) | (top >= 32 ? 0u : ((coset >> nlo) << top));
  cplx<R>* __restrict__ psi = A.psi;

  // ---- load: pairs (pos, pos+1) are adjacent in memory (tile bit 0 = state bit 0)
  for (uint32_t p0 = 2 * threadIdx.x; p0 < M; p0 += 2 * kThreads * kChunk) {
    cplx2<R> v[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const uint32_t pos = p0 + 2 * kThreads * k;
      if (pos < M) v[k] = *reinterpret_cast<const cplx2<R>*>(psi + (C.base | C.dep(pos)));
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const uint32_t pos = p0 + 2 * kThreads * k;
      if (pos < M) {
        T[sw(pos)] = v[k].a;
        T[sw(pos + 1)] = v[k].b;
      }
    }
  }
  __syncthreads();

  // ---- rounds
  const uint32_t ngroups = M >> RB;
  for (uint32_t r = 0; r < A.n_rounds; ++r) {
    const TileRound R_ = A.rounds[r];
    const uint32_t b0 = 1u << R_.tbit[0], b1 = 1u << R_.tbit[1], b2 = 1u << R_.tbit[2],
                   b3 = 1u << R_.tbit[3];
    for (uint32_t g = threadIdx.x; g < ngroups; g += kThreads) {
      uint32_t gpos = g;
      gpos = insert0(gpos, R_.tbit[0]);
      gpos = insert0(gpos, R_.tbit[1]);
      gpos = insert0(gpos, R_.tbit[2]);
      gpos = insert0(gpos, R_.tbit[3]);
      cplx<R> a[RN];
#pragma unroll
      for (int j = 0; j < RN; ++j) {
        const uint32_t off = ((j & 1) ? b0 : 0u) | ((j & 2) ? b1 : 0u) | ((j & 4) ? b2 : 0u) | ((j & 8) ? b3 : 0u);
        a[j] = T[sw(gpos | off)];
      }
      if (R_.diag >= 0) {
        const DiagDev& D = A.diag[R_.diag];
#pragma unroll
        for (int j = 0; j < RN; ++j) {
          const uint32_t off = ((j & 1) ? b0 : 0u) | ((j & 2) ? b1 : 0u) | ((j & 4) ? b2 : 0u) | ((j & 8) ? b3 : 0u);
          a[j] = cmul(a[j], diag_phase<R>(C.base | C.dep(gpos | off), D));
        }
      }
      const uint32_t gglobal = C.base | C.dep(gpos);
      for (int o = R_.op_begin; o < R_.op_end; ++o) apply_op<R>(a, A.ops[o], A.coef, gglobal);
#pragma unroll
      for (int j = 0; j < RN; ++j) {
        const uint32_t off = ((j & 1) ? b0 : 0u) | ((j & 2) ? b1 : 0u) | ((j & 4) ? b2 : 0u) | ((j & 8) ? b3 : 0u);
        T[sw(gpos | off)] = a[j];
      }
    }
    __syncthreads();
  }

  // ---- store
  for (uint32_t p0 = 2 * threadIdx.x; p0 < M; p0 += 2 * kThreads * kChunk) {
    cplx2<R> v[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const uint32_t pos = p0 + 2 * kThreads * k;
      if (pos < M) {
        v[k].a = T[sw(pos)];
        v[k].b = T[sw(pos + 1)];
      }
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const uint32_t pos = p0 + 2 * kThreads * k;
      if (pos < M) *reinterpret_cast<cplx2<R>*>(psi + (C.base | C.dep(pos))) = v[k];
    }
  }
}

}  // namespace

template <class R>
void launch_tile(const TileKArgs<R>& A, hipStream_t s) {
  static bool attr_set = false;
  const size_t lds = sizeof(cplx<R>) << A.m;
  if (!attr_set) {
    hipFuncSetAttribute((const void*)tile_kernel<R>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const uint32_t n_cosets = 1u << (A.n - A.m);
  QS_LAUNCH("tile_pass", s, tile_kernel<R>, dim3(n_cosets), dim3(kThreads), lds, s, A);
}

template void launch_tile<float>(const TileKArgs<float>&, hipStream_t);
template void launch_tile<double>(const TileKArgs<double>&, hipStream_t);

}  // namespace qs
