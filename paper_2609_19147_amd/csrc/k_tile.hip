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
#include "rho.h"

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

// u x + v y as one multiply-add chain per component (four instructions each,
// against five for two complex products and an add).
template <class R>
__device__ __forceinline__ cplx<R> cmul2(cplx<R> u, cplx<R> x, cplx<R> v, cplx<R> y) {
  return {fma(u.re, x.re, fma(-u.im, x.im, fma(v.re, y.re, -v.im * y.im))),
          fma(u.re, x.im, fma(u.im, x.re, fma(v.re, y.im, v.im * y.re)))};
}

template <int S, class R>
__device__ __forceinline__ void op_mat(cplx<R>* a, cptr<cplx<R>> u) {
  const cplx<R> u00 = ldc(u, 0), u01 = ldc(u, 1), u10 = ldc(u, 2), u11 = ldc(u, 3);
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = cmul2(u00, x, u01, y);
    a[j | (1 << S)] = cmul2(u10, x, u11, y);
  }
}

template <int S, class R>
__device__ __forceinline__ void op_diag(cplx<R>* a, cptr<cplx<R>> u) {
  const cplx<R> d0 = ldc(u, 0), d1 = ldc(u, 1);
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

// Unscaled QFT stage on register bit S: a1' = (a0 - a1) t_k with t_k = w E[k],
// w the group twiddle (bits outside the round) and E[k] the intra-round
// factor of the register bits below S.  The inverse stage undoes it:
// a1 <- a1 conj(t_k), then the butterfly.
// kThenH: the Hadamard of bit S follows at once (no later stage of a round
// acts on bit S or is controlled by it): with u = a0 + a1 and
// v = t_k (a0 - a1), a0' = u + v and a1' = 2u - a0' (five multiply-adds and
// four adds per pair instead of twelve operations).
// kSym: E[k + 2^(S-1)] = i E[k], so the upper half of the t_k is the lower
// half times i (register moves and sign flips, no multiplies).
template <int S, class R, bool kInv, bool kThenH = false, bool kSym = false>
__device__ __forceinline__ void op_qft(cplx<R>* a, cplx<R> w, cptr<cplx<R>> E) {
  static_assert(!(kInv && kThenH), "the inverse stage has no fused Hadamard");
  constexpr int K = 1 << S;
  cplx<R> tw[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (kSym && k >= K / 2 && K >= 2)
      tw[k] = {-tw[k - K / 2].im, tw[k - K / 2].re};
    else
      tw[k] = k == 0 ? w : cmul(w, ldc(E, k));
  }
  // pairs (j, j | 2^S) with j = k + hi * 2^(S+1): the twiddle depends on k only
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const cplx<R> t = tw[k];
#pragma unroll
    for (int hi = 0; hi < (RN >> (S + 1)); ++hi) {
      const int j = k + (hi << (S + 1));
      const cplx<R> x = a[j], y = a[j | (1 << S)];
      if constexpr (kInv) {
        const cplx<R> yt = cmulc(y, t);
        a[j] = cadd(x, yt);
        a[j | (1 << S)] = csub(x, yt);
      } else if constexpr (kThenH) {
        const cplx<R> u = cadd(x, y), d = csub(x, y);
        const cplx<R> s0 = {fma(t.re, d.re, fma(-t.im, d.im, u.re)), fma(t.re, d.im, fma(t.im, d.re, u.im))};
        a[j] = s0;
        a[j | (1 << S)] = {fma(R(2), u.re, -s0.re), fma(R(2), u.im, -s0.im)};
      } else {
        a[j] = cadd(x, y);
        a[j | (1 << S)] = cmul(csub(x, y), t);
      }
    }
  }
}

// Twiddle numerator of a stage on bit p of a register whose lowest bit is
// base: the index bits in [base, p).
__device__ __forceinline__ uint32_t stage_low(uint32_t g, int p, int base) {
  return g & ((1u << p) - 1u) & ~((1u << base) - 1u);
}

// ---- straight-line round patterns -------------------------------------------
// Group twiddle of a stage with stage bit p: exp(i pi (g mod 2^p) / 2^p), or the
// square of the previous stage's (bit p + 1 of the same round) when flagged.
template <class R>
__device__ __forceinline__ cplx<R> qft_w(cptr<TileOp> op, uint32_t gglobal, cplx<R> wprev) {
  if (op->square) return cmul(wprev, wprev);
  const int p = op->sbit;
  return cispi<R>(stage_low(gglobal, p, op->base), p);
}

// The four stages of a QFT round; kThenH: each followed by its Hadamard.
template <class R, bool kThenH, bool kSym>
__device__ __forceinline__ void round_qft4(cplx<R>* a, cptr<TileOp> ops, cptr<cplx<R>> coef, uint32_t gglobal) {
  cplx<R> w = qft_w<R>(ops + 0, gglobal, cplx<R>{R(1), R(0)});
  op_qft<3, R, false, kThenH, kSym>(a, w, coef + ops[0].coef);
  w = qft_w<R>(ops + 1, gglobal, w);
  op_qft<2, R, false, kThenH, kSym>(a, w, coef + ops[1].coef);
  w = qft_w<R>(ops + 2, gglobal, w);
  op_qft<1, R, false, kThenH, kSym>(a, w, coef + ops[2].coef);
  w = qft_w<R>(ops + 3, gglobal, w);
  op_qft<0, R, false, kThenH, kSym>(a, w, coef + ops[3].coef);
}

template <class R>
__device__ __forceinline__ void round_h4(cplx<R>* a) {
  op_h<3>(a);
  op_h<2>(a);
  op_h<1>(a);
  op_h<0>(a);
}

template <class R>
__device__ __forceinline__ void round_mat4(cplx<R>* a, cptr<cplx<R>> c) {
  op_mat<0>(a, c);
  op_mat<1>(a, c + 4);
  op_mat<2>(a, c + 8);
  op_mat<3>(a, c + 12);
}

// [[x, -i y], [-i y, x]] with real (x, y) = c: 2 real multiply-adds per output component.
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
// [[x, -y], [y, x]] with real (x, y) = c.
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
// Factored rotations, the common factor applied at the store: [[1, -i t],
// [-i t, 1]] and [[1, -t], [t, 1]], one multiply-add per output component.
template <int S, class R>
__device__ __forceinline__ void op_rxf(cplx<R>* a, R t) {
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = {fma(t, y.im, x.re), fma(-t, y.re, x.im)};
    a[j | (1 << S)] = {fma(t, x.im, y.re), fma(-t, x.re, y.im)};
  }
}
template <int S, class R>
__device__ __forceinline__ void op_ryf(cplx<R>* a, R t) {
#pragma unroll
  for (int j = 0; j < RN; ++j) {
    if (j & (1 << S)) continue;
    const cplx<R> x = a[j], y = a[j | (1 << S)];
    a[j] = {fma(-t, y.re, x.re), fma(-t, y.im, x.im)};
    a[j | (1 << S)] = {fma(t, x.re, y.re), fma(t, x.im, y.im)};
  }
}

// A general single-qubit round as D2 T D1 (RT_ZYZ4 and its two reduced forms).
template <class R, bool kD1, bool kD2>
struct FZyz4 {
  cptr<cplx<R>> c;  // D1[16] if kD1, then D2[16] if kD2, then t[4] as (t, 0)
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const {
    constexpr int o2 = kD1 ? 16 : 0, ot = o2 + (kD2 ? 16 : 0);
    if constexpr (kD1) {
#pragma unroll
      for (int j = 0; j < RN; ++j) a[j] = cmul(a[j], ldc(c, j));
    }
    op_ryf<0>(a, c[ot + 0].re);
    op_ryf<1>(a, c[ot + 1].re);
    op_ryf<2>(a, c[ot + 2].re);
    op_ryf<3>(a, c[ot + 3].re);
    if constexpr (kD2) {
#pragma unroll
      for (int j = 0; j < RN; ++j) a[j] = cmul(a[j], ldc(c, o2 + j));
    }
  }
};

// ---- round patterns as functors: f(a, g) transforms the 16 registers of the
// group whose smallest index is g (index bits outside the round).
template <class R, bool kThenH4, bool kSym>
struct FQft4 {
  cptr<TileOp> ops;
  cptr<cplx<R>> coef;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t g) const {
    round_qft4<R, kThenH4, kSym>(a, ops, coef, g);
  }
};
template <class R>
struct FH4 {
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const { round_h4<R>(a); }
};
template <class R>
struct FMat4 {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const { round_mat4<R>(a, c); }
};
template <class R>
struct FRx4 {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const {
    op_rx<0>(a, ldc(c, 0));
    op_rx<1>(a, ldc(c, 1));
    op_rx<2>(a, ldc(c, 2));
    op_rx<3>(a, ldc(c, 3));
  }
};
template <class R>
struct FRx4F {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const {
    op_rxf<0>(a, c[0].re);
    op_rxf<1>(a, c[1].re);
    op_rxf<2>(a, c[2].re);
    op_rxf<3>(a, c[3].re);
  }
};
template <class R>
struct FRy4F {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const {
    op_ryf<0>(a, c[0].re);
    op_ryf<1>(a, c[1].re);
    op_ryf<2>(a, c[2].re);
    op_ryf<3>(a, c[3].re);
  }
};
template <class R>
struct FRy4 {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const {
    op_ry<0>(a, ldc(c, 0));
    op_ry<1>(a, ldc(c, 1));
    op_ry<2>(a, ldc(c, 2));
    op_ry<3>(a, ldc(c, 3));
  }
};
template <int S, class R>
struct FH1 {
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const { op_h<S>(a); }
};
template <int S, class R>
struct FDiag1 {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const { op_diag<S>(a, c); }
};
template <int S, class R>
struct FMat1 {
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t) const { op_mat<S>(a, c); }
};
// One QFT stage (stage bit p) on register bit S, optionally followed by the
// Hadamard of the same bit.  A lone stage always evaluates its twiddle.
template <int S, class R, bool kThenH, bool kInv>
struct FQft1 {
  cptr<cplx<R>> E;
  int p, base;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t g) const {
    const cplx<R> w = cispi<R>(stage_low(g, p, base), p);
    op_qft<S, R, kInv, kThenH>(a, w, E);
  }
};

// Diagonal slot d of a pass (uniform): its descriptor read with scalar loads.
__device__ __forceinline__ DiagDev diag_slot(const DiagDev* slots, int d) {
  const cptr<DiagDev> S = to_const(slots) + d;
  DiagDev D;
  D.terms = S->terms;
  D.groups = S->groups;
  D.lut = S->lut;
  D.n_groups = S->n_groups;
  D.conj = S->conj;
  D.theta = S->theta;
  D.global = S->global;
  return D;
}

template <class R>
struct RoundLoop {
  const Ctx& C;
  cptr<TileRound> R_;
  cplx<R>* T;
  uint32_t ngroups, nthr;

  template <class F>
  __device__ __forceinline__ void operator()(const F& f) const {
    const int t0 = R_->tbit[0], t1 = R_->tbit[1], t2 = R_->tbit[2], t3 = R_->tbit[3];
    uint32_t loff[RN];
#pragma unroll
    for (int j = 0; j < RN; ++j) loff[j] = R_->loff[j];
    auto place = [&](uint32_t g) {
      g = insert0(g, t0);
      g = insert0(g, t1);
      g = insert0(g, t2);
      return insert0(g, t3);
    };
    for (uint32_t g = threadIdx.x; g < ngroups; g += nthr) {
      const uint32_t gpos = place(g);
      cplx<R>* Tg = T + lds_off(gpos);
      cplx<R> a[RN];
#pragma unroll
      for (int j = 0; j < RN; ++j) a[j] = Tg[loff[j]];
      f(a, C.base | C.dep(gpos));
#pragma unroll
      for (int j = 0; j < RN; ++j) Tg[loff[j]] = a[j];
    }
  }
};

// The same loop over two tiles at once (the fused adjoint step's phi and
// lambda): one set of LDS addresses and one barrier per round for both.
template <class R>
struct RoundLoop2 {
  const Ctx& C;
  cptr<TileRound> R_;
  cplx<R>* T;
  cplx<R>* T1;
  uint32_t ngroups, nthr;

  template <class F>
  __device__ __forceinline__ void operator()(const F& f) const {
    const int t0 = R_->tbit[0], t1 = R_->tbit[1], t2 = R_->tbit[2], t3 = R_->tbit[3];
    uint32_t loff[RN];
#pragma unroll
    for (int j = 0; j < RN; ++j) loff[j] = R_->loff[j];
    for (uint32_t g = threadIdx.x; g < ngroups; g += nthr) {
      uint32_t gpos = insert0(g, t0);
      gpos = insert0(gpos, t1);
      gpos = insert0(gpos, t2);
      gpos = insert0(gpos, t3);
      cplx<R>* Ta = T + lds_off(gpos);
      cplx<R>* Tb = T1 + lds_off(gpos);
      cplx<R> a[RN], b[RN];
#pragma unroll
      for (int j = 0; j < RN; ++j) a[j] = Ta[loff[j]];
#pragma unroll
      for (int j = 0; j < RN; ++j) b[j] = Tb[loff[j]];
      const uint32_t gg = C.base | C.dep(gpos);
      f(a, gg);
      f(b, gg);
#pragma unroll
      for (int j = 0; j < RN; ++j) Ta[loff[j]] = a[j];
#pragma unroll
      for (int j = 0; j < RN; ++j) Tb[loff[j]] = b[j];
    }
  }
};
template <class R, bool kTwo>
struct LoopOf {
  using type = RoundLoop<R>;
  __device__ static type make(const Ctx& C, cptr<TileRound> R_, cplx<R>* T, cplx<R>*, uint32_t ng, uint32_t nt) {
    return type{C, R_, T, ng, nt};
  }
};
template <class R>
struct LoopOf<R, true> {
  using type = RoundLoop2<R>;
  __device__ static type make(const Ctx& C, cptr<TileRound> R_, cplx<R>* T, cplx<R>* T1, uint32_t ng, uint32_t nt) {
    return type{C, R_, T, T1, ng, nt};
  }
};

// RT_DIAG rounds: register j of the group at index g holds index g | b_j with
// b_j the subset j of the round's state bits b[0..3].
template <class R, bool kConj>
struct FDiagLut {
  DiagDev D;
  cptr<int32_t> qt;
  uint32_t b[4];
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t g) const { diag_lut_round<R, kConj>(a, g, b, D, qt); }
};
template <class R, bool kConj>
struct FDiagPair {
  DiagDev D;
  cptr<int32_t> row;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t g) const { diag_pair_round<R, kConj>(a, g, D, row); }
};
template <class R, bool kConj, bool kFactored>
struct FDiagPairRx4 {
  DiagDev D;
  cptr<int32_t> row;
  cptr<cplx<R>> c;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t g) const {
    diag_pair_round<R, kConj>(a, g, D, row);
    if constexpr (kFactored) {
      op_rxf<0>(a, c[0].re);
      op_rxf<1>(a, c[1].re);
      op_rxf<2>(a, c[2].re);
      op_rxf<3>(a, c[3].re);
    } else {
      op_rx<0>(a, ldc(c, 0));
      op_rx<1>(a, ldc(c, 1));
      op_rx<2>(a, ldc(c, 2));
      op_rx<3>(a, ldc(c, 3));
    }
  }
};
template <class R>
struct FDiagAngles {
  DiagDev D;
  const cplx<R>* qp;
  uint32_t b[4];
  __device__ __forceinline__ void operator()(cplx<R>* a, uint32_t g) const {
    diag_apply_angles<R>(a, g, b[0], b[1], b[2], b[3], D, qp);
  }
};

// kDiag: the pass carries diagonal layers.  Passes without them use an
// instantiation that has no phase-evaluation code at all, which keeps the
// butterfly rounds' register allocation and schedule tight.
// Coset `coset` of the pass's tile bits: its index bits outside the tile.
template <class R>
__device__ __forceinline__ Ctx coset_ctx(const TileKArgs<R>& A, uint32_t coset) {
  Ctx C;
  C.L = A.L;
  C.a = A.a;
  const uint32_t nlo = A.a - A.L;  // coset bits placed at [L, a)
  const uint32_t top = A.a + A.h;  // first coset bit above the high tile range
  C.base = ((coset & ((1u << nlo) - 1u)) << A.L) | (top >= 32 ? 0u : ((coset >> nlo) << top));
  return C;
}

// ---- load: pairs (pos, pos+1) are adjacent in memory (tile bit 0 = state bit 0).
// Tiles of >= 1024 amplitudes give every thread a multiple of kChunk pairs,
// so the batch of loads is issued without per-element guards.
// complex128: one 16-byte amplitude per lane and access, consecutive lanes on
// consecutive amplitudes (a pair per lane would be two 16-byte accesses at a
// 32-byte lane stride, each half-filling its requests)
__device__ __forceinline__ void tile_load_c128(const TileKArgs<double>& A, const Ctx& C, cplx<double>* T) {
  const uint32_t M = 1u << A.m, nthr = blockDim.x;
  const cplx<double>* __restrict__ psi = A.psi;
  constexpr int K = 2 * kChunk;
  for (uint32_t p0 = threadIdx.x; p0 < M; p0 += nthr * K) {
    cplx<double> v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t pos = p0 + nthr * k;
      if (pos < M) v[k] = ld_nt(psi + (C.base | C.dep(pos)));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t pos = p0 + nthr * k;
      if (pos < M) T[lds_off(pos)] = v[k];
    }
  }
}

template <class R>
__device__ __forceinline__ void tile_load(const TileKArgs<R>& A, const Ctx& C, cplx<R>* T) {
  const uint32_t M = 1u << A.m, stride = 2 * blockDim.x;
  if (A.init_amp != 0.0) {
    // the uniform initial state, made here instead of read from HBM
    const cplx2<R> v{cplx<R>{(R)A.init_amp, R(0)}, cplx<R>{(R)A.init_amp, R(0)}};
    for (uint32_t pos = 2 * threadIdx.x; pos < M; pos += stride) *reinterpret_cast<cplx2<R>*>(T + lds_off(pos)) = v;
    return;
  }
  if constexpr (sizeof(R) == 8) {
    tile_load_c128(A, C, T);
    return;
  }
  const cplx<R>* __restrict__ psi = A.psi;
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
}

// kTwo: the rounds run on T and T1 together (RoundLoop2).
template <class R, bool kDiag, bool kTwo = false>
__device__ __forceinline__ void tile_rounds(const TileKArgs<R>& A, const Ctx& C, cplx<R>* T, uint32_t nthr,
                                            cplx<R>* T1 = nullptr) {
  // threads [0, nthr) take the register groups; every thread of the workgroup
  // takes part in the barrier after each round
  const uint32_t M = 1u << A.m;
  // the pattern is uniform per round, so the dispatch sits
  // outside the per-thread group loop and every pattern runs its own loop
  // (registers loaded, transformed and stored with no value crossing a join)
  const uint32_t ngroups = M >> RB;
  const cptr<TileRound> rounds = to_const(A.rounds);
  const cptr<TileOp> ops = to_const(A.ops);
  const cptr<cplx<R>> coef = to_const(A.coef);
  for (uint32_t r = 0; r < A.n_rounds; ++r) {
    const cptr<TileRound> R_ = rounds + r;
    const auto L = LoopOf<R, kTwo>::make(C, R_, T, T1, ngroups, nthr);
    switch (R_->type) {
      case RT_DIAG:
        if constexpr (kDiag) {
          const DiagDev D = diag_slot(A.diag, R_->diag);
          const uint32_t b[4] = {C.dep(1u << R_->tbit[0]), C.dep(1u << R_->tbit[1]), C.dep(1u << R_->tbit[2]),
                                 C.dep(1u << R_->tbit[3])};
          if (R_->qcoef >= 0)
            L(FDiagAngles<R>{D, A.coef + R_->qcoef, {b[0], b[1], b[2], b[3]}});
          else if (D.conj)
            L(FDiagLut<R, true>{D, to_const(A.qtab) + R_->qoff, {b[0], b[1], b[2], b[3]}});
          else
            L(FDiagLut<R, false>{D, to_const(A.qtab) + R_->qoff, {b[0], b[1], b[2], b[3]}});
        }
        break;
      case RT_DIAG_PAIR:
        if constexpr (kDiag) {
          const DiagDev D = diag_slot(A.diag, R_->diag);
          if (D.conj)
            L(FDiagPair<R, true>{D, to_const(A.qtab) + R_->qoff});
          else
            L(FDiagPair<R, false>{D, to_const(A.qtab) + R_->qoff});
        }
        break;
      case RT_DIAG_PAIR_RX:
      case RT_DIAG_PAIR_RXF:
        if constexpr (kDiag) {
          const DiagDev D = diag_slot(A.diag, R_->diag);
          const cptr<int32_t> row = to_const(A.qtab) + R_->qoff;
          const cptr<cplx<R>> c = coef + R_->coef4;
          if (R_->type == RT_DIAG_PAIR_RXF) {
            if (D.conj)
              L(FDiagPairRx4<R, true, true>{D, row, c});
            else
              L(FDiagPairRx4<R, false, true>{D, row, c});
          } else {
            if (D.conj)
              L(FDiagPairRx4<R, true, false>{D, row, c});
            else
              L(FDiagPairRx4<R, false, false>{D, row, c});
          }
        }
        break;
      case RT_QFT4:
        L(FQft4<R, false, false>{ops + R_->op_begin, coef});
        break;
      case RT_QFT4_H4:
        L(FQft4<R, true, false>{ops + R_->op_begin, coef});
        break;
      case RT_QFT4S:
        L(FQft4<R, false, true>{ops + R_->op_begin, coef});
        break;
      case RT_QFT4S_H4:
        L(FQft4<R, true, true>{ops + R_->op_begin, coef});
        break;
      case RT_H4:
        L(FH4<R>{});
        break;
      case RT_MAT4:
        L(FMat4<R>{coef + R_->coef4});
        break;
      case RT_MAT4_RX:
        L(FRx4<R>{coef + R_->coef4});
        break;
      case RT_MAT4_RY:
        L(FRy4<R>{coef + R_->coef4});
        break;
      case RT_ZYZ4:
        L(FZyz4<R, true, true>{coef + R_->coef4});
        break;
      case RT_YZ4:
        L(FZyz4<R, false, true>{coef + R_->coef4});
        break;
      case RT_ZY4:
        L(FZyz4<R, true, false>{coef + R_->coef4});
        break;
      case RT_MAT4_RXF:
        L(FRx4F<R>{coef + R_->coef4});
        break;
      case RT_MAT4_RYF:
        L(FRy4F<R>{coef + R_->coef4});
        break;
      case RT_OP1: {
        const cptr<TileOp> op = ops + R_->op_begin;
        const cptr<cplx<R>> c = coef + op->coef;
        const int kind = op->kind == OP_H ? 0 : (op->kind == OP_DIAG ? 1 : 2);
        switch (kind * 4 + (op->rbit & 3)) {
          case 0: L(FH1<0, R>{}); break;
          case 1: L(FH1<1, R>{}); break;
          case 2: L(FH1<2, R>{}); break;
          case 3: L(FH1<3, R>{}); break;
          case 4: L(FDiag1<0, R>{c}); break;
          case 5: L(FDiag1<1, R>{c}); break;
          case 6: L(FDiag1<2, R>{c}); break;
          case 7: L(FDiag1<3, R>{c}); break;
          case 8: L(FMat1<0, R>{c}); break;
          case 9: L(FMat1<1, R>{c}); break;
          case 10: L(FMat1<2, R>{c}); break;
          default: L(FMat1<3, R>{c}); break;
        }
        break;
      }
      case RT_QH1: {
        const cptr<TileOp> op = ops + R_->op_begin;
        const cptr<cplx<R>> E = coef + op->coef;
        const int p = op->sbit, base = op->base;
        switch (op->rbit & 3) {
          case 0: L(FQft1<0, R, true, false>{E, p, base}); break;
          case 1: L(FQft1<1, R, true, false>{E, p, base}); break;
          case 2: L(FQft1<2, R, true, false>{E, p, base}); break;
          default: L(FQft1<3, R, true, false>{E, p, base}); break;
        }
        break;
      }
      default: {  // RT_QFT1
        const cptr<TileOp> op = ops + R_->op_begin;
        const cptr<cplx<R>> E = coef + op->coef;
        const int p = op->sbit, base = op->base;
        switch ((op->kind == OP_QFT_INV ? 4 : 0) + (op->rbit & 3)) {
          case 0: L(FQft1<0, R, false, false>{E, p, base}); break;
          case 1: L(FQft1<1, R, false, false>{E, p, base}); break;
          case 2: L(FQft1<2, R, false, false>{E, p, base}); break;
          case 3: L(FQft1<3, R, false, false>{E, p, base}); break;
          case 4: L(FQft1<0, R, false, true>{E, p, base}); break;
          case 5: L(FQft1<1, R, false, true>{E, p, base}); break;
          case 6: L(FQft1<2, R, false, true>{E, p, base}); break;
          default: L(FQft1<3, R, false, true>{E, p, base}); break;
        }
        break;
      }
    }
    __syncthreads();
  }

}

// Stores the tile; returns this thread's FP64 sum of |psi|^2 over what it
// stored when the pass reports its norm (0 otherwise).
template <class R>
__device__ __forceinline__ double tile_store(const TileKArgs<R>& A, const Ctx& C, const cplx<R>* T, uint32_t nthr) {
  // threads [0, nthr) store the tile
  const uint32_t M = 1u << A.m, stride = 2 * nthr;
  double nacc = 0.0;
  cplx<R>* __restrict__ psi = A.psi;
  // with the pass's butterfly normalisation
  const R sc = (R)A.scale;
  const bool do_scale = A.scale != 1.0;
  if constexpr (sizeof(R) == 8) {
    // complex128: one amplitude per lane and access (as in the load)
    constexpr int K = 2 * kChunk;
    for (uint32_t p0 = threadIdx.x; p0 < M; p0 += nthr * K) {
      cplx<R> v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t pos = p0 + nthr * k;
        if (pos < M) v[k] = T[lds_off(pos)];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t pos = p0 + nthr * k;
        if (pos < M) {
          if (do_scale) v[k] = cscale(v[k], sc);
          st_nt(psi + (C.base | C.dep(pos)), v[k]);
          if (A.norm_part != nullptr) nacc += abs2_d(v[k]);
        }
      }
    }
    return nacc;
  }
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
      if (A.norm_part != nullptr) {
#pragma unroll
        for (int k = 0; k < kChunk; ++k) nacc += abs2_d(v[k].a) + abs2_d(v[k].b);
      }
    }
  } else {
    for (uint32_t pos = 2 * threadIdx.x; pos < M; pos += stride) {
      cplx2<R> v = *reinterpret_cast<const cplx2<R>*>(T + lds_off(pos));
      if (do_scale) {
        v.a = cscale(v.a, sc);
        v.b = cscale(v.b, sc);
      }
      st_nt(reinterpret_cast<cplx2<R>*>(psi + (C.base | C.dep(pos))), v);
      if (A.norm_part != nullptr) nacc += abs2_d(v.a) + abs2_d(v.b);
    }
  }
  return nacc;
}

template <class R, bool kDiag>
__device__ __forceinline__ void tile_body(const TileKArgs<R>& A, const uint32_t coset) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  const Ctx C = coset_ctx(A, coset);
  tile_load<R>(A, C, T);
  __syncthreads();
  tile_rounds<R, kDiag>(A, C, T, blockDim.x);
  const double nacc = tile_store<R>(A, C, T, blockDim.x);
  if (A.norm_part != nullptr) {
    const double t = block_sum_fixed(nacc);
    if (threadIdx.x == 0) A.norm_part[coset] = t;
  }
}

template <class R, bool kDiag>
__global__ void __launch_bounds__(kMaxThreads) tile_kernel(TileKArgs<R> A) {
  tile_body<R, kDiag>(A, A.order ? blockIdx.x : xcd_block(blockIdx.x, gridDim.x));
}

// complex64 passes: registers capped at 128 so that four waves fit per SIMD
// (two 512-thread workgroups of 2^13-amplitude tiles, or four of 2^12, share
// a CU's LDS).
template <bool kDiag>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4)))
tile_kernel_c64(TileKArgs<float> A) {
  tile_body<float, kDiag>(A, A.order ? blockIdx.x : xcd_block(blockIdx.x, gridDim.x));
}

// ---- software-pipelined tile passes ------------------------------------------
// A tile that fills a CU's LDS (2^13 complex128 or 2^14 complex64 amplitudes)
// leaves one workgroup per CU, so a workgroup per coset would load, run its
// rounds and store strictly one after the other.  Instead one workgroup per
// CU walks the cosets w, w + G, w + 2G, ... (G workgroups) and issues the
// loads of its next coset into registers before it runs the current coset's
// rounds: HBM reads overlap the rounds and the stores.  A thread moves
// kPipeK 16-byte accesses per coset (an amplitude pair each for complex64,
// one amplitude for complex128); the first PipeAccess::pre of them are
// prefetched, the rest (complex128 only, whose rounds need the registers)
// are issued at the top of the coset's turn, ahead of the prefetched ones'
// LDS writes.
constexpr int kPipeK = 16;
template <class R>
struct PipeAccess;
template <>
struct PipeAccess<float> {
  using T = cplx2<float>;
  static constexpr uint32_t amps = 2;
  static constexpr int pre = 16;
};
template <>
struct PipeAccess<double> {
  using T = cplx<double>;
  static constexpr uint32_t amps = 1;
  static constexpr int pre = 8;
};

template <class R, int K0, int K1>
__device__ __forceinline__ void pipe_issue(const TileKArgs<R>& A, const Ctx& C, typename PipeAccess<R>::T* v) {
  using E = typename PipeAccess<R>::T;
  constexpr uint32_t apa = PipeAccess<R>::amps;
  const uint32_t step = apa * blockDim.x;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const uint32_t pos = apa * threadIdx.x + step * k;
    v[k - K0] = ld_nt(reinterpret_cast<const E*>(A.psi + (C.base | C.dep(pos))));
  }
}

template <class R, int K0, int K1>
__device__ __forceinline__ void pipe_to_lds(const typename PipeAccess<R>::T* v, cplx<R>* T) {
  using E = typename PipeAccess<R>::T;
  constexpr uint32_t apa = PipeAccess<R>::amps;
  const uint32_t step = apa * blockDim.x;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const uint32_t pos = apa * threadIdx.x + step * k;
    *reinterpret_cast<E*>(T + lds_off(pos)) = v[k - K0];
  }
}

// Requires 2^m = blockDim.x * kPipeK * PipeAccess<R>::amps (checked on the host).
template <class R>
__global__ void __launch_bounds__(kMaxThreads) tile_kernel_pipe(TileKArgs<R> A, uint32_t n_cosets) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  constexpr int P = PipeAccess<R>::pre;
  typename PipeAccess<R>::T v[P];
  const uint32_t G = gridDim.x;
  uint32_t c = A.order ? blockIdx.x : xcd_block(blockIdx.x, G);
  if (c < n_cosets) pipe_issue<R, 0, P>(A, coset_ctx(A, c), v);
  for (; c < n_cosets; c += G) {
    const Ctx C = coset_ctx(A, c);
    __syncthreads();  // the previous coset's store has finished reading the tile
    if constexpr (P < kPipeK) {
      typename PipeAccess<R>::T w[kPipeK - P];
      pipe_issue<R, P, kPipeK>(A, C, w);
      pipe_to_lds<R, 0, P>(v, T);
      pipe_to_lds<R, P, kPipeK>(w, T);
    } else {
      pipe_to_lds<R, 0, P>(v, T);
    }
    __syncthreads();
    if (c + G < n_cosets) pipe_issue<R, 0, P>(A, coset_ctx(A, c + G), v);
    tile_rounds<R, false>(A, C, T, blockDim.x);
    const double nacc = tile_store<R>(A, C, T, blockDim.x);
    if (A.norm_part != nullptr) {
      const double t = block_sum_fixed(nacc);
      if (threadIdx.x == 0) A.norm_part[c] = t;
    }
  }
}

// ---- warp-specialised persistent passes ---------------------------------------
// For complex128 tiles that fill a CU's LDS (2^13 amplitudes) and whose pass
// reports no norm: one persistent workgroup per CU of kWsConsumers threads
// that run the rounds and store each tile, and kWsProducers threads that
// hold the next coset's tile in registers (kWsK 16-byte loads each, issued
// as soon as the current tile is in LDS) and write it into LDS once the
// consumers have stored theirs.  HBM reads overlap the rounds and the
// stores; the LDS hand-over is the only serial step.  Producer and consumer
// code are separate loops (disjoint register live ranges) with the same
// sequence of workgroup barriers: per coset, one per round, one after the
// store and, when a next coset exists, one after its tile is written.
constexpr uint32_t kWsConsumers = 256, kWsProducers = 256;
constexpr int kWsK = 32;  // 16-byte accesses per producer thread and tile

template <class R>
__device__ __forceinline__ void ws_issue(const TileKArgs<R>& A, const Ctx& C, uint32_t pt,
                                         typename PipeAccess<R>::T* v) {
  using E = typename PipeAccess<R>::T;
  constexpr uint32_t apa = PipeAccess<R>::amps;
#pragma unroll
  for (int k = 0; k < kWsK; ++k) {
    const uint32_t pos = apa * (pt + kWsProducers * k);
    v[k] = ld_nt(reinterpret_cast<const E*>(A.psi + (C.base | C.dep(pos))));
  }
}

template <class R>
__device__ __forceinline__ void ws_to_lds(const typename PipeAccess<R>::T* v, uint32_t pt, cplx<R>* T) {
  using E = typename PipeAccess<R>::T;
  constexpr uint32_t apa = PipeAccess<R>::amps;
#pragma unroll
  for (int k = 0; k < kWsK; ++k) *reinterpret_cast<E*>(T + lds_off(apa * (pt + kWsProducers * k))) = v[k];
}

// Requires 2^m = kWsProducers * kWsK * PipeAccess<R>::amps and norm_part == null
// (checked on the host).
template <class R>
__global__ void __launch_bounds__(kWsConsumers + kWsProducers) tile_kernel_ws(TileKArgs<R> A, uint32_t n_cosets) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  const uint32_t G = gridDim.x;
  const uint32_t c0 = A.order ? blockIdx.x : xcd_block(blockIdx.x, G);
  if (c0 >= n_cosets) return;  // the whole workgroup leaves together
  const uint32_t R_ = A.n_rounds;
  if (threadIdx.x >= kWsConsumers) {
    const uint32_t pt = threadIdx.x - kWsConsumers;
    typename PipeAccess<R>::T v[kWsK];
    ws_issue<R>(A, coset_ctx(A, c0), pt, v);
    ws_to_lds<R>(v, pt, T);
    __syncthreads();  // first tile in LDS
    for (uint32_t c = c0; c < n_cosets; c += G) {
      const bool next = c + G < n_cosets;
      if (next) ws_issue<R>(A, coset_ctx(A, c + G), pt, v);
      for (uint32_t r = 0; r < R_; ++r) __syncthreads();  // the consumers' rounds
      __syncthreads();  // the consumers have stored the tile
      if (next) {
        ws_to_lds<R>(v, pt, T);
        __syncthreads();  // next tile in LDS
      }
    }
  } else {
    __syncthreads();  // first tile in LDS
    for (uint32_t c = c0; c < n_cosets; c += G) {
      const bool next = c + G < n_cosets;
      const Ctx C = coset_ctx(A, c);
      tile_rounds<R, false>(A, C, T, kWsConsumers);
      tile_store<R>(A, C, T, kWsConsumers);
      __syncthreads();  // tile read out of LDS
      if (next) __syncthreads();  // next tile in LDS
    }
  }
}

// ---- fused adjoint step ---------------------------------------------------------
// One workgroup per coset undoes the pass on both adjoint states: phi's and
// lambda's tiles are loaded into two LDS tiles, the pass's rounds run on each,
// the cross densities of the layer's parameter bits are summed from the two
// resulting tiles, and both tiles are stored back -- 4 S of HBM traffic per
// layer instead of 6 S for two passes and a separate re-read of both states.
template <class R, bool kDiag>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 2 : 1)))
tile_kernel_dual(TileKArgs<R> A, cplx<R>* lam, RhoTileArgs Q,
                                                                 double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[rho::kRhoMaxWaves][32];
  const uint32_t M = 1u << A.m;
  cplx<R>* T0 = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* T1 = T0 + lds_off(M);
  const uint32_t ntiles = gridDim.x;
  const uint32_t coset = A.order ? blockIdx.x : xcd_block(blockIdx.x, ntiles);
  const Ctx C = coset_ctx(A, coset);
  TileKArgs<R> B = A;
  B.psi = lam;
  tile_load<R>(A, C, T0);
  tile_load<R>(B, C, T1);
  __syncthreads();
  tile_rounds<R, kDiag>(A, C, T0, blockDim.x);
  tile_rounds<R, kDiag>(A, C, T1, blockDim.x);
  if (Q.nbits) rho::accumulate_tile<R>(T0, T1, M, Q, red, partials, coset, ntiles);
  tile_store<R>(A, C, T0, blockDim.x);
  tile_store<R>(B, C, T1, blockDim.x);
}

// The same step with persistent workgroups (as many as fit on the device,
// each walking the cosets c, c + G, c + 2G, ...) that issue the loads of
// their next coset's two tiles into registers before the current coset's
// rounds, cross densities and stores: HBM reads overlap the work of the step,
// which a workgroup per coset (two or four resident per CU, each loading,
// computing and storing in turn) leaves exposed.  complex64 with
// 2^m = blockDim.x * kDualPipeK * 2 (eight 16-byte accesses per thread and
// tile; checked on the host).
constexpr int kDualPipeK = 8;
template <class R, bool kDiag>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(2)))
tile_kernel_dual_pipe(TileKArgs<R> A, cplx<R>* lam, RhoTileArgs Q, double* __restrict__ partials,
                      uint32_t n_cosets) {
  static_assert(sizeof(R) == 4, "complex64 tiles only");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[rho::kRhoMaxWaves][32];
  const uint32_t M = 1u << A.m;
  cplx<R>* T0 = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* T1 = T0 + lds_off(M);
  TileKArgs<R> B = A;
  B.psi = lam;
  typename PipeAccess<R>::T v0[kDualPipeK], v1[kDualPipeK];
  const uint32_t G = gridDim.x;
  uint32_t c = A.order ? blockIdx.x : xcd_block(blockIdx.x, G);
  if (c < n_cosets) {
    const Ctx C = coset_ctx(A, c);
    pipe_issue<R, 0, kDualPipeK>(A, C, v0);
    pipe_issue<R, 0, kDualPipeK>(B, C, v1);
  }
  for (; c < n_cosets; c += G) {
    const Ctx C = coset_ctx(A, c);
    __syncthreads();  // the previous coset's stores have finished reading the tiles
    pipe_to_lds<R, 0, kDualPipeK>(v0, T0);
    pipe_to_lds<R, 0, kDualPipeK>(v1, T1);
    __syncthreads();
    if (c + G < n_cosets) {
      const Ctx Cn = coset_ctx(A, c + G);
      pipe_issue<R, 0, kDualPipeK>(A, Cn, v0);
      pipe_issue<R, 0, kDualPipeK>(B, Cn, v1);
    }
    if constexpr (kDiag) {
      tile_rounds<R, kDiag>(A, C, T0, blockDim.x);
      tile_rounds<R, kDiag>(A, C, T1, blockDim.x);
    } else {
      tile_rounds<R, false, true>(A, C, T0, blockDim.x, T1);
    }
    if (Q.nbits) rho::accumulate_tile<R>(T0, T1, M, Q, red, partials, c, n_cosets);
    tile_store<R>(A, C, T0, blockDim.x);
    tile_store<R>(B, C, T1, blockDim.x);
  }
}

// A batched instance's argument block, read field by field with scalar loads.
template <class R>
__device__ __forceinline__ TileKArgs<R> load_args(const TileKArgs<R>* descs, uint32_t i) {
  const cptr<TileKArgs<R>> P = to_const(descs) + i;
  TileKArgs<R> A;
  A.psi = P->psi;
  A.rounds = P->rounds;
  A.ops = P->ops;
  A.coef = P->coef;
  A.diag = P->diag;
  A.qtab = P->qtab;
  A.L = P->L;
  A.a = P->a;
  A.h = P->h;
  A.m = P->m;
  A.n_rounds = P->n_rounds;
  A.n = P->n;
  A.scale = P->scale;
  A.norm_part = nullptr;  // batched passes never report a norm
  A.init_amp = P->init_amp;
  A.order = 0;
  return A;
}

// Many instances of one tile geometry in one grid: virtual block v (the
// XCD-aware order of the workgroups) runs coset (v & (2^shift - 1)) of
// instance (v >> shift).
template <class R, bool kDiag>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
tile_kernel_batched(const TileKArgs<R>* __restrict__ descs,
                                                                    uint32_t shift) {
  const uint32_t v = xcd_block(blockIdx.x, gridDim.x);
  tile_body<R, kDiag>(load_args(descs, v >> shift), v & ((1u << shift) - 1u));
}

inline uint32_t tile_threads(uint32_t m) {
  uint32_t threads = (1u << m) >> RB;
  return threads < 64 ? 64 : (threads > (uint32_t)kMaxThreads ? (uint32_t)kMaxThreads : threads);
}

template <class R, bool kDiag>
inline uint32_t tile_threads_for(uint32_t m) {
  return tile_threads(m);
}

// Dynamic LDS limit of the tile kernels: the largest tile (2^14 complex64 or
// 2^13 complex128 amplitudes with padding, 139264 bytes) plus headroom, below
// the CU's 160 KB so that the kernels' small static LDS still fits.
constexpr int kTileDynLds = 144 * 1024;

inline size_t tile_lds(uint32_t m, size_t elem) {
  const uint32_t M = 1u << m;
  return elem * (M + ((M >> 5) << 1));
}

}  // namespace

template <class R, bool kDiag>
void launch_tile_batched_k(const TileKArgs<R>* descs_dev, uint32_t count, uint32_t n, uint32_t m, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)tile_kernel_batched<R, kDiag>, kTileDynLds, "tile_pass_batched");
    attr_set = true;
  }
  const uint32_t shift = n - m;
  QS_LAUNCH("tile_pass_batched", s, (tile_kernel_batched<R, kDiag>), dim3(count << shift), dim3(tile_threads_for<R, kDiag>(m)),
            tile_lds(m, sizeof(cplx<R>)), s, descs_dev, shift);
}

template <class R>
void launch_tile_batched(const TileKArgs<R>* descs_dev, uint32_t count, uint32_t n, uint32_t m, bool has_diag,
                         hipStream_t s) {
  if (has_diag)
    launch_tile_batched_k<R, true>(descs_dev, count, n, m, s);
  else
    launch_tile_batched_k<R, false>(descs_dev, count, n, m, s);
}

template <class R, bool kDiag>
void launch_tile_k(const TileKArgs<R>& A, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)tile_kernel<R, kDiag>, kTileDynLds, "tile_pass");
    attr_set = true;
  }
  // one thread per register group of a round, between 64 and 512 threads
  const uint32_t n_cosets = 1u << (A.n - A.m);
  QS_LAUNCH("tile_pass", s, (tile_kernel<R, kDiag>), dim3(n_cosets), dim3(tile_threads_for<R, kDiag>(A.m)),
            tile_lds(A.m, sizeof(cplx<R>)), s, A);
}

template <bool kDiag>
void launch_tile_c64(const TileKArgs<float>& A, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)tile_kernel_c64<kDiag>, kTileDynLds, "tile_pass");
    attr_set = true;
  }
  QS_LAUNCH("tile_pass", s, tile_kernel_c64<kDiag>, dim3(1u << (A.n - A.m)), dim3(tile_threads(A.m)),
            tile_lds(A.m, sizeof(cplx<float>)), s, A);
}

// Workgroups of a pipelined pass: one per compute unit (at most one coset each).
inline uint32_t pipe_grid(uint32_t n_cosets) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return n_cosets < (uint32_t)cus ? n_cosets : (uint32_t)cus;
}

template <class R>
bool pipe_eligible(const TileKArgs<R>& A) {
  // tiles that fill the LDS, without diagonal slots (whose rounds need the
  // registers the prefetch would take)
  return A.diag == nullptr && A.init_amp == 0.0 && A.m == (sizeof(R) == 8 ? 13u : 14u) &&
         (1u << A.m) == tile_threads(A.m) * kPipeK * PipeAccess<R>::amps;
}

// complex128 tiles that fill the LDS (measured: for complex64 the pipelined
// kernel is the faster one)
template <class R>
bool ws_eligible(const TileKArgs<R>& A) {
  return sizeof(R) == 8 && pipe_eligible(A) && A.norm_part == nullptr &&
         (1u << A.m) == kWsProducers * kWsK * PipeAccess<R>::amps;
}

template <class R>
void launch_tile(const TileKArgs<R>& A, hipStream_t s) {
  if (ws_eligible(A)) {
    static bool attr_set = false;
    if (!attr_set) {
      allow_dynamic_lds((const void*)tile_kernel_ws<R>, kTileDynLds, "tile_pass");
      attr_set = true;
    }
    const uint32_t n_cosets = 1u << (A.n - A.m);
    QS_LAUNCH("tile_pass", s, tile_kernel_ws<R>, dim3(pipe_grid(n_cosets)), dim3(kWsConsumers + kWsProducers),
              tile_lds(A.m, sizeof(cplx<R>)), s, A, n_cosets);
    return;
  }
  if (pipe_eligible(A)) {
    static bool attr_set = false;
    if (!attr_set) {
      allow_dynamic_lds((const void*)tile_kernel_pipe<R>, kTileDynLds, "tile_pass");
      attr_set = true;
    }
    const uint32_t n_cosets = 1u << (A.n - A.m);
    QS_LAUNCH("tile_pass", s, tile_kernel_pipe<R>, dim3(pipe_grid(n_cosets)), dim3(tile_threads(A.m)),
              tile_lds(A.m, sizeof(cplx<R>)), s, A, n_cosets);
    return;
  }
  if constexpr (sizeof(R) == 4) {
    if (A.diag != nullptr)
      launch_tile_c64<true>(A, s);
    else
      launch_tile_c64<false>(A, s);
  } else {
    if (A.diag != nullptr)
      launch_tile_k<R, true>(A, s);
    else
      launch_tile_k<R, false>(A, s);
  }
}

template <class R, bool kDiag>
void launch_tile_dual_k(const TileKArgs<R>& A, cplx<R>* lam, const RhoTileArgs& Q, double* partials, size_t lds,
                        hipStream_t s) {
  const uint32_t n_cosets = 1u << (A.n - A.m), threads = tile_threads_for<R, kDiag>(A.m);
  if constexpr (sizeof(R) == 4) {
    if ((1u << A.m) == threads * kDualPipeK * PipeAccess<R>::amps) {
      // persistent: the workgroups that fit on the device at once (a
      // property of the kernel, its block size and LDS, looked up once each)
      static bool attr_set = false;
      static int per_cu[16] = {0};
      if (!attr_set) {
        allow_dynamic_lds((const void*)tile_kernel_dual_pipe<R, kDiag>, kTileDynLds, "tile_pass_dual");
        attr_set = true;
      }
      int& nb = per_cu[A.m & 15];
      if (nb == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)tile_kernel_dual_pipe<R, kDiag>,
                                                          (int)threads, lds) != hipSuccess ||
            nb < 1)
          nb = 1;
      }
      const uint32_t grid = std::min<uint64_t>(n_cosets, (uint64_t)nb * pipe_grid(~0u));
      QS_LAUNCH("tile_pass_dual", s, (tile_kernel_dual_pipe<R, kDiag>), dim3(grid), dim3(threads), lds, s, A, lam, Q,
                partials, n_cosets);
      return;
    }
  }
  static bool attr_set = false;
  if (!attr_set) {
    allow_dynamic_lds((const void*)tile_kernel_dual<R, kDiag>, kTileDynLds, "tile_pass_dual");
    attr_set = true;
  }
  QS_LAUNCH("tile_pass_dual", s, (tile_kernel_dual<R, kDiag>), dim3(n_cosets), dim3(threads), lds, s, A, lam, Q,
            partials);
}

template <class R>
bool launch_tile_dual(const TileKArgs<R>& A, cplx<R>* lam, const RhoTileArgs& Q, double* partials, double* out,
                      hipStream_t s) {
  const size_t lds = 2 * tile_lds(A.m, sizeof(cplx<R>));
  if (lds > (size_t)kTileDynLds || Q.nbits > 32 || A.init_amp != 0.0 || A.norm_part != nullptr) return false;
  for (uint32_t k = 0; k < Q.nbits; ++k)
    if (Q.tbit[k] >= A.m) return false;
  if (A.diag != nullptr)
    launch_tile_dual_k<R, true>(A, lam, Q, partials, lds, s);
  else
    launch_tile_dual_k<R, false>(A, lam, Q, partials, lds, s);
  if (Q.nbits) launch_rho_finalize(partials, 1u << (A.n - A.m), 8 * Q.nbits, out, s);
  return true;
}

template bool launch_tile_dual<float>(const TileKArgs<float>&, cplx<float>*, const RhoTileArgs&, double*, double*,
                                      hipStream_t);
template bool launch_tile_dual<double>(const TileKArgs<double>&, cplx<double>*, const RhoTileArgs&, double*, double*,
                                       hipStream_t);
template void launch_tile<float>(const TileKArgs<float>&, hipStream_t);
template void launch_tile<double>(const TileKArgs<double>&, hipStream_t);
template void launch_tile_batched<float>(const TileKArgs<float>*, uint32_t, uint32_t, uint32_t, bool, hipStream_t);
template void launch_tile_batched<double>(const TileKArgs<double>*, uint32_t, uint32_t, uint32_t, bool, hipStream_t);

}  // namespace qs
