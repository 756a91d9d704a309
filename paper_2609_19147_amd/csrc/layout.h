// Plain-old-data descriptors shared by the host planner and the device kernels.
//
// Everything here is expressed in *state bit positions* (bit p of the basis
// index; qubit q sits at p = n-1-q).  Masks are 32-bit because the library
// caps n at 32 qubits.
#pragma once
#include <stdint.h>

namespace qs {

// ---- tile passes -----------------------------------------------------------
// A tile is the set of basis indices that differ only in the tile bits
// [0, L) U [a, a+h) (a == L gives the contiguous tile [0, L+h)).  Tile
// position j (0 <= j < 2^(L+h)) maps to state offset
//   (j & (2^L-1)) | ((j >> L) << a).
// One workgroup owns one coset of the tile (all other bits fixed), stages its
// 2^(L+h) amplitudes in LDS, and runs a list of rounds.  A round gathers, per
// thread, the 2^RB amplitudes that differ in RB tile bits into registers,
// optionally multiplies them by a diagonal phase, applies its operations
// (butterflies on single register bits) and writes them back.
constexpr int kRoundBits = 4;          // RB: register bits per round
constexpr int kMaxTileBits = 14;       // LDS tile <= 2^14 amplitudes
constexpr int kMaxDiagSlots = 4;       // diagonal layers fused into one pass

enum TileOpKind : int32_t {
  OP_MAT = 0,   // general 2x2: a0' = u00 a0 + u01 a1, a1' = u10 a0 + u11 a1 (coef: u00,u01,u10,u11)
  OP_H = 1,     // Hadamard butterfly, scaled by 1/sqrt(2)
  OP_QFT = 2,   // QFT stage on bit p: H butterfly, then a1' *= exp(i pi (i mod 2^p) / 2^p)
                //   coef: 2^s intra-round twiddles (s = register bit of the op)
                // H and QFT butterflies are applied unscaled (a0 + a1, a0 - a1); the
                // pass multiplies by its accumulated 2^(-k/2) once, at the store.
  OP_DIAG = 3,  // diag(d0, d1) (coef: d0, d1)
  OP_QFT_INV = 4,  // inverse of OP_QFT: a1 *= conj(twiddle), then H butterfly
  OP_GRAD = 5,     // (adjoint only) accumulate 2 Re <lambda|K|phi>, K = coef (2x2)
};

struct TileOp {
  int32_t kind;
  int32_t rbit;    // register bit (0..RB-1) the op acts on
  int32_t sbit;    // state bit position p
  int32_t coef;    // offset into the pass's coefficient array (complex entries)
  int32_t slot;    // OP_GRAD: gradient accumulator index; else -1
  int32_t square;  // OP_QFT: 1 = the group twiddle is the square of the previous op's
  int32_t base;    // OP_QFT / OP_QFT_INV: lowest state bit of the register (the
                   // twiddle reads state bits [base, sbit))
  int32_t pad;
};

// LDS layout of a tile: position j is stored at element j + 2 (j >> 5) (two
// pad elements every 32), which keeps pairs 16-byte aligned, spreads the
// strided round accesses over the banks, and is additive over disjoint bits:
// lds(g | o) = lds(g) + lds(o).
// Round patterns with straight-line code in the kernel (ops of other rounds
// run through a generic per-op loop).
enum TileRoundType : int32_t {
  RT_GENERIC = 0,  // planner-internal only: never reaches a kernel
  RT_QFT4 = 1,     // QFT stages on register bits 3, 2, 1, 0 (the ops, in that order)
  RT_QFT4_H4 = 2,  // RT_QFT4 followed by H on register bits 3, 2, 1, 0
  RT_H4 = 3,       // H on every register bit
  RT_MAT4 = 4,     // one single-qubit op per register bit (any kinds), as 2x2
                   // matrices in coef[coef4 + 4 r ...] for register bit r
                   // (identity where a bit has no op; H unscaled)
  RT_MAT4_RX = 5,  // RT_MAT4 where every matrix is [[a, -ib], [-ib, a]] (a, b real):
                   //   coef[coef4 + r] = (a, b)
  RT_MAT4_RY = 6,  // RT_MAT4 where every matrix is [[a, -b], [b, a]] (a, b real)
  RT_QFT1 = 7,     // one QFT (or inverse QFT) stage, on any register bit
  RT_QH1 = 8,      // one QFT stage followed by H on the same register bit
  RT_OP1 = 9,      // one single-qubit op (MAT, DIAG or H) on any register bit
  RT_DIAG = 10,    // device only: the round's diagonal slot, no ops (a planner round
                   // with a diagonal becomes an RT_DIAG round followed by the round)
  RT_DIAG_PAIR = 11,     // device only: RT_DIAG of a one-group layer whose count is a
                         // sum of distinct bit-pair mismatches (pair table row flags)
  RT_DIAG_PAIR_RX = 12,  // device only: RT_DIAG_PAIR, then the RT_MAT4_RX rotations
  // device only, factored rotations: every a (RX, RY) with |b| <= 8 |a|, the
  // kernel applies [[1, -i t], [-i t, 1]] (RY [[1, -t], [t, 1]]) with
  // coef[coef4 + r] = (t, 0), t = b / a, and the pass's store scale carries
  // the product of the a
  RT_MAT4_RXF = 13,
  RT_MAT4_RYF = 14,
  RT_DIAG_PAIR_RXF = 15,
  // device only: RT_QFT4 / RT_QFT4_H4 whose stages' intra-round factors
  // satisfy E[k + 2^(r-1)] = i E[k] on register bit r >= 1 (the stages of
  // consecutive qubits with no dropped angle): the kernel multiplies out the
  // lower half of each stage's twiddles only
  RT_QFT4S = 16,
  RT_QFT4S_H4 = 17,
  // device only: an RT_MAT4 round whose four matrices are unitary up to a
  // positive factor, each factored as D2 [[1, -t], [t, 1]] D1 with diagonal
  // D1, D2 and |t| <= 8: the kernel multiplies the 16 registers by the
  // product table D1[j] (16 entries), applies the four real factored
  // rotations (t_r = coef[coef4 + o + r].re, o = 16 per table present), then
  // multiplies by D2[j]; the pass scale carries the factors.  RT_YZ4 has no
  // D1 (all ones), RT_ZY4 no D2.
  RT_ZYZ4 = 18,
  RT_YZ4 = 19,
  RT_ZY4 = 20,
};
// The planner splits a round matching none of the patterns into a sequence of
// rounds over the same register bits (RT_MAT4 groups and RT_QFT1 stages).

struct TileRound {
  int32_t tbit[kRoundBits];  // tile-bit positions of register bits 0..RB-1 (ascending)
  int32_t op_begin, op_end;  // ops [op_begin, op_end) of the pass
  int32_t diag;              // -1 or a diagonal slot applied before the ops
  int32_t diag_conj;         // 1: multiply by the conjugate phase (inverse)
  int32_t type;              // TileRoundType
  int32_t coef4;             // RT_MAT4*: coefficient offset of the four matrices
  int32_t qoff;              // diag: word offset of the round's pair table in the pass's
                             // quadratic table, or -1 (evaluate every amplitude's counts)
  int32_t qcoef;             // diag, angle mode: coefficient offset of the six pair
                             // phases exp(i Q_kl); -1: lookup-table mode
  uint32_t loff[1 << kRoundBits];  // LDS element offset of register element j
};

// ---- diagonal layers ----------------------------------------------------------
// phase(i) = prod_g LUT_g[count_g(i)],  count_g(i) = sum over the group's terms.
enum DiagTermForm : int32_t {
  DT_BITS = 0,       // popcount(i & mask)
  DT_SHIFT_XOR = 1,  // popcount((i ^ (i >> shift)) & mask)  (bond p <-> p+shift mismatch)
  DT_SHIFT_AND = 2,  // popcount((i & (i >> shift)) & mask)  (both bits set)
  DT_PARITY = 3,     // parity(i & mask)                      (general Z-string)
  DT_ALL = 4,        // (i & mask) == mask                    (multi-controlled)
};

struct DiagTerm {
  int32_t form;
  int32_t shift;
  uint32_t mask;
  int32_t pad;
};

// 32-bit words per group in a diagonal round's pair table (see the round
// builder): {quadratic flag, q01, q02, q03, q12, q13, q23, pair flag,
// deg_0..deg_3, N_0..N_3}.
constexpr int kPairRowWords = 16;

struct DiagGroup {
  int32_t term_begin, term_end;  // into the layer's term array
  int32_t lut_begin;             // into the layer's LUT (count + 1 entries)
  int32_t lut_len;
};

// ---- GF(2) affine gathers -----------------------------------------------------
// out[y] = in[A y ^ cprime].  Tile subspace V (dimension d = 2c) contains
// span(e_0..e_{c-1}) and A^{-1} span(e_0..e_{c-1}); every workgroup owns one
// coset y0 + V so that both its reads and its writes are aligned runs of 2^c
// amplitudes.
constexpr int kGf2MaxC = 5;
struct Gf2Args {
  uint32_t n, c, d, n_free;
  uint32_t cprime;
  uint32_t acol[32];               // A e_j
  uint32_t free_bits[32];          // coset representative positions
  uint32_t au_hi[1 << kGf2MaxC];   // source offsets for the high source coordinates
  uint32_t t_lo[1 << kGf2MaxC];    // tile coordinate of low source coordinates
  uint32_t t_hi[1 << kGf2MaxC];    // tile coordinate of high source coordinates
  uint32_t v_hi[1 << kGf2MaxC];    // destination offsets for high tile coordinates
  uint32_t hx[1 << kGf2MaxC];      // LDS swizzle: tile coordinate t lives at t ^ hx[t >> c]
};

}  // namespace qs
