// Dense k-qubit blocks (k = 4, 5, 6) on the matrix cores.
//
// A block applies a 2^k x 2^k complex matrix U to the k target bits of every
// basis index: for each assignment of the other bits (a column), the 2^k
// amplitudes along the targets are multiplied by U.  That is a complex matrix
// product Y = U X with X of shape 2^k x (number of columns); the paper names
// generic matrix fusion of such windows as its next extension (Section
// "Limitations and Future Work"), and it is the one layer here whose
// arithmetic intensity (8 2^k flop per amplitude, 2^(k-1) flop per byte in
// complex64) reaches the matrix cores' ridge.
//
// Tiles: the target bits plus the c lowest non-target bits (the columns).
// Every tile bit below the c-th non-target bit is in the tile, so the tile's
// low L >= c bits are the state's low bits and loads/stores move runs of
// 2^L >= 16 consecutive amplitudes; the remaining tile bits are targets, whose
// global offsets come from a small LDS table.  A workgroup (4 waves) stages a
// tile in LDS; wave w takes 16-column blocks w, w + 4, ...; each block's product
// is 4 real MFMA 16x16x4 chains per 16-row tile of U:
//   Yr += Ur Xr + Ui (-Xi),   Yi += Ur Xi + Ui Xr,
// with U's fragments held in registers for the whole kernel and X's read from
// LDS.  Results go back to the same LDS columns (each column block is read and
// written by one wave only, or, for complex64 k = 6, by one pair of waves that
// each compute half of its rows, with a barrier between their reads and
// writes), then the tile is stored.
//
// Operand layouts of V_MFMA_{F32,F64}_16X16X4 (wave64): A[i][kk] in lane
// i + 16 kk, B[kk][j] in lane j + 16 kk; D[i][j] in lane j + 16 (i / 4),
// register i % 4 for F32, and in lane j + 16 (i % 4), register i / 4 for F64
// (checked by a one-hot probe of both builtins).
#include "kernels.h"

namespace qs {

namespace {

constexpr int kDenseThreads = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class R>
struct Acc4;
template <>
struct Acc4<float> {
  typedef f32x4 T;
};
template <>
struct Acc4<double> {
  typedef f64x4 T;
};

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS element of tile position pos (two pad elements every 32).
__device__ __forceinline__ uint32_t dense_lds_off(uint32_t pos) { return pos + ((pos >> 5) << 1); }

// Tile load and store with kIO 16-byte accesses per thread issued before any
// is waited for: a loop that waits for each load before the next pays one
// memory latency per access.  A k-qubit tile (c = 6 column bits) holds
// 2^(k+6) amplitudes: two pair accesses per thread at k = 4, four at k = 5,
// eight (in two batches, the matrix fragments filling the registers) at k = 6.
template <class R, int K>
constexpr int dense_io() { return K == 16 ? 2 : 4; }

template <class R, int kIO, uint32_t NT = kDenseThreads>
__device__ __forceinline__ void dense_load(const cplx<R>* __restrict__ psi, cplx<R>* T, uint32_t M, uint32_t base,
                                           uint32_t L, const uint32_t* hi_tab) {
  const uint32_t Lmask = (1u << L) - 1u, step = 2u * NT;
  for (uint32_t p0 = 2u * threadIdx.x; p0 < M; p0 += step * kIO) {
    cplx2<R> v[kIO];
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + step * k;
      if (p < M) v[k] = ld_nt(reinterpret_cast<const cplx2<R>*>(psi + (base | (p & Lmask) | hi_tab[p >> L])));
    }
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + step * k;
      if (p < M) *reinterpret_cast<cplx2<R>*>(T + dense_lds_off(p)) = v[k];
    }
  }
}

template <class R, int kIO, uint32_t NT = kDenseThreads>
__device__ __forceinline__ void dense_store(cplx<R>* __restrict__ psi, const cplx<R>* T, uint32_t M, uint32_t base,
                                            uint32_t L, const uint32_t* hi_tab) {
  const uint32_t Lmask = (1u << L) - 1u, step = 2u * NT;
  for (uint32_t p0 = 2u * threadIdx.x; p0 < M; p0 += step * kIO) {
    cplx2<R> v[kIO];
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + step * k;
      if (p < M) v[k] = *reinterpret_cast<const cplx2<R>*>(T + dense_lds_off(p));
    }
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + step * k;
      if (p < M) st_nt(reinterpret_cast<cplx2<R>*>(psi + (base | (p & Lmask) | hi_tab[p >> L])), v[k]);
    }
  }
}

// Accesses [K0, K1) of a tile's pair accesses (p = 2 threadIdx.x + 2 NT k, NT
// threads) into registers, and from registers into the LDS tile.
template <class R, int K0, int K1, uint32_t NT = kDenseThreads>
__device__ __forceinline__ void dense_issue(const cplx<R>* __restrict__ psi, uint32_t base, uint32_t L,
                                            const uint32_t* hi_tab, cplx2<R>* v) {
  const uint32_t Lmask = (1u << L) - 1u;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const uint32_t p = 2u * threadIdx.x + 2u * NT * k;
    v[k - K0] = ld_nt(reinterpret_cast<const cplx2<R>*>(psi + (base | (p & Lmask) | hi_tab[p >> L])));
  }
}
template <class R, int K0, int K1, uint32_t NT = kDenseThreads>
__device__ __forceinline__ void dense_put(cplx<R>* T, const cplx2<R>* v) {
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const uint32_t p = 2u * threadIdx.x + 2u * NT * k;
    *reinterpret_cast<cplx2<R>*>(T + dense_lds_off(p)) = v[k - K0];
  }
}

// complex128 k = 4: one 16-byte amplitude per lane and access.
__device__ __forceinline__ void dense_load1(const cplx<double>* __restrict__ psi, cplx<double>* T, uint32_t M,
                                            uint32_t base, uint32_t L, const uint32_t* hi_tab) {
  constexpr int kIO = 8;
  const uint32_t Lmask = (1u << L) - 1u;
  for (uint32_t p0 = threadIdx.x; p0 < M; p0 += kDenseThreads * kIO) {
    cplx<double> v[kIO];
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + kDenseThreads * k;
      if (p < M) v[k] = ld_nt(psi + (base | (p & Lmask) | hi_tab[p >> L]));
    }
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + kDenseThreads * k;
      if (p < M) T[dense_lds_off(p)] = v[k];
    }
  }
}
__device__ __forceinline__ void dense_store1(cplx<double>* __restrict__ psi, const cplx<double>* T, uint32_t M,
                                             uint32_t base, uint32_t L, const uint32_t* hi_tab) {
  constexpr int kIO = 8;
  const uint32_t Lmask = (1u << L) - 1u;
  for (uint32_t p0 = threadIdx.x; p0 < M; p0 += kDenseThreads * kIO) {
    cplx<double> v[kIO];
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + kDenseThreads * k;
      if (p < M) v[k] = T[dense_lds_off(p)];
    }
#pragma unroll
    for (int k = 0; k < kIO; ++k) {
      const uint32_t p = p0 + kDenseThreads * k;
      if (p < M) st_nt(psi + (base | (p & Lmask) | hi_tab[p >> L]), v[k]);
    }
  }
}

// Deposit the low bits of v into the set bits of mask, in increasing order.
__device__ __forceinline__ uint32_t deposit(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    const uint32_t low = mask & (0u - mask);
    if (v & 1u) r |= low;
    v >>= 1;
    mask &= mask - 1u;
  }
  return r;
}

template <class R, int K>
__global__ void __launch_bounds__(kDenseThreads) __attribute__((amdgpu_waves_per_eu(3))) dense_kernel(cplx<R>* __restrict__ psi, const cplx<R>* U_,
                                                              DenseGeom G) {
  constexpr int KS = K / 4;   // 4-deep steps of the contraction
  // 16-row tiles of U per wave: complex64 k = 6 splits its four between the
  // two waves of a pair (each wave holds half of U's fragments, so three
  // waves fit per SIMD); the pair's waves take the same column blocks
  constexpr bool kSplit = sizeof(R) == 4 && K == 64;
  constexpr int RT = kSplit ? 2 : K / 16;
  typedef typename Acc4<R>::T acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t M = 1u << G.m;
  cplx<R>* T = reinterpret_cast<cplx<R>*>(smem_raw);
  uint32_t* hi_tab = reinterpret_cast<uint32_t*>(smem_raw + sizeof(cplx<R>) * dense_lds_off(M));
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t li = lane & 15u, lk = lane >> 4;
  const uint32_t rt0 = kSplit ? 2u * (wave & 1u) : 0u;                    // first row tile
  const uint32_t cb0 = kSplit ? wave >> 1 : wave, cbs = kSplit ? 2u : 4u;  // column blocks

  // global offsets of the high tile bits (all of them targets)
  for (uint32_t h = threadIdx.x; h < (1u << G.n_hi); h += kDenseThreads) {
    uint32_t off = 0;
    for (uint32_t j = 0; j < G.n_hi; ++j)
      if ((h >> j) & 1u) off |= 1u << G.hi_bit[j];
    hi_tab[h] = off;
  }

  // U fragments: A[i][kk] = U[16 (rt0 + rt) + i][4 ks + kk]
  const cptr<cplx<R>> U = to_const(U_);
  R ur[RT][KS], ui[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const uint32_t e = (16u * (rt0 + rt) + li) * K + 4u * ks + lk;
      ur[rt][ks] = U[e].re;
      ui[rt][ks] = U[e].im;
    }
  // tile positions of the rows this lane reads (B operand) and writes (D)
  const uint32_t colmask = (M - 1u) & ~G.rowmask;
  uint32_t brow[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) brow[ks] = deposit(4u * ks + lk, G.rowmask);
  uint32_t drow[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      drow[rt][v] = deposit(16u * (rt0 + rt) + (sizeof(R) == 4 ? 4u * lk + v : lk + 4u * v), G.rowmask);
  const uint32_t ncb = (1u << G.c) >> 4;
  __syncthreads();

  // complex64 k = 6 (2^12-amplitude tiles, eight pair accesses per thread):
  // the first kPre accesses of the next tile are issued before this tile's
  // contraction (the register file holds no more at three waves per SIMD),
  // the rest at the top of the tile's turn.  (Measured: prefetching k = 4 and
  // k = 5 tiles, which are HBM-bound, gains nothing or loses.)
  constexpr int kAcc = K / 8;
  constexpr int kPre = kSplit ? 4 : 0;
  constexpr bool kPipe = kPre > 0;
  const bool pipe = kPipe && M == 2u * kDenseThreads * kAcc;  // full tiles (n - k >= 6)
  auto tile_base = [&](uint32_t t) {
    uint32_t base = 0;
    for (uint32_t j = 0; j < G.n_free; ++j)
      if ((t >> j) & 1u) base |= 1u << G.free_bit[j];
    return base;
  };
  cplx2<R> pre[kPipe ? kPre : 1];
  if constexpr (kPipe) {
    if (pipe && blockIdx.x < G.n_tiles) dense_issue<R, 0, kPre>(psi, tile_base(blockIdx.x), G.L, hi_tab, pre);
  }
  for (uint32_t t = blockIdx.x; t < G.n_tiles; t += gridDim.x) {
    // coset bits of tile t (the state bits outside the tile)
    const uint32_t base = tile_base(t);
    // load: tile bit 0 is state bit 0, so pairs (p, p + 1) are adjacent
    if (kPipe && pipe) {
      if constexpr (kPre < kAcc) {
        cplx2<R> rest[kAcc > kPre ? kAcc - kPre : 1];
        dense_issue<R, kPre, kAcc>(psi, base, G.L, hi_tab, rest);
        dense_put<R, 0, kPre>(T, pre);
        dense_put<R, kPre, kAcc>(T, rest);
      } else {
        dense_put<R, 0, kPre>(T, pre);
      }
    } else if constexpr (sizeof(R) == 8 && K == 16) {
      // complex128, k = 4 (K = 16, memory-bound): one 16-byte amplitude per lane and
      // access (for k = 5 the extra address work costs more than it saves)
      dense_load1(psi, T, M, base, G.L, hi_tab);
    } else {
      dense_load<R, dense_io<R, K>()>(psi, T, M, base, G.L, hi_tab);
    }
    __syncthreads();
    if constexpr (kPipe) {
      if (pipe && t + gridDim.x < G.n_tiles)
        dense_issue<R, 0, kPre>(psi, tile_base(t + gridDim.x), G.L, hi_tab, pre);
    }

    // uniform trip count: with split row tiles the two waves of a pair read
    // all rows of a column block and each writes half of them back in place,
    // so a barrier separates every round's reads from its writes
    const uint32_t trips = (ncb + cbs - 1u) / cbs;
    for (uint32_t it = 0; it < trips; ++it) {
      const uint32_t cb = cb0 + it * cbs;
      const bool active = cb < ncb;
      const uint32_t colp = deposit(16u * (active ? cb : 0u) + li, colmask);
      acc_t yr[RT], yi[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        yr[rt] = acc_t{0, 0, 0, 0};
        yi[rt] = acc_t{0, 0, 0, 0};
      }
      if (active) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const cplx<R> x = T[dense_lds_off(brow[ks] | colp)];
          const R nxi = -x.im;
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            yr[rt] = mfma16(ur[rt][ks], x.re, yr[rt]);
            yr[rt] = mfma16(ui[rt][ks], nxi, yr[rt]);
            yi[rt] = mfma16(ur[rt][ks], x.im, yi[rt]);
            yi[rt] = mfma16(ui[rt][ks], x.re, yi[rt]);
          }
        }
      }
      if constexpr (kSplit) __syncthreads();
      if (active) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int v = 0; v < 4; ++v) T[dense_lds_off(drow[rt][v] | colp)] = cplx<R>{yr[rt][v], yi[rt][v]};
      }
    }
    __syncthreads();
    if constexpr (sizeof(R) == 8 && K == 16) {
      dense_store1(psi, T, M, base, G.L, hi_tab);
    } else {
      dense_store<R, dense_io<R, K>()>(psi, T, M, base, G.L, hi_tab);
    }
    __syncthreads();
  }
}

// complex128 k = 6: the 64 x 64 matrix (64 KB) does not fit the register
// file, so it is staged in LDS next to the tile and each wave reads its A
// fragments from there; otherwise as dense_kernel (f64 MFMA, D[i][j] in lane
// j + 16 (i % 4), register i / 4).  The staged rows are kUsStride = 65
// entries apart: the 16 rows a fragment read touches then fall in 16
// different bank groups (at 64 they would all share one).
constexpr int kUsStride = 65;
constexpr uint32_t kThreads6 = 512;
__global__ void __launch_bounds__(kThreads6) dense_kernel_k6_c128(cplx<double>* __restrict__ psi,
                                                                  const cplx<double>* U_, DenseGeom G) {
  // 512 threads, two waves per SIMD: the waves of a pair take the same
  // column block, each two of U's four 16-row tiles (as the complex64 k = 6
  // split), with a barrier between a column block's reads and its in-place
  // writes
  constexpr int K = 64, RT = 2, KS = K / 4;
  constexpr uint32_t NT = kThreads6;
  typedef f64x4 acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t M = 1u << G.m;
  cplx<double>* T = reinterpret_cast<cplx<double>*>(smem_raw);
  cplx<double>* Us = T + dense_lds_off(M);
  uint32_t* hi_tab = reinterpret_cast<uint32_t*>(Us + K * kUsStride);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t li = lane & 15u, lk = lane >> 4;
  const uint32_t rt0 = 2u * (wave & 1u), cb0 = wave >> 1, cbs = NT / 128u;
  for (uint32_t h = threadIdx.x; h < (1u << G.n_hi); h += NT) {
    uint32_t off = 0;
    for (uint32_t j = 0; j < G.n_hi; ++j)
      if ((h >> j) & 1u) off |= 1u << G.hi_bit[j];
    hi_tab[h] = off;
  }
  for (uint32_t e = threadIdx.x; e < (uint32_t)(K * K); e += NT) Us[(e / K) * kUsStride + e % K] = U_[e];
  const uint32_t colmask = (M - 1u) & ~G.rowmask;
  uint32_t brow[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) brow[ks] = deposit(4u * ks + lk, G.rowmask);
  uint32_t drow[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) drow[rt][v] = deposit(16u * (rt0 + rt) + lk + 4u * v, G.rowmask);
  const uint32_t ncb = (1u << G.c) >> 4;
  const uint32_t trips = (ncb + cbs - 1u) / cbs;
  __syncthreads();

  // the next tile's loads are issued before this tile's contraction (one
  // workgroup per CU: tile and matrix fill the LDS)
  constexpr int kAcc = 4;
  const bool pipe = M == 2u * NT * kAcc;  // full tiles (n - k >= 6)
  auto tile_base = [&](uint32_t t) {
    uint32_t base = 0;
    for (uint32_t j = 0; j < G.n_free; ++j)
      if ((t >> j) & 1u) base |= 1u << G.free_bit[j];
    return base;
  };
  cplx2<double> pre[kAcc];
  if (pipe && blockIdx.x < G.n_tiles) dense_issue<double, 0, kAcc, NT>(psi, tile_base(blockIdx.x), G.L, hi_tab, pre);
  for (uint32_t t = blockIdx.x; t < G.n_tiles; t += gridDim.x) {
    const uint32_t base = tile_base(t);
    if (pipe)
      dense_put<double, 0, kAcc, NT>(T, pre);
    else
      dense_load<double, 2, NT>(psi, T, M, base, G.L, hi_tab);
    __syncthreads();
    if (pipe && t + gridDim.x < G.n_tiles)
      dense_issue<double, 0, kAcc, NT>(psi, tile_base(t + gridDim.x), G.L, hi_tab, pre);
    for (uint32_t it = 0; it < trips; ++it) {
      const uint32_t cb = cb0 + it * cbs;
      const bool active = cb < ncb;
      const uint32_t colp = deposit(16u * (active ? cb : 0u) + li, colmask);
      acc_t yr[RT], yi[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        yr[rt] = acc_t{0, 0, 0, 0};
        yi[rt] = acc_t{0, 0, 0, 0};
      }
      if (active) {
#pragma unroll 4
        for (int ks = 0; ks < KS; ++ks) {
          const cplx<double> x = T[dense_lds_off(brow[ks] | colp)];
          const double nxi = -x.im;
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const cplx<double> u = Us[(16u * (rt0 + rt) + li) * kUsStride + 4u * ks + lk];
            yr[rt] = mfma16(u.re, x.re, yr[rt]);
            yr[rt] = mfma16(u.im, nxi, yr[rt]);
            yi[rt] = mfma16(u.re, x.im, yi[rt]);
            yi[rt] = mfma16(u.im, x.re, yi[rt]);
          }
        }
      }
      __syncthreads();  // both waves of the pair have read the column block
      if (active) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int v = 0; v < 4; ++v) T[dense_lds_off(drow[rt][v] | colp)] = cplx<double>{yr[rt][v], yi[rt][v]};
      }
    }
    __syncthreads();
    dense_store<double, 2, NT>(psi, T, M, base, G.L, hi_tab);
    __syncthreads();
  }
}

}  // namespace

bool dense_supported(int n, int k, bool complex128) {
  (void)complex128;  // complex128 k = 6 stages its matrix in LDS
  return k >= 4 && k <= 6 && n - k >= 4 && n <= 32;
}

DenseGeom dense_geometry(int n, int k, const int* bits_sorted) {
  DenseGeom G{};
  uint32_t tmask = 0;
  for (int j = 0; j < k; ++j) tmask |= 1u << bits_sorted[j];
  const int c = n - k < 6 ? n - k : 6;
  // tile bits: the targets plus the c lowest other bits
  uint32_t bmask = tmask;
  for (int b = 0, got = 0; b < n && got < c; ++b)
    if (!((tmask >> b) & 1u)) {
      bmask |= 1u << b;
      ++got;
    }
  int L = 0;
  while (L < n && ((bmask >> L) & 1u)) ++L;
  G.m = (uint32_t)(k + c);
  G.c = (uint32_t)c;
  G.L = (uint32_t)L;
  // tile position of every tile bit = its rank in bmask
  uint32_t rowmask = 0, pos = 0;
  for (int b = 0; b < n; ++b)
    if ((bmask >> b) & 1u) {
      if ((tmask >> b) & 1u) rowmask |= 1u << pos;
      if ((int)pos >= L) G.hi_bit[G.n_hi++] = (uint32_t)b;
      ++pos;
    }
  G.rowmask = rowmask;
  for (int b = 0; b < n; ++b)
    if (!((bmask >> b) & 1u)) G.free_bit[G.n_free++] = (uint32_t)b;
  G.n_tiles = 1u << G.n_free;
  return G;
}

template <class R>
bool launch_dense(cplx<R>* psi, int n, int k, const int* bits_sorted, const cplx<R>* U_dev, hipStream_t s) {
  if (!dense_supported(n, k, sizeof(R) == 8)) return false;
  const DenseGeom G = dense_geometry(n, k, bits_sorted);
  const uint32_t M = 1u << G.m;
  const size_t lds = sizeof(cplx<R>) * (M + ((M >> 5) << 1)) + 64 * sizeof(uint32_t);
  const uint32_t grid = G.n_tiles < 2048u ? G.n_tiles : 2048u;
  if (k == 4) {
    QS_LAUNCH("dense_k4", s, (dense_kernel<R, 16>), dim3(grid), dim3(kDenseThreads), lds, s, psi, U_dev, G);
  } else if (k == 5) {
    QS_LAUNCH("dense_k5", s, (dense_kernel<R, 32>), dim3(grid), dim3(kDenseThreads), lds, s, psi, U_dev, G);
  } else if constexpr (sizeof(R) == 4) {
    QS_LAUNCH("dense_k6", s, (dense_kernel<R, 64>), dim3(grid), dim3(kDenseThreads), lds, s, psi, U_dev, G);
  } else {
    // the tile, the 64 x 64 complex128 matrix (rows padded) and the offset table: ~136 KB
    const size_t lds6 = lds + sizeof(cplx<double>) * 64 * kUsStride;
    static bool attr_set = false;
    if (!attr_set) {
      allow_dynamic_lds((const void*)dense_kernel_k6_c128, (int)lds6, "dense_k6");
      attr_set = true;
    }
    QS_LAUNCH("dense_k6", s, dense_kernel_k6_c128, dim3(grid), dim3(kThreads6), lds6, s, psi, U_dev, G);
  }
  return true;
}

template bool launch_dense<float>(cplx<float>*, int, int, const int*, const cplx<float>*, hipStream_t);
template bool launch_dense<double>(cplx<double>*, int, int, const int*, const cplx<double>*, hipStream_t);

}  // namespace qs
