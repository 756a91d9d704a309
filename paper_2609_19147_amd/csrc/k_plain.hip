// Plain per-gate kernels: one launch per gate (the per-gate path of the
// paper's pure tier, Appendix A, and the fallback for gates with no cheaper
// structure).  Single-qubit gates update amplitude pairs at stride 2^p;
// controlled gates touch only the control = 1 half (masked updates); phase
// gates touch only the amplitudes whose phase changes; X / CNOT / SWAP only
// move amplitudes.
#include "kernels.h"

namespace qs {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(uint64_t work) {
  uint64_t b = (work + kThreads - 1) / kThreads;
  const uint64_t cap = 256ull * 8 * 16;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

#define GRID_LOOP(t, count)                                                         \
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < (count); \
       t += (uint64_t)gridDim.x * blockDim.x)

template <class R>
struct U2 {
  cplx<R> u[4];
};
template <class R>
struct U4 {
  cplx<R> u[16];
};

template <class R>
__global__ void __launch_bounds__(kThreads) mat1_kernel(cplx<R>* psi, uint64_t count, uint32_t p, U2<R> U) {
  GRID_LOOP(t, count) {
    const uint64_t i0 = insert0_64(t, p), i1 = i0 | (1ull << p);
    const cplx<R> x = psi[i0], y = psi[i1];
    psi[i0] = cadd(cmul(U.u[0], x), cmul(U.u[1], y));
    psi[i1] = cadd(cmul(U.u[2], x), cmul(U.u[3], y));
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) cmat1_kernel(cplx<R>* psi, uint64_t count, uint32_t lo, uint32_t hi,
                                                         uint64_t cbit, uint64_t tbit, U2<R> U) {
  GRID_LOOP(t, count) {
    const uint64_t i0 = insert0_64(insert0_64(t, lo), hi) | cbit, i1 = i0 | tbit;
    const cplx<R> x = psi[i0], y = psi[i1];
    psi[i0] = cadd(cmul(U.u[0], x), cmul(U.u[1], y));
    psi[i1] = cadd(cmul(U.u[2], x), cmul(U.u[3], y));
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) flip_kernel(cplx<R>* psi, uint64_t count, uint32_t p) {
  GRID_LOOP(t, count) {
    const uint64_t i0 = insert0_64(t, p), i1 = i0 | (1ull << p);
    const cplx<R> x = psi[i0], y = psi[i1];
    psi[i0] = y;
    psi[i1] = x;
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) swap_kernel(cplx<R>* psi, uint64_t count, uint32_t lo, uint32_t hi,
                                                        uint64_t m0, uint64_t m1) {
  // swap the amplitude with only bit m0 set against the one with only bit m1 set
  GRID_LOOP(t, count) {
    const uint64_t b = insert0_64(insert0_64(t, lo), hi);
    const uint64_t i0 = b | m0, i1 = b | m1;
    const cplx<R> x = psi[i0], y = psi[i1];
    psi[i0] = y;
    psi[i1] = x;
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) phase_mask_kernel(cplx<R>* psi, uint64_t count, uint32_t mask,
                                                              cplx<R> ph) {
  GRID_LOOP(t, count) {
    uint64_t i = t;
    for (uint32_t m = mask; m; m &= m - 1) {
      const uint32_t b = __builtin_ctz(m);
      i = insert0_64(i, b) | (1ull << b);
    }
    psi[i] = cmul(psi[i], ph);
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) diag1_kernel(cplx<R>* psi, uint64_t count, uint32_t p, cplx<R> d0,
                                                         cplx<R> d1) {
  GRID_LOOP(t, count) {
    const uint64_t i0 = insert0_64(t, p), i1 = i0 | (1ull << p);
    psi[i0] = cmul(psi[i0], d0);
    psi[i1] = cmul(psi[i1], d1);
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) parity_kernel(cplx<R>* psi, uint64_t count, uint32_t mask, cplx<R> even,
                                                          cplx<R> odd) {
  GRID_LOOP(i, count) {
    const bool o = __builtin_popcount((uint32_t)i & mask) & 1;
    psi[i] = cmul(psi[i], o ? odd : even);
  }
}

template <class R>
__global__ void __launch_bounds__(kThreads) mat2_kernel(cplx<R>* psi, uint64_t count, uint32_t lo, uint32_t hi,
                                                        uint64_t ba, uint64_t bb, U4<R> U) {
  GRID_LOOP(t, count) {
    const uint64_t b = insert0_64(insert0_64(t, lo), hi);
    // row index r = (bit a << 1) | bit b  (first listed wire is the most significant)
    const uint64_t idx[4] = {b, b | bb, b | ba, b | ba | bb};
    cplx<R> x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = psi[idx[k]];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cplx<R> acc = cmul(U.u[4 * r], x[0]);
#pragma unroll
      for (int c = 1; c < 4; ++c) acc = cadd(acc, cmul(U.u[4 * r + c], x[c]));
      psi[idx[r]] = acc;
    }
  }
}

struct Bits6 {
  int32_t b[6];
};

template <class R>
__global__ void __launch_bounds__(64) matk_kernel(cplx<R>* psi, uint64_t count, int k, Bits6 bits, Bits6 sorted,
                                                  const cplx<R>* __restrict__ U) {
  GRID_LOOP(t, count) {
    uint64_t b = t;
    for (int j = 0; j < k; ++j) b = insert0_64(b, sorted.b[j]);
    const int d = 1 << k;
    cplx<R> x[64];
    for (int r = 0; r < d; ++r) {
      uint64_t i = b;
      for (int j = 0; j < k; ++j)
        if ((r >> (k - 1 - j)) & 1) i |= 1ull << bits.b[j];
      x[r] = psi[i];
    }
    for (int r = 0; r < d; ++r) {
      cplx<R> acc = {R(0), R(0)};
      for (int c = 0; c < d; ++c) acc = cadd(acc, cmul(U[r * d + c], x[c]));
      uint64_t i = b;
      for (int j = 0; j < k; ++j)
        if ((r >> (k - 1 - j)) & 1) i |= 1ull << bits.b[j];
      psi[i] = acc;
    }
  }
}

}  // namespace

template <class R>
void launch_mat1(cplx<R>* psi, int n, int p, const cplx<R>* u, hipStream_t s) {
  U2<R> U;
  for (int k = 0; k < 4; ++k) U.u[k] = u[k];
  const uint64_t c = 1ull << (n - 1);
  QS_LAUNCH("plain_mat1", s, mat1_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, (uint32_t)p, U);
}
template <class R>
void launch_cmat1(cplx<R>* psi, int n, int pc, int pt, const cplx<R>* u, hipStream_t s) {
  U2<R> U;
  for (int k = 0; k < 4; ++k) U.u[k] = u[k];
  const uint64_t c = 1ull << (n - 2);
  uint32_t lo = pc < pt ? pc : pt, hi = pc < pt ? pt : pc;
  QS_LAUNCH("plain_cmat1", s, cmat1_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, lo, hi, 1ull << pc,
            1ull << pt, U);
}
template <class R>
void launch_flip(cplx<R>* psi, int n, int p, hipStream_t s) {
  const uint64_t c = 1ull << (n - 1);
  QS_LAUNCH("plain_flip", s, flip_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, (uint32_t)p);
}
template <class R>
void launch_cflip(cplx<R>* psi, int n, int pc, int pt, hipStream_t s) {
  const uint64_t c = 1ull << (n - 2);
  uint32_t lo = pc < pt ? pc : pt, hi = pc < pt ? pt : pc;
  // control set, target 0 <-> control set, target 1
  QS_LAUNCH("plain_cflip", s, swap_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, lo, hi, 1ull << pc,
            (1ull << pc) | (1ull << pt));
}
template <class R>
void launch_swap(cplx<R>* psi, int n, int pa, int pb, hipStream_t s) {
  const uint64_t c = 1ull << (n - 2);
  uint32_t lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
  QS_LAUNCH("plain_swap", s, swap_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, lo, hi, 1ull << pa,
            1ull << pb);
}
template <class R>
void launch_phase_mask(cplx<R>* psi, int n, uint32_t mask, cplx<R> ph, hipStream_t s) {
  const uint64_t c = 1ull << (n - __builtin_popcount(mask));
  QS_LAUNCH("plain_phase_mask", s, phase_mask_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, mask, ph);
}
template <class R>
void launch_diag1(cplx<R>* psi, int n, int p, cplx<R> d0, cplx<R> d1, hipStream_t s) {
  const uint64_t c = 1ull << (n - 1);
  QS_LAUNCH("plain_diag1", s, diag1_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, (uint32_t)p, d0, d1);
}
template <class R>
void launch_parity_phase(cplx<R>* psi, int n, uint32_t mask, cplx<R> even, cplx<R> odd, hipStream_t s) {
  const uint64_t c = 1ull << n;
  QS_LAUNCH("plain_parity_phase", s, parity_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, mask, even,
            odd);
}
template <class R>
void launch_mat2(cplx<R>* psi, int n, int pa, int pb, const cplx<R>* u16, hipStream_t s) {
  U4<R> U;
  for (int k = 0; k < 16; ++k) U.u[k] = u16[k];
  const uint64_t c = 1ull << (n - 2);
  uint32_t lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
  QS_LAUNCH("plain_mat2", s, mat2_kernel<R>, dim3(grid_for(c)), dim3(kThreads), 0, s, psi, c, lo, hi, 1ull << pa,
            1ull << pb, U);
}
template <class R>
void launch_matk(cplx<R>* psi, int n, int k, const int* bits, const cplx<R>* u_dev, hipStream_t s) {
  Bits6 b, sorted;
  for (int j = 0; j < 6; ++j) b.b[j] = sorted.b[j] = j < k ? bits[j] : 0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j)
      if (sorted.b[j] < sorted.b[i]) { int t = sorted.b[i]; sorted.b[i] = sorted.b[j]; sorted.b[j] = t; }
  const uint64_t c = 1ull << (n - k);
  uint64_t blocks = (c + 63) / 64;
  if (blocks > 65536) blocks = 65536;
  QS_LAUNCH("plain_matk", s, matk_kernel<R>, dim3((unsigned)blocks), dim3(64), 0, s, psi, c, k, b, sorted, u_dev);
}

#define INST(R)                                                                                      \
  template void launch_mat1<R>(cplx<R>*, int, int, const cplx<R>*, hipStream_t);                   \
  template void launch_cmat1<R>(cplx<R>*, int, int, int, const cplx<R>*, hipStream_t);             \
  template void launch_flip<R>(cplx<R>*, int, int, hipStream_t);                                    \
  template void launch_cflip<R>(cplx<R>*, int, int, int, hipStream_t);                              \
  template void launch_swap<R>(cplx<R>*, int, int, int, hipStream_t);                               \
  template void launch_phase_mask<R>(cplx<R>*, int, uint32_t, cplx<R>, hipStream_t);                \
  template void launch_diag1<R>(cplx<R>*, int, int, cplx<R>, cplx<R>, hipStream_t);                 \
  template void launch_parity_phase<R>(cplx<R>*, int, uint32_t, cplx<R>, cplx<R>, hipStream_t);     \
  template void launch_mat2<R>(cplx<R>*, int, int, int, const cplx<R>*, hipStream_t);               \
  template void launch_matk<R>(cplx<R>*, int, int, const int*, const cplx<R>*, hipStream_t);
INST(float)
INST(double)

}  // namespace qs
