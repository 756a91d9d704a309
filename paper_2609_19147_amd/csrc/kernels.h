// Host-side launchers of the device kernels (one translation unit per kernel
// family).  All launchers enqueue on the given stream and throw qs::Error on a
// launch failure.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev.h"
#include "layout.h"

namespace qs {

// Profiling hooks (implemented in api.cpp): bracket a launch with HIP events
// when profiling is enabled.
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);
void check_launch(const char* name);

#define QS_LAUNCH(name, stream, ...)      \
  do {                                    \
    ::qs::prof_begin(name, stream);       \
    hipLaunchKernelGGL(__VA_ARGS__);      \
    ::qs::check_launch(name);             \
    ::qs::prof_end(stream);               \
  } while (0)

// ---- state initialisation / conversion ----
template <class R> void launch_fill_basis(cplx<R>* psi, uint64_t N, uint64_t index, hipStream_t s);
template <class R> void launch_fill_uniform(cplx<R>* psi, uint64_t N, double v, hipStream_t s);
template <class Rd, class Rs> void launch_convert(cplx<Rd>* dst, const cplx<Rs>* src, uint64_t N, hipStream_t s);
template <class R> void launch_gather(const cplx<R>* psi, const uint64_t* idx, cplx<R>* out, uint64_t count,
                                      hipStream_t s);

// ---- plain per-gate kernels (one launch per gate) ----
template <class R> void launch_mat1(cplx<R>* psi, int n, int p, const cplx<R>* u, hipStream_t s);
template <class R> void launch_cmat1(cplx<R>* psi, int n, int pc, int pt, const cplx<R>* u, hipStream_t s);
template <class R> void launch_flip(cplx<R>* psi, int n, int p, hipStream_t s);
template <class R> void launch_cflip(cplx<R>* psi, int n, int pc, int pt, hipStream_t s);
template <class R> void launch_swap(cplx<R>* psi, int n, int pa, int pb, hipStream_t s);
template <class R> void launch_phase_mask(cplx<R>* psi, int n, uint32_t mask, cplx<R> ph, hipStream_t s);
template <class R> void launch_diag1(cplx<R>* psi, int n, int p, cplx<R> d0, cplx<R> d1, hipStream_t s);
template <class R> void launch_parity_phase(cplx<R>* psi, int n, uint32_t mask, cplx<R> even, cplx<R> odd,
                                            hipStream_t s);
template <class R> void launch_mat2(cplx<R>* psi, int n, int pa, int pb, const cplx<R>* u16, hipStream_t s);
template <class R> void launch_matk(cplx<R>* psi, int n, int k, const int* bits, const cplx<R>* u_dev,
                                    hipStream_t s);

// ---- structured layers ----
template <class R>
struct TileKArgs {
  cplx<R>* psi;
  const TileRound* rounds;
  const TileOp* ops;
  const cplx<R>* coef;
  DiagDev diag[kMaxDiagSlots];
  uint32_t L, a, h, m;
  uint32_t n_rounds;
  uint32_t n;
  double scale;  // 2^(-k/2) for the pass's k unscaled butterflies
};
template <class R> void launch_tile(const TileKArgs<R>& A, hipStream_t s);

template <class R>
void launch_diag(cplx<R>* psi, int n, const DiagDev& D, hipStream_t s);

template <class R>
void launch_gf2(const cplx<R>* in, cplx<R>* out, const Gf2Args& A, hipStream_t s);

// ---- FP64 reductions (deterministic: fixed grid, fixed combination order) ----
// Each writes NV (sum, compensation) pairs per block into partials and then
// folds them into out[NV] (device) with a single-block kernel.
constexpr int kRedBlocks = 1024;
constexpr int kMaxTermsPerLaunch = 8;
template <class R> void launch_norm2(const cplx<R>* psi, uint64_t N, double* partials, double* out, hipStream_t s);
template <class Ra, class Rb>
void launch_overlap(const cplx<Ra>* a, const cplx<Rb>* b, uint64_t N, double* partials, double* out, hipStream_t s);
template <class Ra, class Rb>
void launch_distance2(const cplx<Ra>* a, const cplx<Rb>* b, uint64_t N, double ar, double ai, double bs,
                      double* partials, double* out, hipStream_t s);
// Diagonal Pauli terms: out[t] = sum_i |psi_i|^2 (-1)^{popcount(i & z[t])}, t < nt <= 8.
template <class R>
void launch_expect_z(const cplx<R>* psi, int n, const uint32_t* z, int nt, double* partials, double* out,
                     hipStream_t s);
// Off-diagonal terms sharing x: out[t] = sum_i Re(i^{ny_t} (-1)^{popcount((i^x) & z_t)} conj(psi_i) psi_{i^x}).
template <class R>
void launch_expect_x(const cplx<R>* psi, int n, uint32_t x, const uint32_t* z, const int* ny, int nt,
                     double* partials, double* out, hipStream_t s);

}  // namespace qs
