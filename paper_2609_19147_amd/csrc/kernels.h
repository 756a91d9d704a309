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
// Raise the dynamic LDS limit of a kernel (QS_EDEVICE on failure).
void allow_dynamic_lds(const void* kernel, int bytes, const char* name);

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
  const DiagDev* diag;  // the pass's diagonal slots (device memory), or null
  const int32_t* qtab;  // pair coefficients of the diagonal rounds (TileRound::qoff)
  uint32_t L, a, h, m;
  uint32_t n_rounds;
  uint32_t n;
  double scale;       // 2^(-k/2) for the pass's k unscaled butterflies
  double* norm_part;  // null, or one FP64 sum of |psi|^2 as stored per tile
  double init_amp;    // 0: load the tile; else the tile starts as this real
                      // amplitude everywhere (a uniform state made on load)
  uint32_t order;     // workgroup -> coset: 0 XCD-blocked (each XCD a contiguous
                      // range of cosets), 1 launch order (concurrent workgroups
                      // of all XCDs on neighbouring cosets)
};
template <class R> void launch_tile(const TileKArgs<R>& A, hipStream_t s);
// Fused adjoint step (declared here, RhoTileArgs below): the pass A undone on
// two states at once -- A.psi (phi) and lam, each staged in LDS -- followed
// by the cross densities of the requested tile bits Q.tbit[0 .. Q.nbits)
// (positions in the pass's tile) between the two resulting tiles, folded into
// out[8 Q.nbits] (device) through partials (rho_tile_partials doubles).  The
// sums are of the tiles as staged, before the pass's butterfly
// normalisation A.scale is applied on the store: true sums = scale^2 x out.
// Returns false (nothing launched) when two tiles do not fit in LDS.
struct RhoTileArgs;
template <class R>
bool launch_tile_dual(const TileKArgs<R>& A, cplx<R>* lam, const RhoTileArgs& Q, double* partials, double* out,
                      hipStream_t s);
// count instances of one geometry (n qubits, m tile bits), descriptors in device
// memory; has_diag: some descriptor has a diagonal slot.
template <class R>
void launch_tile_batched(const TileKArgs<R>* descs_dev, uint32_t count, uint32_t n, uint32_t m, bool has_diag,
                         hipStream_t s);

// Diagonal observable value(i) = c0 + sum_g w[g] count_g(i) (count terms as in
// the phase layers), expectation sum_i |psi_i|^2 value(i), for count instances
// of n qubits at once; out[k] receives instance k's expectation (device).
struct ObsDev {
  const void* psi;  // cplx<R>*
  const DiagTerm* terms;
  const DiagGroup* groups;
  const double* w;
  int32_t n_groups;
  int32_t pad;
  double c0;
  // per group g, kObsNbrStride int32: [0, 32) neighbour masks N_p, [32, 64)
  // degrees deg_p, [64] = 1 when the group is a set of distinct bit pairs
  // (every term DT_SHIFT_XOR), so that flipping a zero bit p changes the
  // count by deg_p - 2 popcount(N_p & i); 0 otherwise
  const int32_t* nbr;
};
constexpr int kObsNbrStride = 65;
template <class R>
void launch_batch_observable(const ObsDev* obs_dev, uint32_t count, uint32_t n, double* partials, double* out,
                             hipStream_t s);
size_t batch_observable_partials(uint32_t count, uint32_t n);  // doubles needed for partials

template <class R>
void launch_diag(cplx<R>* psi, int n, const DiagDev& D, hipStream_t s);

// Dense k-qubit block (matrix cores): psi <- U on the k bits bits_sorted
// (ascending); U_dev is 2^k x 2^k row-major in device memory with index bit u
// of rows and columns on bits_sorted[u].  Supported for k = 4..6 with n >= k + 4
// (complex128: k <= 5); returns false, launching nothing, otherwise.
struct DenseGeom {
  uint32_t m, c, L;        // tile bits, column bits, low tile bits equal to state bits [0, L)
  uint32_t rowmask;        // tile positions of the targets
  uint32_t n_hi;           // tile bits at positions >= L (all targets) ...
  uint32_t hi_bit[6];      // ... and their state bits
  uint32_t n_free;         // state bits outside the tile (ascending) ...
  uint32_t free_bit[32];
  uint32_t n_tiles;        // 2^n_free
};
bool dense_supported(int n, int k, bool complex128);
DenseGeom dense_geometry(int n, int k, const int* bits_sorted);
template <class R>
bool launch_dense(cplx<R>* psi, int n, int k, const int* bits_sorted, const cplx<R>* U_dev, hipStream_t s);

template <class R>
void launch_gf2(const cplx<R>* in, cplx<R>* out, const Gf2Args& A, hipStream_t s, double* norm_part = nullptr);
// Norm partials of a gather: one per wavefront of each coset tile (four
// wavefronts per tile).
inline uint64_t gf2_norm_slots(const Gf2Args& A) { return 4ull << (A.n - A.d); }
// out[0] = sum of count FP64 partials in a fixed order (compensated);
// scratch holds 2 kRedBlocks doubles.
void launch_fold_partials(const double* partials, uint64_t count, double* scratch, double* out, hipStream_t s);

// ---- FP64 reductions (deterministic: fixed grid, fixed combination order) ----
// Each writes NV (sum, compensation) pairs per block into partials and then
// folds them into out[NV] (device), one workgroup per output.
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

// ---- read-out ----
// Shot sampling: out[k] = the first index whose cumulative probability exceeds
// u[k] ||psi||^2 (cumulative sums hierarchical, FP64, fixed order); u and out
// in device memory; scratch needs sample_scratch_doubles(n) doubles.
struct SampleGeom {
  uint32_t sub_len, subs_per_block;
  uint64_t n_sub, n_blk;
};
SampleGeom sample_geometry(int n);
size_t sample_scratch_doubles(int n);
template <class R>
void launch_sample(const cplx<R>* psi, int n, const double* u_dev, uint64_t count, uint64_t* out_dev,
                   double* scratch, hipStream_t s);

// Allocation-free sampling (qs_sample_noalloc): its scratch is one static
// device array per GPU, sized for states of up to kNoAllocSampleMaxQubits
// qubits and kNoAllocSampleMaxDraws draws per call.  Layout (doubles): the
// norm reduction's partials (2 kRedBlocks) and result (8), the sampling sums
// of a kNoAllocSampleMaxQubits-qubit state, the uniforms, the drawn indices.
constexpr int kNoAllocSampleMaxQubits = 26;
constexpr uint64_t kNoAllocSampleMaxDraws = 1ull << 16;
struct NoAllocSampleScratch {
  double* norm_partials;
  double* norm_out;
  double* sums;
  double* u;
  uint64_t* out;
};
// The array's device address on `device` (looked up with that device current
// on the first call for it, then cached); fails with QS_EDEVICE if the lookup
// fails.
NoAllocSampleScratch noalloc_sample_scratch(int device);
// Marginal over k <= 16 state bits sel[0] < sel[1] < ...: out[bin] (device),
// bin bit j = state bit sel[j].
struct MarginalArgs {
  uint32_t k, chunks;
  uint64_t chunk_len;
  uint32_t sel[32];
};
MarginalArgs marginal_geometry(int n, const int* sel_bits, int k);
size_t marginal_partials(const MarginalArgs& A);
template <class R>
void launch_marginal(const cplx<R>* psi, const MarginalArgs& A, double* partials, double* out, hipStream_t s);

// ---- adjoint support ----
// out = H psi for a sum of Pauli terms c_t X^{x_t} Z^{z_t} (c_t complex: the
// coefficient times i^{#Y}): out_i = sum_t c_t (-1)^{popcount(j & z_t)} psi_j
// with j = i ^ x_t.  The terms of one X mask form a group whose coefficient
// of j is c0 + sum_k w_k count_k(j), count_k one of the diagonal layers' count
// forms (DT_BITS: single Z, DT_SHIFT_XOR: Z pairs at one distance, DT_PARITY:
// longer Z strings), so that equal-coefficient Z and ZZ terms cost one
// popcount together.  Groups and counts in device memory.
struct PauliGroup {
  uint32_t x;
  int32_t k0, nk;  // counts [k0, k0 + nk)
  int32_t pad;
  double c0re, c0im;
};
struct PauliCount {
  int32_t form;  // DT_BITS, DT_SHIFT_XOR or DT_PARITY
  uint32_t shift, mask;
  int32_t pad;
  double wre, wim;
};
template <class R>
void launch_pauli_apply(const cplx<R>* psi, cplx<R>* out, int n, const PauliGroup* groups, int n_groups,
                        const PauliCount* counts, hipStream_t s);
// rho[r][c] = sum over pairs on bit b of conj(lam_r) phi_c (8 doubles: re/im of
// rho00, rho01, rho10, rho11).
template <class R>
void launch_pair_rho(const cplx<R>* phi, const cplx<R>* lam, int n, int b, double* partials, double* out,
                     hipStream_t s);
// The same eight sums for several bits at once, over the tiles of a tile-pass
// geometry ([0, L) U [a, a + h), m = L + h): tbit[] are tile positions.
// out[8 j + v] for requested bit j.  Returns false (nothing launched) when the
// two staged tiles do not fit in LDS; partials needs rho_tile_partials doubles.
struct RhoTileArgs {
  uint32_t L, a, h, m;
  uint32_t nbits;
  uint32_t tbit[32];
};
size_t rho_tile_partials(int n, const RhoTileArgs& A);
// out[v] = sum over tiles of partials[v ntiles + tile] for v < nvals (compensated, fixed order).
void launch_rho_finalize(const double* partials, uint32_t ntiles, uint32_t nvals, double* out, hipStream_t s);
bool rho_tile_fits(uint32_t m, size_t amp_bytes);  // both tiles of 2^m amplitudes fit in LDS
template <class R>
bool launch_rho_tile(const cplx<R>* phi, const cplx<R>* lam, int n, const RhoTileArgs& A, double* partials,
                     double* out, hipStream_t s);
// out[g] = sum_x count_g(x) Im(conj(lam_x) phi_x) for groups [g0, g0 + ng), ng <= 8.
template <class R>
void launch_diag_grad(const cplx<R>* phi, const cplx<R>* lam, int n, const DiagDev& D, int g0, int ng,
                      double* partials, double* out, hipStream_t s);

}  // namespace qs
