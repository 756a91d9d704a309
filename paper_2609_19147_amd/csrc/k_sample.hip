// Read-out from the device state: shot sampling of the basis-state
// distribution p_i = |psi_i|^2 / ||psi||^2 and marginal distributions over a
// subset of qubits (the paper's measurement and sampling workloads, Sections
// "State Management" and "Algorithm Implementations").
//
// Sampling, for caller-provided uniform numbers u in [0, 1): the drawn index
// is the first i whose cumulative probability mass exceeds u ||psi||^2.  The
// cumulative sums are hierarchical and FP64 with a fixed order everywhere:
// 64-amplitude sub-block sums (one wavefront each), block sums over 2^14
// amplitudes, an exclusive scan of the block sums by one workgroup; then one
// wavefront per sample searches the block prefixes, scans the block's
// sub-block sums and finally the sub-block's 64 probabilities.
#include "kernels.h"

#include <mutex>
#include <string>

#include "planner.h"

namespace qs {

void check_hip(hipError_t e, const char* what);

namespace {

constexpr int kSampThreads = 256;
constexpr int kScanThreads = 1024;

template <class R>
__device__ __forceinline__ double prob(const cplx<R>& a) {
  const double x = (double)a.re, y = (double)a.im;
  return x * x + y * y;
}

// Fixed-order inclusive scan across a wavefront.
__device__ __forceinline__ double wave_scan(double x, uint32_t lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// sub[s] = sum of the probabilities of amplitudes [s sub_len, (s + 1) sub_len),
// sub_len <= 64, one wavefront per sub-block.
template <class R>
__global__ void __launch_bounds__(kSampThreads) sub_sums_kernel(const cplx<R>* __restrict__ psi, uint64_t n_sub,
                                                                uint32_t sub_len, double* __restrict__ sub) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t waves = (uint64_t)gridDim.x * (kSampThreads / 64);
  for (uint64_t s = blockIdx.x * (uint64_t)(kSampThreads / 64) + (threadIdx.x >> 6); s < n_sub; s += waves) {
    const double p = lane < sub_len ? prob(psi[s * sub_len + lane]) : 0.0;
    const double t = wave_sum(p);
    if (lane == 0) sub[s] = t;
  }
}

// blk[b] = sum of its subs_per_block sub-block sums, in order.
__global__ void __launch_bounds__(kSampThreads) block_sums_kernel(const double* __restrict__ sub, uint64_t n_blk,
                                                                  uint32_t subs_per_block, double* __restrict__ blk) {
  for (uint64_t b = blockIdx.x * (uint64_t)kSampThreads + threadIdx.x; b < n_blk;
       b += (uint64_t)gridDim.x * kSampThreads) {
    double t = 0.0;
    for (uint32_t j = 0; j < subs_per_block; ++j) t += sub[b * subs_per_block + j];
    blk[b] = t;
  }
}

// P[0..n] = exclusive prefix of blk[0..n) (P[n] = total); one workgroup.
__global__ void __launch_bounds__(kScanThreads) block_scan_kernel(const double* __restrict__ blk, uint64_t n,
                                                                  double* __restrict__ P) {
  __shared__ double tot[kScanThreads];
  const uint64_t chunk = (n + kScanThreads - 1) / kScanThreads;
  const uint64_t b0 = threadIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
  double t = 0.0;
  for (uint64_t b = b0; b < b1; ++b) t += blk[b];
  tot[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int k = 0; k < kScanThreads; ++k) {
      const double v = tot[k];
      tot[k] = run;
      run += v;
    }
    P[n] = run;
  }
  __syncthreads();
  double run = tot[threadIdx.x];
  for (uint64_t b = b0; b < b1; ++b) {
    P[b] = run;
    run += blk[b];
  }
}

// One wavefront per sample.
template <class R>
__global__ void __launch_bounds__(kSampThreads) sample_kernel(const cplx<R>* __restrict__ psi,
                                                              const double* __restrict__ sub,
                                                              const double* __restrict__ P, uint64_t n_blk,
                                                              uint32_t subs_per_block, uint32_t sub_len,
                                                              const double* __restrict__ u, uint64_t count,
                                                              uint64_t* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t k = blockIdx.x * (uint64_t)(kSampThreads / 64) + (threadIdx.x >> 6);
  if (k >= count) return;
  const double total = P[n_blk];
  double t = u[k] * total;
  // block: last b with P[b] <= t (P is non-decreasing, P[0] = 0); requiring
  // P[b] < total as well keeps a product u total that rounded up to total in
  // the last block with mass
  uint64_t lo = 0, hi = n_blk - 1;
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) / 2;
    if (P[mid] <= t && P[mid] < total) lo = mid;
    else hi = mid - 1;
  }
  const uint64_t b = lo;
  t -= P[b];
  // sub-block: subs_per_block <= 256 sums, 4 per lane, scanned in order
  double s4[4], run = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t idx = lane * 4 + j;
    s4[j] = idx < subs_per_block ? sub[b * subs_per_block + idx] : 0.0;
    run += s4[j];
  }
  const double incl = wave_scan(run, lane);
  double excl = incl - run;
  // the first sub-block whose inclusive sum exceeds t; if rounding leaves t at
  // or past the block's total, the last sub-block with mass
  int pick = -1, last = -1;
  double before = 0.0, before_last = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int idx = (int)(lane * 4 + j);
    if (s4[j] > 0.0) {
      if (pick < 0 && excl + s4[j] > t) {
        pick = idx;
        before = excl;
      }
      last = idx;
      before_last = excl;
    }
    excl += s4[j];
  }
  // the smallest lane holding a pick wins; else the largest lane holding mass
  const uint64_t hit = __ballot(pick >= 0);
  uint32_t sb;
  double sbefore;
  if (hit) {
    const int src = __builtin_ctzll(hit);
    sb = (uint32_t)__shfl(pick, src, 64);
    sbefore = __shfl(before, src, 64);
  } else {
    const uint64_t has = __ballot(last >= 0);
    const int src = has ? 63 - __builtin_clzll(has) : 0;
    sb = has ? (uint32_t)__shfl(last, src, 64) : 0u;
    sbefore = has ? __shfl(before_last, src, 64) : 0.0;
  }
  t -= sbefore;
  // amplitude within the sub-block
  const uint64_t base = (b * subs_per_block + sb) * sub_len;
  const double p = lane < sub_len ? prob(psi[base + lane]) : 0.0;
  const double pin = wave_scan(p, lane);
  const uint64_t over = __ballot(p > 0.0 && pin > t);
  const uint64_t mass = __ballot(p > 0.0);
  uint32_t idx;
  if (over) idx = (uint32_t)__builtin_ctzll(over);
  else idx = mass ? (uint32_t)(63 - __builtin_clzll(mass)) : 0u;
  if (lane == 0) out[k] = base + idx;
}

// Marginal: out_partial[bin * chunks + c] = sum over the chunk c of the other
// qubits' index values r of p(compose(bin, r)).
template <class R>
__global__ void __launch_bounds__(kSampThreads) marginal_kernel(const cplx<R>* __restrict__ psi, MarginalArgs A,
                                                                double* __restrict__ partials) {
  const uint32_t bin = blockIdx.x / A.chunks, c = blockIdx.x % A.chunks;
  uint64_t bpart = 0;
  for (uint32_t j = 0; j < A.k; ++j)
    if ((bin >> j) & 1u) bpart |= 1ull << A.sel[j];
  const uint64_t r0 = (uint64_t)c * A.chunk_len, r1 = r0 + A.chunk_len;
  double s = 0.0;
  for (uint64_t r = r0 + threadIdx.x; r < r1; r += kSampThreads) {
    uint64_t i = r;
    for (uint32_t j = 0; j < A.k; ++j) {  // ascending: open a zero at every selected bit
      const uint64_t lo = i & ((1ull << A.sel[j]) - 1ull);
      i = ((i >> A.sel[j]) << (A.sel[j] + 1)) | lo;
    }
    s += prob(psi[i | bpart]);
  }
  __shared__ double red[kSampThreads];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int stride = kSampThreads / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) red[threadIdx.x] += red[threadIdx.x + stride];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kSampThreads) marginal_finalize(const double* __restrict__ partials,
                                                                  uint32_t bins, uint32_t chunks,
                                                                  double* __restrict__ out) {
  for (uint32_t b = blockIdx.x * kSampThreads + threadIdx.x; b < bins; b += gridDim.x * kSampThreads) {
    double t = 0.0;
    for (uint32_t c = 0; c < chunks; ++c) t += partials[(size_t)b * chunks + c];
    out[b] = t;
  }
}

inline unsigned grid_of(uint64_t work, int per_block, unsigned cap) {
  uint64_t g = (work + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

SampleGeom sample_geometry(int n) {
  SampleGeom G;
  G.sub_len = n >= 6 ? 64u : (1u << n);
  const uint32_t blk_len = n >= 14 ? (1u << 14) : (1u << n);
  G.subs_per_block = blk_len / G.sub_len;
  G.n_blk = (1ull << n) / blk_len;
  G.n_sub = G.n_blk * G.subs_per_block;
  return G;
}

size_t sample_scratch_doubles(int n) {
  const SampleGeom G = sample_geometry(n);
  return G.n_sub + G.n_blk + (G.n_blk + 1);
}

template <class R>
void launch_sample(const cplx<R>* psi, int n, const double* u_dev, uint64_t count, uint64_t* out_dev,
                   double* work, hipStream_t s) {
  const SampleGeom G = sample_geometry(n);
  double* sub = work;
  double* blk = sub + G.n_sub;
  double* P = blk + G.n_blk;
  QS_LAUNCH("sample_sub_sums", s, sub_sums_kernel<R>, dim3(grid_of(G.n_sub, kSampThreads / 64, 65536)),
            dim3(kSampThreads), 0, s, psi, G.n_sub, G.sub_len, sub);
  QS_LAUNCH("sample_block_sums", s, block_sums_kernel, dim3(grid_of(G.n_blk, kSampThreads, 4096)),
            dim3(kSampThreads), 0, s, sub, G.n_blk, G.subs_per_block, blk);
  QS_LAUNCH("sample_scan", s, block_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, blk, G.n_blk, P);
  if (count)
    QS_LAUNCH("sample_draw", s, sample_kernel<R>, dim3(grid_of(count, kSampThreads / 64, 1u << 30)),
              dim3(kSampThreads), 0, s, psi, sub, P, G.n_blk, G.subs_per_block, G.sub_len, u_dev, count,
              out_dev);
}

// ---- allocation-free sampling ----------------------------------------------
// Static scratch of qs_sample_noalloc, one copy per GPU (kept until the
// process ends): nothing in it needs clearing, since every region is written
// before it is read within a call.  Calls that overlap on one GPU share it.
namespace {
constexpr size_t kNaNormDoubles = 2 * (size_t)kRedBlocks + 8;
constexpr size_t kNaSumDoubles = ((size_t)1 << (kNoAllocSampleMaxQubits - 6)) +
                                 2 * ((size_t)1 << (kNoAllocSampleMaxQubits - 14)) + 1;
constexpr size_t kNaDoubles = kNaNormDoubles + kNaSumDoubles + 2 * kNoAllocSampleMaxDraws;
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kNaDoubles];

NoAllocSampleScratch noalloc_sample_scratch(int device) {
  if (device < 0 || device >= kNaMaxDevices) fail(QS_EINVAL, "device ordinal out of range");
  double* base;
  {
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[device]) {
      // the array's address differs per device: look it up with that device current
      int prev = 0;
      check_hip(hipGetDevice(&prev), "hipGetDevice");
      if (prev != device) check_hip(hipSetDevice(device), "hipSetDevice");
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (prev != device) (void)hipSetDevice(prev);
      check_hip(e, "hipGetSymbolAddress(scratch)");
      g_na_ptr[device] = (double*)p;
    }
    base = g_na_ptr[device];
  }
  NoAllocSampleScratch S;
  S.norm_partials = base;
  S.norm_out = base + 2 * (size_t)kRedBlocks;
  S.sums = base + kNaNormDoubles;
  S.u = S.sums + kNaSumDoubles;
  S.out = (uint64_t*)(S.u + kNoAllocSampleMaxDraws);
  return S;
}

size_t marginal_partials(const MarginalArgs& A) { return ((size_t)1 << A.k) * A.chunks; }

MarginalArgs marginal_geometry(int n, const int* sel_bits, int k) {
  MarginalArgs A{};
  A.k = (uint32_t)k;
  for (int j = 0; j < k; ++j) A.sel[j] = (uint32_t)sel_bits[j];
  const uint64_t rest = 1ull << (n - k);
  const uint32_t bins = 1u << k;
  // about 4096 workgroups in all, chunks of at least 4096 index values
  uint64_t chunks = 4096 / bins;
  if (chunks < 1) chunks = 1;
  while (chunks > 1 && rest / chunks < 4096) chunks >>= 1;
  if (chunks > rest) chunks = rest;
  A.chunks = (uint32_t)chunks;
  A.chunk_len = rest / chunks;
  return A;
}

template <class R>
void launch_marginal(const cplx<R>* psi, const MarginalArgs& A, double* partials, double* out, hipStream_t s) {
  const uint32_t bins = 1u << A.k;
  QS_LAUNCH("marginal", s, marginal_kernel<R>, dim3(bins * A.chunks), dim3(kSampThreads), 0, s, psi, A, partials);
  QS_LAUNCH("marginal_finalize", s, marginal_finalize, dim3(grid_of(bins, kSampThreads, 256)), dim3(kSampThreads),
            0, s, partials, bins, A.chunks, out);
}

template void launch_sample<float>(const cplx<float>*, int, const double*, uint64_t, uint64_t*, double*, hipStream_t);
template void launch_sample<double>(const cplx<double>*, int, const double*, uint64_t, uint64_t*, double*,
                                    hipStream_t);
template void launch_marginal<float>(const cplx<float>*, const MarginalArgs&, double*, double*, hipStream_t);
template void launch_marginal<double>(const cplx<double>*, const MarginalArgs&, double*, double*, hipStream_t);

}  // namespace qs
