// Streaming-ceiling probe: what HBM bandwidth plain streams and the tile
// passes' access patterns reach on this device, with no arithmetic of the
// method.  A tile pass reads and writes 2S bytes per pass; its achievable
// rate depends on the run length 2^L of its high-bit tiles and on the order
// in which workgroups take cosets, so the probe times, on a 2^n-amplitude
// complex64 state (S = 8 * 2^n bytes):
//   - hipMemcpyAsync device to device (the runtime's blit), 2S;
//   - a non-temporal streaming copy with K 16-byte accesses in flight per
//     thread, out of place and in place, 2S; a read-only stream (S) and a
//     write-only stream (S);
//   - tile-pattern passes: each workgroup loads one coset of the tile bits
//     [0, L) U [a, a + h) into LDS (padded as in the tile kernel), optionally
//     runs R rounds of four unscaled Hadamard butterflies, and stores it back,
//     in XCD-blocked or launch coset order.
// Output: one JSON object per line ({"probe", "bytes", "best_ms", "GBs"}).
// Usage: ceiling_probe [n]   (n = 30 by default; needs 2 * 8 * 2^n bytes).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define PROBE_CHECK(x)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::printf("{\"error\": \"%s at line %d\"}\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 ld_stream(const f4* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(f4* p, f4 v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ uint32_t xcd_blocked(uint32_t w, uint32_t grid) {
  return (grid & 7u) == 0u ? (w & 7u) * (grid >> 3) + (w >> 3) : w;
}

// Each block moves K * 256 consecutive 16-byte words.
template <int K>
__global__ void __launch_bounds__(256) copy_stream(const f4* __restrict__ in, f4* __restrict__ out) {
  const uint64_t base = (uint64_t)blockIdx.x * K * 256 + threadIdx.x;
  f4 v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = ld_stream(in + base + k * 256);
#pragma unroll
  for (int k = 0; k < K; ++k) st_stream(out + base + k * 256, v[k]);
}

template <int K>
__global__ void __launch_bounds__(256) read_stream(const f4* __restrict__ in, float* __restrict__ sink) {
  const uint64_t base = (uint64_t)blockIdx.x * K * 256 + threadIdx.x;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < K; ++k) acc += ld_stream(in + base + k * 256);
  if (acc.x == 1234.5f) sink[0] = acc.y;  // keeps the loads; never true for the zero state
}

template <int K>
__global__ void __launch_bounds__(256) write_stream(f4* __restrict__ out) {
  const uint64_t base = (uint64_t)blockIdx.x * K * 256 + threadIdx.x;
  const f4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < K; ++k) st_stream(out + base + k * 256, v);
}

struct Geo {
  uint32_t L, a, h, m;
};

__device__ __forceinline__ uint64_t coset_base(const Geo& G, uint32_t coset) {
  const uint32_t nlo = G.a - G.L, top = G.a + G.h;
  return ((uint64_t)(coset & ((1u << nlo) - 1u)) << G.L) | ((uint64_t)(coset >> nlo) << top);
}
__device__ __forceinline__ uint64_t tile_dep(const Geo& G, uint32_t pos) {
  return (pos & ((1u << G.L) - 1u)) | ((uint64_t)(pos >> G.L) << G.a);
}
__device__ __forceinline__ uint32_t lds_pad(uint32_t pos) { return pos + ((pos >> 5) << 1); }
__device__ __forceinline__ uint32_t insert_zero(uint32_t x, uint32_t b) {
  return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1u));
}

// R rounds of four unscaled Hadamard butterflies on tile bits 4r .. 4r + 3 (mod m).
__device__ void h4_rounds(float2* T, uint32_t m, int R) {
  const uint32_t ng = (1u << m) >> 4;
  for (int r = 0; r < R; ++r) {
    uint32_t tb[4];
    for (int k = 0; k < 4; ++k) tb[k] = (4u * r + k) % m;
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (tb[j] < tb[i]) {
          const uint32_t t = tb[i];
          tb[i] = tb[j];
          tb[j] = t;
        }
    for (uint32_t g = threadIdx.x; g < ng; g += blockDim.x) {
      uint32_t gp = g;
      for (int k = 0; k < 4; ++k) gp = insert_zero(gp, tb[k]);
      float2 a[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        uint32_t o = gp;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if ((j >> k) & 1) o |= 1u << tb[k];
        a[j] = T[lds_pad(o)];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (!(j & (1 << s))) {
            const float2 x = a[j], y = a[j | (1 << s)];
            a[j] = make_float2(x.x + y.x, x.y + y.y);
            a[j | (1 << s)] = make_float2(x.x - y.x, x.y - y.y);
          }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        uint32_t o = gp;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if ((j >> k) & 1) o |= 1u << tb[k];
        T[lds_pad(o)] = make_float2(a[j].x * 0.25f, a[j].y * 0.25f);
      }
    }
    __syncthreads();
  }
}

// One coset per workgroup: 2^m = 16 * 2 * blockDim.x amplitudes (checked on the host).
__global__ void __launch_bounds__(1024) tile_pattern(float2* psi, Geo G, int xcd_order, int R) {
  extern __shared__ __align__(16) float2 T[];
  const uint32_t coset = xcd_order ? xcd_blocked(blockIdx.x, gridDim.x) : blockIdx.x;
  const uint64_t base = coset_base(G, coset);
  const uint32_t stride = 2 * blockDim.x;
  f4 v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    v[k] = ld_stream(reinterpret_cast<const f4*>(psi + (base | tile_dep(G, 2 * threadIdx.x + stride * k))));
#pragma unroll
  for (int k = 0; k < 8; ++k) *reinterpret_cast<f4*>(T + lds_pad(2 * threadIdx.x + stride * k)) = v[k];
  __syncthreads();
  h4_rounds(T, G.m, R);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = *reinterpret_cast<const f4*>(T + lds_pad(2 * threadIdx.x + stride * k));
#pragma unroll
  for (int k = 0; k < 8; ++k)
    st_stream(reinterpret_cast<f4*>(psi + (base | tile_dep(G, 2 * threadIdx.x + stride * k))), v[k]);
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 30;
  if (n < 24 || n > 31) {
    std::printf("{\"error\": \"n must lie in 24..31\"}\n");
    return 2;
  }
  const uint64_t N = 1ull << n, bytes = N * 8, words = bytes / 16;
  float2 *A = nullptr, *B = nullptr;
  float* sink = nullptr;
  PROBE_CHECK(hipMalloc(&A, bytes));
  PROBE_CHECK(hipMalloc(&B, bytes));
  PROBE_CHECK(hipMalloc(&sink, 64));
  PROBE_CHECK(hipMemset(A, 0, bytes));
  PROBE_CHECK(hipMemset(B, 0, bytes));
  hipEvent_t e0, e1;
  PROBE_CHECK(hipEventCreate(&e0));
  PROBE_CHECK(hipEventCreate(&e1));
  auto timeit = [&](const char* name, double moved, auto launch) {
    launch();
    PROBE_CHECK(hipGetLastError());
    PROBE_CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int r = 0; r < 5; ++r) {
      PROBE_CHECK(hipEventRecord(e0, 0));
      launch();
      PROBE_CHECK(hipEventRecord(e1, 0));
      PROBE_CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
      best = ms < best ? ms : best;
    }
    std::printf("{\"probe\": \"%s\", \"bytes\": %.0f, \"best_ms\": %.4f, \"GBs\": %.1f}\n", name, moved, best,
                moved / (best * 1e-3) / 1e9);
    std::fflush(stdout);
  };
  const double two = 2.0 * bytes, one = 1.0 * bytes;
  timeit("hipMemcpyAsync_d2d", two, [&] { PROBE_CHECK(hipMemcpyAsync(B, A, bytes, hipMemcpyDeviceToDevice, 0)); });
  timeit("copy_K4", two, [&] { copy_stream<4><<<words / (256 * 4), 256>>>((const f4*)A, (f4*)B); });
  timeit("copy_K8", two, [&] { copy_stream<8><<<words / (256 * 8), 256>>>((const f4*)A, (f4*)B); });
  timeit("copy_in_place_K8", two, [&] { copy_stream<8><<<words / (256 * 8), 256>>>((const f4*)A, (f4*)A); });
  timeit("read_K8", one, [&] { read_stream<8><<<words / (256 * 8), 256>>>((const f4*)A, sink); });
  timeit("write_K8", one, [&] { write_stream<8><<<words / (256 * 8), 256>>>((f4*)B); });
  PROBE_CHECK(hipFuncSetAttribute((const void*)tile_pattern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  144 * 1024));
  // the 30-qubit benchmark plan's geometries (13-bit tiles) and longer-run ones
  const uint32_t nn = (uint32_t)n;
  const Geo geos[] = {{13, 13, 0, 13}, {5, nn - 8, 8, 13}, {4, 13, 9, 13}, {8, nn - 5, 5, 13},
                      {14, 14, 0, 14}, {6, nn - 8, 8, 14}, {6, 14, 8, 14}, {7, nn - 7, 7, 14}};
  for (int R : {0, 4}) {
    for (const Geo& g : geos) {
      if (g.a + g.h > (uint32_t)n || g.L > g.a) continue;
      const uint32_t threads = (1u << g.m) / 16;  // 16 amplitudes per thread
      const uint32_t cosets = 1u << (n - g.m);
      const size_t lds = 8 * ((1u << g.m) + (((1u << g.m) >> 5) << 1));
      for (int x = 1; x >= 0; --x) {
        char name[128];
        std::snprintf(name, sizeof name, "tile L%u a%u h%u m%u rounds%d %s", g.L, g.a, g.h, g.m, R,
                      x ? "xcd_blocked" : "launch_order");
        timeit(name, two, [&] { tile_pattern<<<cosets, threads, lds>>>(A, g, x, R); });
      }
    }
  }
  PROBE_CHECK(hipFree(A));
  PROBE_CHECK(hipFree(B));
  PROBE_CHECK(hipFree(sink));
  return 0;
}
