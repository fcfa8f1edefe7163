// Memory-system probes for the measurement side (not part of the walk
// library): random gathers of fixed granules over a power-of-two buffer, a
// streaming read, and a single-lane pointer chase.  They set the gather
// roofline the walk kernels are compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // SplitMix64 finaliser (Steele, Lea, Flood 2014)
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

// Item i reads granule mix64(i ^ seed) mod n_gran, V 16-byte vectors (V = 0:
// one 4-byte word).  Four items per round keep four gathers in flight.
template <int V>
__global__ __launch_bounds__(256) void k_gather(const uint4* __restrict__ buf, uint64_t gmask, uint64_t n_items,
                                                uint64_t seed, uint64_t* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += 4 * stride) {
    uint64_t g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = mix64((i + u * stride) ^ seed) & gmask;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i + u * stride >= n_items) break;
      if constexpr (V == 0) {
        acc ^= reinterpret_cast<const uint32_t*>(buf)[g[u]];
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const uint4 q = buf[g[u] * V + k];
          acc ^= q.x ^ q.y ^ q.z ^ q.w;
        }
      }
    }
  }
  if (acc == 0x12345678u) sink[0] = acc;  // keeps the loads alive
}

__global__ __launch_bounds__(256) void k_stream(const uint4* __restrict__ buf, uint64_t n_vec,
                                                uint64_t* __restrict__ sink) {
  uint32_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vec; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 q = buf[i];
    acc ^= q.x ^ q.y ^ q.z ^ q.w;
  }
  if (acc == 0x12345678u) sink[0] = acc;
}

// One lane follows next[] for `hops` dependent loads; next is a permutation.
__global__ void k_chase(const uint32_t* __restrict__ next, uint64_t hops, uint32_t start, uint64_t* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t c = start;
  for (uint64_t h = 0; h < hops; ++h) c = next[c];
  out[0] = c;
}

}  // namespace

extern "C" {

// granule_bytes: 4, 16, 64 or 128; n_granules a power of two; buf holds
// n_granules * granule_bytes bytes.  Returns 0 or a HIP error code.
int n2vm_gather(const void* buf, uint64_t n_granules, uint32_t granule_bytes, uint64_t n_items, uint64_t seed,
                uint64_t* d_sink, int grid, void* stream) {
  if (!buf || !d_sink || n_granules == 0 || (n_granules & (n_granules - 1))) return (int)hipErrorInvalidValue;
  const uint64_t mask = n_granules - 1;
  hipStream_t st = (hipStream_t)stream;
  const uint4* b = (const uint4*)buf;
  switch (granule_bytes) {
    case 4: hipLaunchKernelGGL(k_gather<0>, dim3(grid), dim3(256), 0, st, b, mask, n_items, seed, d_sink); break;
    case 16: hipLaunchKernelGGL(k_gather<1>, dim3(grid), dim3(256), 0, st, b, mask, n_items, seed, d_sink); break;
    case 64: hipLaunchKernelGGL(k_gather<4>, dim3(grid), dim3(256), 0, st, b, mask, n_items, seed, d_sink); break;
    case 128: hipLaunchKernelGGL(k_gather<8>, dim3(grid), dim3(256), 0, st, b, mask, n_items, seed, d_sink); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int n2vm_stream(const void* buf, uint64_t nbytes, uint64_t* d_sink, int grid, void* stream) {
  if (!buf || !d_sink || nbytes % 16) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint4*)buf, nbytes / 16, d_sink);
  return (int)hipGetLastError();
}

int n2vm_chase(const uint32_t* next, uint64_t hops, uint32_t start, uint64_t* d_out, void* stream) {
  if (!next || !d_out) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, (hipStream_t)stream, next, hops, start, d_out);
  return (int)hipGetLastError();
}

}  // extern "C"
