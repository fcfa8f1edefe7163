// Graph preparation kernels: CSR validation, statistics and the per-row
// inclusive weight prefix used by the O(log d) sampling paths.
//
// The CSR store with sorted rows is the paper's default adjacency structure
// (Methods, "Succinct data structures" and "Available data-structure
// trade-offs"); the degree of v is offsets[v+1] - offsets[v].
#include "n2v_device.hpp"
#include "n2v_internal.hpp"

namespace n2v {

namespace {

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

// One wavefront per row (grid-stride).  Rows whose offsets are inconsistent
// are flagged and never dereferenced.
__global__ __launch_bounds__(256) void k_validate_stats(const uint64_t* __restrict__ O, int64_t n,
                                                        const int32_t* __restrict__ D, uint64_t m,
                                                        const uint32_t* __restrict__ W,
                                                        unsigned long long* __restrict__ stats) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  uint64_t err = 0, maxd = 0, maxs = 0, sumd2 = 0;
  if (wave == 0 && (O[0] != 0 || O[n] != m)) err |= kErrOffsets;
  for (int64_t v = wave; v < n; v += nwaves) {
    const uint64_t lo = O[v], hi = O[v + 1];
    if (hi < lo || hi > m) {
      err |= kErrOffsets;
      continue;
    }
    uint64_t s = 0;
    for (uint64_t e = lo + lane; e < hi; e += 64) {
      const int32_t x = D[e];
      if (x < 0 || (int64_t)x >= n) err |= kErrRange;
      if (e > lo && D[e - 1] >= x) err |= kErrOrder;
      s += W ? (uint64_t)W[e] : 1ull;
    }
    s = wave_sum_u64(s);
    const uint64_t d = hi - lo;
    maxd = d > maxd ? d : maxd;
    maxs = s > maxs ? s : maxs;
    sumd2 += d * d;
  }
  err = wave_or_u64(err);
  if (lane == 0) {
    if (err) atomicOr(stats + 0, (unsigned long long)err);
    atomicMax(stats + 1, (unsigned long long)maxd);
    atomicMax(stats + 2, (unsigned long long)maxs);
    atomicAdd(stats + 3, (unsigned long long)sumd2);
  }
}

// R[e] = sum of W over row entries up to and including e (row-local).
template <typename RT>
__global__ __launch_bounds__(256) void k_row_prefix(const uint64_t* __restrict__ O, int64_t n,
                                                    const uint32_t* __restrict__ W,
                                                    RT* __restrict__ R) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const uint64_t lo = O[v], hi = O[v + 1];
    uint64_t carry = 0;
    for (uint64_t base = lo; base < hi; base += 64) {
      const uint64_t e = base + lane;
      uint64_t x = e < hi ? (uint64_t)W[e] : 0ull;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, (unsigned)o, 64);
        if (lane >= o) x += y;
      }
      if (e < hi) R[e] = (RT)(carry + x);
      carry += __shfl(x, 63, 64);
    }
  }
}

__global__ __launch_bounds__(256) void k_node_records(const uint64_t* __restrict__ O, int64_t n,
                                                      const uint32_t* __restrict__ R, uint4* __restrict__ NR) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = O[v];
    const uint64_t d = O[v + 1] - lo;
    NR[v] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)d, d ? R[lo + d - 1] : 0u);
  }
}

int prep_blocks(int64_t n) {
  int64_t waves = n;  // one wave per row
  int64_t blocks = (waves + 3) / 4;
  if (blocks > 256 * 32) blocks = 256 * 32;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

template <typename T>
__global__ void k_prefix_heads(const T* __restrict__ R, uint64_t nh, T* __restrict__ HR) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += stride) HR[i] = R[i << 5];
}

// Hub sets.  One block per hub: every entry of the hub's row sets its bit
// (bits of one 32-bit word may come from several lanes: atomic or).
__global__ __launch_bounds__(256) void k_hub_bits(const uint64_t* __restrict__ O, const int32_t* __restrict__ D,
                                                  const int32_t* __restrict__ hubs, uint64_t lines,
                                                  uint32_t* __restrict__ sets) {
  const int32_t h = hubs[blockIdx.x];
  uint32_t* const set = sets + (uint64_t)blockIdx.x * lines * 16u;
  const uint64_t a = O[h], b = O[h + 1];
  for (uint64_t k = a + threadIdx.x; k < b; k += blockDim.x) {
    const uint32_t x = (uint32_t)D[k];
    const uint32_t line = x / kHubLineIds, bit = x - line * kHubLineIds;
    atomicOr(set + (uint64_t)line * 16u + (bit >> 5), 1u << (bit & 31u));
  }
}

// One block per hub: word 15 of every line = members in the earlier lines
// (each thread counts a contiguous range of lines; a block scan of the
// counts gives the range's base).
__global__ __launch_bounds__(256) void k_hub_ranks(uint64_t lines, uint32_t* __restrict__ sets,
                                                   const int32_t* __restrict__ hubs, int32_t* __restrict__ hub_of) {
  __shared__ uint32_t part[256];
  uint32_t* const set = sets + (uint64_t)blockIdx.x * lines * 16u;
  const uint64_t per = (lines + blockDim.x - 1) / blockDim.x;
  const uint64_t l0 = min(lines, (uint64_t)threadIdx.x * per), l1 = min(lines, l0 + per);
  uint32_t cnt = 0;
  for (uint64_t l = l0; l < l1; ++l)
    for (int w = 0; w < 15; ++w) cnt += (uint32_t)__popc(set[l * 16u + (uint64_t)w]);
  part[threadIdx.x] = cnt;
  __syncthreads();
  // inclusive scan of the 256 counts (Hillis-Steele)
  for (unsigned off = 1; off < blockDim.x; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t base = part[threadIdx.x] - cnt;
  for (uint64_t l = l0; l < l1; ++l) {
    uint32_t c = 0;
    for (int w = 0; w < 15; ++w) c += (uint32_t)__popc(set[l * 16u + (uint64_t)w]);
    set[l * 16u + 15u] = base;
    base += c;
  }
  if (threadIdx.x == 0) hub_of[hubs[blockIdx.x]] = (int32_t)blockIdx.x;
}

}  // namespace

hipError_t launch_hub_sets(const uint64_t* O, const int32_t* D, const int32_t* hubs, uint32_t n_hubs,
                           uint64_t lines, uint32_t* sets, int32_t* hub_of, hipStream_t st) {
  if (n_hubs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hub_bits, dim3(n_hubs), dim3(256), 0, st, O, D, hubs, lines, sets);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hub_ranks, dim3(n_hubs), dim3(256), 0, st, lines, sets, hubs, hub_of);
  return hipGetLastError();
}

hipError_t launch_prefix_heads(const void* R, uint32_t r_bytes, uint64_t m, void* HR, hipStream_t st) {
  const uint64_t nh = (m + 31) >> 5;
  if (nh == 0) return hipSuccess;
  uint64_t blocks = (nh + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  if (r_bytes == 4)
    hipLaunchKernelGGL(k_prefix_heads<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, st, (const uint32_t*)R, nh,
                       (uint32_t*)HR);
  else
    hipLaunchKernelGGL(k_prefix_heads<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, st, (const uint64_t*)R, nh,
                       (uint64_t*)HR);
  return hipGetLastError();
}

hipError_t launch_dest_heads(const int32_t* D, uint64_t m, int32_t* HD, hipStream_t st) {
  const uint64_t nh = (m + 31) >> 5;
  if (nh == 0) return hipSuccess;
  uint64_t blocks = (nh + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  hipLaunchKernelGGL(k_prefix_heads<int32_t>, dim3((unsigned)blocks), dim3(256), 0, st, D, nh, HD);
  return hipGetLastError();
}

hipError_t launch_validate_stats(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
                                 const uint32_t* W, uint64_t* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_validate_stats, dim3(prep_blocks(n)), dim3(256), 0, st, O, n, D, m, W,
                     (unsigned long long*)stats);
  return hipGetLastError();
}

hipError_t launch_node_records(const uint64_t* O, int64_t n, const uint32_t* R, uint4* NR, hipStream_t st) {
  hipLaunchKernelGGL(k_node_records, dim3(prep_blocks(n)), dim3(256), 0, st, O, n, R, NR);
  return hipGetLastError();
}

hipError_t launch_row_prefix(const uint64_t* O, int64_t n, const uint32_t* W, void* R,
                             uint32_t r_bytes, hipStream_t st) {
  if (r_bytes == 4)
    hipLaunchKernelGGL(k_row_prefix<uint32_t>, dim3(prep_blocks(n)), dim3(256), 0, st, O, n, W,
                       (uint32_t*)R);
  else
    hipLaunchKernelGGL(k_row_prefix<uint64_t>, dim3(prep_blocks(n)), dim3(256), 0, st, O, n, W,
                       (uint64_t*)R);
  return hipGetLastError();
}

}  // namespace n2v
