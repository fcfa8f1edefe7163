// Common-neighbour lists of edges, built once per graph.
//
// A second-order step from v after t needs the positions j in N(v) whose
// candidate is a common neighbour (x in N(t), x != t), the prefix of their
// weights and the position of t in N(v) (Methods, "Efficient sampling for
// Node2Vec RWs": the in-out bias is 1 exactly on N(t), Eq. 3).  Building that
// list (a merge or a probe of two rows) dominates the step when the rows are
// long, and walks cross the same edges again and again.  The graph is
// immutable, so the list of an edge t -> v is a pure function of the graph:
// these kernels store it, indexed by the edge's position e in the CSR
// (v = D[e], e in t's row), and the walk kernels read it instead of
// rebuilding it.  Each entry is {R_v[j], inclusive prefix of the listed
// weights, j, 0}: exactly the values the list routes compute, so walks stay
// bit-identical.  Each edge has a 32-byte record {first entry, entries,
// position of t in N(v) or ~0, total listed weight} {weight of t in N(v), 0,
// 0, 0}, so a step reads everything it needs before the draw in one line;
// first entry ~0 marks an edge whose list is not kept.
//
// Passes (one wavefront per edge; the lanes split the shorter of N(t) and
// N(v) and bisect the other; walking N(t) yields the positions in N(v) in
// increasing order too, so a ballot keeps the entries sorted):
//   k_edge_src            source row of every entry, and the build work
//   k_edge_lists_measure  per edge: number of common neighbours, position of t in N(v)
//   (the kept edges are chosen and their lists laid out on the device: a sum
//    of the counts, a sort by saved work per entry when they exceed the
//    budget, an exclusive scan of the kept counts, the 32-byte records)
//   k_edge_lists_fill     per kept edge: the entries, in increasing j
#include <hipcub/hipcub.hpp>

#include "n2v_device.hpp"
#include "n2v_internal.hpp"

namespace n2v {

namespace {

__device__ __forceinline__ int64_t wave_index() { return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ __forceinline__ int64_t wave_count() { return ((int64_t)gridDim.x * blockDim.x) >> 6; }

// position of x in A[0, n) (n >= 1), or ~0
__device__ __forceinline__ uint32_t find_in_row(const int32_t* __restrict__ A, uint32_t n, int32_t x) {
  int32_t val;
  const uint32_t p = floor_search(A, 0u, n, A[0], x, val);
  return val == x ? p : 0xFFFFFFFFu;
}

// The two rows of edge e = (t -> v).
struct EdgeRows {
  uint64_t lot, lov;
  uint32_t dt, dv;
  int32_t t;
};

// Candidate i of the shorter row of an edge, searched in the longer one:
// whether it is a listed common neighbour, and its position p in N(v).
__device__ __forceinline__ bool chunk_hit(const int32_t* __restrict__ D, const EdgeRows& r, uint32_t i, uint32_t* p) {
  if (r.dt <= r.dv) {  // candidates from N(t), positions by bisection in N(v)
    if (i >= r.dt) return false;
    const int32_t x = D[r.lot + i];
    if (x == r.t) return false;
    *p = find_in_row(D + r.lov, r.dv, x);
    return *p != 0xFFFFFFFFu;
  }
  if (i >= r.dv) return false;  // candidates from N(v), membership by bisection in N(t)
  const int32_t x = D[r.lov + i];
  *p = i;
  return x != r.t && find_in_row(D + r.lot, r.dt, x) != 0xFFFFFFFFu;
}

__device__ __forceinline__ EdgeRows edge_rows(const uint64_t* __restrict__ O, const int32_t* __restrict__ D,
                                              const int32_t* __restrict__ src, uint64_t e) {
  EdgeRows r;
  r.t = src[e];
  const int32_t v = D[e];
  r.lot = O[r.t];
  r.dt = (uint32_t)(O[r.t + 1] - r.lot);
  r.lov = O[v];
  r.dv = (uint32_t)(O[v + 1] - r.lov);
  return r;
}

// Per edge: {entries, position of t in N(v) or ~0, total listed weight,
// weight of t in N(v) (0 when t is not in it)}.
__global__ __launch_bounds__(256) void k_edge_lists_measure(const uint64_t* __restrict__ O,
                                                            const int32_t* __restrict__ D,
                                                            const int32_t* __restrict__ src, uint64_t m,
                                                            const uint32_t* __restrict__ R,
                                                            uint4* __restrict__ meas) {
  const int lane = threadIdx.x & 63;
  for (uint64_t e = (uint64_t)wave_index(); e < m; e += (uint64_t)wave_count()) {
    const EdgeRows r = edge_rows(O, D, src, e);
    uint32_t c = 0, cw = 0;
    const uint32_t span = r.dt <= r.dv ? r.dt : r.dv;
    if (r.dv > 0) {
      for (uint32_t c0 = 0; c0 < span; c0 += 64) {
        uint32_t p = 0;
        const bool hit = chunk_hit(D, r, c0 + lane, &p);
        const uint32_t w = hit ? (p ? R[r.lov + p] - R[r.lov + p - 1] : R[r.lov + p]) : 0u;
        c += (uint32_t)__popcll(__ballot(hit));
        cw += (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(w), 63);
      }
    }
    if (lane == 0) {
      const uint32_t pt = r.dv > 0 ? find_in_row(D + r.lov, r.dv, r.t) : 0xFFFFFFFFu;
      const uint32_t wt = pt == 0xFFFFFFFFu ? 0u : (pt ? R[r.lov + pt] - R[r.lov + pt - 1] : R[r.lov + pt]);
      meas[e] = make_uint4(c, pt, cw, wt);
    }
  }
}

__global__ __launch_bounds__(256) void k_edge_lists_fill(const uint64_t* __restrict__ O, const int32_t* __restrict__ D,
                                                         const int32_t* __restrict__ src, uint64_t m,
                                                         const uint32_t* __restrict__ R,
                                                         const uint4* __restrict__ info, uint4* __restrict__ ent) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (uint64_t e = (uint64_t)wave_index(); e < m; e += (uint64_t)wave_count()) {
    const uint4 inf = info[2 * e];
    if (inf.x == 0xFFFFFFFFu || inf.y == 0) continue;  // not kept, or empty
    const uint64_t off = inf.x;
    const EdgeRows r = edge_rows(O, D, src, e);
    const uint32_t span = r.dt <= r.dv ? r.dt : r.dv;
    uint64_t k = 0;
    uint32_t E = 0;  // listed weight so far (part of the row sum, which fits 32 bits)
    for (uint32_t c0 = 0; c0 < span; c0 += 64) {
      uint32_t p = 0;
      const bool hit = chunk_hit(D, r, c0 + lane, &p);
      const uint32_t rv = hit ? R[r.lov + p] : 0u;
      const uint32_t w = hit ? (p ? rv - R[r.lov + p - 1] : rv) : 0u;
      const uint32_t incl = wave_incl_scan_u32(w);
      const uint64_t mk = __ballot(hit);
      if (hit) ent[off + k + (uint64_t)__popcll(mk & lt)] = make_uint4(rv, E + incl, p, 0u);
      k += (uint64_t)__popcll(mk);
      E += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    }
  }
}

// Source row of every entry (one wavefront per row), and into *work the
// build work sum over entries of min(d_t, d_v) * bits(max(d_t, d_v)).
__global__ __launch_bounds__(256) void k_edge_src(const uint64_t* __restrict__ O, int64_t n,
                                                  const int32_t* __restrict__ D, int32_t* __restrict__ src,
                                                  unsigned long long* __restrict__ work) {
  const int lane = threadIdx.x & 63;
  uint64_t acc = 0;
  for (int64_t t = wave_index(); t < n; t += wave_count()) {
    const uint64_t a = O[t], b = O[t + 1];
    const uint64_t dt = b - a;
    for (uint64_t k = a + lane; k < b; k += 64) {
      src[k] = (int32_t)t;
      const int32_t v = D[k];
      const uint64_t dv = O[v + 1] - O[v];
      const uint64_t mx = dt > dv ? dt : dv, mn = dt > dv ? dv : dt;
      acc += mn * (uint64_t)(64 - __clzll((long long)(mx | 1)));
    }
  }
  acc = wave_incl_scan_u64(acc);
  if (lane == 63 && acc) atomicAdd(work, (unsigned long long)acc);
}

// Per edge: the list length (for the scans and the sum), and the sort key
// of an edge's saved work per stored entry, (d_t + d_v) / (entries + 4), as
// the bits of a positive float (which order like the floats).
__global__ __launch_bounds__(256) void k_edge_counts(const uint64_t* __restrict__ O, const int32_t* __restrict__ D,
                                                     const int32_t* __restrict__ src, const uint4* __restrict__ meas,
                                                     uint64_t m, uint64_t* __restrict__ cnt,
                                                     uint32_t* __restrict__ key, uint32_t* __restrict__ idx,
                                                     unsigned long long* __restrict__ all) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    const uint32_t c = meas[e].x;
    cnt[e] = c;
    acc += c;
    if (key) {
      const int32_t t = src[e], v = D[e];
      const float deg = (float)((O[t + 1] - O[t]) + (O[v + 1] - O[v]));
      key[e] = __float_as_uint(deg / ((float)c + 4.0f));
      idx[e] = (uint32_t)e;
    }
  }
  acc = wave_incl_scan_u64(acc);
  if ((threadIdx.x & 63) == 63 && acc) atomicAdd(all, (unsigned long long)acc);
}

// In decreasing saved work per entry (sorted order i -> edge idx[i], with
// cum[i] the inclusive sum of the list lengths so far): an edge keeps its list
// when the lists up to it fit the budget, or when it is empty.
__global__ __launch_bounds__(256) void k_edge_keep(const uint32_t* __restrict__ idx, const uint64_t* __restrict__ cum,
                                                   const uint4* __restrict__ meas, uint64_t m, uint64_t budget,
                                                   uint8_t* __restrict__ keep) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint32_t e = idx[i];
    keep[e] = (cum[i] <= budget || meas[e].x == 0) ? 1 : 0;
  }
}

// Kept list lengths (0 for the others), the input of the offset scan.
__global__ __launch_bounds__(256) void k_edge_sizes(const uint4* __restrict__ meas, const uint8_t* __restrict__ keep,
                                                    uint64_t m, uint64_t* __restrict__ sz) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
    sz[e] = (!keep || keep[e]) ? meas[e].x : 0u;
}

// The 32-byte records from the measure and the offsets; tot[0] += kept edges,
// tot[1] = entries of all kept lists.
__global__ __launch_bounds__(256) void k_edge_info(const uint4* __restrict__ meas, const uint8_t* __restrict__ keep,
                                                   const uint64_t* __restrict__ off, uint64_t m,
                                                   uint4* __restrict__ info, unsigned long long* __restrict__ tot) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t kept = 0;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    const uint4 me = meas[e];
    const bool k = !keep || keep[e];
    // t's position in N(v) stays in an edge without a list (return-only steps read it)
    info[2 * e] = k ? make_uint4((uint32_t)off[e], me.x, me.y, me.z) : make_uint4(0xFFFFFFFFu, 0u, me.y, 0u);
    info[2 * e + 1] = make_uint4(me.w, 0u, 0u, 0u);
    kept += k ? 1u : 0u;
    if (e == m - 1) tot[1] = off[e] + (k ? me.x : 0u);
  }
  kept = wave_incl_scan_u64(kept);
  if ((threadIdx.x & 63) == 63 && kept) atomicAdd(&tot[0], (unsigned long long)kept);
}

__global__ __launch_bounds__(256) void k_gather_counts(const uint32_t* __restrict__ idx,
                                                       const uint64_t* __restrict__ cnt, uint64_t m,
                                                       uint64_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) out[i] = cnt[idx[i]];
}

unsigned flat_blocks(uint64_t items) {
  uint64_t b = (items + 255) / 256;
  if (b > 256 * 32) b = 256 * 32;
  return (unsigned)(b ? b : 1);
}

unsigned edge_blocks(uint64_t edges) {
  uint64_t b = (edges + 3) / 4;
  if (b > 256 * 64) b = 256 * 64;
  return (unsigned)(b ? b : 1);
}

}  // namespace

hipError_t launch_edge_lists_measure(const uint64_t* O, const int32_t* D, const int32_t* src, uint64_t m,
                                     const uint32_t* R, uint4* meas, hipStream_t st) {
  hipLaunchKernelGGL(k_edge_lists_measure, dim3(edge_blocks(m)), dim3(256), 0, st, O, D, src, m, R, meas);
  return hipGetLastError();
}

hipError_t launch_edge_src(const uint64_t* O, int64_t n, const int32_t* D, int32_t* src, unsigned long long* work,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_edge_src, dim3(edge_blocks((uint64_t)n)), dim3(256), 0, st, O, n, D, src, work);
  return hipGetLastError();
}

hipError_t launch_edge_counts(const uint64_t* O, const int32_t* D, const int32_t* src, const uint4* meas, uint64_t m,
                              uint64_t* cnt, uint32_t* key, uint32_t* idx, unsigned long long* all, hipStream_t st) {
  hipLaunchKernelGGL(k_edge_counts, dim3(flat_blocks(m)), dim3(256), 0, st, O, D, src, meas, m, cnt, key, idx, all);
  return hipGetLastError();
}

hipError_t edge_keep_by_gain(const uint32_t* key, const uint32_t* idx, uint32_t* key_s, uint32_t* idx_s,
                             const uint64_t* cnt, uint64_t* cnt_s, uint64_t* cum, const uint4* meas, uint64_t m,
                             uint64_t budget, uint8_t* keep, hipStream_t st) {
  // lengths in sorted order, then their inclusive sum
  size_t b1 = 0, b2 = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, b1, key, key_s, idx, idx_s, (int)m, 0, 32, st);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::InclusiveSum(nullptr, b2, cnt_s, cum, (int)m, st);
  if (e != hipSuccess) return e;
  void* tmp = nullptr;
  e = hipMalloc(&tmp, std::max(b1, b2));
  if (e != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortPairsDescending(tmp, b1, key, key_s, idx, idx_s, (int)m, 0, 32, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gather_counts, dim3(flat_blocks(m)), dim3(256), 0, st, idx_s, cnt, m, cnt_s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipcub::DeviceScan::InclusiveSum(tmp, b2, cnt_s, cum, (int)m, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_edge_keep, dim3(flat_blocks(m)), dim3(256), 0, st, idx_s, cum, meas, m, budget, keep);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  return e;
}

hipError_t edge_layout(const uint4* meas, const uint8_t* keep, uint64_t m, uint64_t* sz, uint64_t* off, uint4* info,
                       unsigned long long* tot, hipStream_t st) {
  hipLaunchKernelGGL(k_edge_sizes, dim3(flat_blocks(m)), dim3(256), 0, st, meas, keep, m, sz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t b = 0;
  e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, sz, off, (int)m, st);
  if (e != hipSuccess) return e;
  void* tmp = nullptr;
  e = hipMalloc(&tmp, b ? b : 1);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(tmp, b, sz, off, (int)m, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_edge_info, dim3(flat_blocks(m)), dim3(256), 0, st, meas, keep, off, m, info, tot);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  return e;
}

hipError_t launch_edge_lists_fill(const uint64_t* O, const int32_t* D, const int32_t* src, uint64_t m,
                                  const uint32_t* R, const uint4* info, uint4* ent, hipStream_t st) {
  hipLaunchKernelGGL(k_edge_lists_fill, dim3(edge_blocks(m)), dim3(256), 0, st, O, D, src, m, R, info, ent);
  return hipGetLastError();
}

}  // namespace n2v
