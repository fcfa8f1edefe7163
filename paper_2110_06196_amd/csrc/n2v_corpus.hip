// Training corpora from device walks: context slots of every walk position
// (window-based SkipGram / CBOW, and Walklets with a stride) and scale-free
// negative samples (nodes drawn with probability proportional to out-degree).
//
// Both kernels are write-bound streams.  A block owns a tile of consecutive
// walk positions; what it reads is staged in LDS and what it writes leaves in
// consecutive words, so global loads and stores coalesce.
#include "n2v_device.hpp"
#include "n2v_internal.hpp"

namespace n2v {
namespace {

constexpr uint32_t kCtxTile = 1024;  // positions per contexts tile
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

// Contexts with the tile's walk words and a halo of H = min(window * stride,
// L - 1) positions on each side in LDS (H small enough to fit).  Position p of
// the tile sits at ys[H + p]; its column (or kNoNode when it holds no node) at
// col[p].  The slot at offset o * stride lies in the same walk exactly when
// the column plus that offset stays in [0, L), and then it is ys[H + p + o s].
//
// Output word u of the tile holds slot u mod 2w of position u / 2w.  Each lane
// walks its words 256 apart, advancing (position, slot) by (256 / 2w,
// 256 mod 2w) with one carry instead of dividing per word.
__global__ __launch_bounds__(256) void k_contexts_lds(const int32_t* __restrict__ Y, uint64_t n_pos, uint32_t L,
                                                      uint32_t window, uint32_t stride, uint32_t H,
                                                      int32_t* __restrict__ C) {
  extern __shared__ int32_t sm[];
  int32_t* ys = sm;                                          // [kCtxTile + 2H]
  uint32_t* col = reinterpret_cast<uint32_t*>(sm + kCtxTile + 2 * H);  // [kCtxTile]
  const uint32_t W2 = 2u * window;
  const uint32_t dq = 256u / W2, dr = 256u - dq * W2;
  const uint32_t t = threadIdx.x;
  for (uint64_t e0 = (uint64_t)blockIdx.x * kCtxTile; e0 < n_pos; e0 += (uint64_t)gridDim.x * kCtxTile) {
    const uint32_t np = (uint32_t)(n_pos - e0 < kCtxTile ? n_pos - e0 : kCtxTile);
    const uint64_t row0 = e0 / L;
    const uint32_t i0 = (uint32_t)(e0 - row0 * L);
    __syncthreads();  // the previous tile's readers are done
    for (uint32_t x = t; x < np + 2 * H; x += 256) {
      const int64_t gpos = (int64_t)e0 - (int64_t)H + (int64_t)x;
      ys[x] = (gpos >= 0 && gpos < (int64_t)n_pos) ? Y[gpos] : -1;
    }
    __syncthreads();
    for (uint32_t p = t; p < np; p += 256) {
      uint64_t row;
      uint32_t i;
      split_pos(row0, i0, p, L, &row, &i);
      col[p] = ys[H + p] >= 0 ? i : kNoNode;
    }
    __syncthreads();
    const uint32_t words = np * W2;
    int32_t* __restrict__ out = C + e0 * W2;
    uint32_t pos = t / W2, slot = t - (t / W2) * W2;
    for (uint32_t u = t; u < words; u += 256) {
      const uint32_t c = col[pos];
      const int32_t o = (int32_t)slot - (int32_t)window + (slot >= window ? 1 : 0);
      const int64_t os = (int64_t)o * (int64_t)stride;
      const int64_t j = (int64_t)c + os;
      int32_t v = -1;
      // in the walk: |os| <= min(window * stride, L - 1) = H, so the index stays in the tile
      if (c != kNoNode && j >= 0 && j < (int64_t)L) v = ys[(int64_t)(H + pos) + os];
      out[u] = v;
      pos += dq;
      slot += dr;
      if (slot >= W2) {
        slot -= W2;
        ++pos;
      }
    }
  }
}

// Contexts for halos too wide for LDS: the same word order, slots gathered
// from global memory.
__global__ __launch_bounds__(256) void k_contexts_global(const int32_t* __restrict__ Y, uint64_t n_pos, uint32_t L,
                                                         uint32_t window, uint32_t stride, int32_t* __restrict__ C) {
  const uint32_t W2 = 2u * window;
  const uint32_t dq = 256u / W2, dr = 256u - dq * W2;
  const uint32_t t = threadIdx.x;
  for (uint64_t e0 = (uint64_t)blockIdx.x * 256; e0 < n_pos; e0 += (uint64_t)gridDim.x * 256) {
    const uint64_t np = n_pos - e0 < 256 ? n_pos - e0 : 256;
    const uint64_t row0 = e0 / L;
    const uint32_t i0 = (uint32_t)(e0 - row0 * L);
    const uint64_t words = np * W2;
    int32_t* __restrict__ out = C + e0 * W2;
    uint32_t pos = t / W2, slot = t - (t / W2) * W2;
    for (uint64_t u = t; u < words; u += 256) {
      uint64_t row;
      uint32_t i;
      split_pos(row0, i0, pos, L, &row, &i);
      const int32_t* __restrict__ y = Y + row * L;
      const int64_t o = slot < window ? (int64_t)slot - (int64_t)window : (int64_t)slot - (int64_t)window + 1;
      const int64_t j = (int64_t)i + o * (int64_t)stride;
      int32_t v = -1;
      if (j >= 0 && j < (int64_t)L && y[i] >= 0) v = y[j];
      out[u] = v;
      pos += dq;
      slot += dr;
      if (slot >= W2) {
        slot -= W2;
        ++pos;
      }
    }
  }
}

// Guide table of the degree-proportional draw (cut-point method, Chen and
// Asau 1974): with 2^s buckets of the 64-bit draw r, bucket b = r >> (64 - s)
// starts at T_b = floor((b << (64 - s)) * m / 2^64), and G[b] is the node whose
// offset interval [O[v], O[v+1]) holds T_b.  G[2^s] = n - 1 closes the table.
// When m < 2^32 the offsets are also copied to 32 bits (O32), halving the
// bytes the searches pull through the caches.
__global__ __launch_bounds__(256) void k_neg_guide(const uint64_t* __restrict__ O, int64_t n, uint32_t s,
                                                   int32_t* __restrict__ G, uint32_t* __restrict__ O32) {
  const uint64_t nb = 1ull << s;
  const uint64_t m = O[n];
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += step) {
    if (b == nb) {
      G[b] = (int32_t)(n - 1);
      continue;
    }
    const uint64_t T = scale_draw(b << (64 - s), m);
    int64_t lo = 0, hi = n;  // O[lo] <= T < O[hi]
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (O[mid] <= T) lo = mid;
      else hi = mid;
    }
    G[b] = (int32_t)lo;
  }
  if (O32)
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= (uint64_t)n; v += step)
      O32[v] = (uint32_t)O[v];
}

// The node v with O[v] <= T < O[v+1] for the draw r, T = floor(r m / 2^64).
// Draws of one bucket have T between T_b and T_{b+1}, so v lies in
// [G[b], G[b+1]]; a bucket that no offset boundary crosses (G[b] == G[b+1])
// needs no offset read at all.
template <typename OT>
__device__ __forceinline__ int32_t neg_draw(const OT* __restrict__ O, const int32_t* __restrict__ G, uint32_t s,
                                            uint64_t m, uint64_t r) {
  const uint64_t b = r >> (64 - s);
  int64_t lo = G[b], hi = (int64_t)G[b + 1] + 1;  // O[lo] <= T < O[hi]
  if (hi - lo > 1) {
    const uint64_t T = scale_draw(r, m);
    do {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if ((uint64_t)O[mid] <= T) lo = mid;
      else hi = mid;
    } while (hi - lo > 1);
  }
  return (int32_t)lo;
}

// A block owns P = 2^lgP consecutive walk positions (P n_neg words staged in
// LDS); item it of the tile is position it mod P, negative pair it / P, and
// one Philox block gives the pair's two 64-bit draws.  The staged tile then
// leaves in consecutive words.
template <typename OT>
__global__ __launch_bounds__(256) void k_negatives(const OT* __restrict__ O, uint64_t m,
                                                   const int32_t* __restrict__ G, uint32_t s,
                                                   const int32_t* __restrict__ Y, uint64_t n_pos, uint32_t L,
                                                   uint32_t n_neg, uint32_t lgP, uint64_t seed, uint64_t wid_base,
                                                   int32_t* __restrict__ N) {
  extern __shared__ int32_t sm[];  // [P * n_neg]
  const uint32_t P = 1u << lgP;
  const uint32_t npairs = (n_neg + 1u) / 2u;
  const uint32_t t = threadIdx.x;
  for (uint64_t e0 = (uint64_t)blockIdx.x * P; e0 < n_pos; e0 += (uint64_t)gridDim.x * P) {
    const uint32_t np = (uint32_t)(n_pos - e0 < P ? n_pos - e0 : P);
    const uint64_t row0 = e0 / L;
    const uint32_t i0 = (uint32_t)(e0 - row0 * L);
    __syncthreads();  // the previous tile's readers are done
    for (uint32_t it = t; it < P * npairs; it += 256) {
      const uint32_t pos = it & (P - 1u), jp = it >> lgP;
      if (pos >= np) continue;
      int32_t v0 = -1, v1 = -1;
      if (m > 0 && Y[e0 + pos] >= 0) {
        uint64_t row;
        uint32_t i;
        split_pos(row0, i0, pos, L, &row, &i);
        const uint64_t wid = wid_base + row;
        uint32_t w[4];
        philox_words(seed, i, (uint32_t)wid, (uint32_t)(wid >> 32), 0x80000000u + jp, w);
        v0 = neg_draw(O, G, s, m, (uint64_t)w[0] | ((uint64_t)w[1] << 32));
        if (2u * jp + 1u < n_neg) v1 = neg_draw(O, G, s, m, (uint64_t)w[2] | ((uint64_t)w[3] << 32));
      }
      sm[pos * n_neg + 2u * jp] = v0;
      if (2u * jp + 1u < n_neg) sm[pos * n_neg + 2u * jp + 1u] = v1;
    }
    __syncthreads();
    int32_t* __restrict__ out = N + e0 * n_neg;
    for (uint32_t x = t; x < np * n_neg; x += 256) out[x] = sm[x];
  }
}

int stream_blocks(uint64_t tiles, const DevInfo& di) {
  const uint64_t cap = (uint64_t)(di.cus > 0 ? di.cus : 256) * 32;
  return (int)(tiles < cap ? (tiles ? tiles : 1) : cap);
}

constexpr size_t kCorpusLdsBytes = 64 * 1024;

}  // namespace

uint32_t neg_guide_shift(int64_t n) {
  int s = 1;
  while (s < (int)kNegGuideMaxShift && (1ll << s) < n) ++s;
  s += kNegGuideShiftAdjust;
  return s < 1 ? 1u : (s > (int)kNegGuideMaxShift ? kNegGuideMaxShift : (uint32_t)s);
}

size_t neg_guide_bytes(uint32_t shift, int64_t n, uint64_t m) {
  size_t b = ((1ull << shift) + 1) * sizeof(int32_t);
  if (m < (1ull << 32)) b += ((size_t)n + 1) * sizeof(uint32_t);
  return b;
}

hipError_t launch_contexts(const int32_t* Y, uint64_t n_walks, uint32_t L, uint32_t window, uint32_t stride,
                           int32_t* C, const DevInfo& di, hipStream_t st) {
  const uint64_t n_pos = n_walks * L;
  if (n_pos == 0) return hipSuccess;
  const uint64_t reach = (uint64_t)window * stride;
  const uint64_t H = reach < (uint64_t)L - 1 ? reach : (uint64_t)L - 1;
  const size_t lds = (2 * (size_t)kCtxTile + 2 * H) * sizeof(int32_t);
  if (lds <= kCorpusLdsBytes) {
    hipLaunchKernelGGL(k_contexts_lds, dim3(stream_blocks((n_pos + kCtxTile - 1) / kCtxTile, di)), dim3(256), lds,
                       st, Y, n_pos, L, window, stride, (uint32_t)H, C);
  } else {
    hipLaunchKernelGGL(k_contexts_global, dim3(stream_blocks((n_pos + 255) / 256, di)), dim3(256), 0, st, Y, n_pos,
                       L, window, stride, C);
  }
  return hipGetLastError();
}

// The guide buffer holds G (2^shift + 1 int32) and, when m < 2^32, O32 (n + 1
// uint32) right after it.
static uint32_t* guide_o32(const GraphDev& g, int32_t* guide, uint32_t shift) {
  return g.m < (1ull << 32) ? reinterpret_cast<uint32_t*>(guide + (1ull << shift) + 1) : nullptr;
}

hipError_t launch_neg_guide(const GraphDev& g, int32_t* guide, uint32_t shift, const DevInfo& di, hipStream_t st) {
  const uint64_t items = ((1ull << shift) + 1) > (uint64_t)g.n + 1 ? ((1ull << shift) + 1) : (uint64_t)g.n + 1;
  hipLaunchKernelGGL(k_neg_guide, dim3(stream_blocks((items + 255) / 256, di)), dim3(256), 0, st, g.O, g.n, shift,
                     guide, guide_o32(g, guide, shift));
  return hipGetLastError();
}

hipError_t launch_negatives(const GraphDev& g, const int32_t* guide, uint32_t shift, const int32_t* Y,
                            uint64_t n_walks, uint32_t L, uint32_t n_neg, uint64_t seed, uint64_t wid_base,
                            int32_t* N, const DevInfo& di, hipStream_t st) {
  const uint64_t n_pos = n_walks * L;
  if (n_pos == 0) return hipSuccess;
  if ((size_t)n_neg * sizeof(int32_t) > kCorpusLdsBytes) return hipErrorInvalidValue;
  uint32_t lgP = 8;  // 256 positions per tile while P n_neg words fit the LDS budget
  while (lgP > 0 && ((size_t)n_neg << lgP) * sizeof(int32_t) > kCorpusLdsBytes) --lgP;
  const size_t lds = ((size_t)n_neg << lgP) * sizeof(int32_t);
  const dim3 grid(stream_blocks((n_pos + (1u << lgP) - 1) >> lgP, di));
  const uint32_t* o32 = guide ? guide_o32(g, const_cast<int32_t*>(guide), shift) : nullptr;
  if (o32)
    hipLaunchKernelGGL(k_negatives<uint32_t>, grid, dim3(256), lds, st, o32, g.m, guide, shift, Y, n_pos, L, n_neg,
                       lgP, seed, wid_base, N);
  else
    hipLaunchKernelGGL(k_negatives<uint64_t>, grid, dim3(256), lds, st, g.O, g.m, guide, shift, Y, n_pos, L, n_neg,
                       lgP, seed, wid_base, N);
  return hipGetLastError();
}

}  // namespace n2v
