// Walk kernels for gfx950 (wave64).
//
// Every kernel computes the same walk, defined in the paper's Methods, "First
// and second-order RW-based embedding methods": the un-normalised weight of
// candidate x in N(v) is pi_vx = alpha(t,x) * w_vx with alpha = 1/p (x == t),
// 1 (x in N(t)), 1/q (otherwise) (Eq. 1; the in-out / return split of Eq. 2-3
// and its set-difference and binary-search reformulations), and the next node
// is drawn on the fly ("Efficient sampling for Node2Vec RWs", steps 1-4):
// biased weights, cumulative sum, uniform value in [0, total), first index
// whose cumulative sum exceeds it.  The paper's eight specialised variants
// (weighted? x p == 1? x q == 1?) become the kernel families below; they are
// bit-identical because a common positive factor on every weight never
// changes the selected index:  B c > floor(r c S / 2^64)  <=>  B > floor(r S / 2^64)
// for integers B, c, S.
//
//  * k_walk_lane   one lane per walker, O(log d) per step:
//      - first order, unweighted: j = floor(r d / 2^64)
//      - first order, weighted:   first j with R_j > floor(r S_v / 2^64), R = row prefix
//      - node2vec with 1/q == 1:  only x == t is re-weighted, so
//        B_j = C16 R_j + (P16 - C16) w_t [j >= pos(t)]  (mod 2^64, exact since
//        B_j < 2^64), searched by bisection; pos(t) by bisection for t in N(v).
//  * k_walk_group  G lanes per walker (node2vec with 1/q != 1): the row of v is
//      streamed in chunks of G candidates; each candidate is classified
//      return / common / far against N(t), which sits in LDS when the previous
//      row was short enough to stage (ping-pong buffers), else is probed in
//      global memory; uint64 group reductions give block sums, and a second
//      pass over a single block finds the selected index with a group scan and
//      a ballot.
#include "n2v_device.hpp"
#include "n2v_internal.hpp"

#include <map>
#include <mutex>
#include <utility>

namespace n2v {

namespace {

enum { kFoUnw = 0, kFoW = 1, kRetUnw = 2, kRetW = 3 };

template <int MODE, typename RT>
__global__ __launch_bounds__(256) void k_walk_lane(WalkArgs a) {
  const uint64_t* __restrict__ O = a.g.O;
  const int32_t* __restrict__ D = a.g.D;
  const uint32_t* __restrict__ W = a.g.W;
  const RT* __restrict__ R = (const RT*)a.g.R;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nwalks; w += stride) {
    int32_t* __restrict__ row = a.Y + w * a.L;
    const int32_t start = a.starts[w % a.ns];
    const uint64_t wid = a.wid_base + w;
    uint32_t len = 0;
    if (start >= 0 && (int64_t)start < a.g.n) {
      row[0] = start;
      len = 1;
      int32_t v = start, t = -1;
      for (uint32_t s = 1; s < a.L; ++s) {
        const uint64_t lo = O[v];
        const uint32_t d = (uint32_t)(O[v + 1] - lo);
        if (d == 0) break;  // dead end
        const uint64_t r = philox_draw(a.seed, s, wid);
        uint32_t j;
        if (MODE == kFoUnw || (MODE == kRetUnw && t < 0)) {
          j = (uint32_t)scale_draw(r, d);
        } else if (MODE == kFoW || (MODE == kRetW && t < 0)) {
          const uint64_t total = (uint64_t)R[lo + d - 1];
          if (total == 0) break;  // every candidate has weight zero
          j = upper_bound_gt(R + lo, d, scale_draw(r, total));
        } else {
          const uint32_t pt = lower_bound_i32(D + lo, d, t);
          const bool has_t = pt < d && D[lo + pt] == t;
          uint64_t wt = 0;
          if (has_t) wt = (MODE == kRetW) ? (uint64_t)W[lo + pt] : 1ull;
          const uint64_t S = (MODE == kRetW) ? (uint64_t)R[lo + d - 1] : (uint64_t)d;
          const uint64_t corr = ((uint64_t)a.P16 - (uint64_t)kC16) * wt;  // mod 2^64
          const uint64_t total = (uint64_t)kC16 * S + corr;
          if (total == 0) break;
          const uint64_t T = scale_draw(r, total);
          uint32_t jl = 0, jh = d - 1;
          while (jl < jh) {
            const uint32_t mid = jl + ((jh - jl) >> 1);
            const uint64_t Rm = (MODE == kRetW) ? (uint64_t)R[lo + mid] : (uint64_t)(mid + 1);
            const uint64_t Bm = (uint64_t)kC16 * Rm + (mid >= pt ? corr : 0ull);
            if (Bm > T) jh = mid;
            else jl = mid + 1;
          }
          j = jl;
        }
        const int32_t x = D[lo + j];
        row[s] = x;
        len = s + 1;
        t = v;
        v = x;
      }
    }
    for (uint32_t s = len; s < a.L; ++s) row[s] = -1;
    if (a.lens) a.lens[w] = (int32_t)len;
  }
}

__device__ __forceinline__ bool lds_contains(const int32_t* A, uint32_t n, int32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (A[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && A[lo] == x;
}

__device__ __forceinline__ bool global_contains(const int32_t* __restrict__ A, uint32_t n, int32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (A[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && A[lo] == x;
}

template <int G, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_walk_group(WalkArgs a, int tile) {
  extern __shared__ int32_t lds[];
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const int gib = threadIdx.x / G;
  const int gpb = blockDim.x / G;
  int32_t* const bufA = lds + (size_t)gib * 2 * tile;
  int32_t* const bufB = bufA + tile;
  const uint64_t ngroups = (uint64_t)gridDim.x * gpb;
  const uint64_t* __restrict__ O = a.g.O;
  const int32_t* __restrict__ D = a.g.D;
  const uint32_t* __restrict__ W = a.g.W;

  for (uint64_t w = (uint64_t)blockIdx.x * gpb + gib; w < a.nwalks; w += ngroups) {
    int32_t* __restrict__ row = a.Y + w * a.L;
    const int32_t start = a.starts[w % a.ns];
    const uint64_t wid = a.wid_base + w;
    uint32_t len = 0;
    int32_t ob = -1;  // output window: this lane holds slot s0 + gl
    uint32_t s0 = 0;
    if (start >= 0 && (int64_t)start < a.g.n) {
      if (gl == 0) ob = start;
      len = 1;
      int32_t v = start, t = -1;
      uint64_t tlo = 0;
      uint32_t td = 0;
      bool t_in_lds = false;
      int32_t* cur = bufA;  // N(t) when staged
      int32_t* nxt = bufB;  // N(v) being staged
      for (uint32_t s = 1; s < a.L; ++s) {
        const uint64_t lo = O[v];
        const uint32_t d = (uint32_t)(O[v + 1] - lo);
        if (d == 0) break;
        const bool second = a.second_order && t >= 0;
        const bool stage = d <= (uint32_t)tile;
        const uint32_t nc = (d + G - 1) / G;   // chunks of G candidates
        const uint32_t bs = (nc + G - 1) / G;  // chunks per block (at most G blocks)

        auto alpha = [&](int32_t x) -> uint64_t {
          if (!second) return 1ull;
          if (x == t) return (uint64_t)a.P16;
          const bool common = t_in_lds ? lds_contains(cur, td, x) : global_contains(D + tlo, td, x);
          return common ? (uint64_t)kC16 : (uint64_t)a.Q16;
        };

        // Pass 1: block sums of the biased weights; lane k keeps block k.
        uint64_t acc = 0, blk = 0;
        for (uint32_t c = 0; c < nc; ++c) {
          const uint32_t j = c * G + gl;
          if (j < d) {
            const int32_t x = D[lo + j];
            if (stage) nxt[j] = x;
            const uint64_t wt = WEIGHTED ? (uint64_t)W[lo + j] : 1ull;
            acc += wt * alpha(x);
          }
          if ((c + 1) % bs == 0 || c + 1 == nc) {
            const uint64_t sb = grp_sum<G>(acc);
            if ((uint32_t)gl == c / bs) blk = sb;
            acc = 0;
          }
        }
        const uint64_t incl = grp_incl_scan<G>(blk, gl);
        const uint64_t total = grp_bcast<G>(incl, G - 1);
        if (total == 0) break;
        const uint64_t T = scale_draw(philox_draw(a.seed, s, wid), total);
        const uint64_t bm = grp_ballot<G>(incl > T, gbase);
        const int kb = __ffsll((unsigned long long)bm) - 1;
        uint64_t base = grp_bcast<G>(incl - blk, kb);

        // Pass 2: rescan block kb only.
        int32_t xsel = -1;
        const uint32_t cend = min((uint32_t)(kb + 1) * bs, nc);
        for (uint32_t c = (uint32_t)kb * bs; c < cend; ++c) {
          const uint32_t j = c * G + gl;
          uint64_t b = 0;
          int32_t x = -1;
          if (j < d) {
            x = stage ? nxt[j] : D[lo + j];
            const uint64_t wt = WEIGHTED ? (uint64_t)W[lo + j] : 1ull;
            b = wt * alpha(x);
          }
          const uint64_t inc = grp_incl_scan<G>(b, gl);
          const uint64_t m2 = grp_ballot<G>(base + inc > T, gbase);
          if (m2) {
            xsel = grp_bcast_i32<G>(x, __ffsll((unsigned long long)m2) - 1);
            break;
          }
          base += grp_bcast<G>(inc, G - 1);
        }
        if (xsel < 0) break;  // unreachable: block kb's prefix exceeds T

        if ((uint32_t)gl == s % G) ob = xsel;
        if (s % G == G - 1) {
          row[s0 + gl] = ob;
          s0 += G;
          ob = -1;
        }
        len = s + 1;
        t = v;
        tlo = lo;
        td = d;
        t_in_lds = stage;
        int32_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
        v = xsel;
        // the staged row is read by other lanes of the group at the next step
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    for (uint32_t s = s0; s < a.L; s += G) {
      const uint32_t idx = s + gl;
      if (idx < a.L) row[idx] = (s == s0 && idx < len) ? ob : -1;
    }
    if (a.lens && gl == 0) a.lens[w] = (int32_t)len;
  }
}

// Grid size: enough blocks to fill every CU at the kernel's occupancy, never
// more than the work needs (the kernels loop over walkers).
template <typename K>
int grid_for(K kernel, size_t lds_bytes, uint64_t work_blocks, const DevInfo& di) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair((const void*)kernel, lds_bytes);
    auto it = cache.find(key);
    if (it != cache.end()) {
      per_cu = it->second;
    } else {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds_bytes) != hipSuccess ||
          per_cu < 1)
        per_cu = 1;
      cache[key] = per_cu;
    }
  }
  uint64_t full = (uint64_t)per_cu * (uint64_t)(di.cus > 0 ? di.cus : 256);
  uint64_t g = work_blocks < full ? work_blocks : full;
  return (int)(g < 1 ? 1 : g);
}

template <int MODE, typename RT>
hipError_t go_lane(const WalkArgs& a, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  auto k = k_walk_lane<MODE, RT>;
  int blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : grid_for(k, 0, (a.nwalks + 255) / 256, di);
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int G, bool WEIGHTED>
hipError_t go_group(const WalkArgs& a, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  auto k = k_walk_group<G, WEIGHTED>;
  const int gpb = 256 / G;
  const size_t lds = (size_t)gpb * 2 * (size_t)cfg.lds_tile * sizeof(int32_t);
  int blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : grid_for(k, lds, (a.nwalks + gpb - 1) / gpb, di);
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, st, a, cfg.lds_tile);
  return hipGetLastError();
}

template <bool WEIGHTED>
hipError_t go_group_g(const WalkArgs& a, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  switch (cfg.lanes_per_walker) {
    case 4: return go_group<4, WEIGHTED>(a, cfg, di, st);
    case 8: return go_group<8, WEIGHTED>(a, cfg, di, st);
    case 16: return go_group<16, WEIGHTED>(a, cfg, di, st);
    case 32: return go_group<32, WEIGHTED>(a, cfg, di, st);
    default: return go_group<64, WEIGHTED>(a, cfg, di, st);
  }
}

}  // namespace

hipError_t launch_walks(const WalkArgs& a, Path path, const LaunchCfg& cfg, const DevInfo& di,
                        hipStream_t st) {
  if (a.nwalks == 0) return hipSuccess;
  const bool weighted = a.g.W != nullptr;
  const bool r64 = a.g.r_bytes == 8;
  switch (path) {
    case Path::kFirstOrder:
      if (!weighted) return go_lane<kFoUnw, uint32_t>(a, cfg, di, st);
      return r64 ? go_lane<kFoW, uint64_t>(a, cfg, di, st) : go_lane<kFoW, uint32_t>(a, cfg, di, st);
    case Path::kReturnOnly:
      if (!weighted) return go_lane<kRetUnw, uint32_t>(a, cfg, di, st);
      return r64 ? go_lane<kRetW, uint64_t>(a, cfg, di, st) : go_lane<kRetW, uint32_t>(a, cfg, di, st);
    default:
      return weighted ? go_group_g<true>(a, cfg, di, st) : go_group_g<false>(a, cfg, di, st);
  }
}

}  // namespace n2v
