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
//  * k_walk_n2v    G lanes per walker (node2vec with 1/q != 1).  With R the row
//      prefix of v, a special list C of the positions of common neighbours
//      (x in N(t), x != t; the in-out bias is 1 exactly there, Eq. 3 and the
//      set difference N(v) minus N(t) that follows it) and the position pt of
//      t (return bias), the cumulative sum is
//        B_j = Q16 R_j + (C16 - Q16) sum_{c in C, c <= j} w_c + (P16 - Q16) w_t [j >= pt]
//      (mod 2^64; exact because the true B_j < 2^64).  C is built by the
//      cheapest (by a latency estimate) of three equivalent routes: probe
//      every y in N(t) into N(v) by bisection (short N(t), long N(v): the
//      typical leaf-to-hub step), stream N(v) and test each x against N(t)
//      (kept in LDS when the previous row fit a ping-pong tile, else bisected
//      in global memory), or merge both rows, a window of N(t) at a time in
//      LDS.  The draw is then located by a ballot over B at the listed
//      positions and a G-ary search of the segment between two of them.  C is
//      kept in LDS one page at a time: the first pass counts every common
//      neighbour (so the total is exact) and stores the first page; later
//      pages are listed only if the draw lands beyond the stored ones.  A
//      two-pass stream of the biased weights (block sums, then a scan of one
//      block) remains as a route that can be forced for testing.
//
// Walks are handed to groups (lanes, for k_walk_lane) from a per-stream
// device counter, a few at a time, so that heavy-tailed walk costs do not
// leave a launch waiting on its slowest fixed share.
#include "n2v_device.hpp"
#include "n2v_internal.hpp"

#include <cstddef>
#include <map>
#include <mutex>
#include <utility>

namespace n2v {

namespace {

enum { kFoUnw = 0, kFoW = 1, kRetUnw = 2, kRetW = 3 };

// Output rows leave in whole 64-byte lines: a slot is staged until the slot
// that ends its line (by address) is drawn, then the line is stored at once; a
// line written piecemeal costs one write per piece once the random reads of
// the walk have pushed it out of the cache.  Only the row's first and last
// lines can be partial.

// One whole walk (row w of request a) by one lane.  `st` is the lane's output
// stage in LDS: slot k of the current line at st[64 * k].
template <int MODE, typename RT>
__device__ __forceinline__ void lane_walk(const WalkArgs& a, uint64_t w, int32_t* st) {
  const uint64_t* __restrict__ O = a.g.O;
  const int32_t* __restrict__ D = a.g.D;
  const RT* __restrict__ R = (const RT*)a.g.R;
  {
    int32_t* __restrict__ row = a.Y + w * a.L;
    const int32_t start = a.starts[w % a.ns];
    const uint64_t wid = a.wid_base + w;
    uint32_t len = 0;
    // slot of row position 0 within its line; every line before the one
    // holding position s has been stored once s is staged
    const uint32_t roff = (uint32_t)(((uintptr_t)row >> 2) & (kOutStage - 1));
    auto put = [&](uint32_t s, int32_t x) {
      const uint32_t k = (roff + s) & (kOutStage - 1);
      st[64 * k] = x;
      if (k == kOutStage - 1) {
        if (s >= kOutStage - 1) {
          int4* __restrict__ dst = (int4*)(row + (s - (kOutStage - 1)));
#pragma unroll
          for (uint32_t q = 0; q < kOutStage / 4; ++q)
            dst[q] = make_int4(st[64 * (4 * q)], st[64 * (4 * q + 1)], st[64 * (4 * q + 2)], st[64 * (4 * q + 3)]);
        } else {
          for (uint32_t p = 0; p <= s; ++p) row[p] = st[64 * ((roff + p) & (kOutStage - 1))];
        }
      }
    };
    if (start >= 0 && (int64_t)start < a.g.n) {
      put(0, start);
      len = 1;
      int32_t v = start, t = -1;
      uint64_t epos = 0;  // position of the edge t -> v in the entries
      for (uint32_t s = 1; s < a.L; ++s) {
        uint64_t lo;
        uint32_t d;
        uint64_t rowsum = 0;  // S_v from the node record when there is one
        constexpr bool kRec = (MODE == kFoW || MODE == kRetW) && sizeof(RT) == 4;
        if (kRec && a.g.NR) {
          const uint4 rec = a.g.NR[v];
          lo = (uint64_t)rec.x | ((uint64_t)rec.y << 32);
          d = rec.z;
          rowsum = rec.w;
        } else {
          lo = O[v];
          d = (uint32_t)(O[v + 1] - lo);
        }
        if (d == 0) break;  // dead end
        const uint64_t r = philox_draw(a.seed, s, wid);
        uint32_t j;
        if (MODE == kFoUnw || (MODE == kRetUnw && t < 0)) {
          j = (uint32_t)scale_draw(r, d);
        } else if (MODE == kFoW || (MODE == kRetW && t < 0)) {
          const uint64_t total = (kRec && a.g.NR) ? rowsum : (uint64_t)R[lo + d - 1];
          if (total == 0) break;  // every candidate has weight zero
          j = upper_bound_interp(R + lo, d, scale_draw(r, total), total);
        } else {
          uint32_t pt;
          uint64_t wt = 0;
          if (kRec && MODE == kRetW && a.g.pair_info != nullptr) {
            // the 32-byte record of the edge t -> v (built at upload for every
            // edge) holds t's position in N(v), all ones when t is not a
            // neighbour of v, and t's weight there (0): read beside the node
            // record instead of a search of N(v) for t
            pt = a.g.pair_info[2 * epos].z;
            wt = a.g.pair_info[2 * epos + 1].x;
          } else {
            int32_t vt;
            pt = floor_search(D + lo, 0u, d, D[lo], t, vt);
            if (vt == t) wt = (MODE == kRetW) ? (uint64_t)a.g.W[lo + pt] : 1ull;
          }
          const uint64_t S =
              (MODE == kRetW) ? ((kRec && a.g.NR) ? rowsum : (uint64_t)R[lo + d - 1]) : (uint64_t)d;
          const uint64_t corr = ((uint64_t)a.P16 - (uint64_t)kC16) * wt;  // mod 2^64
          const uint64_t total = (uint64_t)kC16 * S + corr;
          if (total == 0) break;
          const uint64_t T = scale_draw(r, total);
          // B_m = C16 R_m (+ corr from t's position on): the row prefix scaled
          // and shifted at one position, searched like the first-order prefix
          j = first_above_interp(d, T, total, [&](uint32_t m) -> uint64_t {
            const uint64_t Rm = (MODE == kRetW) ? (uint64_t)R[lo + m] : (uint64_t)(m + 1);
            return (uint64_t)kC16 * Rm + (m >= pt ? corr : 0ull);
          });
        }
        const int32_t x = D[lo + j];
        put(s, x);
        len = s + 1;
        t = v;
        v = x;
        epos = lo + j;
      }
    }
    // staged slots [s0, len) (the start of len's line, or 0), then the padding
    const uint32_t lk = (roff + len) & (kOutStage - 1);
    const uint32_t s0 = len > lk ? len - lk : 0u;
    for (uint32_t p = s0; p < a.L; ++p) row[p] = p < len ? st[64 * ((roff + p) & (kOutStage - 1))] : -1;
    if (a.lens) a.lens[w] = (int32_t)len;
    if (a.steps && len > 1) atomicAdd(a.steps, (unsigned long long)(len - 1));
  }
}

template <int MODE, typename RT>
__global__ __launch_bounds__(256) void k_walk_lane(WalkArgs a, unsigned long long* ctr, uint32_t chunk) {
  __shared__ int32_t stage[256 * kOutStage];
  int32_t* const st = stage + (threadIdx.x / 64u) * (64u * kOutStage) + (threadIdx.x & 63u);
  if (ctr) {
    // a wave takes 64 * chunk walks at a time from the launch counter
    const int lane = threadIdx.x & 63;
    const uint64_t span = 64ull * chunk;
    while (true) {
      unsigned long long c = 0;
      if (lane == 0) c = atomicAdd(ctr, (unsigned long long)span);
      const uint64_t base = wave_read_u64((uint64_t)c, 0);
      if (base >= a.nwalks) break;
      const uint64_t end = min(base + span, a.nwalks);
      for (uint64_t w = base + lane; w < end; w += 64) lane_walk<MODE, RT>(a, w, st);
    }
    return;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nwalks; w += stride)
    lane_walk<MODE, RT>(a, w, st);
}

__device__ __forceinline__ bool lds_contains(const int32_t* A, uint32_t n, int32_t x) {
  if (n == 0) return false;
  int32_t val;
  floor_search(A, 0u, n, A[0], x, val);
  return val == x;
}

__device__ __forceinline__ bool global_contains(const int32_t* __restrict__ A, uint32_t n, int32_t x) {
  if (n == 0) return false;
  int32_t val;
  floor_search(A, 0u, n, A[0], x, val);
  return val == x;
}

// ---------------------------------------------------------------------------
// node2vec kernel: G lanes per walker.
// ---------------------------------------------------------------------------
enum { kModeAuto = 0, kModeTwoPass = 1, kModeProbe = 2, kModeStream = 3, kModeMerge = 4, kModeHubSets = 5,
       kModeSetProbe = 6, kModeSetStream = 7 };

// Membership of node y in a hub set (one bit, one word of the line).
__device__ __forceinline__ bool set_member(const uint32_t* __restrict__ set, uint32_t y) {
  const uint32_t line = y / kHubLineIds, b = y - line * kHubLineIds;
  return (set[(uint64_t)line * 16u + (b >> 5)] >> (b & 31u)) & 1u;
}

// Membership of y in a hub set and, when it is a member, its position in the
// hub's row: the members before it are the line's count word plus the bits
// below y in the line (one 64-byte line read).
__device__ __forceinline__ bool set_rank(const uint32_t* __restrict__ set, uint32_t y, uint32_t& pos) {
  const uint32_t line = y / kHubLineIds, b = y - line * kHubLineIds;
  const uint4* __restrict__ q = (const uint4*)(set + (uint64_t)line * 16u);
  const uint4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  const uint32_t w[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                          q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
  const uint32_t wi = b >> 5, bit = b & 31u;
  uint32_t cnt = w[15], word = 0;
#pragma unroll
  for (uint32_t k = 0; k < 15; ++k) {
    cnt += k < wi ? (uint32_t)__popc(w[k]) : 0u;
    word = k == wi ? w[k] : word;
  }
  pos = cnt + (uint32_t)__popc(word & ((1u << bit) - 1u));
  return (word >> bit) & 1u;
}


__device__ __forceinline__ uint32_t ceil_log2p1(uint32_t x) {  // ceil(log2(x + 1))
  return 32u - (uint32_t)__clz(x);
}

// First j in [lo, hi) with pred(j) (pred monotone in j); hi if none.  Group
// cooperative: each round the G lanes probe G evenly spaced points.
template <int G, typename P>
__device__ __forceinline__ uint32_t gary_first(uint32_t lo, uint32_t hi, int gl, int gbase, P pred) {
  while (hi - lo > (uint32_t)G) {
    const uint32_t step = (hi - lo + G - 1) / G;
    const uint32_t j = lo + (uint32_t)(gl + 1) * step - 1;
    const bool real = j < hi;
    const bool pr = real ? pred(j) : true;
    const uint64_t m = grp_ballot<G>(pr, gbase);
    if (m == 0) return hi;  // lane G-1 probed hi - 1 and it is false
    const int f = __ffsll((unsigned long long)m) - 1;
    const uint32_t jf = (uint32_t)grp_bcast_i32<G>((int32_t)j, f);
    lo = lo + (uint32_t)f * step;  // every probe below lane f is false
    if (jf < hi) hi = jf;          // the probe of lane f is true
  }
  const uint32_t j = lo + (uint32_t)gl;
  const bool pr = j < hi && pred(j);
  const uint64_t m = grp_ballot<G>(pr, gbase);
  return m ? lo + (uint32_t)(__ffsll((unsigned long long)m) - 1) : hi;
}

// gary_first that also reads the destination row X[j] in its final round, so
// that the chosen candidate's destination comes with the search; xok is false
// when no index in [lo, hi) satisfies pred (then the caller reads it).
template <int G, typename P>
__device__ __forceinline__ uint32_t gary_first_x(uint32_t lo, uint32_t hi, int gl, int gbase, P pred,
                                                 const int32_t* __restrict__ X, int32_t& xo, bool& xok) {
  while (hi - lo > (uint32_t)G) {
    const uint32_t step = (hi - lo + G - 1) / G;
    const uint32_t j = lo + (uint32_t)(gl + 1) * step - 1;
    const bool real = j < hi;
    const bool pr = real ? pred(j) : true;
    const uint64_t m = grp_ballot<G>(pr, gbase);
    if (m == 0) {
      xok = false;
      return hi;
    }
    const int f = __ffsll((unsigned long long)m) - 1;
    const uint32_t jf = (uint32_t)grp_bcast_i32<G>((int32_t)j, f);
    lo = lo + (uint32_t)f * step;
    if (jf < hi) hi = jf;
  }
  const uint32_t j = lo + (uint32_t)gl;
  bool pr = false;
  int32_t xv = 0;
  if (j < hi) {
    pr = pred(j);
    xv = X[j];
  }
  const uint64_t m = grp_ballot<G>(pr, gbase);
  xok = m != 0;
  if (!xok) return hi;
  const int f = __ffsll((unsigned long long)m) - 1;
  xo = grp_bcast_i32<G>(xv, f);
  return lo + (uint32_t)f;
}

// First k in [0, nc) whose stored list entry satisfies pred (monotone in k),
// or nc, by G-ary rounds; the final round's window starts one entry early, so
// the entries at k and k - 1 (when they exist) come with it: ek = entry k
// (k < nc), ekm = entry k - 1 (k > 0).
template <int G, typename P>
__device__ __forceinline__ uint32_t list_search(const uint4* __restrict__ ent, uint32_t nc, int gl, int gbase, P pred,
                                                uint4& ek, uint4& ekm) {
  uint32_t lo = 0, hi = nc;
  while (hi - lo > (uint32_t)G - 2u) {
    const uint32_t step = (hi - lo + G - 1) / G;
    const uint32_t j = lo + (uint32_t)(gl + 1) * step - 1;
    const bool pr = j < hi ? pred(ent[j]) : true;
    const uint64_t m = grp_ballot<G>(pr, gbase);
    if (m == 0) {  // every probe false, the last one at hi - 1: the answer is hi
      lo = hi;
      break;
    }
    const int f = __ffsll((unsigned long long)m) - 1;
    const uint32_t jf = (uint32_t)grp_bcast_i32<G>((int32_t)j, f);
    lo = lo + (uint32_t)f * step;
    if (jf < hi) hi = jf;
  }
  // window [b, b + G) holds lo - 1 .. hi (hi - lo <= G - 2); hi is true or nc
  const uint32_t b = lo > 0 ? lo - 1 : 0u;
  const uint32_t j = b + (uint32_t)gl;
  uint4 en = make_uint4(0u, 0u, 0u, 0u);
  if (j < nc) en = ent[j];
  const bool pr = j >= lo && j < hi && pred(en);
  const uint64_t m = grp_ballot<G>(pr, gbase);
  const uint32_t k = m ? b + (uint32_t)(__ffsll((unsigned long long)m) - 1) : hi;
  auto take = [&](uint32_t lane_idx) {
    uint4 r;
    r.x = (uint32_t)grp_bcast_i32<G>((int32_t)en.x, (int)lane_idx);
    r.y = (uint32_t)grp_bcast_i32<G>((int32_t)en.y, (int)lane_idx);
    r.z = (uint32_t)grp_bcast_i32<G>((int32_t)en.z, (int)lane_idx);
    r.w = 0u;
    return r;
  };
  if (k < nc) ek = take(k - b);
  if (k > 0) ekm = take(k - 1 - b);
  return k;
}

// gary_first over a row of a prefix array V (positions lo + j) with a
// predicate on (V[lo + j], j), monotone in j, through the row's heads
// H[b] = V[32 b]: a long range first searches the heads of its whole 32-entry
// blocks (contiguous: a few lines instead of one line per probe), then the
// at most 32 entries between the last false head and the first true one.
//
// X, when given, is the row's destination array (X[j] = D[lo + j]): the
// destination of the answer is returned in xo (xok true) from the final round.
template <int G, typename RT, typename P>
__device__ __forceinline__ uint32_t gary_first_heads(const RT* __restrict__ V, const RT* __restrict__ H, uint64_t lo,
                                                     uint32_t jlo, uint32_t jhi, int gl, int gbase, P pred,
                                                     const int32_t* __restrict__ X, int32_t& xo, bool& xok) {
  auto direct = [&](uint32_t j) { return pred((uint64_t)V[lo + j], j); };
  // a range of more than 64 entries holds at least two heads
  if (H == nullptr || jhi - jlo <= 64u || jhi - jlo <= 2u * G) return gary_first_x<G>(jlo, jhi, gl, gbase, direct, X, xo, xok);
  const uint64_t a = lo + jlo, e = lo + jhi;
  const uint64_t hb0 = (a + 31) >> 5, hb1 = (e - 1) >> 5;  // blocks whose head lies in [a, e)
  const uint32_t nh = (uint32_t)(hb1 - hb0 + 1);
  const uint32_t k = gary_first<G>(0u, nh, gl, gbase, [&](uint32_t i) {
    return pred((uint64_t)H[hb0 + i], (uint32_t)(((hb0 + i) << 5) - lo));
  });
  uint64_t sb, se;  // the answer is the first true position in [sb, se), or none (jhi)
  if (k == 0) {
    sb = a;
    se = (hb0 << 5) + 1;
  } else if (k == nh) {
    sb = (hb1 << 5) + 1;
    se = e;
  } else {
    sb = ((hb0 + k - 1) << 5) + 1;
    se = ((hb0 + k) << 5) + 1;
  }
  return gary_first_x<G>((uint32_t)(sb - lo), (uint32_t)(se - lo), gl, gbase, direct, X, xo, xok);
}

// Splitters of a long sorted row A[0..n) (n >= 4G): the group loads A[l n / G]
// for its G lanes into LDS (one coalesced round), and every lane can then
// bisect a key among the splitters in LDS and the key's 1/G slice of A in
// global memory.  spl must hold G entries.
template <int G>
__device__ __forceinline__ void load_splitters(const int32_t* __restrict__ A, uint32_t n, int32_t* spl, int gl) {
  spl[gl] = A[(uint32_t)(((uint64_t)gl * n) / G)];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Floor search of y in the row D[P, P + n) (n >= G) that starts from the
// slice between the splitters around y: the splitter below y is the slice's
// first entry, so its value comes from LDS.  A slice longer than 1024 entries
// continues through its heads HD[i] = D[32 i] (contiguous, a few lines) and
// then one 32-entry block of D, instead of bisecting D itself (a line per
// probe).  Returns the position in the row and its value as floor_search does
// (value != y when y is not in the row).
template <int G>
__device__ __forceinline__ uint32_t split_floor(const int32_t* __restrict__ D, const int32_t* __restrict__ HD,
                                                uint64_t P, uint32_t n, const int32_t* spl, int32_t y, int32_t& val) {
  // first splitter index l with spl[l] > y (spl[0] = D[P]); 0 -> y < D[P]
  int lo = 0, hi = G;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (spl[mid] <= y) lo = mid + 1;
    else hi = mid;
  }
  if (lo == 0) {
    val = spl[0];  // above y
    return 0;
  }
  const uint32_t b = (uint32_t)(((uint64_t)(lo - 1) * n) / G);
  const uint32_t e = lo < G ? (uint32_t)(((uint64_t)lo * n) / G) : n;
  const int32_t vb = spl[lo - 1];
  if (HD == nullptr || e - b <= 1024u) return floor_search(D + P, b, e - b, vb, y, val);
  const uint64_t s0 = P + b, s1 = P + e;                    // D[s0] = vb <= y
  const uint64_t hb0 = (s0 + 31) >> 5, hb1 = (s1 - 1) >> 5;  // heads inside the slice (at least 32)
  const int32_t h0 = HD[hb0];
  if (h0 > y) return b + floor_search(D + s0, 0u, (uint32_t)((hb0 << 5) - s0), vb, y, val);
  int32_t hv;
  const uint32_t i = floor_search(HD + hb0, 0u, (uint32_t)(hb1 - hb0 + 1), h0, y, hv);
  const uint64_t B = (hb0 + i) << 5;
  const uint32_t len = (uint32_t)(s1 - B < 32u ? s1 - B : 32u);
  return (uint32_t)(B - P) + floor_search(D + B, 0u, len, hv, y, val);
}

// One whole walk (row w of request a) by one group of G lanes; mem is the
// group's LDS region of group_lds_words(tile, cap, G) words.  FULL adds the
// approximated step and the forced two-pass route to the exact routes; HEADS
// the head search of long splitter slices (graphs with rows longer than
// kHeadsMinDegree, which alone carry destination heads).
// Fused context output (CTX): the walk's positions go to a ring of rp
// (a power of two >= 2 h + 1) words in LDS after the group's region, and the
// 2 window context slots of position i (the nodes at i + o stride, o = -window
// .. -1, 1 .. window, or -1 outside the walk) are written to
// C[row][i][*] once position i + h is drawn, or when the walk ends.
struct CtxArgs {
  int32_t* C = nullptr;
  uint32_t window = 0, stride = 0, h = 0, rp = 0;
};

// LISTS: every edge of the graph keeps a stored list and the route is
// automatic, so a second-order step always searches a stored list and the
// list-building routes are left out (fewer live registers: no spills).
template <int G, bool WEIGHTED, typename RT, bool FULL, bool HEADS = false, bool CTX = false, bool LISTS = false>
__device__ __forceinline__ void group_walk(const WalkArgs& a, uint64_t w, int32_t* mem, int tile, int cap,
                                           int mode_knob, const CtxArgs& cx = CtxArgs{}) {
  if constexpr (LISTS) {
    // the lists-only variant stages no row and builds no list: said at
    // compile time, the staging code and its state drop out
    tile = 0;
    cap = 0;
    mode_knob = kModeAuto;
  }
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  int32_t* const bufA = mem;
  int32_t* const bufB = bufA + tile;
  uint32_t* const lpos = (uint32_t*)(bufB + tile);
  uint32_t* const lw = lpos + cap;
  int32_t* const win = (int32_t*)(lw + cap);
  // Output in whole lines (by address): groups of 16 or more lanes hold one
  // slot per lane and store G slots (one to four lines) at once; narrower
  // groups collect a line of kOutStage slots in LDS (after the merge window)
  // and store it together.
  constexpr uint32_t OW = G >= 16 ? (uint32_t)G : kOutStage;
  int32_t* const ostage = win + 2 * G;
  int32_t* const ring = mem + group_lds_words(tile, cap, G);  // CTX only
  // context slots of position i of this walk's row; positions beyond `last`
  // are outside the walk
  auto emit = [&](uint32_t i, int64_t last) {
    const uint32_t W2 = 2u * cx.window;
    int32_t* __restrict__ out = cx.C + (w * a.L + i) * (uint64_t)W2;
    for (uint32_t c = (uint32_t)(threadIdx.x & (G - 1)); c < W2; c += G) {
      const int64_t o = c < cx.window ? (int64_t)c - (int64_t)cx.window : (int64_t)c - (int64_t)cx.window + 1;
      const int64_t j = (int64_t)i + o * (int64_t)cx.stride;
      out[c] = (j >= 0 && j <= last) ? ring[(uint32_t)j & (cx.rp - 1u)] : -1;
    }
  };
  const uint64_t* __restrict__ O = a.g.O;
  const int32_t* __restrict__ D = a.g.D;
  const RT* __restrict__ R = (const RT*)a.g.R;
  const RT* __restrict__ HR = (const RT*)a.g.HR;
  const int32_t* __restrict__ HD = HEADS ? a.g.HD : nullptr;
  const uint64_t lt_mask = (gl == 0) ? 0ull : ((~0ull) >> (64 - gl));  // group lanes below gl
  const uint64_t P16 = a.P16, Q16 = a.Q16;
  const uint64_t cdel = (uint64_t)kC16 - Q16;  // common minus far, mod 2^64
  const uint64_t rdel = P16 - Q16;             // return minus far, mod 2^64

  {
    int32_t* __restrict__ row = a.Y + w * a.L;
    const int32_t start = a.starts[w % a.ns];
    const uint64_t wid = a.wid_base + w;
    uint32_t len = 0;
    // Row position s sits in slot (roff + s) mod OW of an OW-slot piece that
    // starts on a line boundary; ob (G >= 16) is this lane's slot of the
    // current piece.  Every piece before the one holding position s has been
    // stored once s is staged.
    const uint32_t roff = (uint32_t)(((uintptr_t)row >> 2) & (OW - 1));
    int32_t ob = -1;
    int32_t nf = (int32_t)(OW - 1 - roff);  // the next position that ends a piece
    auto put = [&](uint32_t s, int32_t x) {
      const uint32_t k = (uint32_t)((int32_t)s - nf - 1) & (OW - 1);
      if constexpr (G >= 16) {
        if ((uint32_t)gl == k) ob = x;
      } else {
        if (gl == 0) ostage[k] = x;
      }
      if ((int32_t)s != nf) return;
      const int32_t ps = nf - (int32_t)(OW - 1);  // the piece's first position
      nf += OW;
      if constexpr (G >= 16) {
        if (ps + gl >= 0) row[ps + gl] = ob;
      } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // OW / G back-to-back stores cover the line (only the row's first
        // line can start before the row)
#pragma unroll
        for (int32_t kk = 0; kk < (int32_t)OW; kk += G)
          if (ps + kk + gl >= 0) row[ps + kk + gl] = ostage[kk + gl];
      }
    };
    if (start >= 0 && (int64_t)start < a.g.n) {
      if constexpr (CTX) {
        if (gl == 0) ring[0] = start;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        put(0, start);
      }
      len = 1;
      int32_t v = start, t = -1;
      uint64_t tlo = 0;
      uint32_t td = 0;
      uint64_t epos = 0;  // position of the edge t -> v in N(t)
      int32_t tset = -1;  // hub set of t, or -1
      bool t_in_lds = false;
      int32_t* cur = bufA;  // N(t) when staged
      int32_t* nxt = bufB;  // N(v) being staged
      // Draws depend on (step, walk) only: group lane gl holds the draw of
      // step s1 + gl, all G computed together in the vector unit once every G
      // steps, instead of one scalar Philox evaluation per step.
      uint64_t rdraw = 0;
      for (uint32_t s = 1; s < a.L; ++s) {
        // row offset, degree and row weight sum: one 16-byte node record when
        // the graph has them, else the offsets and the row's last prefix entry
        uint64_t lo, Srec = 0;
        uint32_t d;
        constexpr bool kRec = WEIGHTED && sizeof(RT) == 4;
        if (kRec && a.g.NR) {
          const uint4 rec = a.g.NR[v];
          lo = (uint64_t)rec.x | ((uint64_t)rec.y << 32);
          d = rec.z;
          Srec = rec.w;
        } else {
          lo = O[v];
          d = (uint32_t)(O[v + 1] - lo);
        }
        if (d == 0) break;  // dead end
        int32_t vset = -1;  // hub set of v, or -1
        if constexpr (HEADS) {
          if (a.g.hub_of != nullptr && d >= a.g.hub_min_deg) vset = a.g.hub_of[v];
        }
        const uint32_t sk = (s - 1u) & (uint32_t)(G - 1);
        if (sk == 0) rdraw = philox_draw(a.seed, s + (uint32_t)gl, wid);
        const uint64_t r = grp_bcast<G>(rdraw, (int)sk);
        auto Rv = [&](uint32_t j) -> uint64_t {
          return WEIGHTED ? (uint64_t)R[lo + j] : (uint64_t)j + 1ull;
        };
        // weight of candidate j as a difference of the row prefix: the walk
        // reads one array (R) instead of two (R and W)
        auto Wv = [&](uint32_t j) -> uint64_t {
          if (!WEIGHTED) return 1ull;
          const uint64_t hi = (uint64_t)R[lo + j];
          return j ? hi - (uint64_t)R[lo + j - 1] : hi;
        };
        const uint64_t S = (kRec && a.g.NR) ? Srec : Rv(d - 1);  // row weight sum
        uint32_t jsel = 0xFFFFFFFFu;
        int32_t xq = 0;      // D[lo + jsel] when the final search round fetched it
        bool xq_ok = false;
        bool staged = false;
        bool stop = false;

        auto member = [&](int32_t x) -> bool {
          return t_in_lds ? lds_contains(cur, td, x) : global_contains(D + tlo, td, x);
        };

        // Two-pass streaming over the biased weights (also the fallback when
        // the list of common neighbours does not fit in LDS).
        auto two_pass = [&]() {
          const uint32_t nc = (d + G - 1) / G;
          const uint32_t bs = (nc + G - 1) / G;
          const bool stg = d <= (uint32_t)tile;
          auto alpha = [&](int32_t x) -> uint64_t {
            if (x == t) return P16;
            return member(x) ? (uint64_t)kC16 : Q16;
          };
          uint64_t acc = 0, blk = 0;
          for (uint32_t c = 0; c < nc; ++c) {
            const uint32_t j = c * G + gl;
            if (j < d) {
              const int32_t x = D[lo + j];
              if (stg) nxt[j] = x;
              const uint64_t wt = Wv(j);
              acc += wt * alpha(x);
            }
            if ((c + 1) % bs == 0 || c + 1 == nc) {
              const uint64_t sb = grp_sum<G>(acc);
              if ((uint32_t)gl == c / bs) blk = sb;
              acc = 0;
            }
          }
          staged = stg;
          const uint64_t incl = grp_incl_scan<G>(blk, gl);
          const uint64_t total = grp_bcast<G>(incl, G - 1);
          if (total == 0) {
            stop = true;
            return;
          }
          const uint64_t T = scale_draw(r, total);
          const uint64_t bm = grp_ballot<G>(incl > T, gbase);
          const int kb = __ffsll((unsigned long long)bm) - 1;
          uint64_t base = grp_bcast<G>(incl - blk, kb);
          const uint32_t cend = min((uint32_t)(kb + 1) * bs, nc);
          for (uint32_t c = (uint32_t)kb * bs; c < cend; ++c) {
            const uint32_t j = c * G + gl;
            uint64_t b = 0;
            if (j < d) {
              const int32_t x = stg ? nxt[j] : D[lo + j];
              const uint64_t wt = Wv(j);
              b = wt * alpha(x);
            }
            const uint64_t inc = grp_incl_scan<G>(b, gl);
            const uint64_t m2 = grp_ballot<G>(base + inc > T, gbase);
            if (m2) {
              jsel = c * G + (uint32_t)(__ffsll((unsigned long long)m2) - 1);
              break;
            }
            base += grp_bcast<G>(inc, G - 1);
          }
        };

        // Approximated step (Methods, "Approximated RWs"): only the Sorted
        // Unique Sub-Sample of k neighbours is considered, one uniform position
        // per bucket of length floor(d / k) (the last bucket takes the
        // remainder); the biased weights are normalised over the sub-sample.
        auto approx_step = [&]() {
          const uint32_t k = a.k_approx;
          const uint32_t blen = d / k;
          auto pos_of = [&](uint32_t i) -> uint32_t {
            uint32_t o[4];
            philox_words(a.seed, s, (uint32_t)wid, (uint32_t)(wid >> 32), 1u + i / 2u, o);
            const uint64_t rr = (i & 1u) ? ((uint64_t)o[2] | ((uint64_t)o[3] << 32))
                                         : ((uint64_t)o[0] | ((uint64_t)o[1] << 32));
            const uint32_t st = i * blen;
            const uint32_t ln = (i + 1 < k) ? blen : d - st;
            return st + (uint32_t)scale_draw(rr, ln);
          };
          const bool second = a.second_order && t >= 0;
          // a long N(t) outside LDS: bisections start from its splitters
          const bool split_t = second && !t_in_lds && td >= 4u * G;
          if (split_t) load_splitters<G>(D + tlo, td, win, gl);
          auto weight = [&](uint32_t p) -> uint64_t {
            const int32_t x = D[lo + p];
            const uint64_t wt = Wv(p);
            if (!second) return wt;
            if (x == t) return wt * P16;
            bool common;
            if (split_t) {
              int32_t val;
              split_floor<G>(D, HD, tlo, td, win, x, val);
              common = val == x;
            } else {
              common = member(x);
            }
            return wt * (common ? (uint64_t)kC16 : Q16);
          };
          const uint32_t nc = (k + G - 1) / G;
          const uint32_t bs = (nc + G - 1) / G;
          uint64_t acc = 0, blk = 0;
          for (uint32_t c = 0; c < nc; ++c) {
            const uint32_t i = c * G + gl;
            if (i < k) acc += weight(pos_of(i));
            if ((c + 1) % bs == 0 || c + 1 == nc) {
              const uint64_t sb = grp_sum<G>(acc);
              if ((uint32_t)gl == c / bs) blk = sb;
              acc = 0;
            }
          }
          const uint64_t incl = grp_incl_scan<G>(blk, gl);
          const uint64_t total = grp_bcast<G>(incl, G - 1);
          if (total == 0) {
            stop = true;
            return;
          }
          const uint64_t T = scale_draw(r, total);
          const uint64_t bm = grp_ballot<G>(incl > T, gbase);
          const int kb = __ffsll((unsigned long long)bm) - 1;
          uint64_t base = grp_bcast<G>(incl - blk, kb);
          const uint32_t cend = min((uint32_t)(kb + 1) * bs, nc);
          for (uint32_t c = (uint32_t)kb * bs; c < cend; ++c) {
            const uint32_t i = c * G + gl;
            uint64_t b = 0;
            uint32_t p = 0;
            if (i < k) {
              p = pos_of(i);
              b = weight(p);
            }
            const uint64_t inc = grp_incl_scan<G>(b, gl);
            const uint64_t m2 = grp_ballot<G>(base + inc > T, gbase);
            if (m2) {
              jsel = (uint32_t)grp_bcast_i32<G>((int32_t)p, __ffsll((unsigned long long)m2) - 1);
              break;
            }
            base += grp_bcast<G>(inc, G - 1);
          }
        };

        if (FULL && a.k_approx != 0 && d > a.k_approx) {
          if constexpr (FULL) approx_step();
        } else if (!a.second_order || t < 0) {
          // First-order step (also the first step of a node2vec walk).
          if (S == 0) break;
          const uint64_t T = scale_draw(r, S);
          if (WEIGHTED) {
            jsel = gary_first_heads<G>(
                R, HR, lo, 0u, d, gl, gbase, [&](uint64_t v, uint32_t) { return v > T; }, D + lo, xq, xq_ok);
          } else {
            jsel = (uint32_t)T;
          }
          if (a.second_order && d <= (uint32_t)tile) {
            for (uint32_t j = gl; j < d; j += G) nxt[j] = D[lo + j];
            staged = true;
          }
        } else {
          // An edge t -> v whose common-neighbour list is stored (built at
          // upload, the same list the routes below build): search it.
          bool cached = false;
          if constexpr (WEIGHTED && sizeof(RT) == 4) {
            if (a.g.pair_info != nullptr && mode_knob == kModeAuto) {
              const uint4 inf = a.g.pair_info[2 * epos];
              const uint32_t wtc = a.g.pair_info[2 * epos + 1].x;
              cached = inf.x != 0xFFFFFFFFu;
              if (cached) {
                const uint4* __restrict__ ent = a.g.pair_ent + inf.x;
                const uint32_t nc = inf.y, ptc = inf.z;
                const bool has_t = ptc != 0xFFFFFFFFu;
                const uint64_t CW = inf.w;
                const uint64_t retw = rdel * (uint64_t)wtc;  // wtc = 0 when t is not in N(v)
                const uint64_t total = Q16 * S + cdel * CW + retw;
                if (total == 0) break;
                const uint64_t T = scale_draw(r, total);
                // first listed entry with B > T, B = Q16 R_j + cdel E_j + retw [j >= pt]
                uint4 ek, ekm;
                const uint32_t k = list_search<G>(ent, nc, gl, gbase, [&](const uint4& en) {
                  return Q16 * (uint64_t)en.x + cdel * (uint64_t)en.y + ((has_t && en.z >= ptc) ? retw : 0ull) > T;
                }, ek, ekm);
                uint32_t seg_lo = 0, seg_hi = d;
                uint64_t Eprev = CW;
                if (k < nc) {
                  seg_hi = ek.z;
                  Eprev = 0;
                  if (k > 0) {
                    seg_lo = ekm.z + 1;
                    Eprev = ekm.y;
                  }
                } else if (nc > 0) {
                  seg_lo = ekm.z + 1;
                }
                const uint64_t base = cdel * Eprev;
                jsel = gary_first_heads<G>(
                    R, HR, lo, seg_lo, seg_hi, gl, gbase,
                    [&](uint64_t v, uint32_t j) { return Q16 * v + base + ((has_t && j >= ptc) ? retw : 0ull) > T; },
                    D + lo, xq, xq_ok);
              }
            }
          }
          if (!LISTS && !cached) {
            int mode = mode_knob;
            if (mode == kModeAuto || mode == kModeHubSets) {
              // dependent-latency estimate: global load = 100, LDS load = 15
              // splitters cut a bisection of a row of n >= 4G by log2(G) global rounds for one round
              auto glob = [&](uint32_t n) -> uint32_t {
                return n >= 4u * G ? 100u * (ceil_log2p1(n) - ceil_log2p1(G - 1)) + 15u * ceil_log2p1(G) : 100u * ceil_log2p1(n);
              };
              const uint64_t probe = (uint64_t)((td + 1 + G - 1) / G) * glob(d) + (d >= 4u * G ? 100u : 0u);
              const uint64_t stream = (uint64_t)((d + G - 1) / G) *
                                          (100u + (t_in_lds ? 15u * ceil_log2p1(td) : glob(td))) +
                                      (!t_in_lds && td >= 4u * G ? 100u : 0u);
              // a merge round streams two lines where a probe round of G keys
              // reads G random lines per level: once the two rows are too long
              // for the caches to hold them (2^14 entries together), the merge
              // is priced for the traffic it saves (measured on a 20M-node
              // graph with 1.25M-entry rows: a round at 240 -> 60 took node2vec
              // (1, 2) from 21.6 to 14.4 s; 30 gave 14.5, 15 gave 18.1; without
              // the length gate the 64-graph plan without stored lists lost 12%,
              // and a gate at 2^16 gave 18.4 s)
              const bool uncached = (uint64_t)d + td >= (1u << 14);
              const uint64_t merge = (uint64_t)(((uint64_t)d + td + 2u * G - 1) / (2u * G)) *
                                     (uncached ? (t_in_lds ? 40u : 60u) : (t_in_lds ? 150u : 240u));
              mode = probe < stream ? (probe <= merge ? kModeProbe : kModeMerge)
                                    : (stream <= merge ? kModeStream : kModeMerge);
              if constexpr (HEADS) {
                // a hub set answers a key with one line read: the keys of N(t)
                // against v's set (positions included), or the candidates of
                // N(v) against t's set
                uint64_t best = probe < stream ? (probe < merge ? probe : merge) : (stream < merge ? stream : merge);
                // a set lookup is a random line: past the caches it costs
                // twice its latency price against the streamed merge
                // (20M-node graph: 14.5 -> 14.1 s; four times: 16.5 s)
                const uint64_t sprobe =
                    (uint64_t)((td + 1 + G - 1) / G) * ((t_in_lds ? 15u : 100u) + 100u) * (uncached ? 2u : 1u);
                const uint64_t sstream = (uint64_t)((d + G - 1) / G) * 200u * (uncached ? 2u : 1u);
                if (mode_knob == kModeHubSets) {
                  if (vset >= 0) mode = kModeSetProbe;
                  else if (tset >= 0) mode = kModeSetStream;
                } else {
                  if (vset >= 0 && sprobe < best) {
                    best = sprobe;
                    mode = kModeSetProbe;
                  }
                  if (tset >= 0 && sstream < best) mode = kModeSetStream;
                }
              }
            }
            if (FULL && mode == kModeTwoPass) {
              if constexpr (FULL) two_pass();
            } else {
              // List the positions j in N(v) whose candidate is a common
              // neighbour (x in N(t), x != t), in increasing j, one LDS page of
              // `cap` entries at a time.  Every route visits keys in an order
              // that makes the hit positions increase, so a page can be resumed
              // from the key after its last stored hit.
              uint32_t cnt = 0, pt = 0, stored = 0, resume = 0;
              bool has_t = false, first = true;
              uint64_t acc = 0;
              auto append = [&](bool hit, uint32_t pos, uint32_t key0) {
                const uint64_t m = grp_ballot<G>(hit, gbase);
                if (m == 0) return;
                if (hit) {
                  // a listed position gets its weight after the route (below);
                  // a hit beyond the page adds its weight to the first pass's sum now
                  const uint32_t idx = stored + (uint32_t)__popcll(m & lt_mask);
                  if (idx < (uint32_t)cap) lpos[idx] = pos;
                  else if (first) acc += (uint32_t)Wv(pos);
                }
                const uint32_t nh = (uint32_t)__popcll(m);
                const uint32_t room = (uint32_t)cap - stored;
                if (room > 0 && nh >= room) {
                  uint64_t mm = m;  // the room-th hit fills the page's last slot
                  for (uint32_t i = 1; i < room; ++i) mm &= mm - 1;
                  resume = key0 + (uint32_t)(__ffsll((unsigned long long)mm) - 1) + 1;
                }
                cnt += nh;
                stored = min((uint32_t)cap, stored + nh);
              };
              // keys [from, end): probe route keys are N(t) then t itself; stream
              // route keys are the candidates of N(v).  Later pages stop once full.
              auto gen = [&](uint32_t from) {
                if (mode == kModeProbe) {
                  const uint32_t nk = td + 1;
                  const bool split = d >= 4u * G;
                  if (split) load_splitters<G>(D + lo, d, win, gl);
                  for (uint32_t c = from; c < nk; c += G) {
                    if (!first && stored >= (uint32_t)cap) break;
                    const uint32_t k = c + gl;
                    const bool act = k < nk;
                    const bool tkey = k == td;
                    int32_t y = t;
                    if (act && !tkey) y = t_in_lds ? cur[k] : D[tlo + k];
                    uint32_t pos = 0;
                    bool hit = false;
                    if (act) {
                      int32_t val;
                      pos = split ? split_floor<G>(D, HD, lo, d, win, y, val) : floor_search(D + lo, 0u, d, D[lo], y, val);
                      hit = val == y;
                    }
                    const uint64_t mt = grp_ballot<G>(hit && tkey, gbase);
                    if (mt) {
                      has_t = true;
                      pt = (uint32_t)grp_bcast_i32<G>((int32_t)pos, __ffsll((unsigned long long)mt) - 1);
                    }
                    // a self-loop at t puts t in N(t): that candidate is a return, not common
                    append(hit && !tkey && y != t, pos, c);
                  }
                } else if (HEADS && mode == kModeSetProbe) {
                  // keys N(t) then t, as the probe route, each looked up in
                  // v's set: membership and position from one line
                  const uint32_t* __restrict__ vs = a.g.hub_sets + (uint64_t)vset * a.g.hub_lines * 16u;
                  const uint32_t nk = td + 1;
                  for (uint32_t c = from; c < nk; c += G) {
                    if (!first && stored >= (uint32_t)cap) break;
                    const uint32_t k = c + gl;
                    const bool act = k < nk;
                    const bool tkey = k == td;
                    int32_t y = t;
                    if (act && !tkey) y = t_in_lds ? cur[k] : D[tlo + k];
                    uint32_t pos = 0;
                    const bool hit = act && set_rank(vs, (uint32_t)y, pos);
                    const uint64_t mt = grp_ballot<G>(hit && tkey, gbase);
                    if (mt) {
                      has_t = true;
                      pt = (uint32_t)grp_bcast_i32<G>((int32_t)pos, __ffsll((unsigned long long)mt) - 1);
                    }
                    append(hit && !tkey && y != t, pos, c);
                  }
                } else if (HEADS && mode == kModeSetStream) {
                  // candidates of N(v), as the stream route, each looked up in t's set
                  const uint32_t* __restrict__ ts = a.g.hub_sets + (uint64_t)tset * a.g.hub_lines * 16u;
                  const bool stg = first && d <= (uint32_t)tile;
                  for (uint32_t c = from; c < d; c += G) {
                    if (!first && stored >= (uint32_t)cap) break;
                    const uint32_t j = c + gl;
                    const bool act = j < d;
                    int32_t x = 0;
                    if (act) {
                      x = D[lo + j];
                      if (stg) nxt[j] = x;
                    }
                    const bool isret = act && x == t;
                    const uint64_t mt = grp_ballot<G>(isret, gbase);
                    if (mt) {
                      has_t = true;
                      pt = c + (uint32_t)(__ffsll((unsigned long long)mt) - 1);
                    }
                    const bool in_t = act && !isret && set_member(ts, (uint32_t)x);
                    append(in_t, j, c);
                  }
                  if (first) staged = stg;
                } else if (mode == kModeMerge) {
                  // co-iterate N(v) (candidates, global) and N(t) (B): invariant
                  // "every element of B before ib is below N(v)[ia]".  A round
                  // stages 2G elements of B in LDS, takes 2G candidates (two per
                  // lane), decides every candidate that is at most the window's
                  // last element by bisecting the window, and advances ia past
                  // the decided candidates, or ib by 2G when some candidate lies
                  // beyond the window.
                  constexpr uint32_t W2 = 2u * G;
                  const bool stg = first && d <= (uint32_t)tile;
                  auto Bv = [&](uint32_t k) -> int32_t { return t_in_lds ? cur[k] : D[tlo + k]; };
                  uint32_t ia = from, ib = 0;
                  if (ia > 0 && ia < d) {
                    const int32_t a0 = D[lo + ia];
                    ib = gary_first<G>(0u, td, gl, gbase, [&](uint32_t k) { return Bv(k) >= a0; });
                  }
                  while (ia < d) {
                    if (!first && stored >= (uint32_t)cap) break;
                    const uint32_t j0 = ia + gl, j1 = j0 + G;
                    const bool act0 = j0 < d, act1 = j1 < d;
                    int32_t x0 = 0x7FFFFFFF, x1 = 0x7FFFFFFF;
                    if (act0) x0 = D[lo + j0];
                    if (act1) x1 = D[lo + j1];
                    const uint32_t nb = ib < td ? min(W2, td - ib) : 0u;
                    const int32_t b0 = (uint32_t)gl < nb ? Bv(ib + gl) : 0x7FFFFFFF;
                    const int32_t b1 = (uint32_t)gl + G < nb ? Bv(ib + G + gl) : 0x7FFFFFFF;
                    if (stg) {
                      if (act0) nxt[j0] = x0;
                      if (act1) nxt[j1] = x1;
                    }
                    win[gl] = b0;
                    win[G + gl] = b1;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    // B beyond this window is empty when nb < 2G: then every candidate is decided
                    const int32_t blast = nb == W2 ? grp_bcast_i32<G>(b1, G - 1) : 0x7FFFFFFF;
                    const bool res0 = act0 && x0 <= blast, res1 = act1 && x1 <= blast;
                    const bool ret0 = res0 && x0 == t, ret1 = res1 && x1 == t;
                    const uint64_t mt0 = grp_ballot<G>(ret0, gbase), mt1 = grp_ballot<G>(ret1, gbase);
                    if (mt0 | mt1) {
                      has_t = true;
                      pt = mt0 ? ia + (uint32_t)(__ffsll((unsigned long long)mt0) - 1)
                               : ia + G + (uint32_t)(__ffsll((unsigned long long)mt1) - 1);
                    }
                    const bool in0 = res0 && !ret0 && nb > 0 && lds_contains(win, nb, x0);
                    const bool in1 = res1 && !ret1 && nb > 0 && lds_contains(win, nb, x1);
                    append(in0, j0, ia);
                    append(in1, j1, ia + G);
                    const uint32_t nact = min(W2, d - ia);
                    const uint32_t nres = (uint32_t)__popcll(grp_ballot<G>(res0, gbase)) +
                                          (uint32_t)__popcll(grp_ballot<G>(res1, gbase));
                    if (nres == nact) {
                      ia += nact;
                    } else {
                      ia += nres;  // decided candidates are a prefix: the candidates are sorted
                      ib += W2;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                  }
                  if (first) staged = stg;
                } else {
                  const bool stg = first && d <= (uint32_t)tile;
                  const bool split = !t_in_lds && td >= 4u * G;
                  if (split) load_splitters<G>(D + tlo, td, win, gl);
                  for (uint32_t c = from; c < d; c += G) {
                    if (!first && stored >= (uint32_t)cap) break;
                    const uint32_t j = c + gl;
                    const bool act = j < d;
                    int32_t x = 0;
                    if (act) {
                      x = D[lo + j];
                      if (stg) nxt[j] = x;
                    }
                    const bool isret = act && x == t;
                    const uint64_t mt = grp_ballot<G>(isret, gbase);
                    if (mt) {
                      has_t = true;
                      pt = c + (uint32_t)(__ffsll((unsigned long long)mt) - 1);
                    }
                    bool in_t;
                    if (t_in_lds) {
                      in_t = act && !isret && lds_contains(cur, td, x);
                    } else {
                      if (split) {
                        in_t = false;
                        if (act && !isret) {
                          int32_t val;
                          split_floor<G>(D, HD, tlo, td, win, x, val);
                          in_t = val == x;
                        }
                      } else {
                        in_t = act && !isret && global_contains(D + tlo, td, x);
                      }
                    }
                    append(act && !isret && in_t, j, c);
                  }
                  if (first) staged = stg;
                }
                // Weights of the page's positions: one gather over the list, off the
                // chain of dependent loads of the route's rounds.
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (uint32_t k = gl; k < stored; k += 2 * G) {
                  const uint32_t k2 = k + G;
                  const bool two = k2 < stored;
                  const uint32_t w1 = (uint32_t)Wv(lpos[k]);
                  const uint32_t w2 = two ? (uint32_t)Wv(lpos[k2]) : 0u;
                  lw[k] = w1;
                  if (two) lw[k2] = w2;
                  if (first) acc += (uint64_t)w1 + w2;
                }
                // the page is read by other lanes of the group
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
              };
              gen(0);  // first pass: every hit counted, first page stored
              first = false;
              const uint64_t CW = grp_sum<G>(acc);
              const uint64_t wt = has_t ? Wv(pt) : 0ull;
              const uint64_t retw = rdel * wt;
              const uint64_t total = Q16 * S + cdel * CW + retw;
              if (total == 0) break;
              const uint64_t T = scale_draw(r, total);
              // B_j = Q16 R_j + cdel * (common weight up to j) + retw [j >= pt]:
              // find the first listed position with B > T, then the segment
              // before it holds no common neighbour.
              uint64_t E = 0, Eprev = CW;
              uint32_t seg_lo = 0, seg_hi = d, lastpos = 0, left = cnt, page = stored;
              bool found = false, any = false;
              while (true) {
                for (uint32_t c = 0; c < page; c += G) {
                  const uint32_t k = c + gl;
                  const bool act = k < page;
                  const uint32_t p = act ? lpos[k] : 0u;
                  const uint64_t wk = act ? (uint64_t)lw[k] : 0ull;
                  const uint64_t inc = grp_incl_scan<G>(wk, gl);
                  const uint64_t Ek = E + inc;
                  const uint64_t Bk = Q16 * Rv(p) + cdel * Ek + ((has_t && p >= pt) ? retw : 0ull);
                  const uint64_t m = grp_ballot<G>(act && Bk > T, gbase);
                  if (m) {
                    const int f = __ffsll((unsigned long long)m) - 1;
                    Eprev = grp_bcast<G>(Ek - wk, f);
                    seg_hi = (uint32_t)grp_bcast_i32<G>((int32_t)p, f);
                    const uint32_t pprev = (uint32_t)grp_bcast_i32<G>((int32_t)p, f > 0 ? f - 1 : 0);
                    seg_lo = f > 0 ? pprev + 1 : (any ? lastpos + 1 : 0u);
                    found = true;
                    break;
                  }
                  const uint32_t nact = min((uint32_t)G, page - c);
                  lastpos = (uint32_t)grp_bcast_i32<G>((int32_t)p, (int)nact - 1);
                  any = true;
                  E += grp_bcast<G>(inc, G - 1);
                }
                left -= page;
                if (found || left == 0) break;
                // the draw lies beyond this page: list the next one
                stored = 0;
                const uint32_t from = resume;
                gen(from);
                page = stored;
                if (page == 0) break;  // unreachable: `left` hits remain after `from`
              }
              if (!found) {
                seg_lo = any ? lastpos + 1 : 0u;
                seg_hi = d;
                Eprev = CW;
              }
              const uint64_t base = cdel * Eprev;
              if constexpr (WEIGHTED) {
                jsel = gary_first_heads<G>(
                    R, HR, lo, seg_lo, seg_hi, gl, gbase,
                    [&](uint64_t v, uint32_t j) { return Q16 * v + base + ((has_t && j >= pt) ? retw : 0ull) > T; },
                    D + lo, xq, xq_ok);
              } else {
                jsel = gary_first<G>(seg_lo, seg_hi, gl, gbase, [&](uint32_t j) {
                  return Q16 * Rv(j) + base + ((has_t && j >= pt) ? retw : 0ull) > T;
                });
              }
            }
          }
        }
        if (stop || jsel >= d) break;  // total weight zero (jsel >= d is unreachable)
        const int32_t xsel = xq_ok ? xq : D[lo + jsel];

        if constexpr (CTX) {
          if (gl == 0) ring[s & (cx.rp - 1u)] = xsel;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (s >= cx.h) emit(s - cx.h, (int64_t)s);
        } else {
          put(s, xsel);
        }
        len = s + 1;
        t = v;
        tlo = lo;
        td = d;
        tset = vset;
        epos = lo + jsel;
        t_in_lds = staged;
        if (staged) {
          int32_t* tmp = cur;
          cur = nxt;
          nxt = tmp;
        }
        v = xsel;
        // the staged row and the list are read by other lanes of the group
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if constexpr (CTX) {
      // positions whose right neighbours ran past the end (the drawn steps
      // emitted positions [max(h, 1) - h, len - 1 - h]; with h = 0, that is a
      // one-slot walk, the start is left), then the padding
      const uint32_t first = len > cx.h ? len - cx.h : 0u;
      for (uint32_t i = first; i < len; ++i) emit(i, (int64_t)len - 1);
      if (cx.h == 0 && len > 0) emit(0u, 0);
      const uint32_t W2 = 2u * cx.window;
      int32_t* __restrict__ pad = cx.C + (w * a.L + len) * (uint64_t)W2;
      const uint64_t words = (uint64_t)(a.L - len) * W2;
      for (uint64_t u = (uint64_t)gl; u < words; u += G) pad[u] = -1;
    } else {
      // positions [s0, len) (from the start of len's piece, or 0) are staged,
      // the rest are padding
      if constexpr (G < 16) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t s0 = nf >= (int32_t)(OW - 1) ? (uint32_t)(nf - (int32_t)(OW - 1)) : 0u;
        for (uint32_t p = s0 + (uint32_t)gl; p < a.L; p += G)
          row[p] = p < len ? ostage[(uint32_t)((int32_t)p - nf - 1) & (OW - 1)] : -1;
      } else {
      const uint32_t lk = (roff + len) & (OW - 1);
      const uint32_t s0 = len > lk ? len - lk : 0u;
      const int64_t first = (int64_t)s0 - (int64_t)((roff + s0) & (OW - 1));
      for (int64_t base = first; base < (int64_t)a.L; base += OW) {
        for (uint32_t kk = (uint32_t)gl; kk < OW; kk += G) {
          const int64_t p = base + kk;
          if (p >= (int64_t)s0 && p < (int64_t)a.L) {
            int32_t val = -1;
            if (p < (int64_t)len) {
              if constexpr (G >= 16) val = ob;
              else val = ostage[kk];
            }
            row[p] = val;
          }
        }
      }
      }
    }
    if (a.lens && gl == 0) a.lens[w] = (int32_t)len;
    if (a.steps && gl == 0 && len > 1) atomicAdd(a.steps, (unsigned long long)(len - 1));
  }
}

// Occupancy bounds (measured): one walker per wavefront runs 8 waves per SIMD
// with scalar spills; 4- and 8-lane groups run 5 and 6 waves with a few vector
// spills; the lists-only 4-lane variant runs 7 (72 registers, a 20-byte spill:
// faster than 6 waves without spill and than 8 with more).
template <int G, bool WEIGHTED, typename RT, bool FULL, bool HEADS, bool LISTS = false>
__global__ __launch_bounds__(256, G == 64 ? 8 : (G == 4 ? (LISTS ? 7 : 5) : (G == 8 ? 6 : 1))) void k_walk_n2v(WalkArgs a, int tile, int cap, int mode_knob,
                                                                                   unsigned long long* ctr, uint32_t chunk) {
  extern __shared__ int32_t lds[];
  // with one walker per wavefront the group index is uniform: say so, so that
  // per-walker state (walk index, counters, draws) lives in scalar registers
  const int gib = G == 64 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x / 64u) : (int)(threadIdx.x / G);
  const int gpb = blockDim.x / G;
  int32_t* const mem = lds + (size_t)gib * group_lds_words(tile, cap, G);
  // With a launch counter, groups take `chunk` walks at a time (walk costs are
  // heavy-tailed: fixed shares leave a long tail); without, fixed shares.
  const int gl = (threadIdx.x & 63) & (G - 1);
  const uint64_t ngroups = (uint64_t)gridDim.x * gpb;
  uint64_t w = ctr ? 0 : (uint64_t)blockIdx.x * gpb + gib, e = 0;
  while (true) {
    if (ctr) {
      if (w >= e) {
        unsigned long long c = 0;
        if (gl == 0) c = atomicAdd(ctr, (unsigned long long)chunk);
        w = grp_bcast<G>((uint64_t)c, 0);
        e = min(w + chunk, a.nwalks);
      }
    }
    if (w >= a.nwalks) break;
    group_walk<G, WEIGHTED, RT, FULL, HEADS, false, LISTS>(a, w, mem, tile, cap, mode_knob);
    w += ctr ? 1 : ngroups;
  }
}

// Fused walk -> contexts: the node2vec kernel's walker loop with context
// output (every kind runs through the group routine: its first-order branch
// serves first-order walks and the first step of node2vec walks).
template <int G, bool WEIGHTED, typename RT, bool LISTS = false>
__global__ __launch_bounds__(256, LISTS ? 7 : 1) void k_walk_ctx(WalkArgs a, int tile, int cap, CtxArgs cx,
                                                                  unsigned long long* ctr, uint32_t chunk) {
  extern __shared__ int32_t lds[];
  const int gib = G == 64 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x / 64u) : (int)(threadIdx.x / G);
  const int gpb = blockDim.x / G;
  int32_t* const mem = lds + (size_t)gib * (group_lds_words(tile, cap, G) + cx.rp);
  const int gl = (threadIdx.x & 63) & (G - 1);
  const uint64_t ngroups = (uint64_t)gridDim.x * gpb;
  uint64_t w = ctr ? 0 : (uint64_t)blockIdx.x * gpb + gib, e = 0;
  while (true) {
    if (ctr) {
      if (w >= e) {
        unsigned long long c = 0;
        if (gl == 0) c = atomicAdd(ctr, (unsigned long long)chunk);
        w = grp_bcast<G>((uint64_t)c, 0);
        e = min(w + chunk, a.nwalks);
      }
    }
    if (w >= a.nwalks) break;
    group_walk<G, WEIGHTED, RT, false, false, true, LISTS>(a, w, mem, tile, cap, kModeAuto, cx);
    w += ctr ? 1 : ngroups;
  }
}

// ---------------------------------------------------------------------------
// Persistent batched kernel: groups pop walk chunks (request, first row, end
// row) from a device queue ordered longest-estimated-first and run each walk
// with the same per-walk routines as the plain kernels.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ void lane_dispatch(const WalkArgs& a, uint64_t w, int32_t* st) {
  const bool weighted = a.g.W != nullptr;
  const bool r64 = a.g.r_bytes == 8;
  if (a.path == (uint32_t)Path::kFirstOrder) {
    if (!weighted) lane_walk<kFoUnw, uint32_t>(a, w, st);
    else if (r64) lane_walk<kFoW, uint64_t>(a, w, st);
    else lane_walk<kFoW, uint32_t>(a, w, st);
  } else {
    if (!weighted) lane_walk<kRetUnw, uint32_t>(a, w, st);
    else if (r64) lane_walk<kRetW, uint64_t>(a, w, st);
    else lane_walk<kRetW, uint32_t>(a, w, st);
  }
}

// The batched kernel reads its requests from a table in device memory.  A
// pointer read from memory carries no address space, so loads through it
// would compile to flat loads (which also wait on the LDS counter).  Every
// array a request points to is in global memory: this mirror of WalkArgs,
// with the same layout, types the pointers so, and the kernel converts them
// once per chunk.
#define N2V_GLOBAL __attribute__((address_space(1)))
struct GraphDevG {
  const N2V_GLOBAL uint64_t* O;
  const N2V_GLOBAL int32_t* D;
  const N2V_GLOBAL uint32_t* W;
  const N2V_GLOBAL void* R;
  uint32_t r_bytes;
  int64_t n;
  uint64_t m;
  const N2V_GLOBAL uint4* NR;
  const N2V_GLOBAL void* HR;
  const N2V_GLOBAL int32_t* HD;
  const N2V_GLOBAL uint4* pair_info;
  const N2V_GLOBAL uint4* pair_ent;
  const N2V_GLOBAL int32_t* hub_of;
  const N2V_GLOBAL uint32_t* hub_sets;
  uint64_t hub_lines;
  uint32_t hub_min_deg;
  uint32_t hub_pad;
};
struct WalkArgsG {
  GraphDevG g;
  const N2V_GLOBAL int32_t* starts;
  uint64_t ns;
  uint64_t nwalks;
  uint32_t L;
  uint32_t second_order;
  uint32_t P16, Q16;
  uint64_t seed;
  uint64_t wid_base;
  N2V_GLOBAL int32_t* Y;
  N2V_GLOBAL int32_t* lens;
  uint32_t path;
  uint32_t k_approx;
  N2V_GLOBAL unsigned long long* steps;
};
static_assert(sizeof(WalkArgsG) == sizeof(WalkArgs) && offsetof(WalkArgsG, g.NR) == offsetof(WalkArgs, g.NR) &&
                  offsetof(WalkArgsG, g.HR) == offsetof(WalkArgs, g.HR) &&
                  offsetof(WalkArgsG, g.HD) == offsetof(WalkArgs, g.HD) &&
                  offsetof(WalkArgsG, g.pair_ent) == offsetof(WalkArgs, g.pair_ent) &&
                  offsetof(WalkArgsG, g.hub_sets) == offsetof(WalkArgs, g.hub_sets) &&
                  offsetof(WalkArgsG, g.hub_min_deg) == offsetof(WalkArgs, g.hub_min_deg) &&
                  offsetof(WalkArgsG, starts) == offsetof(WalkArgs, starts) &&
                  offsetof(WalkArgsG, seed) == offsetof(WalkArgs, seed) && offsetof(WalkArgsG, Y) == offsetof(WalkArgs, Y) &&
                  offsetof(WalkArgsG, path) == offsetof(WalkArgs, path) &&
                  offsetof(WalkArgsG, steps) == offsetof(WalkArgs, steps),
              "WalkArgsG mirrors WalkArgs");

__device__ __forceinline__ WalkArgs from_global(const WalkArgsG& r) {
  WalkArgs a;
  a.g.O = (const uint64_t*)r.g.O;
  a.g.D = (const int32_t*)r.g.D;
  a.g.W = (const uint32_t*)r.g.W;
  a.g.R = (const void*)r.g.R;
  a.g.r_bytes = r.g.r_bytes;
  a.g.n = r.g.n;
  a.g.m = r.g.m;
  a.g.NR = (const uint4*)r.g.NR;
  a.g.HR = (const void*)r.g.HR;
  a.g.HD = (const int32_t*)r.g.HD;
  a.g.pair_info = (const uint4*)r.g.pair_info;
  a.g.pair_ent = (const uint4*)r.g.pair_ent;
  a.g.hub_of = (const int32_t*)r.g.hub_of;
  a.g.hub_sets = (const uint32_t*)r.g.hub_sets;
  a.g.hub_lines = r.g.hub_lines;
  a.g.hub_min_deg = r.g.hub_min_deg;
  a.starts = (const int32_t*)r.starts;
  a.ns = r.ns;
  a.nwalks = r.nwalks;
  a.L = r.L;
  a.second_order = r.second_order;
  a.P16 = r.P16;
  a.Q16 = r.Q16;
  a.seed = r.seed;
  a.wid_base = r.wid_base;
  a.Y = (int32_t*)r.Y;
  a.lens = (int32_t*)r.lens;
  a.path = r.path;
  a.k_approx = r.k_approx;
  a.steps = (unsigned long long*)r.steps;
  return a;
}

// A wavefront pops one chunk at a time, so the request it serves is uniform
// across the wave: the request record is read with scalar loads and lives in
// scalar registers (with 16 groups of 4 lanes per wave, per-group requests
// held the record in vector registers and spilled), and the wave's groups
// run walks of one request, hence of one length.  The lanes of a lane-path
// chunk take one walk each; the groups of a node2vec chunk take every
// (64 / G)-th walk of it.
// W32: every request's graph is weighted with 32-bit prefixes, so only those
// walk variants are compiled in (fewer live registers, fewer spills).
template <int G, bool FULL, bool W32, bool LISTS = false>
__global__ __launch_bounds__(256, G == 64 ? 7 : (G == 4 ? (LISTS ? 7 : 5) : 1)) void k_walk_queue(const WalkArgs* __restrict__ reqs,
                                                    const QueueChunk* __restrict__ chunks, uint32_t nchunks,
                                                    uint32_t* __restrict__ head, int tile, int cap,
                                                    int mode_knob) {
  extern __shared__ int32_t lds[];
  constexpr uint32_t GPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const uint32_t giw = (uint32_t)lane / G;  // group index within the wavefront
  // the wavefront's LDS: its groups' regions, or its lanes' output stages
  int32_t* const wmem = lds + (size_t)(threadIdx.x / 64u) * queue_wave_words(tile, cap, G);
  int32_t* const mem = wmem + (size_t)giw * group_lds_words(tile, cap, G);
  int32_t* const st = wmem + lane;
  while (true) {
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(head, 1u);
    c = (uint32_t)__builtin_amdgcn_readlane((int)c, 0);
    if (c >= nchunks) break;  // every wavefront exits once the queue is drained
    // the previous chunk's LDS reads by other lanes come before this chunk's writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const QueueChunk ch = chunks[c];
    const WalkArgs a = from_global(((const WalkArgsG*)reqs)[ch.req]);
    if (a.path != (uint32_t)Path::kGeneric) {
      for (uint64_t w = ch.w0 + (uint64_t)lane; w < ch.w1; w += 64) {
        if constexpr (W32) {
          if (a.path == (uint32_t)Path::kFirstOrder) lane_walk<kFoW, uint32_t>(a, w, st);
          else lane_walk<kRetW, uint32_t>(a, w, st);
        } else {
          lane_dispatch<G>(a, w, st);
        }
      }
    } else if (W32) {
      for (uint64_t w = ch.w0 + giw; w < ch.w1; w += GPW)
        group_walk<G, true, uint32_t, FULL, false, false, LISTS>(a, w, mem, tile, cap, mode_knob);
    } else if (a.g.W == nullptr) {
      for (uint64_t w = ch.w0 + giw; w < ch.w1; w += GPW) group_walk<G, false, uint32_t, FULL>(a, w, mem, tile, cap, mode_knob);
    } else if (a.g.r_bytes == 8) {
      for (uint64_t w = ch.w0 + giw; w < ch.w1; w += GPW) group_walk<G, true, uint64_t, FULL>(a, w, mem, tile, cap, mode_knob);
    } else {
      for (uint64_t w = ch.w0 + giw; w < ch.w1; w += GPW) group_walk<G, true, uint32_t, FULL>(a, w, mem, tile, cap, mode_knob);
    }
  }
}

__global__ void k_reset_counter(uint32_t* head) { *head = 0u; }
__global__ void k_reset_counter64(unsigned long long* c) { *c = 0ull; }

}  // namespace

unsigned long long* counter_slot(const DevInfo& di, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return nullptr;
  }
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, unsigned long long*> slot;
  static std::map<int, std::pair<unsigned long long*, int>> slab;  // device -> (slab, slots used)
  constexpr int kSlab = 512;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(di.device, st);
  auto it = slot.find(key);
  if (it != slot.end()) return it->second;
  auto& sb = slab[di.device];
  if (sb.first == nullptr || sb.second == kSlab) {
    void* p = nullptr;
    if (hipMalloc(&p, kSlab * sizeof(unsigned long long)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    sb = std::make_pair((unsigned long long*)p, 0);
  }
  unsigned long long* c = sb.first + sb.second++;
  slot.emplace(key, c);
  return c;
}

void reset_counter(unsigned long long* c, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter64, dim3(1), dim3(1), 0, st, c);
}

std::mutex& counter_mutex() {
  static std::mutex mu;
  return mu;
}

namespace {

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
  return with_walk_counter(di, st, [&](unsigned long long* ctr) {
    // a wave's share in units of 64 walks decides its chunk
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, a, ctr, walk_chunk(a.nwalks / 64, (uint64_t)blocks * 4));
    return hipGetLastError();
  });
}

template <int G, bool WEIGHTED, typename RT>
hipError_t go_n2v(const WalkArgs& a, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  const bool full = a.k_approx != 0 || cfg.mode == kModeTwoPass;
  // 64-lane groups on graphs with destination heads or hub sets take the
  // variant that searches heads and looks keys up in the sets
  const bool heads = G == 64 && (a.g.HD != nullptr || a.g.hub_sets != nullptr);
  // 4-lane groups on graphs whose edges all keep a stored list (automatic
  // route) take the variant without the list-building routes
  const bool lists = G == 4 && WEIGHTED && sizeof(RT) == 4 && cfg.lists && !full && cfg.mode == kModeAuto;
  auto k = full ? (heads ? k_walk_n2v<G, WEIGHTED, RT, true, G == 64> : k_walk_n2v<G, WEIGHTED, RT, true, false>)
                : (heads ? k_walk_n2v<G, WEIGHTED, RT, false, G == 64>
                         : (lists ? k_walk_n2v<G, WEIGHTED, RT, false, false, G == 4 && WEIGHTED && sizeof(RT) == 4>
                                  : k_walk_n2v<G, WEIGHTED, RT, false, false>));
  const int gpb = 256 / G;
  // the lists-only variant stages no row and builds no list in LDS
  const int tile = lists ? 0 : cfg.lds_tile, cap = lists ? 0 : cfg.list_cap;
  const size_t lds = (size_t)gpb * group_lds_words(tile, cap, G) * sizeof(int32_t);
  int blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : grid_for(k, lds, (a.nwalks + gpb - 1) / gpb, di);
  return with_walk_counter(di, st, [&](unsigned long long* ctr) {
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, st, a, tile, cap, cfg.mode, ctr,
                       walk_chunk(a.nwalks, (uint64_t)blocks * gpb));
    return hipGetLastError();
  });
}

template <bool WEIGHTED, typename RT>
hipError_t go_n2v_g(const WalkArgs& a, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  switch (cfg.lanes_per_walker) {
    case 4: return go_n2v<4, WEIGHTED, RT>(a, cfg, di, st);
    case 8: return go_n2v<8, WEIGHTED, RT>(a, cfg, di, st);
    case 16: return go_n2v<16, WEIGHTED, RT>(a, cfg, di, st);
    case 32: return go_n2v<32, WEIGHTED, RT>(a, cfg, di, st);
    default: return go_n2v<64, WEIGHTED, RT>(a, cfg, di, st);
  }
}

// The queue kernel carries the approximated step and the forced two-pass
// route only when a request of the launch needs them.
inline bool queue_full(const LaunchCfg& cfg) { return cfg.full != 0 || cfg.mode == kModeTwoPass; }

// 4-lane groups whose requests' graphs are all weighted (32-bit prefixes)
// and keep a stored list for every edge: the lists-only queue kernel, which
// stages no row and builds no list in LDS.
inline bool queue_lists(const LaunchCfg& cfg) {
  return cfg.lanes_per_walker == 4 && cfg.w32 && cfg.lists && !queue_full(cfg) && cfg.mode == kModeAuto;
}

template <int G>
auto queue_kernel(const LaunchCfg& cfg) {
  const bool full = queue_full(cfg);
  if (G == 4 && queue_lists(cfg)) return k_walk_queue<G, false, true, true>;
  if (cfg.w32) return full ? k_walk_queue<G, true, true> : k_walk_queue<G, false, true>;
  return full ? k_walk_queue<G, true, false> : k_walk_queue<G, false, false>;
}

template <int G>
hipError_t go_queue(const WalkArgs* reqs, const QueueChunk* chunks, uint32_t nchunks, uint32_t* head,
                    const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  auto k = queue_kernel<G>(cfg);
  const int gpb = 256 / G;
  const bool lists = queue_lists(cfg);
  const int tile = lists ? 0 : cfg.lds_tile, cap = lists ? 0 : cfg.list_cap;
  const size_t lds = 4 * (size_t)queue_wave_words(tile, cap, G) * sizeof(int32_t);
  int blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : grid_for(k, lds, ((uint64_t)nchunks + gpb - 1) / gpb, di);
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, head);
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, st, reqs, chunks, nchunks, head, tile, cap, cfg.mode);
  return hipGetLastError();
}

}  // namespace

int queue_grid_blocks(const LaunchCfg& cfg, const DevInfo& di, uint32_t nchunks) {
  const int G = cfg.lanes_per_walker == 4 ? 4 : (cfg.lanes_per_walker == 16 ? 16 : (cfg.lanes_per_walker == 32 ? 32 : 64));
  const int gpb = 256 / G;
  const bool lists = queue_lists(cfg);
  const size_t lds = 4 * (size_t)queue_wave_words(lists ? 0 : cfg.lds_tile, lists ? 0 : cfg.list_cap, G) * sizeof(int32_t);
  const uint64_t work = ((uint64_t)nchunks + gpb - 1) / gpb;
  if (G == 4) return grid_for(queue_kernel<4>(cfg), lds, work, di);
  if (G == 16) return grid_for(queue_kernel<16>(cfg), lds, work, di);
  if (G == 32) return grid_for(queue_kernel<32>(cfg), lds, work, di);
  return grid_for(queue_kernel<64>(cfg), lds, work, di);
}

hipError_t launch_queue(const WalkArgs* d_reqs, const QueueChunk* d_chunks, uint32_t nchunks,
                        uint32_t* d_head, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st) {
  if (nchunks == 0) return hipSuccess;
  switch (cfg.lanes_per_walker) {
    case 4: return go_queue<4>(d_reqs, d_chunks, nchunks, d_head, cfg, di, st);
    case 16: return go_queue<16>(d_reqs, d_chunks, nchunks, d_head, cfg, di, st);
    case 32: return go_queue<32>(d_reqs, d_chunks, nchunks, d_head, cfg, di, st);
    default: return go_queue<64>(d_reqs, d_chunks, nchunks, d_head, cfg, di, st);
  }
}

namespace {
template <int G, bool WEIGHTED, typename RT>
hipError_t go_ctx(const WalkArgs& a, const LaunchCfg& cfg, const CtxArgs& cx, const DevInfo& di, hipStream_t st) {
  // 4-lane groups on graphs whose edges all keep a stored list (automatic
  // route): the lists-only variant, as for the walk kernel
  constexpr bool kL = G == 4 && WEIGHTED && sizeof(RT) == 4;
  const bool lists = kL && cfg.lists && cfg.mode == kModeAuto;
  auto k = lists ? k_walk_ctx<G, WEIGHTED, RT, kL> : k_walk_ctx<G, WEIGHTED, RT>;
  const int gpb = 256 / G;
  const int tile = lists ? 0 : cfg.lds_tile, cap = lists ? 0 : cfg.list_cap;
  const size_t lds = (size_t)gpb * (group_lds_words(tile, cap, G) + cx.rp) * sizeof(int32_t);
  int blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : grid_for(k, lds, (a.nwalks + gpb - 1) / gpb, di);
  return with_walk_counter(di, st, [&](unsigned long long* ctr) {
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, st, a, tile, cap, cx, ctr,
                       walk_chunk(a.nwalks, (uint64_t)blocks * gpb));
    return hipGetLastError();
  });
}

template <int G>
hipError_t go_ctx_g(const WalkArgs& a, const LaunchCfg& cfg, const CtxArgs& cx, const DevInfo& di, hipStream_t st) {
  if (a.g.W == nullptr) return go_ctx<G, false, uint32_t>(a, cfg, cx, di, st);
  return a.g.r_bytes == 8 ? go_ctx<G, true, uint64_t>(a, cfg, cx, di, st) : go_ctx<G, true, uint32_t>(a, cfg, cx, di, st);
}
}  // namespace

size_t ctx_block_lds_bytes(int lanes_per_walker, int tile, int cap, uint32_t rp) {
  return (size_t)(256 / lanes_per_walker) * ((size_t)group_lds_words(tile, cap, lanes_per_walker) + rp) * 4;
}

hipError_t launch_walks_ctx(const WalkArgs& a, const LaunchCfg& cfg, int32_t* C, uint32_t window, uint32_t stride,
                            uint32_t h, uint32_t rp, const DevInfo& di, hipStream_t st) {
  if (a.nwalks == 0) return hipSuccess;
  CtxArgs cx;
  cx.C = C;
  cx.window = window;
  cx.stride = stride;
  cx.h = h;
  cx.rp = rp;
  switch (cfg.lanes_per_walker) {
    case 4: return go_ctx_g<4>(a, cfg, cx, di, st);
    case 16: return go_ctx_g<16>(a, cfg, cx, di, st);
    default: return go_ctx_g<64>(a, cfg, cx, di, st);
  }
}

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
      if (!weighted) return go_n2v_g<false, uint32_t>(a, cfg, di, st);
      return r64 ? go_n2v_g<true, uint64_t>(a, cfg, di, st) : go_n2v_g<true, uint32_t>(a, cfg, di, st);
  }
}

}  // namespace n2v
