// Elias-Fano edge store on the GPU (Methods, "Edge Encoding", "Operations on
// Elias-Fano", "Efficient implementation of Elias-Fano"): construction from a
// CSR graph, select and rank, and every exact walk kind over the store.  Only
// where the neighbours come from changes; the walks are the CSR walks, bit for
// bit.
//
// Layout: edge code phi_k(a, b) = a 2^k + b, k = ceil(log2 n), u = n 2^k;
// l = floor(log2(u / m)) low bits per code in L (field i = bits [i l, i l + l),
// least significant first); the one of code i at bit (code_i >> l) + i of H,
// ((u - 1) >> l) + 1 zeros; S1[j] / S0[j] = position of one / zero number
// j 2^lgq.  rank(x) counts the codes strictly below x, so the row of node a is
// [rank(phi(a, 0)), rank(phi(a + 1, 0))) and neighbour j of a is
// select(rank(phi(a, 0)) + j) & (2^k - 1).
#include "n2v_device.hpp"
#include "n2v_internal.hpp"

namespace n2v {
namespace {

// Bit position of set bit number r (from 0, least significant first) of b,
// which has more than r set bits: a popcount bisection over halves (the word
// half first, then 32-bit arithmetic).
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t b, uint32_t r) {
  uint32_t x = (uint32_t)b, pos = 0;
  uint32_t c = (uint32_t)__popc(x);
  if (r >= c) { r -= c; x = (uint32_t)(b >> 32); pos = 32; }
  c = (uint32_t)__popc(x & 0xFFFFu);
  if (r >= c) { r -= c; x >>= 16; pos += 16; }
  c = (uint32_t)__popc(x & 0xFFu);
  if (r >= c) { r -= c; x >>= 8; pos += 8; }
  c = (uint32_t)__popc(x & 0xFu);
  if (r >= c) { r -= c; x >>= 4; pos += 4; }
  c = (uint32_t)__popc(x & 0x3u);
  if (r >= c) { r -= c; x >>= 2; pos += 2; }
  if (r >= (x & 1u)) pos += 1;
  return pos;
}

// From word w of H whose wanted bits (ones, or zeros when ZEROS) below the
// start are already masked out of b, the word holding wanted bit number r and
// that bit's position, reading two words per round (both loads in flight).
// The word after H's last lies in the same allocation (L, S1 or S0 follow),
// and the wanted bit always lies inside H, so the read ahead stays in bounds.
template <bool ZEROS>
__device__ __forceinline__ uint64_t ef_scan(const uint64_t* __restrict__ H, uint64_t w, uint64_t b, uint64_t r) {
  while (true) {
    const uint32_t c = (uint32_t)__popcll(b);
    if (r < c) break;
    r -= c;
    const uint64_t b1 = ZEROS ? ~H[w + 1] : H[w + 1];
    const uint64_t b2 = ZEROS ? ~H[w + 2] : H[w + 2];
    const uint32_t c1 = (uint32_t)__popcll(b1);
    if (r < c1) {
      b = b1;
      w += 1;
      break;
    }
    r -= c1;
    b = b2;
    w += 2;
  }
  return (w << 6) + nth_set_bit(b, (uint32_t)r);
}

__device__ __forceinline__ uint64_t ef_low(const EFDev& e, uint64_t i) {
  if (e.l == 0) return 0;
  const uint64_t bit = i * e.l;
  if (e.l <= 32) {
    // the field lies inside the 64 bits from the 32-bit word holding its first
    // bit: two word loads side by side and one funnel shift, no branch (the
    // word after L's last is S1's first, inside the same allocation)
    const uint32_t* __restrict__ L32 = reinterpret_cast<const uint32_t*>(e.L);
    const uint64_t w32 = bit >> 5;
    const uint32_t v = __builtin_amdgcn_alignbit(L32[w32 + 1], L32[w32], (uint32_t)bit & 31u);
    return e.l == 32 ? (uint64_t)v : (uint64_t)(v & ((1u << e.l) - 1u));
  }
  const uint64_t w = bit >> 6;
  const uint32_t o = (uint32_t)(bit & 63);
  uint64_t v = e.L[w] >> o;
  if (o + e.l > 64) v |= e.L[w + 1] << (64 - o);
  return v & ((1ull << e.l) - 1);
}

// Position of one number i (i < m): from the sample of its quantum, count
// ones word by word.
__device__ __forceinline__ uint64_t ef_one_pos(const EFDev& e, uint64_t i) {
  const uint64_t j = i >> e.lgq;
  const uint64_t p = e.S1[j];
  const uint64_t r = i - (j << e.lgq);
  const uint64_t w = p >> 6;
  return ef_scan<false>(e.H, w, e.H[w] & (~0ull << (p & 63)), r);
}

// Position of zero number z (z < n_zeros).
__device__ __forceinline__ uint64_t ef_zero_pos(const EFDev& e, uint64_t z) {
  const uint64_t j = z >> e.lgq;
  const uint64_t p = e.S0[j];
  const uint64_t r = z - (j << e.lgq);
  const uint64_t w = p >> 6;
  return ef_scan<true>(e.H, w, ~e.H[w] & (~0ull << (p & 63)), r);
}

// select(i): the i-th smallest code (i < m).
__device__ __forceinline__ uint64_t ef_select(const EFDev& e, uint64_t i) {
  return ((ef_one_pos(e, i) - i) << e.l) | ef_low(e, i);
}

// The codes with high part hx: index i of the first one, and (when c is not
// null) how many.  Their ones follow zero number hx - 1 (or start H when
// hx = 0) and run up to zero number hx; the run is measured a 64-byte line
// of H (8 words, loaded together) at a time.
__device__ __forceinline__ void ef_bucket(const EFDev& e, uint64_t hx, uint64_t* i, uint64_t* c) {
  uint64_t q = 0;
  *i = 0;
  if (hx > 0) {
    const uint64_t p0 = ef_zero_pos(e, hx - 1);
    *i = p0 - (hx - 1);
    q = p0 + 1;
  }
  if (!c) return;
  uint64_t n = 0;
  while (q < e.h_bits) {
    const uint32_t s = (uint32_t)(q & 63);
    const uint64_t rem = e.H[q >> 6] >> s;
    const uint32_t left = 64u - s;
    const uint64_t full = left == 64u ? ~0ull : ((1ull << left) - 1);
    if (rem == full) {
      n += left;
      q += left;
      continue;
    }
    n += (uint64_t)__builtin_ctzll(~rem);
    break;
  }
  *c = n;
}

// First index in [i, i + c) of the bucket whose low part is >= xl (low parts
// increase inside a bucket), or i + c: a bisection over the packed low parts.
__device__ __forceinline__ uint64_t ef_low_bound(const EFDev& e, uint64_t i, uint64_t c, uint64_t xl) {
  uint64_t lo = i, hi = i + c;
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (ef_low(e, mid) < xl) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// rank(x): codes strictly below x.  Codes with high part below hx = x >> l
// come before the bucket of hx; inside the bucket they are ordered by their
// low parts.
__device__ __forceinline__ uint64_t ef_rank(const EFDev& e, uint64_t x) {
  if (e.m == 0) return 0;
  const uint64_t hx = x >> e.l;
  if (hx >= e.n_zeros) return e.m;
  const uint64_t xl = e.l ? (x & ((1ull << e.l) - 1)) : 0;
  uint64_t i, c = 0;
  ef_bucket(e, hx, &i, xl == 0 ? nullptr : &c);  // a row start (low part 0) needs no run length
  return xl == 0 ? i : ef_low_bound(e, i, c, xl);
}

// rank(x), and whether x is present (the code at the rank equals x).
__device__ __forceinline__ uint64_t ef_rank_has(const EFDev& e, uint64_t x, bool* has) {
  *has = false;
  if (e.m == 0) return 0;
  const uint64_t hx = x >> e.l;
  if (hx >= e.n_zeros) return e.m;
  uint64_t i, c;
  ef_bucket(e, hx, &i, &c);
  const uint64_t xl = e.l ? (x & ((1ull << e.l) - 1)) : 0;
  const uint64_t j = ef_low_bound(e, i, c, xl);
  *has = j < i + c && ef_low(e, j) == xl;
  return j;
}

// Is x a code of the list?
__device__ __forceinline__ bool ef_contains(const EFDev& e, uint64_t x) {
  bool has;
  (void)ef_rank_has(e, x, &has);
  return has;
}

// The row of node v: lo = rank(phi(v, 0)) and d = rank(phi(v + 1, 0)) - lo.
// When phi(v, 0) has no low bits (l <= k) both ranks are zero positions, the
// second hx1 - hx0 zeros after the first: one select and a continued word
// scan instead of two selects.
__device__ __forceinline__ void ef_row(const EFDev& e, int32_t v, uint64_t* lo, uint32_t* d) {
  const uint64_t x0 = (uint64_t)(uint32_t)v << e.k, x1 = ((uint64_t)(uint32_t)v + 1) << e.k;
  if (e.l > e.k || e.m == 0) {
    *lo = ef_rank(e, x0);
    *d = (uint32_t)(ef_rank(e, x1) - *lo);
    return;
  }
  const uint64_t hx0 = x0 >> e.l, hx1 = x1 >> e.l;
  if (hx0 >= e.n_zeros) {
    *lo = e.m;
    *d = 0;
    return;
  }
  uint64_t i0 = 0, q = 0;  // zero number hx0 - 1 ends the codes below x0; the scan goes on from q
  if (hx0 > 0) {
    const uint64_t p0 = ef_zero_pos(e, hx0 - 1);
    i0 = p0 - (hx0 - 1);
    q = p0 + 1;
  }
  *lo = i0;
  if (hx1 >= e.n_zeros) {
    *d = (uint32_t)(e.m - i0);
    return;
  }
  // zero number hx1 - 1: the (hx1 - 1 - (hx0 ? hx0 : 0))-th zero from q (0-based)
  const uint64_t r = (hx1 - 1) - (hx0 > 0 ? hx0 : 0);
  const uint64_t w = q >> 6;
  const uint64_t p1 = ef_scan<true>(e.H, w, ~e.H[w] & (~0ull << (q & 63)), r);
  *d = (uint32_t)(p1 - (hx1 - 1) - i0);
}

__device__ __forceinline__ int32_t ef_nbr(const EFDev& e, uint64_t idx) {
  return (int32_t)(ef_select(e, idx) & ((1ull << e.k) - 1));
}

// ---------------------------------------------------------------------------
// Construction from a validated CSR.
// ---------------------------------------------------------------------------
constexpr uint32_t kEfChunk = 4096;

// Last a in [alo, ahi] with O[a] <= i (rows may be empty), given O[alo] <= i.
__device__ __forceinline__ int64_t src_of(const uint64_t* __restrict__ O, int64_t alo, int64_t ahi, uint64_t i) {
  while (alo < ahi) {
    const int64_t mid = alo + ((ahi - alo + 1) >> 1);
    if (O[mid] <= i) alo = mid;
    else ahi = mid - 1;
  }
  return alo;
}

// Every entry sets its bit of H and ORs its low part into L (both zeroed).
// A block takes a chunk of entries and narrows the source search to the
// rows the chunk spans.
__global__ __launch_bounds__(256) void k_ef_fill(const uint64_t* __restrict__ O, int64_t n,
                                                 const int32_t* __restrict__ D, EFDev e, uint64_t* H, uint64_t* L) {
  __shared__ int64_t rows[2];
  for (uint64_t e0 = (uint64_t)blockIdx.x * kEfChunk; e0 < e.m; e0 += (uint64_t)gridDim.x * kEfChunk) {
    const uint64_t e1 = e0 + kEfChunk < e.m ? e0 + kEfChunk : e.m;
    __syncthreads();
    if (threadIdx.x == 0) {
      rows[0] = src_of(O, 0, n - 1, e0);
      rows[1] = src_of(O, 0, n - 1, e1 - 1);
    }
    __syncthreads();
    const int64_t a0 = rows[0], a1 = rows[1];
    for (uint64_t i = e0 + threadIdx.x; i < e1; i += 256) {
      const int64_t a = src_of(O, a0, a1, i);
      const uint64_t code = ((uint64_t)a << e.k) | (uint64_t)(uint32_t)D[i];
      const uint64_t p = (code >> e.l) + i;
      atomicOr((unsigned long long*)&H[p >> 6], 1ull << (p & 63));
      if (e.l) {
        const uint64_t low = code & ((1ull << e.l) - 1);
        const uint64_t bit = i * e.l;
        const uint64_t w = bit >> 6;
        const uint32_t o = (uint32_t)(bit & 63);
        atomicOr((unsigned long long*)&L[w], low << o);
        if (o + e.l > 64) atomicOr((unsigned long long*)&L[w + 1], low >> (64 - o));
      }
    }
  }
}

// Quantum indexes, straight from the CSR: one number i sits at
// (code_i >> l) + i; zero number z sits after the codes whose high part is at
// most z, i.e. at z + #{codes < (z + 1) 2^l}.
__global__ __launch_bounds__(256) void k_ef_index(const uint64_t* __restrict__ O, int64_t n,
                                                  const int32_t* __restrict__ D, EFDev e, uint64_t s1_len,
                                                  uint64_t s0_len, uint64_t* S1, uint64_t* S0) {
  const uint64_t kmask = (1ull << e.k) - 1;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < s1_len + s0_len;
       j += (uint64_t)gridDim.x * blockDim.x) {
    if (j < s1_len) {
      const uint64_t i = j << e.lgq;
      const int64_t a = src_of(O, 0, n - 1, i);
      const uint64_t code = ((uint64_t)a << e.k) | (uint64_t)(uint32_t)D[i];
      S1[j] = (code >> e.l) + i;
    } else {
      const uint64_t z = (j - s1_len) << e.lgq;
      const uint64_t y = (z + 1) << e.l;
      const uint64_t a = y >> e.k;
      uint64_t c = e.m;
      if (a < (uint64_t)n) {
        const uint64_t lo = O[a];
        c = lo + lower_bound_i32(D + lo, (uint32_t)(O[a + 1] - lo), (int32_t)(y & kmask));
      }
      S0[j - s1_len] = z + c;
    }
  }
}

__global__ __launch_bounds__(256) void k_ef_select_bulk(EFDev e, const uint64_t* __restrict__ idx, uint64_t count,
                                                        uint64_t* __restrict__ out) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x)
    out[t] = idx[t] < e.m ? ef_select(e, idx[t]) : ~0ull;
}

__global__ __launch_bounds__(256) void k_ef_rank_bulk(EFDev e, const uint64_t* __restrict__ x, uint64_t count,
                                                      uint64_t* __restrict__ out) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x)
    out[t] = ef_rank(e, x[t]);
}

// ---------------------------------------------------------------------------
// Walks.  The arithmetic is that of the CSR kernels; the row of v is
// [rank(phi(v, 0)), rank(phi(v + 1, 0))), weights are differences of the row
// prefix R, and t is found in N(v) by rank(phi(v, t)).
// ---------------------------------------------------------------------------
enum { kEfFoUnw = 0, kEfFoW = 1, kEfRetUnw = 2, kEfRetW = 3 };

template <typename RT>
__device__ __forceinline__ uint64_t weight_at(const RT* __restrict__ R, uint64_t lo, uint32_t j) {
  const uint64_t hi = (uint64_t)R[lo + j];
  return j ? hi - (uint64_t)R[lo + j - 1] : hi;
}

template <int MODE, typename RT>
__device__ __forceinline__ void lane_walk_ef(const WalkArgs& a, const EFDev& e, uint64_t w) {
  const RT* __restrict__ R = (const RT*)a.g.R;
  int32_t* __restrict__ row = a.Y + w * a.L;
  const int32_t start = a.starts[w % a.ns];
  const uint64_t wid = a.wid_base + w;
  uint32_t len = 0;
  if (start >= 0 && (int64_t)start < a.g.n) {
    row[0] = start;
    len = 1;
    int32_t v = start, t = -1;
    uint64_t lo;
    uint32_t dnext;
    ef_row(e, v, &lo, &dnext);
    for (uint32_t s = 1; s < a.L; ++s) {
      const uint32_t d = dnext;
      if (d == 0) break;  // dead end
      const uint64_t r = philox_draw(a.seed, s, wid);
      uint32_t j;
      if (MODE == kEfFoUnw || (MODE == kEfRetUnw && t < 0)) {
        j = (uint32_t)scale_draw(r, d);
      } else if (MODE == kEfFoW || (MODE == kEfRetW && t < 0)) {
        const uint64_t total = (uint64_t)R[lo + d - 1];
        if (total == 0) break;
        j = upper_bound_interp(R + lo, d, scale_draw(r, total), total);
      } else {
        const uint64_t tc = ((uint64_t)v << e.k) | (uint64_t)(uint32_t)t;
        const uint64_t rt = ef_rank(e, tc);
        const uint32_t pt = (uint32_t)(rt - lo);  // entries of N(v) below t
        const bool has_t = pt < d && ef_select(e, rt) == tc;
        uint64_t wt = 0;
        if (has_t) wt = (MODE == kEfRetW) ? weight_at(R, lo, pt) : 1ull;
        const uint64_t S = (MODE == kEfRetW) ? (uint64_t)R[lo + d - 1] : (uint64_t)d;
        const uint64_t corr = ((uint64_t)a.P16 - (uint64_t)kC16) * wt;  // mod 2^64
        const uint64_t total = (uint64_t)kC16 * S + corr;
        if (total == 0) break;
        const uint64_t T = scale_draw(r, total);
        j = first_above_interp(d, T, total, [&](uint32_t m) -> uint64_t {
          const uint64_t Rm = (MODE == kEfRetW) ? (uint64_t)R[lo + m] : (uint64_t)(m + 1);
          return (uint64_t)kC16 * Rm + (m >= pt ? corr : 0ull);
        });
      }
      const int32_t x = ef_nbr(e, lo + j);
      row[s] = x;
      len = s + 1;
      t = v;
      v = x;
      ef_row(e, v, &lo, &dnext);
    }
  }
  for (uint32_t s = len; s < a.L; ++s) row[s] = -1;
  if (a.lens) a.lens[w] = (int32_t)len;
  if (a.steps && len > 1) atomicAdd(a.steps, (unsigned long long)(len - 1));
}

template <int MODE, typename RT>
__global__ __launch_bounds__(256, 8) void k_walk_lane_ef(WalkArgs a, EFDev e, unsigned long long* ctr, uint32_t chunk) {
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
      for (uint64_t w = base + lane; w < end; w += 64) lane_walk_ef<MODE, RT>(a, e, w);
    }
    return;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nwalks; w += stride)
    lane_walk_ef<MODE, RT>(a, e, w);
}

// node2vec with 1/q != 1: one wavefront per walk, two passes over the biased
// weights of N(v) (block sums, then a scan of the block holding the draw).
// Rows of at most kEfTile entries are decoded into LDS as they are streamed,
// so the next step tests membership in N(t) by bisecting LDS; longer rows of
// t are tested in the store itself.
constexpr uint32_t kEfTile = 512;
constexpr uint32_t kEfList = kEfTile;  // common-neighbour list of the probe route (in the idle tile)
constexpr uint32_t kEfList2 = 256;     // common-neighbour list of the stream route (its own buffer)

__device__ __forceinline__ bool lds_has(const int32_t* A, uint32_t n, int32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (A[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && A[lo] == x;
}

// Cooperative decode of codes [i0, i0 + n) (n <= 64, wave-uniform) by the
// whole wavefront, lane g getting code i0 + g: the ones of consecutive codes
// are consecutive ones of H, so from the position `pos` of one number i0 the
// lanes read 64 consecutive words of H at once, count their ones (a wave
// scan), find the word holding their one by a bisection over the lanes'
// counts (cross-lane reads) and its bit by a popcount bisection; the low
// parts are consecutive fields of L.  Returns the lane's code; pos becomes
// the position after the last decoded one (one select for a whole row).
__device__ __forceinline__ uint64_t ef_decode_chunk(const EFDev& e, uint64_t i0, uint32_t n, uint64_t& pos, int gl) {
  uint64_t code = 0, mine = 0;
  uint32_t got = 0;
  uint64_t w0 = pos >> 6;
  uint64_t mask0 = ~0ull << (pos & 63);
  while (got < n) {
    const uint64_t wi = w0 + (uint64_t)gl;
    const uint64_t word = (wi << 6) < e.h_bits ? e.H[wi] & (gl == 0 ? mask0 : ~0ull) : 0ull;
    const uint32_t incl = wave_incl_scan_u32((uint32_t)__popcll(word));
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t r = (uint32_t)gl - got;  // this lane's one within the round
    const bool want = (uint32_t)gl >= got && (uint32_t)gl < n && r < total;
    // first lane whose inclusive count exceeds r (every lane takes part in the reads)
    int lo = 0, hi = 63;
    for (int it = 0; it < 6; ++it) {
      const int mid = (lo + hi) >> 1;
      const uint32_t cm = (uint32_t)__shfl((int)incl, mid, 64);
      if (cm > r) hi = mid;
      else lo = mid + 1;
    }
    const int L = lo;
    const uint32_t cL = (uint32_t)__shfl((int)incl, L, 64);
    const uint32_t wlo = (uint32_t)__shfl((int)(uint32_t)word, L, 64);
    const uint32_t whi = (uint32_t)__shfl((int)(uint32_t)(word >> 32), L, 64);
    if (want) {
      const uint64_t wL = (uint64_t)wlo | ((uint64_t)whi << 32);
      const uint32_t excl = cL - (uint32_t)__popcll(wL);
      const uint64_t p = ((w0 + (uint64_t)L) << 6) + nth_set_bit(wL, r - excl);
      mine = p;
      code = ((p - (i0 + (uint64_t)gl)) << e.l) | ef_low(e, i0 + (uint64_t)gl);
    }
    got += total < n - got ? total : n - got;
    w0 += 64;
    mask0 = ~0ull;
  }
  const uint64_t plast = (uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)mine, (int)(n - 1)) |
                         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mine >> 32), (int)(n - 1)) << 32);
  pos = plast + 1;
  return code;
}

// Positions of zeros z0 .. z0 + cnt - 1 of H (cnt <= 64, zero z0 + cnt - 1
// exists), lane j getting zero z0 + j (other lanes: unspecified).  From the
// quantum sample at or before z0 the wavefront reads 64 words of H at a time,
// counts their zeros (a wave scan), and each lane finds the word of its zero
// by a bisection over the lanes' counts and its bit by a popcount bisection:
// one round per 4096 bits, where a one-lane select scans word by word.
__device__ __forceinline__ uint64_t wave_zero_positions(const EFDev& e, uint64_t z0, uint32_t cnt, int gl) {
  const uint64_t js = z0 >> e.lgq;
  const uint64_t p = e.S0[js];  // position of zero js 2^lgq
  const uint32_t skip = (uint32_t)(z0 - (js << e.lgq));
  const uint32_t want = skip + (uint32_t)gl;  // this lane's zero, counted from the one at p
  const uint32_t last = skip + cnt - 1u;
  const uint64_t hw = (e.h_bits + 63) >> 6;
  const uint32_t tail = (uint32_t)(e.h_bits & 63);
  uint64_t w0 = p >> 6;
  uint64_t mask0 = ~0ull << (p & 63);
  uint32_t got = 0;
  uint64_t mine = 0;
  while (got <= last) {
    const uint64_t wi = w0 + (uint64_t)gl;
    uint64_t word = 0;
    if (wi < hw) {
      word = ~e.H[wi] & (gl == 0 ? mask0 : ~0ull);
      if (wi == hw - 1 && tail) word &= (1ull << tail) - 1;  // no zeros past the end of H
    }
    const uint32_t incl = wave_incl_scan_u32((uint32_t)__popcll(word));
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t r = want - got;
    const bool here = (uint32_t)gl < cnt && want >= got && r < total;
    int lo = 0, hi = 63;  // first lane whose inclusive count exceeds r
    for (int it = 0; it < 6; ++it) {
      const int mid = (lo + hi) >> 1;
      const uint32_t cm = (uint32_t)__shfl((int)incl, mid, 64);
      if (cm > r) hi = mid;
      else lo = mid + 1;
    }
    const uint32_t cL = (uint32_t)__shfl((int)incl, lo, 64);
    const uint32_t wlo = (uint32_t)__shfl((int)(uint32_t)word, lo, 64);
    const uint32_t whi = (uint32_t)__shfl((int)(uint32_t)(word >> 32), lo, 64);
    if (here) {
      const uint64_t wL = (uint64_t)wlo | ((uint64_t)whi << 32);
      mine = ((w0 + (uint64_t)lo) << 6) + nth_set_bit(wL, r - (cL - (uint32_t)__popcll(wL)));
    }
    got += total;
    w0 += 64;
    mask0 = ~0ull;
  }
  return mine;
}

// When a row spans nb = 2^(k - l) < 64 buckets of high parts (l <= k), the
// wavefront keeps the row's bucket boundaries: lane j <= nb holds the position
// of zero hx0 - 1 + j, hx0 = v nb (-1 for the zero before H when v = 0).  The
// row is [zb_0 - (hx0 - 1), zb_nb - (hx0 + nb - 1)), and bucket b holds the
// codes [zb_b + 1 - (hx0 + b), +(zb_(b+1) - zb_b - 1)).  One cooperative
// decode per step replaces the word-by-word zero scans of every rank into the
// row (a hub's row spans thousands of words).
__device__ __forceinline__ int64_t ef_row_bounds(const EFDev& e, int32_t v, uint32_t nb, int gl, uint64_t* lo,
                                                 uint32_t* d) {
  const uint64_t hx0 = (uint64_t)(uint32_t)v * nb;
  int64_t zb;
  if (hx0 > 0) {
    zb = (int64_t)wave_zero_positions(e, hx0 - 1, nb + 1, gl);
  } else {
    const int64_t z = (int64_t)wave_zero_positions(e, 0, nb, gl);  // lane j: zero j
    const int src = gl > 0 ? gl - 1 : 0;
    const int64_t zs = (int64_t)(((uint64_t)(uint32_t)__shfl((int)(uint32_t)((uint64_t)z >> 32), src, 64) << 32) |
                                 (uint64_t)(uint32_t)__shfl((int)(uint32_t)(uint64_t)z, src, 64));
    zb = gl == 0 ? -1 : zs;
  }
  const int64_t z0 = (int64_t)wave_read_u64((uint64_t)zb, 0);
  const int64_t z1 = (int64_t)wave_read_u64((uint64_t)zb, (int)nb);
  *lo = (uint64_t)(z0 + 1) - hx0;
  *d = (uint32_t)(((uint64_t)(z1 + 1) - (hx0 + nb)) - *lo);
  return zb;
}

// The boundaries of bucket b of the row whose boundaries the lanes hold (every
// lane of the wavefront takes part: call from uniform control flow).
__device__ __forceinline__ void ef_bucket_of(int64_t zb, uint32_t b, int64_t* za, int64_t* zc) {
  auto rd = [&](uint32_t src) {
    return (int64_t)(((uint64_t)(uint32_t)__shfl((int)(uint32_t)((uint64_t)zb >> 32), (int)src, 64) << 32) |
                     (uint64_t)(uint32_t)__shfl((int)(uint32_t)(uint64_t)zb, (int)src, 64));
  };
  *za = rd(b);
  *zc = rd(b + 1);
}

// rank of the code hx0 2^l + y' (y' = y, a node id) inside its row, from the
// bucket boundaries za, zc of its bucket b = y >> l, and whether it is present.
__device__ __forceinline__ uint64_t ef_rank_in_bucket(const EFDev& e, uint64_t hx0, uint32_t y, int64_t za,
                                                      int64_t zc, bool* has) {
  const uint32_t b = y >> e.l;
  const uint64_t xl = e.l ? ((uint64_t)y & ((1ull << e.l) - 1)) : 0;
  const uint64_t i = (uint64_t)(za + 1) - (hx0 + b);
  const uint64_t c = (uint64_t)(zc - za - 1);
  const uint64_t j = xl == 0 ? i : ef_low_bound(e, i, c, xl);
  *has = j < i + c && ef_low(e, j) == xl;
  return j;
}

// First j in [lo, hi) with pred(j) (monotone), or hi: 64 evenly spaced
// probes per round across the wavefront.
template <typename P>
__device__ __forceinline__ uint32_t wave_first(uint32_t lo, uint32_t hi, int gl, P pred) {
  while (hi - lo > 64u) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t j = lo + (uint32_t)(gl + 1) * step - 1;
    const bool pr = j < hi ? pred(j) : true;
    const uint64_t m = grp_ballot<64>(pr, 0);
    if (m == 0) return hi;
    const int f = __ffsll((unsigned long long)m) - 1;
    const uint32_t jf = (uint32_t)grp_bcast_i32<64>((int32_t)j, f);
    lo = lo + (uint32_t)f * step;
    if (jf < hi) hi = jf;
  }
  const uint32_t j = lo + (uint32_t)gl;
  const uint64_t m = grp_ballot<64>(j < hi && pred(j), 0);
  return m ? lo + (uint32_t)(__ffsll((unsigned long long)m) - 1) : hi;
}

template <bool WEIGHTED, typename RT>
__device__ __forceinline__ void wave_walk_ef(const WalkArgs& a, const EFDev& e, uint64_t w, int gl, int32_t* bufA,
                                             int32_t* bufB, uint32_t* lbuf) {
  constexpr int G = 64;
  const RT* __restrict__ R = (const RT*)a.g.R;
  const uint64_t P16 = a.P16, Q16 = a.Q16;
  int32_t* __restrict__ row = a.Y + w * a.L;
  const int32_t start = a.starts[w % a.ns];
  const uint64_t wid = a.wid_base + w;
  uint32_t len = 0;
  if (start >= 0 && (int64_t)start < a.g.n) {
    if (gl == 0) row[0] = start;
    len = 1;
    int32_t v = start, t = -1;
    int32_t* cur = bufA;  // decoded N(t) when t_in_lds
    int32_t* nxt = bufB;  // N(v) being decoded
    bool t_in_lds = false;
    uint32_t td = 0;
    uint64_t tlo = 0;
    uint64_t lo;
    uint32_t dnext;
    // bucket boundaries of the rows of v and t (lanes 0 .. nb), when a row
    // spans fewer than 64 buckets
    const bool use_b = e.l <= e.k && e.k - e.l < 6;
    const uint32_t nb = use_b ? 1u << (e.k - e.l) : 0u;
    int64_t vb = 0, tb = 0;
    if (use_b) vb = ef_row_bounds(e, v, nb, gl, &lo, &dnext);
    else ef_row(e, v, &lo, &dnext);
    const uint64_t lt_mask = gl == 0 ? 0ull : (~0ull >> (64 - gl));
    auto Rv = [&](uint32_t j) -> uint64_t { return WEIGHTED ? (uint64_t)R[lo + j] : (uint64_t)j + 1ull; };
    // lane gl holds the draw of step s1 + gl: one vector Philox evaluation
    // every 64 steps instead of a scalar one per step
    uint64_t rdraw = 0;
    for (uint32_t s = 1; s < a.L; ++s) {
      const uint32_t d = dnext;
      if (d == 0) break;
      const uint32_t sk = (s - 1u) & 63u;
      if (sk == 0) rdraw = philox_draw(a.seed, s + (uint32_t)gl, wid);
      const uint64_t r = wave_read_u64(rdraw, (int)sk);
      bool stage = a.second_order && d <= kEfTile;
      uint32_t jsel = d;
      if (!a.second_order || t < 0) {
        const uint64_t S = WEIGHTED ? (uint64_t)R[lo + d - 1] : (uint64_t)d;
        if (S == 0) break;
        const uint64_t T = scale_draw(r, S);
        jsel = WEIGHTED ? upper_bound_gt(R + lo, d, T) : (uint32_t)T;
        if (stage) {
          uint64_t hpos = ef_one_pos(e, lo);
          for (uint32_t c = 0; c < d; c += G) {
            const uint32_t nn = d - c < (uint32_t)G ? d - c : (uint32_t)G;
            const uint64_t code = ef_decode_chunk(e, lo + c, nn, hpos, gl);
            if (c + (uint32_t)gl < d) nxt[c + gl] = (int32_t)(code & ((1ull << e.k) - 1));
          }
        }
      } else {
        bool done = false;
        // The positions in N(v) of the common neighbours (x in N(t), x != t),
        // their weight sum and the position of t, by one of two routes; then
        // the draw is located through them and a search of the row prefix
        // between two of them, B_j = Q16 R_j + (C16 - Q16) sum_{common c <= j}
        // w_c + (P16 - Q16) w_t [j >= pt] (mod 2^64, exact).  A list longer than
        // its LDS buffer falls back to the two-pass stream below.
        uint32_t* lpos = lbuf;
        uint32_t lcap = kEfList2;
        uint32_t cnt = 0, pt = 0;
        bool has_t = false;
        uint64_t cw = 0;
        // route by a dependent-load estimate per 64 keys: a decoded candidate
        // tested in LDS ~3, in the store ~17 (rank: a zero select, the bucket's
        // run, a bisection of its low parts); a key of N(t) ranked into N(v)
        // ~16 from LDS, ~19 decoded from the store
        const uint64_t c_stream = (uint64_t)((d + G - 1) / G) * (t_in_lds ? 3u : 17u);
        const uint64_t c_probe = (uint64_t)((td + 1 + G - 1) / G) * (t_in_lds ? 16u : 19u);
        if (c_probe < c_stream) {
          // Probe route: rank every key of N(t) (and t) into N(v).  Hits come
          // in increasing position.  The list goes to the tile of N(v) when the
          // row is too long to stage, else to the list buffer (and the row is
          // not staged for the next step).
          if (d > kEfTile) {
            lpos = reinterpret_cast<uint32_t*>(nxt);
            lcap = kEfList;
          }
          stage = false;
          const uint64_t vc0 = (uint64_t)v << e.k;
          for (uint32_t c = 0; c < td + 1; c += G) {
            const uint32_t k = c + (uint32_t)gl;
            const bool tkey = k == td;
            bool hit = false;
            uint32_t pos = 0;
            int32_t y = t;
            if (k < td) y = t_in_lds ? cur[k] : ef_nbr(e, tlo + k);
            if (use_b) {
              int64_t za, zc;
              ef_bucket_of(vb, (uint32_t)y >> e.l, &za, &zc);
              if (k <= td) pos = (uint32_t)(ef_rank_in_bucket(e, (uint64_t)(uint32_t)v * nb, (uint32_t)y, za, zc, &hit) - lo);
            } else if (k <= td) {
              pos = (uint32_t)(ef_rank_has(e, vc0 | (uint64_t)(uint32_t)y, &hit) - lo);
            }
            const uint64_t mt = grp_ballot<G>(hit && tkey, 0);
            if (mt) {
              has_t = true;
              pt = (uint32_t)grp_bcast_i32<G>((int32_t)pos, __ffsll((unsigned long long)mt) - 1);
            }
            // a self-loop at t puts t in N(t): that candidate is a return, not common
            const bool common = hit && !tkey && y != t;
            const uint64_t m = grp_ballot<G>(common, 0);
            if (common) {
              cw += WEIGHTED ? weight_at(R, lo, pos) : 1ull;
              const uint32_t idx = cnt + (uint32_t)__popcll(m & lt_mask);
              if (idx < lcap) lpos[idx] = pos;
            }
            cnt += (uint32_t)__popcll(m);
          }
        } else {
          // Stream route: N(v) decoded 64 codes at a time from one select
          // (staged in LDS when short), each candidate tested against N(t)
          // in LDS or in the store.
          uint64_t hpos = ef_one_pos(e, lo);
          const uint64_t tc0 = (uint64_t)t << e.k;
          const uint64_t kmask = (1ull << e.k) - 1;
          for (uint32_t c = 0; c < d; c += G) {
            const uint32_t nn = d - c < (uint32_t)G ? d - c : (uint32_t)G;
            const uint64_t code = ef_decode_chunk(e, lo + c, nn, hpos, gl);
            const uint32_t j = c + (uint32_t)gl;
            const bool act = j < d;
            const int32_t x = (int32_t)(code & kmask);
            if (act && stage) nxt[j] = x;
            const bool isret = act && x == t;
            const uint64_t mt = grp_ballot<G>(isret, 0);
            if (mt) {
              has_t = true;
              pt = c + (uint32_t)(__ffsll((unsigned long long)mt) - 1);
            }
            bool common;
            if (!t_in_lds && use_b) {
              int64_t za, zc;
              ef_bucket_of(tb, (uint32_t)x >> e.l, &za, &zc);
              bool h = false;
              if (act && !isret) (void)ef_rank_in_bucket(e, (uint64_t)(uint32_t)t * nb, (uint32_t)x, za, zc, &h);
              common = act && !isret && h;
            } else {
              common = act && !isret && (t_in_lds ? lds_has(cur, td, x) : ef_contains(e, tc0 | (uint64_t)(uint32_t)x));
            }
            const uint64_t m = grp_ballot<G>(common, 0);
            if (common) {
              cw += WEIGHTED ? weight_at(R, lo, j) : 1ull;
              const uint32_t idx = cnt + (uint32_t)__popcll(m & lt_mask);
              if (idx < lcap) lpos[idx] = j;
            }
            cnt += (uint32_t)__popcll(m);
          }
        }
        if (cnt <= lcap) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const uint64_t cdel = (uint64_t)kC16 - Q16, rdel = P16 - Q16;
          const uint64_t CW = grp_sum<G>(cw);
          const uint64_t wt = has_t ? (WEIGHTED ? weight_at(R, lo, pt) : 1ull) : 0ull;
          const uint64_t retw = rdel * wt;
          const uint64_t S = WEIGHTED ? (uint64_t)R[lo + d - 1] : (uint64_t)d;
          const uint64_t total = Q16 * S + cdel * CW + retw;
          if (total == 0) break;
          const uint64_t T = scale_draw(r, total);
          // first listed position whose B exceeds T: the segment before it
          // holds no common neighbour
          uint64_t E = 0, Eseg = CW;
          uint32_t seg_lo = 0, seg_end = d, lastpos = 0;
          bool found = false, any = false;
          for (uint32_t c = 0; c < cnt; c += G) {
            const uint32_t k = c + (uint32_t)gl;
            const bool act = k < cnt;
            const uint32_t p = act ? lpos[k] : 0u;
            const uint64_t wk = act ? (WEIGHTED ? weight_at(R, lo, p) : 1ull) : 0ull;
            const uint64_t inc = grp_incl_scan<G>(wk, gl);
            const uint64_t Ek = E + inc;
            const uint64_t Bk = Q16 * Rv(p) + cdel * Ek + ((has_t && p >= pt) ? retw : 0ull);
            const uint64_t mb = grp_ballot<G>(act && Bk > T, 0);
            if (mb) {
              const int f = __ffsll((unsigned long long)mb) - 1;
              Eseg = grp_bcast<G>(Ek - wk, f);
              seg_end = (uint32_t)grp_bcast_i32<G>((int32_t)p, f);
              const uint32_t pprev = (uint32_t)grp_bcast_i32<G>((int32_t)p, f > 0 ? f - 1 : 0);
              seg_lo = f > 0 ? pprev + 1 : (any ? lastpos + 1 : 0u);
              found = true;
              break;
            }
            const uint32_t nact = min((uint32_t)G, cnt - c);
            lastpos = (uint32_t)grp_bcast_i32<G>((int32_t)p, (int)nact - 1);
            any = true;
            E += grp_bcast<G>(inc, G - 1);
          }
          if (!found) seg_lo = any ? lastpos + 1 : 0u;
          // first j in [seg_lo, seg_end) with B_j > T (common weight Eseg
          // there); none: the listed position seg_end itself
          const uint64_t base = cdel * Eseg;
          jsel = wave_first(seg_lo, seg_end, gl, [&](uint32_t j) {
            return Q16 * Rv(j) + base + ((has_t && j >= pt) ? retw : 0ull) > T;
          });
          done = true;
        }
        if (!done) {
        const uint64_t tc0 = (uint64_t)t << e.k;
        auto bias_of = [&](uint32_t j, int32_t x) -> uint64_t {
          const uint64_t wt = WEIGHTED ? weight_at(R, lo, j) : 1ull;
          if (x == t) return wt * P16;
          const bool common = t_in_lds ? lds_has(cur, td, x) : ef_contains(e, tc0 | (uint64_t)(uint32_t)x);
          return wt * (common ? (uint64_t)kC16 : Q16);
        };
        const uint32_t nc = (d + G - 1) / G;
        const uint32_t bs = (nc + G - 1) / G;
        uint64_t acc = 0, blk = 0;
        for (uint32_t c = 0; c < nc; ++c) {
          const uint32_t j = c * G + (uint32_t)gl;
          if (j < d) {
            const int32_t x = ef_nbr(e, lo + j);
            if (stage) nxt[j] = x;
            acc += bias_of(j, x);
          }
          if ((c + 1) % bs == 0 || c + 1 == nc) {
            const uint64_t sb = grp_sum<G>(acc);
            if ((uint32_t)gl == c / bs) blk = sb;
            acc = 0;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint64_t incl = grp_incl_scan<G>(blk, gl);
        const uint64_t total = grp_bcast<G>(incl, G - 1);
        if (total == 0) break;
        const uint64_t T = scale_draw(r, total);
        const uint64_t bm = grp_ballot<G>(incl > T, 0);
        const int kb = __ffsll((unsigned long long)bm) - 1;
        uint64_t base = grp_bcast<G>(incl - blk, kb);
        const uint32_t cend = min((uint32_t)(kb + 1) * bs, nc);
        for (uint32_t c = (uint32_t)kb * bs; c < cend; ++c) {
          const uint32_t j = c * G + (uint32_t)gl;
          uint64_t b = 0;
          if (j < d) b = bias_of(j, stage ? nxt[j] : ef_nbr(e, lo + j));
          const uint64_t inc = grp_incl_scan<G>(b, gl);
          const uint64_t m2 = grp_ballot<G>(base + inc > T, 0);
          if (m2) {
            jsel = c * G + (uint32_t)(__ffsll((unsigned long long)m2) - 1);
            break;
          }
          base += grp_bcast<G>(inc, G - 1);
        }
        }
      }
      if (jsel >= d) break;  // unreachable: the draw lies below the total
      // the staged row is read by other lanes of the wave from here on
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int32_t x = stage ? nxt[jsel] : ef_nbr(e, lo + jsel);
      if (gl == 0) row[s] = x;
      len = s + 1;
      t = v;
      td = d;
      tlo = lo;
      t_in_lds = stage;
      if (stage) {
        int32_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
      }
      v = x;
      tb = vb;
      if (use_b) vb = ef_row_bounds(e, v, nb, gl, &lo, &dnext);
      else ef_row(e, v, &lo, &dnext);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  for (uint32_t s = len + (uint32_t)gl; s < a.L; s += G) row[s] = -1;
  if (gl == 0) {
    if (a.lens) a.lens[w] = (int32_t)len;
    if (a.steps && len > 1) atomicAdd(a.steps, (unsigned long long)(len - 1));
  }
}

template <bool WEIGHTED, typename RT>
__global__ __launch_bounds__(256, 8) void k_walk_n2v_ef(WalkArgs a, EFDev e, unsigned long long* ctr, uint32_t chunk) {
  __shared__ int32_t tiles[4][2][kEfTile];
  __shared__ uint32_t lists[4][kEfList2];
  const int gl = threadIdx.x & 63;
  // the wave index is uniform: per-walker state goes to scalar registers
  const int wv = (int)__builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
  // with a launch counter waves take `chunk` walks at a time, else fixed shares
  uint64_t w = ctr ? 0 : (uint64_t)blockIdx.x * (blockDim.x / 64) + wv, end = 0;
  while (true) {
    if (ctr && w >= end) {
      unsigned long long c = 0;
      if (gl == 0) c = atomicAdd(ctr, (unsigned long long)chunk);
      w = wave_read_u64((uint64_t)c, 0);
      end = min(w + chunk, a.nwalks);
    }
    if (w >= a.nwalks) break;
    wave_walk_ef<WEIGHTED, RT>(a, e, w, gl, tiles[wv][0], tiles[wv][1], lists[wv]);
    w += ctr ? 1 : waves;
  }
}

// Scale-free negatives: the node owning entry T of the edge list is the
// source of code T, select(T) >> k.  Same tiles and counters as the CSR form.
__global__ __launch_bounds__(256) void k_negatives_ef(EFDev e, const int32_t* __restrict__ Y, uint64_t n_pos,
                                                      uint32_t L, uint32_t n_neg, uint32_t lgP, uint64_t seed,
                                                      uint64_t wid_base, int32_t* __restrict__ N) {
  extern __shared__ int32_t sm[];  // [P * n_neg]
  const uint32_t P = 1u << lgP;
  const uint32_t npairs = (n_neg + 1u) / 2u;
  const uint32_t t = threadIdx.x;
  for (uint64_t e0 = (uint64_t)blockIdx.x * P; e0 < n_pos; e0 += (uint64_t)gridDim.x * P) {
    const uint32_t np = (uint32_t)(n_pos - e0 < P ? n_pos - e0 : P);
    const uint64_t row0 = e0 / L;
    const uint32_t i0 = (uint32_t)(e0 - row0 * L);
    __syncthreads();
    for (uint32_t it = t; it < P * npairs; it += 256) {
      const uint32_t pos = it & (P - 1u), jp = it >> lgP;
      if (pos >= np) continue;
      int32_t v0 = -1, v1 = -1;
      if (e.m > 0 && Y[e0 + pos] >= 0) {
        uint64_t row;
        uint32_t i;
        split_pos(row0, i0, pos, L, &row, &i);
        const uint64_t wid = wid_base + row;
        uint32_t wd[4];
        philox_words(seed, i, (uint32_t)wid, (uint32_t)(wid >> 32), 0x80000000u + jp, wd);
        v0 = (int32_t)(ef_select(e, scale_draw((uint64_t)wd[0] | ((uint64_t)wd[1] << 32), e.m)) >> e.k);
        if (2u * jp + 1u < n_neg)
          v1 = (int32_t)(ef_select(e, scale_draw((uint64_t)wd[2] | ((uint64_t)wd[3] << 32), e.m)) >> e.k);
      }
      sm[pos * n_neg + 2u * jp] = v0;
      if (2u * jp + 1u < n_neg) sm[pos * n_neg + 2u * jp + 1u] = v1;
    }
    __syncthreads();
    int32_t* __restrict__ out = N + e0 * n_neg;
    for (uint32_t x = t; x < np * n_neg; x += 256) out[x] = sm[x];
  }
}

int ef_blocks(uint64_t items, const DevInfo& di) {
  const uint64_t want = (items + 255) / 256;
  const uint64_t cap = (uint64_t)(di.cus > 0 ? di.cus : 256) * 16;
  return (int)(want < cap ? (want ? want : 1) : cap);
}

}  // namespace

void ef_shape(int64_t n, uint64_t m, uint32_t lgq, EFDev* e, uint64_t* h_words, uint64_t* l_words,
              uint64_t* s1_len, uint64_t* s0_len) {
  uint32_t k = 0;
  while ((1ll << k) < n) ++k;
  e->k = k;
  e->u = (uint64_t)n << k;
  e->m = m;
  uint32_t l = 0;
  if (m > 0) {
    const uint64_t ratio = e->u / m;
    while (l < 63 && (ratio >> (l + 1)) > 0) ++l;
  }
  e->l = l;
  e->lgq = lgq;
  e->n_zeros = ((e->u - 1) >> l) + 1;
  e->h_bits = m + e->n_zeros;
  *h_words = (e->h_bits + 63) / 64;
  *l_words = (m * l + 63) / 64;
  *s1_len = (m + (1ull << lgq) - 1) >> lgq;
  *s0_len = (e->n_zeros + (1ull << lgq) - 1) >> lgq;
}

hipError_t launch_ef_build(const uint64_t* O, int64_t n, const int32_t* D, const EFDev& e, const DevInfo& di,
                           hipStream_t st) {
  uint64_t hw, lw, n1, n0;
  EFDev tmp;
  ef_shape(n, e.m, e.lgq, &tmp, &hw, &lw, &n1, &n0);
  if (e.m > 0) {
    hipLaunchKernelGGL(k_ef_fill, dim3(ef_blocks((e.m + kEfChunk - 1) / kEfChunk * 256, di)), dim3(256), 0, st, O,
                       n, D, e, const_cast<uint64_t*>(e.H), const_cast<uint64_t*>(e.L));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k_ef_index, dim3(ef_blocks(n1 + n0, di)), dim3(256), 0, st, O, n, D, e, n1, n0,
                     const_cast<uint64_t*>(e.S1), const_cast<uint64_t*>(e.S0));
  return hipGetLastError();
}

hipError_t launch_ef_select(const EFDev& e, const uint64_t* idx, uint64_t count, uint64_t* out, const DevInfo& di,
                            hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ef_select_bulk, dim3(ef_blocks(count, di)), dim3(256), 0, st, e, idx, count, out);
  return hipGetLastError();
}

hipError_t launch_ef_rank(const EFDev& e, const uint64_t* x, uint64_t count, uint64_t* out, const DevInfo& di,
                          hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ef_rank_bulk, dim3(ef_blocks(count, di)), dim3(256), 0, st, e, x, count, out);
  return hipGetLastError();
}

hipError_t launch_walks_ef(const WalkArgs& a, Path path, const EFDev& e, const DevInfo& di, hipStream_t st) {
  if (a.nwalks == 0) return hipSuccess;
  const bool weighted = a.g.R != nullptr;
  const bool r64 = a.g.r_bytes == 8;
  const dim3 lane_grid(ef_blocks(a.nwalks, di));
  const uint32_t lane_chunk = walk_chunk(a.nwalks / 64, (uint64_t)lane_grid.x * 4);
  auto lane = [&](auto kernel) {
    return with_walk_counter(di, st, [&](unsigned long long* ctr) {
      hipLaunchKernelGGL(kernel, lane_grid, dim3(256), 0, st, a, e, ctr, lane_chunk);
      return hipGetLastError();
    });
  };
  switch (path) {
    case Path::kFirstOrder:
      if (!weighted) return lane(k_walk_lane_ef<kEfFoUnw, uint32_t>);
      return r64 ? lane(k_walk_lane_ef<kEfFoW, uint64_t>) : lane(k_walk_lane_ef<kEfFoW, uint32_t>);
    case Path::kReturnOnly:
      if (!weighted) return lane(k_walk_lane_ef<kEfRetUnw, uint32_t>);
      return r64 ? lane(k_walk_lane_ef<kEfRetW, uint64_t>) : lane(k_walk_lane_ef<kEfRetW, uint32_t>);
    default: {
      const dim3 wave_grid(ef_blocks(a.nwalks * 64, di));
      const uint32_t chunk = walk_chunk(a.nwalks, (uint64_t)wave_grid.x * 4);
      return with_walk_counter(di, st, [&](unsigned long long* ctr) {
        if (!weighted)
          hipLaunchKernelGGL((k_walk_n2v_ef<false, uint32_t>), wave_grid, dim3(256), 0, st, a, e, ctr, chunk);
        else if (r64)
          hipLaunchKernelGGL((k_walk_n2v_ef<true, uint64_t>), wave_grid, dim3(256), 0, st, a, e, ctr, chunk);
        else
          hipLaunchKernelGGL((k_walk_n2v_ef<true, uint32_t>), wave_grid, dim3(256), 0, st, a, e, ctr, chunk);
        return hipGetLastError();
      });
    }
  }
  return hipGetLastError();
}

hipError_t launch_negatives_ef(const EFDev& e, const int32_t* Y, uint64_t n_walks, uint32_t L, uint32_t n_neg,
                               uint64_t seed, uint64_t wid_base, int32_t* N, const DevInfo& di, hipStream_t st) {
  const uint64_t n_pos = n_walks * L;
  if (n_pos == 0) return hipSuccess;
  constexpr size_t kLds = 64 * 1024;
  if ((size_t)n_neg * sizeof(int32_t) > kLds) return hipErrorInvalidValue;
  uint32_t lgP = 8;
  while (lgP > 0 && ((size_t)n_neg << lgP) * sizeof(int32_t) > kLds) --lgP;
  const size_t lds = ((size_t)n_neg << lgP) * sizeof(int32_t);
  hipLaunchKernelGGL(k_negatives_ef, dim3(ef_blocks(((n_pos + (1u << lgP) - 1) >> lgP) * 256, di)), dim3(256), lds,
                     st, e, Y, n_pos, L, n_neg, lgP, seed, wid_base, N);
  return hipGetLastError();
}

}  // namespace n2v
