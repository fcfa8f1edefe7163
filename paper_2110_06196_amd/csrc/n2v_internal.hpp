// Internal interface between the host runtime (n2v_api.cpp) and the kernels
// (n2v_walk.hip, n2v_prep.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

namespace n2v {

// Resident graph: borrowed CSR plus library-owned derived arrays.
struct GraphDev {
  const uint64_t* O = nullptr;  // [n+1]
  const int32_t* D = nullptr;   // [m]
  const uint32_t* W = nullptr;  // [m] or null (unweighted)
  const void* R = nullptr;      // per-row inclusive weight prefix, [m], uint32 or uint64
  uint32_t r_bytes = 0;         // 0 (unweighted), 4 or 8
  int64_t n = 0;
  uint64_t m = 0;
  // Weighted graphs with 32-bit row sums: per node {O[v] lo, O[v] hi, d_v,
  // S_v} in one 16-byte record, so a step reads its row's offset, degree and
  // weight sum with one load.  Null otherwise.
  const uint4* NR = nullptr;
  // Weighted CSR graphs: the prefix at every 32nd entry, HR[i] = R[32 i]
  // (ceil(m / 32) entries of r_bytes).  A search over a long row first
  // searches the row's heads, which are contiguous, then one 32-entry block of
  // R.  Null otherwise.
  const void* HR = nullptr;
  // CSR graphs with a row longer than kHeadsMinDegree: the destination at
  // every 32nd entry, HD[i] = D[32 i] (ceil(m / 32) entries).  A bisection over
  // a long splitter slice of a row searches the slice's heads, then one
  // 32-entry block of D.  Null otherwise.
  const int32_t* HD = nullptr;
  // Stored common-neighbour lists of edges (weighted graphs with 32-bit
  // prefixes, see n2v_pairs.hip), indexed by the edge's CSR position e
  // (t -> v = D[e]): pair_info[2e] = {first entry, entries, position of t in
  // N(v) or ~0, total listed weight}, pair_info[2e + 1] = {weight of t in
  // N(v), 0, 0, 0}; first entry ~0 when the list is not kept; pair_ent =
  // entries {R_v[j], inclusive listed weight, j, 0} in increasing j.  Null
  // when the graph has none.
  const uint4* pair_info = nullptr;
  const uint4* pair_ent = nullptr;
  // Membership sets of the hubs (rows of degree at least hub_min_deg, the
  // longest first, within a memory budget): one bit per node id, in 64-byte
  // lines of 15 words (480 ids) plus a 16th word holding the number of
  // members in the set's earlier lines, so one line gives both whether x is
  // in N(h) and, if so, its position in N(h).  hub_of[v] = index of v's set,
  // or -1.  Null when the graph has none.
  const int32_t* hub_of = nullptr;
  const uint32_t* hub_sets = nullptr;
  uint64_t hub_lines = 0;    // lines per set: ceil(n / 480)
  uint32_t hub_min_deg = 0;  // rows shorter than this have no set
  uint32_t hub_pad = 0;
};

// Node ids per 64-byte line of a hub set.
constexpr uint32_t kHubLineIds = 480;

// Rows at which a 64-way splitter slice exceeds 1024 entries.
constexpr uint64_t kHeadsMinDegree = 64ull * 1024;

// Which kernel family serves a request.
enum class Path : int {
  kFirstOrder = 0,  // lane per walker: unweighted multiply-shift / weighted prefix search
  kReturnOnly = 1,  // node2vec with Q16 == 65536: lane per walker, O(log d) per step
  kGeneric = 2      // node2vec with Q16 != 65536: G lanes per walker
};

// One walk request as the kernels see it.
struct WalkArgs {
  GraphDev g;
  const int32_t* starts;
  uint64_t ns;
  uint64_t nwalks;  // ns * walks_per_start
  uint32_t L;
  uint32_t second_order;  // 0: first order (alpha = 1 everywhere)
  uint32_t P16, Q16;
  uint64_t seed;
  uint64_t wid_base;
  int32_t* Y;
  int32_t* lens;
  uint32_t path;      // Path, used by the batched kernel
  uint32_t k_approx;  // 0: exact steps; k: steps from rows longer than k use k sub-sampled neighbours
  unsigned long long* steps;  // if non-null: += sum over walks of (len - 1)
};

// A slice [w0, w1) of the walk rows of request `req`, for the batched kernel.
struct QueueChunk {
  uint32_t req;
  uint32_t pad;
  uint64_t w0, w1;
};

struct LaunchCfg {
  int lanes_per_walker = 16;  // generic path
  int lds_tile = 512;         // entries of N(t) per walker kept in LDS
  int list_cap = 256;         // common-neighbour list entries per walker in LDS
  int mode = 0;               // 0 auto, 1 two-pass streaming, 2 probe N(t), 3 stream N(v)
  int grid_blocks = 0;        // 0 = derive from occupancy
  int full = 1;               // queue kernel with approximated steps and the two-pass route (0: exact routes only)
  int w32 = 0;                // queue kernel for weighted graphs with 32-bit prefixes only (every request's graph)
  int lists = 0;              // every edge of every graph of the launch keeps a stored list
};

// Output slots per 64-byte line: what a walker group of fewer than 16 lanes
// collects in LDS before storing it, and what a one-lane walker stages.
constexpr uint32_t kOutStage = 16;

// LDS words per walker group of g lanes: two staging tiles of the previous
// row, the common-neighbour list (positions, weights), a 2g-entry merge
// window (also the splitters of a long row) and, for g < 16, the output stage.
__host__ __device__ constexpr int group_lds_words(int tile, int cap, int g) {
  return 2 * tile + 2 * cap + 2 * g + (g < 16 ? (int)kOutStage : 0);
}

// LDS words per wavefront of the batched kernel, which runs walker groups and
// one-lane walkers in turn: the groups' regions or the one-lane walkers'
// output stages (one line per lane), whichever is larger.
__host__ __device__ constexpr int queue_wave_words(int tile, int cap, int g) {
  return (64 / g) * group_lds_words(tile, cap, g) > 64 * (int)kOutStage ? (64 / g) * group_lds_words(tile, cap, g)
                                                                         : 64 * (int)kOutStage;
}

// LDS bytes of a 256-thread block for a launch shape (the batched kernel's,
// which is never less than the plain node2vec kernel's).
inline size_t block_lds_bytes(int lanes_per_walker, int tile, int cap) {
  return 4 * (size_t)queue_wave_words(tile, cap, lanes_per_walker) * 4;
}

// Device facts used to size grids.
struct DevInfo {
  int device = 0;
  int cus = 0;
  size_t lds_per_block_max = 0;
};

// Walk counters: every stream of a device has one, allocated at the stream's
// first launch and kept until the process ends.  counter_slot returns it, or
// null (the kernels then use fixed shares) when the stream is being captured
// or no counter can be had.
unsigned long long* counter_slot(const DevInfo& di, hipStream_t st);
// Enqueues a kernel on st that zeroes *c.
void reset_counter(unsigned long long* c, hipStream_t st);
std::mutex& counter_mutex();

// Walks a group takes from the launch counter at a time: one while a group's
// share of the launch is small (a grid sized to the walks keeps every group
// busy), up to 8 for long launches (fewer atomics, a tail of a few walks).
inline uint32_t walk_chunk(uint64_t nwalks, uint64_t groups) {
  const uint64_t share = groups ? nwalks / groups : nwalks;
  return (uint32_t)std::min<uint64_t>(8, std::max<uint64_t>(1, share / 64));
}

// Runs launch(counter) with the stream's counter zeroed right before it on the
// stream: the reset and the launch are enqueued under one lock, so launches
// from several threads onto one stream cannot interleave between them.
template <typename F>
hipError_t with_walk_counter(const DevInfo& di, hipStream_t st, F&& launch) {
  unsigned long long* c = counter_slot(di, st);
  if (!c) return launch((unsigned long long*)nullptr);
  std::lock_guard<std::mutex> lk(counter_mutex());
  reset_counter(c, st);
  return launch(c);
}

hipError_t launch_walks(const WalkArgs& a, Path path, const LaunchCfg& cfg, const DevInfo& di,
                        hipStream_t st);
// Fused walk -> contexts (groups of 4, 16 or 64 lanes; a ring of rp words per
// group after its region): the context slots of walk a into C.
size_t ctx_block_lds_bytes(int lanes_per_walker, int tile, int cap, uint32_t rp);
hipError_t launch_walks_ctx(const WalkArgs& a, const LaunchCfg& cfg, int32_t* C, uint32_t window, uint32_t stride,
                            uint32_t h, uint32_t rp, const DevInfo& di, hipStream_t st);
// Grid of the persistent batched kernel for this shape.
int queue_grid_blocks(const LaunchCfg& cfg, const DevInfo& di, uint32_t nchunks);
// Persistent batched launch: resets *d_head (device) with a kernel, then the
// queue kernel drains d_chunks.  Graph-capturable (no memset nodes).
hipError_t launch_queue(const WalkArgs* d_reqs, const QueueChunk* d_chunks, uint32_t nchunks,
                        uint32_t* d_head, const LaunchCfg& cfg, const DevInfo& di, hipStream_t st);

// Graph preparation.  stats: [0] error flags, [1] max degree, [2] max row sum,
// [3] sum of degree^2 (device uint64[4], zeroed by the caller).
hipError_t launch_validate_stats(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
                                 const uint32_t* W, uint64_t* stats, hipStream_t st);
hipError_t launch_node_records(const uint64_t* O, int64_t n, const uint32_t* R, uint4* NR, hipStream_t st);
// HR[i] = R[32 i] for i < ceil(m / 32); R of r_bytes (4 or 8) per entry.
hipError_t launch_prefix_heads(const void* R, uint32_t r_bytes, uint64_t m, void* HR, hipStream_t st);
// HD[i] = D[32 i] for i < ceil(m / 32).
hipError_t launch_dest_heads(const int32_t* D, uint64_t m, int32_t* HD, hipStream_t st);
// Hub sets (zeroed by the caller): the members' bits of every hub, then the
// per-line member counts before each line; hub_of[hubs[i]] = i (hub_of set
// to -1 by the caller).
hipError_t launch_hub_sets(const uint64_t* O, const int32_t* D, const int32_t* hubs, uint32_t n_hubs,
                           uint64_t lines, uint32_t* sets, int32_t* hub_of, hipStream_t st);
// Passes of the edge-list builder (n2v_pairs.hip).
hipError_t launch_edge_lists_measure(const uint64_t* O, const int32_t* D, const int32_t* src, uint64_t m,
                                     const uint32_t* R, uint4* meas, hipStream_t st);
// Source row of every entry; *work += sum of min(d_t, d_v) bits(max(d_t, d_v)) (zeroed by the caller).
hipError_t launch_edge_src(const uint64_t* O, int64_t n, const int32_t* D, int32_t* src, unsigned long long* work,
                           hipStream_t st);
// cnt[e] = list length of edge e; *all += their sum (zeroed by the caller);
// key / idx (when key is non-null): sort keys of saved work per entry, identity.
hipError_t launch_edge_counts(const uint64_t* O, const int32_t* D, const int32_t* src, const uint4* meas, uint64_t m,
                              uint64_t* cnt, uint32_t* key, uint32_t* idx, unsigned long long* all, hipStream_t st);
// keep[e] = 1 for the edges whose lists are kept under `budget` entries, in
// decreasing saved work per entry (empty lists always); synchronous.
hipError_t edge_keep_by_gain(const uint32_t* key, const uint32_t* idx, uint32_t* key_s, uint32_t* idx_s,
                             const uint64_t* cnt, uint64_t* cnt_s, uint64_t* cum, const uint4* meas, uint64_t m,
                             uint64_t budget, uint8_t* keep, hipStream_t st);
// Records of every edge (keep null: all kept) at the exclusive scan of the
// kept lengths; tot[0] += kept edges, tot[1] = entries (zeroed by the caller); synchronous.
hipError_t edge_layout(const uint4* meas, const uint8_t* keep, uint64_t m, uint64_t* sz, uint64_t* off, uint4* info,
                       unsigned long long* tot, hipStream_t st);
hipError_t launch_edge_lists_fill(const uint64_t* O, const int32_t* D, const int32_t* src, uint64_t m,
                                  const uint32_t* R, const uint4* info, uint4* ent, hipStream_t st);
hipError_t launch_row_prefix(const uint64_t* O, int64_t n, const uint32_t* W, void* R,
                             uint32_t r_bytes, hipStream_t st);

// Elias-Fano edge store (n2v_ef.hip): the edge codes phi_k(a, b) = a 2^k + b
// of the CSR entries, l low bits each in L, high parts as inverted unary gaps
// in H (the one of element i is bit (code_i >> l) + i), and quantum indexes
// S1[j] / S0[j] = position of one / zero number j 2^lgq.
struct EFDev {
  const uint64_t* H = nullptr;
  const uint64_t* L = nullptr;
  const uint64_t* S1 = nullptr;
  const uint64_t* S0 = nullptr;
  uint32_t k = 0, l = 0, lgq = 0, pad = 0;
  uint64_t u = 0, m = 0, n_zeros = 0, h_bits = 0;
};
// Shape of the edge list of a graph on n >= 1 nodes with m entries.
void ef_shape(int64_t n, uint64_t m, uint32_t lgq, EFDev* e, uint64_t* h_words, uint64_t* l_words,
              uint64_t* s1_len, uint64_t* s0_len);
// Fill H, L (zeroed by the caller), S1, S0 of `e` from a validated CSR.
hipError_t launch_ef_build(const uint64_t* O, int64_t n, const int32_t* D, const EFDev& e, const DevInfo& di,
                           hipStream_t st);
hipError_t launch_ef_select(const EFDev& e, const uint64_t* idx, uint64_t count, uint64_t* out, const DevInfo& di,
                            hipStream_t st);
hipError_t launch_ef_rank(const EFDev& e, const uint64_t* x, uint64_t count, uint64_t* out, const DevInfo& di,
                          hipStream_t st);
// Walks over the Elias-Fano store (a.g.R holds the row prefix of weighted graphs).
hipError_t launch_walks_ef(const WalkArgs& a, Path path, const EFDev& e, const DevInfo& di, hipStream_t st);
hipError_t launch_negatives_ef(const EFDev& e, const int32_t* Y, uint64_t n_walks, uint32_t L, uint32_t n_neg,
                               uint64_t seed, uint64_t wid_base, int32_t* N, const DevInfo& di, hipStream_t st);

// Training corpora (n2v_corpus.hip).
hipError_t launch_contexts(const int32_t* Y, uint64_t n_walks, uint32_t L, uint32_t window, uint32_t stride,
                           int32_t* C, const DevInfo& di, hipStream_t st);
constexpr uint32_t kMaxWindow = 1u << 16;     // context window bound (tile words stay in 32 bits)
constexpr uint32_t kMaxNegatives = 1u << 14;  // negatives per position (one position's staging fits LDS)
constexpr uint32_t kMaxFusedHalo = 1023;      // fused contexts: window * stride (ring of 2048 words per walker)

// Negative sampling searches through a guide table of 2^shift + 1 int32
// entries per graph (shift = neg_guide_shift(n), at most kNegGuideMaxShift).
constexpr uint32_t kNegGuideMaxShift = 28;
constexpr int kNegGuideShiftAdjust = -1;  // 2^shift: the power of two at or above n, times 2^adjust
uint32_t neg_guide_shift(int64_t n);
size_t neg_guide_bytes(uint32_t shift, int64_t n, uint64_t m);
hipError_t launch_neg_guide(const GraphDev& g, int32_t* guide, uint32_t shift, const DevInfo& di, hipStream_t st);
hipError_t launch_negatives(const GraphDev& g, const int32_t* guide, uint32_t shift, const int32_t* Y,
                            uint64_t n_walks, uint32_t L, uint32_t n_neg, uint64_t seed, uint64_t wid_base,
                            int32_t* N, const DevInfo& di, hipStream_t st);

enum : uint64_t {
  kErrOffsets = 1,   // O[0] != 0, O not monotone or O[n] != m
  kErrOrder = 2,     // a row not strictly increasing
  kErrRange = 4      // destination outside [0, n)
};

}  // namespace n2v
