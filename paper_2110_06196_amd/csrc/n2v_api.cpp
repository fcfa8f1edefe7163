// C ABI of the walk library: argument validation, graph registry, variant
// dispatch and tuning.  Declarations and semantics: include/n2vwalk.h.
#include "n2vwalk.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "n2v_internal.hpp"
#include "n2v_runtime.hpp"

namespace n2v {

thread_local std::string t_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(N2V_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

std::mutex g_mu;
std::unordered_map<uint64_t, GraphRec*> g_graphs;
uint64_t g_next_graph = 1;
bool g_tune_set = false;
n2v_tuning_t g_tune{};

std::mutex g_dev_mu;
std::unordered_map<int, DevInfo> g_devs;

}  // namespace

int q16_of(double x, uint32_t* out) {
  if (!(x > 0.0) || !std::isfinite(x)) return N2V_ERR_INVALID_ARG;
  const double r = std::nearbyint(65536.0 / x);  // round to nearest, ties to even
  if (!(r >= 1.0) || !(r <= 4294967295.0)) return N2V_ERR_INVALID_ARG;
  *out = (uint32_t)r;
  return N2V_OK;
}

int current_devinfo(DevInfo* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_devs.find(dev);
  if (it == g_devs.end()) {
    DevInfo di;
    di.device = dev;
    e = hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    di.lds_per_block_max = (size_t)lds;
    it = g_devs.emplace(dev, di).first;
  }
  *out = it->second;
  return N2V_OK;
}

GraphRec* find_graph(n2v_graph g) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_graphs.find(g);
  return it == g_graphs.end() ? nullptr : it->second;
}

// Launch configuration for one request on one graph.  The automatic choice
// follows the graph's stationary mean degree sum(d^2)/sum(d): the expected
// number of candidates per step of a long walk.
LaunchCfg choose_cfg(const GraphRec& gr, const DevInfo& di, uint64_t nwalks) {
  LaunchCfg c;
  const double ed = gr.n_entries ? (double)gr.sum_deg_sq / (double)gr.n_entries : 0.0;
  c.lanes_per_walker = ed > 256 ? 64 : (ed > 48 ? 32 : 16);
  // LDS per group: a short staging tile and a long common-neighbour list (a
  // list overflow costs a two-pass stream of the row; a miss in the tile only
  // a bisection in global memory); 8 blocks of 256 threads fit one CU.
  c.lds_tile = c.lanes_per_walker == 64 ? 64 : (c.lanes_per_walker == 32 ? 64 : 32);
  c.list_cap = c.lanes_per_walker == 64 ? 512 : (c.lanes_per_walker == 32 ? 256 : 128);
  c.mode = 0;
  // When every edge keeps a stored common-neighbour list, a step is a few short
  // searches: groups of 4 lanes, 16 walks per wavefront, keep more loads in
  // flight than one walk per wavefront (2.6x on a 1M-node Chung-Lu graph at
  // p = 0.25, q = 4, 10M walks), once the launch has the walks to fill the
  // chip that way; below about 80 walks per CU one walk per wavefront, whose
  // wide searches take fewer rounds, is faster (measured on the same graph).
  // A step on the stored-list path reads nothing from LDS, so the tile and
  // the list capacity stay small.
  const uint64_t cus = di.cus > 0 ? (uint64_t)di.cus : 256;
  if (gr.pair_lists > 0 && gr.pair_lists == gr.n_entries && nwalks >= 96 * cus) {
    c.lanes_per_walker = 4;
    c.lds_tile = 16;
    c.list_cap = 32;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_tune_set) {
    if (g_tune.lanes_per_walker) c.lanes_per_walker = (int)g_tune.lanes_per_walker;
    if (g_tune.lds_tile) c.lds_tile = (int)g_tune.lds_tile;
    if (g_tune.list_cap) c.list_cap = (int)g_tune.list_cap;
    c.mode = (int)g_tune.route;
  }
  // keep the per-block LDS inside the hardware limit
  auto bytes = [&]() { return block_lds_bytes(c.lanes_per_walker, c.lds_tile, c.list_cap); };
  while (bytes() > di.lds_per_block_max && (c.lds_tile > 1 || c.list_cap > 1)) {
    if (c.lds_tile >= c.list_cap && c.lds_tile > 1) c.lds_tile /= 2;
    else c.list_cap /= 2;
  }
  return c;
}

int check_tuning(const n2v_tuning_t& t) {
  const uint32_t g = t.lanes_per_walker;
  if (g != 0 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64)
    return fail(N2V_ERR_INVALID_ARG, "lanes_per_walker must be 4, 8, 16, 32 or 64");
  if (t.lds_tile > (1u << 16) || t.list_cap > (1u << 16))
    return fail(N2V_ERR_INVALID_ARG, "lds_tile / list_cap too large");
  if (t.route > N2V_ROUTE_HUB_SETS) return fail(N2V_ERR_INVALID_ARG, "unknown route");
  if (t.flags & ~(uint32_t)N2V_TUNE_GENERIC_ONLY) return fail(N2V_ERR_INVALID_ARG, "unknown flags");
  return N2V_OK;
}

void apply_tuning_override(LaunchCfg* c, const DevInfo& di, const n2v_tuning_t* fixed) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const n2v_tuning_t* t = fixed ? fixed : (g_tune_set ? &g_tune : nullptr);
    if (!t) return;
    if (t->lanes_per_walker) c->lanes_per_walker = (int)t->lanes_per_walker;
    if (t->lds_tile) c->lds_tile = (int)t->lds_tile;
    if (t->list_cap) c->list_cap = (int)t->list_cap;
    c->mode = (int)t->route;
  }
  // the queue kernel has groups of 4, 16, 32 and 64 lanes
  if (c->lanes_per_walker != 4 && c->lanes_per_walker < 16) c->lanes_per_walker = 16;
  auto bytes = [&]() { return block_lds_bytes(c->lanes_per_walker, c->lds_tile, c->list_cap); };
  while (bytes() > di.lds_per_block_max && (c->lds_tile > 1 || c->list_cap > 1)) {
    if (c->lds_tile >= c->list_cap && c->lds_tile > 1) c->lds_tile /= 2;
    else c->list_cap /= 2;
  }
  c->grid_blocks = 0;
}

bool generic_only() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tune_set && (g_tune.flags & N2V_TUNE_GENERIC_ONLY);
}

// Validate a walk request and fill the kernel arguments.
int prepare_request(const GraphRec& gr, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                    uint32_t walks_per_start, uint32_t walk_len, double p, double q, uint64_t seed,
                    uint64_t walk_id_base, int32_t* d_walks, int32_t* d_lens, uint32_t k_approx,
                    WalkArgs* a, Path* path) {
  if (walk_len == 0) return fail(N2V_ERR_INVALID_ARG, "walk_len must be >= 1");
  // lengths are int32 and the kernels index a row's slots in 32-bit arithmetic
  if (walk_len > (1u << 30)) return fail(N2V_ERR_INVALID_ARG, "walk_len %u above 2^30", walk_len);
  if (walks_per_start == 0) return fail(N2V_ERR_INVALID_ARG, "walks_per_start must be >= 1");
  if (kind != N2V_FIRST_ORDER && kind != N2V_NODE2VEC) return fail(N2V_ERR_INVALID_ARG, "bad kind");
  if (n_starts > 0 && (!d_starts || !d_walks))
    return fail(N2V_ERR_INVALID_ARG, "starts and walks must be non-NULL");
  const unsigned __int128 nw = (unsigned __int128)n_starts * walks_per_start;
  if (nw * walk_len >= ((unsigned __int128)1 << 62)) return fail(N2V_ERR_INVALID_ARG, "output too large");
  uint32_t P16 = kC16Host, Q16 = kC16Host;
  if (kind == N2V_NODE2VEC) {
    if (q16_of(p, &P16) != N2V_OK) return fail(N2V_ERR_INVALID_ARG, "p=%g gives no Q16 value in [1, 2^32-1]", p);
    if (q16_of(q, &Q16) != N2V_OK) return fail(N2V_ERR_INVALID_ARG, "q=%g gives no Q16 value in [1, 2^32-1]", q);
    uint64_t amax = kC16Host;
    if (P16 > amax) amax = P16;
    if (Q16 > amax) amax = Q16;
    if ((unsigned __int128)gr.max_row_wsum * amax > (unsigned __int128)UINT64_MAX)
      return fail(N2V_ERR_OVERFLOW, "max row weight sum %llu * %llu does not fit in 64 bits",
                  (unsigned long long)gr.max_row_wsum, (unsigned long long)amax);
  }
  a->g = gr.dev;
  a->starts = d_starts;
  a->ns = n_starts;
  a->nwalks = (uint64_t)nw;
  a->L = walk_len;
  a->second_order = kind == N2V_NODE2VEC ? 1u : 0u;
  a->P16 = P16;
  a->Q16 = Q16;
  a->seed = seed;
  a->wid_base = walk_id_base;
  a->Y = d_walks;
  a->lens = d_lens;
  // Variant dispatch (the paper's eight specialisations): first order and
  // node2vec with p = q = 1 share the first-order kernels; node2vec with
  // 1/q == 1 only re-weights the return edge; everything else is generic.
  // Approximated walks (sub-sampled rows) always run on the G-lanes kernel.
  if (generic_only() || k_approx > 0) *path = Path::kGeneric;
  else if (kind == N2V_FIRST_ORDER || (P16 == kC16Host && Q16 == kC16Host)) {
    *path = Path::kFirstOrder;
    a->second_order = 0;
  } else if (Q16 == kC16Host) *path = Path::kReturnOnly;
  else *path = Path::kGeneric;
  a->path = (uint32_t)*path;
  a->k_approx = k_approx;
  a->steps = nullptr;
  return N2V_OK;
}

}  // namespace n2v

using namespace n2v;

extern "C" {

const char* n2v_last_error(void) { return t_err.c_str(); }

}  // extern "C"

namespace n2v {
namespace {

// Validate a CSR on the device and collect its statistics: h = {error bits,
// max degree, max row weight sum, sum of squared degrees}.
// Host-side argument checks of a CSR upload (before any device call).
int check_csr_args(const uint64_t* d_offsets, uint64_t n_nodes, const int32_t* d_dst, uint64_t n_entries) {
  if (!d_offsets) return fail(N2V_ERR_INVALID_ARG, "offsets is NULL");
  if (n_entries > 0 && !d_dst) return fail(N2V_ERR_INVALID_ARG, "dst is NULL");
  if (n_nodes > (uint64_t)INT32_MAX) return fail(N2V_ERR_INVALID_ARG, "node ids must fit in int32");
  if (n_entries >= ((uint64_t)1 << 62)) return fail(N2V_ERR_INVALID_ARG, "too many entries");
  return N2V_OK;
}

int validate_csr(const uint64_t* d_offsets, uint64_t n_nodes, const int32_t* d_dst, uint64_t n_entries,
                 const uint32_t* d_weights, hipStream_t st, uint64_t h[4]) {
  uint64_t* d_stats = nullptr;
  hipError_t e = hipMalloc(&d_stats, 4 * sizeof(uint64_t));
  if (e != hipSuccess) return fail(N2V_ERR_NOMEM, "hipMalloc stats: %s", hipGetErrorString(e));
  h[0] = h[1] = h[2] = h[3] = 0;
  e = hipMemsetAsync(d_stats, 0, 4 * sizeof(uint64_t), st);
  if (e == hipSuccess) e = launch_validate_stats(d_offsets, (int64_t)n_nodes, d_dst, n_entries, d_weights, d_stats, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h, d_stats, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(d_stats);
  if (e != hipSuccess) return hip_fail(e, "graph validation");
  if (h[0]) {
    return fail(N2V_ERR_UNSORTED, "invalid CSR:%s%s%s", (h[0] & kErrOffsets) ? " offsets" : "",
                (h[0] & kErrOrder) ? " row-not-strictly-increasing" : "",
                (h[0] & kErrRange) ? " destination-out-of-range" : "");
  }
  return N2V_OK;
}

GraphRec* new_record(uint64_t n_nodes, uint64_t n_entries, const uint64_t h[4], bool weighted, int device) {
  GraphRec* gr = new GraphRec();
  gr->dev.n = (int64_t)n_nodes;
  gr->dev.m = n_entries;
  gr->n_nodes = n_nodes;
  gr->n_entries = n_entries;
  gr->max_degree = h[1];
  gr->max_row_wsum = h[2];
  gr->sum_deg_sq = h[3];
  gr->weighted = weighted ? 1u : 0u;
  gr->device = device;
  return gr;
}

// The per-row inclusive weight prefix (owned), 32-bit when every row sum fits.
int build_prefix(GraphRec* gr, const uint64_t* d_offsets, const uint32_t* d_weights, hipStream_t st,
                 bool node_records) {
  if (!d_weights || gr->n_entries == 0) return N2V_OK;
  const uint32_t rb = gr->max_row_wsum <= 0xFFFFFFFFull ? 4u : 8u;
  void* R = nullptr;
  hipError_t e = hipMalloc(&R, (size_t)gr->n_entries * rb);
  if (e != hipSuccess)
    return fail(N2V_ERR_NOMEM, "hipMalloc prefix (%llu bytes): %s", (unsigned long long)(gr->n_entries * rb),
                hipGetErrorString(e));
  e = launch_row_prefix(d_offsets, gr->dev.n, d_weights, R, rb, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    hipFree(R);
    return hip_fail(e, "row prefix");
  }
  gr->dev.R = R;
  gr->dev.r_bytes = rb;
  gr->owned_bytes += gr->n_entries * rb;
  if (rb == 4 && node_records) {
    uint4* NR = nullptr;
    e = hipMalloc(&NR, (size_t)gr->dev.n * sizeof(uint4));
    if (e != hipSuccess)
      return fail(N2V_ERR_NOMEM, "hipMalloc node records: %s", hipGetErrorString(e));
    e = launch_node_records(d_offsets, gr->dev.n, (const uint32_t*)R, NR, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      hipFree(NR);
      return hip_fail(e, "node records");
    }
    gr->dev.NR = NR;
    gr->owned_bytes += (uint64_t)gr->dev.n * sizeof(uint4);
  }
  if (node_records) {
    const uint64_t hbytes = ((gr->n_entries + 31) >> 5) * rb;
    void* HR = nullptr;
    e = hipMalloc(&HR, (size_t)hbytes);
    if (e != hipSuccess) return fail(N2V_ERR_NOMEM, "hipMalloc prefix heads: %s", hipGetErrorString(e));
    e = launch_prefix_heads(R, rb, gr->n_entries, HR, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      hipFree(HR);
      return hip_fail(e, "prefix heads");
    }
    gr->dev.HR = HR;
    gr->owned_bytes += hbytes;
  }
  return N2V_OK;
}

// Stored common-neighbour lists of edges (n2v_pairs.hip), for weighted graphs
// with 32-bit prefixes and at most kListMaxEntries entries, when measuring
// them takes at most kListWorkCap bisection reads and device memory allows.
// Every edge's list is kept when all fit the budget of min(kListBudgetMax,
// 256 m) bytes (16 B per entry, so 16 entries per graph entry); otherwise the
// edges in decreasing order of saved merge work per stored entry,
// (d_t + d_v) / (entries + 4), up to the first that does not fit (and every
// empty list).  The selection and the layout run on the device.
constexpr uint64_t kListMaxEntries = 1ull << 28;
constexpr uint64_t kListWorkCap = 1ull << 37;
constexpr uint64_t kListBudgetMax = 32ull << 30;

// Device temporaries of one build, freed when it ends.
struct DeviceTemps {
  std::vector<void*> p;
  ~DeviceTemps() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, count ? count * sizeof(T) : 1);
    if (e == hipSuccess) p.push_back(q);
    *out = (T*)q;
    return e;
  }
};

void free_edge_lists(GraphDev& g) {
  if (g.pair_info) (void)hipFree(const_cast<uint4*>(g.pair_info));
  if (g.pair_ent) (void)hipFree(const_cast<uint4*>(g.pair_ent));
  g.pair_info = nullptr;
  g.pair_ent = nullptr;
}

int build_edge_lists(GraphRec* gr, hipStream_t st) {
  GraphDev& g = gr->dev;
  const uint64_t n = gr->n_nodes, m = gr->n_entries;
  if (!g.R || g.r_bytes != 4 || m == 0 || m > kListMaxEntries) return N2V_OK;
  DeviceTemps tmp;
  // The lists change no walk: when device memory runs short the graph is
  // registered without them; any other failure is reported.
  auto hipf = [&](hipError_t e, const char* what) -> int {
    free_edge_lists(g);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return N2V_OK;
    }
    return hip_fail(e, what);
  };
  // scalars: [0] build work, [1] entries of all lists, [2] kept edges, [3] kept entries
  unsigned long long* d_sc;
  int32_t* d_src;
  uint4* d_meas;
  hipError_t e;
  if ((e = tmp.alloc(&d_sc, 4)) != hipSuccess || (e = tmp.alloc(&d_src, m)) != hipSuccess)
    return hipf(e, "allocation");
  unsigned long long h_sc[4] = {0, 0, 0, 0};
  if ((e = hipMemsetAsync(d_sc, 0, sizeof(h_sc), st)) != hipSuccess ||
      (e = launch_edge_src(g.O, (int64_t)n, g.D, d_src, d_sc, st)) != hipSuccess ||
      (e = hipMemcpyAsync(h_sc, d_sc, sizeof(h_sc), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hipf(e, "edge list work");
  if (h_sc[0] > kListWorkCap) return N2V_OK;
  if ((e = tmp.alloc(&d_meas, m)) != hipSuccess) return hipf(e, "allocation");
  if ((e = launch_edge_lists_measure(g.O, g.D, d_src, m, (const uint32_t*)g.R, d_meas, st)) != hipSuccess)
    return hipf(e, "edge list measure");
  // entries are addressed by 32-bit offsets: the budget stays below 2^31 of them
  const uint64_t budget = std::min<uint64_t>(kListBudgetMax, 256ull * m) / sizeof(uint4);
  uint64_t* d_cnt;
  if ((e = tmp.alloc(&d_cnt, m)) != hipSuccess) return hipf(e, "allocation");
  if ((e = launch_edge_counts(g.O, g.D, d_src, d_meas, m, d_cnt, nullptr, nullptr, d_sc + 1, st)) != hipSuccess ||
      (e = hipMemcpyAsync(h_sc, d_sc, sizeof(h_sc), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hipf(e, "edge list sizes");
  uint8_t* d_keep = nullptr;  // null: every list is kept
  if (h_sc[1] > budget) {
    uint32_t *d_key, *d_idx, *d_key_s, *d_idx_s;
    uint64_t *d_cnt_s, *d_cum;
    if ((e = tmp.alloc(&d_keep, m)) != hipSuccess || (e = tmp.alloc(&d_key, m)) != hipSuccess ||
        (e = tmp.alloc(&d_idx, m)) != hipSuccess || (e = tmp.alloc(&d_key_s, m)) != hipSuccess ||
        (e = tmp.alloc(&d_idx_s, m)) != hipSuccess || (e = tmp.alloc(&d_cnt_s, m)) != hipSuccess ||
        (e = tmp.alloc(&d_cum, m)) != hipSuccess)
      return hipf(e, "allocation");
    if ((e = launch_edge_counts(g.O, g.D, d_src, d_meas, m, d_cnt, d_key, d_idx, d_sc + 3, st)) != hipSuccess ||
        (e = edge_keep_by_gain(d_key, d_idx, d_key_s, d_idx_s, d_cnt, d_cnt_s, d_cum, d_meas, m, budget, d_keep, st)) !=
            hipSuccess ||
        (e = hipMemsetAsync(d_sc + 2, 0, 2 * sizeof(unsigned long long), st)) != hipSuccess)
      return hipf(e, "edge list selection");
  }
  uint64_t *d_sz, *d_off;
  uint4* d_info = nullptr;
  if ((e = tmp.alloc(&d_sz, m)) != hipSuccess || (e = tmp.alloc(&d_off, m)) != hipSuccess) return hipf(e, "allocation");
  if ((e = hipMalloc((void**)&d_info, 2 * m * sizeof(uint4))) != hipSuccess) return hipf(e, "allocation");
  g.pair_info = d_info;
  if ((e = edge_layout(d_meas, d_keep, m, d_sz, d_off, d_info, d_sc + 2, st)) != hipSuccess ||
      (e = hipMemcpyAsync(h_sc, d_sc, sizeof(h_sc), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hipf(e, "edge list layout");
  const uint64_t total = h_sc[3], kept = h_sc[2];
  uint4* d_ent = nullptr;
  if ((e = hipMalloc((void**)&d_ent, (total ? total : 1) * sizeof(uint4))) != hipSuccess) return hipf(e, "allocation");
  g.pair_ent = d_ent;
  if ((e = launch_edge_lists_fill(g.O, g.D, d_src, m, (const uint32_t*)g.R, d_info, d_ent, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hipf(e, "edge list fill");
  gr->owned_bytes += 2 * m * sizeof(uint4) + total * sizeof(uint4);
  gr->pair_lists = kept;
  gr->pair_entries = total;
  return N2V_OK;
}

// Hub membership sets (see GraphDev): for the rows of degree at least
// 2^k (k from the upload flags; automatic: kHubSetMinDegree, and only for
// graphs where some edge keeps no stored list, since a step with a stored
// list builds nothing), longest first, within min(kHubSetBudgetMax, a
// quarter of the free device memory).  They change no walk.
constexpr uint64_t kHubSetMinDegree = 4096;
constexpr uint64_t kHubSetBudgetMax = 16ull << 30;

int build_hub_sets(GraphRec* gr, uint32_t flags, hipStream_t st) {
  GraphDev& g = gr->dev;
  if (flags & N2V_UPLOAD_NO_HUB_SETS) return N2V_OK;
  const uint32_t k = (flags >> 8) & 31u;
  uint64_t min_deg = k ? (1ull << k) : kHubSetMinDegree;
  if (!k && gr->pair_lists == gr->n_entries) return N2V_OK;
  if (gr->max_degree < min_deg || gr->n_nodes == 0) return N2V_OK;
  const uint64_t n = gr->n_nodes;
  std::vector<uint64_t> hO(n + 1);
  hipError_t e = hipMemcpy(hO.data(), g.O, (n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hub sets: offsets");
  std::vector<int32_t> hubs;
  for (uint64_t v = 0; v < n; ++v)
    if (hO[v + 1] - hO[v] >= min_deg) hubs.push_back((int32_t)v);
  std::stable_sort(hubs.begin(), hubs.end(), [&](int32_t a, int32_t b) {
    return hO[a + 1] - hO[a] > hO[b + 1] - hO[b];
  });
  const uint64_t lines = (n + kHubLineIds - 1) / kHubLineIds;
  const uint64_t set_bytes = lines * 64;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return N2V_OK;
  }
  const uint64_t budget = std::min<uint64_t>(kHubSetBudgetMax, (uint64_t)free_b / 4);
  const uint64_t keep = std::min<uint64_t>(hubs.size(), budget / set_bytes);
  if (keep == 0) return N2V_OK;
  hubs.resize(keep);
  int32_t* d_hub_of = nullptr;
  uint32_t* d_sets = nullptr;
  int32_t* d_hubs = nullptr;
  auto undo = [&](hipError_t err, const char* what) -> int {
    if (d_hub_of) (void)hipFree(d_hub_of);
    if (d_sets) (void)hipFree(d_sets);
    if (d_hubs) (void)hipFree(d_hubs);
    if (err == hipErrorOutOfMemory) {  // the sets change no walk: go on without them
      (void)hipGetLastError();
      return N2V_OK;
    }
    return hip_fail(err, what);
  };
  if ((e = hipMalloc((void**)&d_hub_of, n * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc((void**)&d_sets, keep * set_bytes)) != hipSuccess ||
      (e = hipMalloc((void**)&d_hubs, keep * sizeof(int32_t))) != hipSuccess)
    return undo(e, "hub sets: allocation");
  if ((e = hipMemsetAsync(d_hub_of, 0xFF, n * sizeof(int32_t), st)) != hipSuccess ||
      (e = hipMemsetAsync(d_sets, 0, keep * set_bytes, st)) != hipSuccess ||
      (e = hipMemcpyAsync(d_hubs, hubs.data(), keep * sizeof(int32_t), hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = launch_hub_sets(g.O, g.D, d_hubs, (uint32_t)keep, lines, d_sets, d_hub_of, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return undo(e, "hub sets: build");
  (void)hipFree(d_hubs);
  g.hub_of = d_hub_of;
  g.hub_sets = d_sets;
  g.hub_lines = lines;
  g.hub_min_deg = (uint32_t)std::min<uint64_t>(min_deg, 0xFFFFFFFFull);
  gr->hub_count = keep;
  gr->owned_bytes += n * sizeof(int32_t) + keep * set_bytes;
  return N2V_OK;
}

n2v_graph register_graph(GraphRec* gr) {
  std::lock_guard<std::mutex> lk(g_mu);
  gr->handle = g_next_graph++;
  g_graphs[gr->handle] = gr;
  return gr->handle;
}

void free_record(GraphRec* gr) {
  if (gr->dev.R) hipFree(const_cast<void*>(gr->dev.R));
  if (gr->dev.NR) hipFree(const_cast<uint4*>(gr->dev.NR));
  if (gr->dev.HR) hipFree(const_cast<void*>(gr->dev.HR));
  if (gr->dev.HD) hipFree(const_cast<int32_t*>(gr->dev.HD));
  if (gr->dev.hub_of) hipFree(const_cast<int32_t*>(gr->dev.hub_of));
  if (gr->dev.hub_sets) hipFree(const_cast<uint32_t*>(gr->dev.hub_sets));
  free_edge_lists(gr->dev);
  if (gr->neg_guide) hipFree(gr->neg_guide);
  if (gr->ef_mem) hipFree(gr->ef_mem);
  delete gr;
}

}  // namespace
}  // namespace n2v

extern "C" {

int n2v_graph_upload(const uint64_t* d_offsets, uint64_t n_nodes, const int32_t* d_dst,
                     uint64_t n_entries, const uint32_t* d_weights, uint32_t flags,
                     void* hip_stream, n2v_graph* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  *out = 0;
  if ((flags & ~(uint32_t)(N2V_UPLOAD_NO_PAIR_LISTS | N2V_UPLOAD_NO_HUB_SETS | N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(31))) != 0)
    return fail(N2V_ERR_INVALID_ARG, "flags: unknown bits 0x%x", flags);
  int rc = check_csr_args(d_offsets, n_nodes, d_dst, n_entries);
  if (rc != N2V_OK) return rc;
  DevInfo di;
  rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  uint64_t h[4];
  rc = validate_csr(d_offsets, n_nodes, d_dst, n_entries, d_weights, st, h);
  if (rc != N2V_OK) return rc;
  GraphRec* gr = new_record(n_nodes, n_entries, h, d_weights != nullptr, di.device);
  gr->dev.O = d_offsets;
  gr->dev.D = d_dst;
  gr->dev.W = d_weights;
  rc = build_prefix(gr, d_offsets, d_weights, st, true);
  if (rc == N2V_OK && gr->max_degree > kHeadsMinDegree) {
    const uint64_t hbytes = ((n_entries + 31) >> 5) * sizeof(int32_t);
    int32_t* HD = nullptr;
    hipError_t e = hipMalloc((void**)&HD, (size_t)hbytes);
    if (e != hipSuccess) {
      rc = fail(N2V_ERR_NOMEM, "hipMalloc destination heads: %s", hipGetErrorString(e));
    } else {
      e = launch_dest_heads(d_dst, n_entries, HD, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        hipFree(HD);
        rc = hip_fail(e, "destination heads");
      } else {
        gr->dev.HD = HD;
        gr->owned_bytes += hbytes;
      }
    }
  }
  if (rc == N2V_OK && !(flags & N2V_UPLOAD_NO_PAIR_LISTS)) {
    try {
      rc = build_edge_lists(gr, st);
    } catch (const std::bad_alloc&) {  // host memory for the layout: go on without lists
      free_edge_lists(gr->dev);
      rc = N2V_OK;
    }
  }
  if (rc == N2V_OK) {
    try {
      rc = build_hub_sets(gr, flags, st);
    } catch (const std::bad_alloc&) {  // host memory for the selection: go on without sets
      rc = N2V_OK;
    }
  }
  if (rc != N2V_OK) {
    free_record(gr);
    return rc;
  }
  *out = register_graph(gr);
  return N2V_OK;
}

int n2v_graph_upload_ef(const uint64_t* d_offsets, uint64_t n_nodes, const int32_t* d_dst,
                        uint64_t n_entries, const uint32_t* d_weights, uint32_t quantum,
                        void* hip_stream, n2v_graph* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  *out = 0;
  if (n_nodes == 0) return fail(N2V_ERR_INVALID_ARG, "an Elias-Fano graph needs at least one node");
  if (quantum == 0) quantum = 256;
  uint32_t lgq = 0;
  while ((1u << lgq) < quantum) ++lgq;
  if ((1u << lgq) != quantum || quantum < 8 || quantum > 65536)
    return fail(N2V_ERR_INVALID_ARG, "quantum %u is not a power of two in [8, 65536]", quantum);
  int rc = check_csr_args(d_offsets, n_nodes, d_dst, n_entries);
  if (rc != N2V_OK) return rc;
  DevInfo di;
  rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  uint64_t h[4];
  rc = validate_csr(d_offsets, n_nodes, d_dst, n_entries, d_weights, st, h);
  if (rc != N2V_OK) return rc;
  GraphRec* gr = new_record(n_nodes, n_entries, h, d_weights != nullptr, di.device);
  gr->storage = N2V_STORAGE_EF;
  gr->ef_quantum = quantum;
  uint64_t hw, lw, n1, n0;
  ef_shape((int64_t)n_nodes, n_entries, lgq, &gr->ef, &hw, &lw, &n1, &n0);
  const uint64_t words = hw + lw + n1 + n0;
  hipError_t e = hipMalloc(&gr->ef_mem, (size_t)(words ? words : 1) * sizeof(uint64_t));
  if (e != hipSuccess) {
    free_record(gr);
    return fail(N2V_ERR_NOMEM, "hipMalloc Elias-Fano store (%llu words): %s", (unsigned long long)words,
                hipGetErrorString(e));
  }
  uint64_t* base = (uint64_t*)gr->ef_mem;
  gr->ef.H = base;
  gr->ef.L = base + hw;
  gr->ef.S1 = base + hw + lw;
  gr->ef.S0 = base + hw + lw + n1;
  gr->owned_bytes += words * sizeof(uint64_t);
  e = hipMemsetAsync(gr->ef_mem, 0, (size_t)(hw + lw) * sizeof(uint64_t), st);
  if (e == hipSuccess) e = launch_ef_build(d_offsets, (int64_t)n_nodes, d_dst, gr->ef, di, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    free_record(gr);
    return hip_fail(e, "Elias-Fano build");
  }
  rc = build_prefix(gr, d_offsets, d_weights, st, false);
  if (rc != N2V_OK) {
    free_record(gr);
    return rc;
  }
  *out = register_graph(gr);
  return N2V_OK;
}

int n2v_ef_info(n2v_graph g, n2v_ef_info_t* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
  if (gr->storage != N2V_STORAGE_EF) return fail(N2V_ERR_INVALID_ARG, "graph %llu is not an Elias-Fano graph",
                                                 (unsigned long long)g);
  uint64_t hw, lw, n1, n0;
  EFDev tmp;
  ef_shape(gr->dev.n, gr->n_entries, gr->ef.lgq, &tmp, &hw, &lw, &n1, &n0);
  std::memset(out, 0, sizeof(*out));
  out->k = gr->ef.k;
  out->l = gr->ef.l;
  out->quantum = gr->ef_quantum;
  out->u = gr->ef.u;
  out->n_codes = gr->ef.m;
  out->n_zeros = gr->ef.n_zeros;
  out->h_bits = gr->ef.h_bits;
  out->h_words = hw;
  out->l_words = lw;
  out->s1_len = n1;
  out->s0_len = n0;
  out->d_H = gr->ef.H;
  out->d_L = gr->ef.L;
  out->d_S1 = gr->ef.S1;
  out->d_S0 = gr->ef.S0;
  return N2V_OK;
}

static int ef_bulk(n2v_graph g, const uint64_t* d_in, uint64_t count, uint64_t* d_out, void* hip_stream,
                   bool select) {
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
  if (gr->storage != N2V_STORAGE_EF) return fail(N2V_ERR_INVALID_ARG, "graph %llu is not an Elias-Fano graph",
                                                 (unsigned long long)g);
  if (count > 0 && (!d_in || !d_out)) return fail(N2V_ERR_INVALID_ARG, "arrays must be non-NULL");
  DevInfo di;
  int rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  hipError_t e = select ? launch_ef_select(gr->ef, d_in, count, d_out, di, (hipStream_t)hip_stream)
                        : launch_ef_rank(gr->ef, d_in, count, d_out, di, (hipStream_t)hip_stream);
  return e == hipSuccess ? N2V_OK : hip_fail(e, select ? "select launch" : "rank launch");
}

int n2v_ef_select(n2v_graph g, const uint64_t* d_idx, uint64_t count, uint64_t* d_out, void* hip_stream) {
  return ef_bulk(g, d_idx, count, d_out, hip_stream, true);
}

int n2v_ef_rank(n2v_graph g, const uint64_t* d_x, uint64_t count, uint64_t* d_out, void* hip_stream) {
  return ef_bulk(g, d_x, count, d_out, hip_stream, false);
}

int n2v_graph_info(n2v_graph g, n2v_graph_info_t* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
  out->n_nodes = gr->n_nodes;
  out->n_entries = gr->n_entries;
  out->max_degree = gr->max_degree;
  out->max_row_wsum = gr->max_row_wsum;
  out->sum_deg_sq = gr->sum_deg_sq;
  out->weighted = gr->weighted;
  out->prefix_bytes = gr->dev.r_bytes;
  out->device_bytes = gr->owned_bytes;
  out->storage = gr->storage;
  out->ef_quantum = gr->ef_quantum;
  out->pair_lists = gr->pair_lists;
  out->pair_entries = gr->pair_entries;
  out->hub_sets = gr->hub_count;
  out->hub_min_degree = gr->dev.hub_min_deg;
  return N2V_OK;
}

int n2v_graph_release(n2v_graph g) {
  GraphRec* gr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find(g);
    if (it == g_graphs.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
    gr = it->second;
    g_graphs.erase(it);
  }
  free_record(gr);
  return N2V_OK;
}

int n2v_walk_contexts(const int32_t* d_walks, uint64_t n_walks, uint32_t walk_len, uint32_t window,
                      uint32_t stride, int32_t* d_contexts, void* hip_stream) {
  if (walk_len == 0 || window == 0 || stride == 0) return fail(N2V_ERR_INVALID_ARG, "walk_len, window and stride must be >= 1");
  if (window > kMaxWindow) return fail(N2V_ERR_INVALID_ARG, "window %u above %u", window, kMaxWindow);
  if (n_walks > 0 && (!d_walks || !d_contexts)) return fail(N2V_ERR_INVALID_ARG, "walks and contexts must be non-NULL");
  if ((unsigned __int128)n_walks * walk_len * window >= ((unsigned __int128)1 << 60))
    return fail(N2V_ERR_INVALID_ARG, "output too large");
  DevInfo di;
  int rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  hipError_t e = launch_contexts(d_walks, n_walks, walk_len, window, stride, d_contexts, di, (hipStream_t)hip_stream);
  return e == hipSuccess ? N2V_OK : hip_fail(e, "contexts launch");
}

int n2v_walks_contexts(n2v_graph g, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                       uint32_t walks_per_start, uint32_t walk_len, double p, double q, uint64_t seed,
                       uint64_t walk_id_base, uint32_t window, uint32_t stride, int32_t* d_contexts,
                       int32_t* d_lens, void* hip_stream) {
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
  if (gr->storage != N2V_STORAGE_CSR) return fail(N2V_ERR_INVALID_ARG, "fused contexts need a CSR graph");
  if (window == 0 || stride == 0) return fail(N2V_ERR_INVALID_ARG, "window and stride must be >= 1");
  if (walk_len == 0) return fail(N2V_ERR_INVALID_ARG, "walk_len must be >= 1");
  const uint64_t hh = std::min<uint64_t>((uint64_t)window * stride, (uint64_t)walk_len - 1);
  if (hh > kMaxFusedHalo)
    return fail(N2V_ERR_INVALID_ARG, "window * stride %llu above the fused limit %u (materialise the walks)",
                (unsigned long long)hh, kMaxFusedHalo);
  if ((unsigned __int128)n_starts * walks_per_start * walk_len * window >= ((unsigned __int128)1 << 60))
    return fail(N2V_ERR_INVALID_ARG, "output too large");
  WalkArgs a;
  Path path;
  int rc = prepare_request(*gr, kind, d_starts, n_starts, walks_per_start, walk_len, p, q, seed, walk_id_base,
                           d_contexts, d_lens, 0u, &a, &path);
  if (rc != N2V_OK) return rc;
  a.Y = nullptr;  // no walk array: the kernel writes contexts only
  DevInfo di;
  rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  uint32_t rp = 1;
  while (rp < 2 * hh + 1) rp <<= 1;
  LaunchCfg cfg = choose_cfg(*gr, di, a.nwalks);
  cfg.lists = gr->pair_lists > 0 && gr->pair_lists == gr->n_entries ? 1 : 0;
  // groups of 4, 16 or 64 lanes (the narrowest at or above the chosen width)
  // whose block, rings included, fits the LDS
  cfg.lanes_per_walker = cfg.lanes_per_walker <= 4 ? 4 : (cfg.lanes_per_walker <= 16 ? 16 : 64);
  while (ctx_block_lds_bytes(cfg.lanes_per_walker, cfg.lds_tile, cfg.list_cap, rp) > di.lds_per_block_max) {
    if (cfg.lanes_per_walker < 64) {
      cfg.lanes_per_walker = cfg.lanes_per_walker == 4 ? 16 : 64;
    } else if (cfg.lds_tile > 1 || cfg.list_cap > 1) {
      if (cfg.lds_tile >= cfg.list_cap && cfg.lds_tile > 1) cfg.lds_tile /= 2;
      else cfg.list_cap /= 2;
    } else {
      return fail(N2V_ERR_INVALID_ARG, "context ring of %u words does not fit the LDS", rp);
    }
  }
  hipError_t e = launch_walks_ctx(a, cfg, d_contexts, window, stride, (uint32_t)hh, rp, di, (hipStream_t)hip_stream);
  return e == hipSuccess ? N2V_OK : hip_fail(e, "fused contexts launch");
}

int n2v_negative_samples(n2v_graph g, const int32_t* d_walks, uint64_t n_walks, uint32_t walk_len,
                         uint32_t n_neg, uint64_t seed, uint64_t walk_id_base, int32_t* d_negatives,
                         void* hip_stream) {
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
  if (walk_len == 0 || n_neg == 0) return fail(N2V_ERR_INVALID_ARG, "walk_len and n_neg must be >= 1");
  if (n_neg > kMaxNegatives) return fail(N2V_ERR_INVALID_ARG, "n_neg %u above %u", n_neg, kMaxNegatives);
  if (n_walks > 0 && (!d_walks || !d_negatives)) return fail(N2V_ERR_INVALID_ARG, "walks and negatives must be non-NULL");
  if ((unsigned __int128)n_walks * walk_len * n_neg >= ((unsigned __int128)1 << 60))
    return fail(N2V_ERR_INVALID_ARG, "output too large");
  if (n_walks == 0) return N2V_OK;
  DevInfo di;
  int rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  if (di.device != gr->device) return fail(N2V_ERR_INVALID_ARG, "graph lives on device %d, current is %d", gr->device, di.device);
  hipStream_t st = (hipStream_t)hip_stream;
  if (gr->storage == N2V_STORAGE_EF) {
    hipError_t e = launch_negatives_ef(gr->ef, d_walks, n_walks, walk_len, n_neg, seed, walk_id_base, d_negatives,
                                       di, st);
    return e == hipSuccess ? N2V_OK : hip_fail(e, "negatives launch");
  }
  int32_t* guide = nullptr;
  uint32_t shift = 0;
  if (gr->n_entries > 0) {
    // The guide table is built once, on this stream, and finished before any
    // call (on any stream) can use it.
    std::lock_guard<std::mutex> lk(g_mu);
    if (!gr->neg_guide) {
      const uint32_t s = neg_guide_shift(gr->dev.n);
      int32_t* t = nullptr;
      hipError_t e = hipMalloc(&t, neg_guide_bytes(s, gr->dev.n, gr->dev.m));
      if (e != hipSuccess) return fail(N2V_ERR_NOMEM, "guide table: %s", hipGetErrorString(e));
      e = launch_neg_guide(gr->dev, t, s, di, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        hipFree(t);
        return hip_fail(e, "guide table");
      }
      gr->neg_guide = t;
      gr->neg_shift = s;
    }
    guide = gr->neg_guide;
    shift = gr->neg_shift;
  }
  hipError_t e = launch_negatives(gr->dev, guide, shift, d_walks, n_walks, walk_len, n_neg, seed, walk_id_base,
                                  d_negatives, di, st);
  return e == hipSuccess ? N2V_OK : hip_fail(e, "negatives launch");
}

int n2v_set_tuning(const n2v_tuning_t* tuning) {
  if (tuning) {
    const int rc = check_tuning(*tuning);
    if (rc != N2V_OK) return rc;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune_set = tuning != nullptr;
  if (tuning) g_tune = *tuning;
  return N2V_OK;
}

static int walks_common(n2v_graph g, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                        uint32_t walks_per_start, uint32_t walk_len, double p, double q,
                        uint64_t seed, uint64_t walk_id_base, int32_t* d_walks, int32_t* d_lens,
                        uint32_t k_approx, void* hip_stream) {
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph %llu", (unsigned long long)g);
  WalkArgs a;
  Path path;
  int rc = prepare_request(*gr, kind, d_starts, n_starts, walks_per_start, walk_len, p, q, seed,
                           walk_id_base, d_walks, d_lens, k_approx, &a, &path);
  if (rc != N2V_OK) return rc;
  if (gr->storage == N2V_STORAGE_EF && k_approx > 0)
    return fail(N2V_ERR_INVALID_ARG, "approximated walks need a CSR graph");
  if (a.nwalks == 0) return N2V_OK;
  DevInfo di;
  rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  if (gr->storage == N2V_STORAGE_EF) {
    hipError_t e = launch_walks_ef(a, path, gr->ef, di, (hipStream_t)hip_stream);
    return e == hipSuccess ? N2V_OK : hip_fail(e, "walk launch");
  }
  LaunchCfg cfg = choose_cfg(*gr, di, a.nwalks);
  cfg.lists = gr->pair_lists > 0 && gr->pair_lists == gr->n_entries ? 1 : 0;
  hipError_t e = launch_walks(a, path, cfg, di, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "walk launch");
  return N2V_OK;
}

int n2v_walks_first_order(n2v_graph g, const int32_t* d_starts, uint64_t n_starts,
                          uint32_t walks_per_start, uint32_t walk_len, uint64_t seed,
                          uint64_t walk_id_base, int32_t* d_walks, int32_t* d_lens,
                          void* hip_stream) {
  return walks_common(g, N2V_FIRST_ORDER, d_starts, n_starts, walks_per_start, walk_len, 1.0, 1.0,
                      seed, walk_id_base, d_walks, d_lens, 0u, hip_stream);
}

int n2v_walks_node2vec(n2v_graph g, const int32_t* d_starts, uint64_t n_starts,
                       uint32_t walks_per_start, uint32_t walk_len, double p, double q,
                       uint64_t seed, uint64_t walk_id_base, int32_t* d_walks, int32_t* d_lens,
                       void* hip_stream) {
  return walks_common(g, N2V_NODE2VEC, d_starts, n_starts, walks_per_start, walk_len, p, q, seed,
                      walk_id_base, d_walks, d_lens, 0u, hip_stream);
}

int n2v_walks_approximated(n2v_graph g, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                           uint32_t walks_per_start, uint32_t walk_len, double p, double q,
                           uint32_t k, uint64_t seed, uint64_t walk_id_base, int32_t* d_walks,
                           int32_t* d_lens, void* hip_stream) {
  if (k == 0) return fail(N2V_ERR_INVALID_ARG, "k must be >= 1");
  return walks_common(g, kind, d_starts, n_starts, walks_per_start, walk_len, p, q, seed, walk_id_base,
                      d_walks, d_lens, k, hip_stream);
}

}  // extern "C"
