// Batched and served forms of the walk generator: chunk queues ordered
// longest-estimated-first, a launch-shape autotuner, hipGraph capture of the
// persistent launch, and a server that admits requests by memory footprint and
// runs them in bounded quanta of the persistent kernel (continuous batching).
#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "n2v_runtime.hpp"

namespace n2v {
namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// Estimated cost of one walk step, in work units, from the graph's stationary
// mean degree E = sum(d^2) / sum(d) and the kernel family: the lane paths cost
// O(log d) dependent loads, the node2vec path a few bisections plus a list.
double step_cost(const GraphRec& gr, Path path) {
  const double E = gr.n_entries ? (double)gr.sum_deg_sq / (double)gr.n_entries : 1.0;
  const double l = std::log2(1.0 + E);
  switch (path) {
    case Path::kFirstOrder: return 1.0 + 0.1 * l;
    case Path::kReturnOnly: return 2.0 + 0.2 * l;
    default: return 6.0 + l;
  }
}

struct Prepared {
  WalkArgs args;
  double walk_cost;         // estimated units per walk row
  bool full_lists = false;  // every edge of the graph keeps a stored common-neighbour list
};

int prepare_all(const n2v_request_desc_t* reqs, uint32_t n, std::vector<Prepared>* out) {
  out->clear();
  out->reserve(n);
  for (uint32_t i = 0; i < n; ++i) {
    const n2v_request_desc_t& r = reqs[i];
    GraphRec* gr = find_graph(r.graph);
    if (!gr) return fail(N2V_ERR_BAD_HANDLE, "request %u: unknown graph", i);
    if (gr->storage != N2V_STORAGE_CSR) return fail(N2V_ERR_INVALID_ARG, "request %u: batches need a CSR graph", i);
    Prepared p;
    Path path;
    int rc = prepare_request(*gr, r.kind, r.d_starts, r.n_starts, r.walks_per_start, r.walk_len, r.p,
                             r.q, r.seed, r.walk_id_base, r.d_walks, r.d_lens, r.k_approx, &p.args, &path);
    if (rc != N2V_OK) return fail(rc, "request %u: %s", i, t_err.c_str());
    p.walk_cost = (double)(r.walk_len > 1 ? r.walk_len - 1 : 1) * step_cost(*gr, path);
    p.full_lists = gr->pair_lists > 0 && gr->pair_lists == gr->n_entries;
    out->push_back(p);
  }
  return N2V_OK;
}

// Whether any request takes approximated steps (the queue kernel then needs
// its full instantiation).
bool needs_full(const std::vector<Prepared>& reqs) {
  for (const Prepared& r : reqs)
    if (r.args.k_approx != 0) return true;
  return false;
}

// Whether every request's graph is weighted with 32-bit prefixes (the queue
// kernel then carries only those walk variants).
bool weighted32(const WalkArgs& a) { return a.g.W != nullptr && a.g.r_bytes == 4; }
int all_w32(const std::vector<Prepared>& reqs) {
  for (const Prepared& r : reqs)
    if (!weighted32(r.args)) return 0;
  return 1;
}

// Whether every node2vec request's graph keeps a stored list for every edge.
int all_lists(const std::vector<Prepared>& reqs) {
  for (const Prepared& r : reqs)
    if (r.args.path == (uint32_t)Path::kGeneric && !r.full_lists) return 0;
  return 1;
}

// Split every request into chunks of roughly `target` units and order them
// longest-estimated-first.  A wavefront runs one chunk at a time: lane-path
// chunks are whole multiples of 64 rows (one per lane) and node2vec chunks
// whole multiples of `unit` rows (the wavefront's walker groups).
// frac < 1 chunks only the first ceil(frac * n) rows of each request (an
// autotuning sample).
std::vector<QueueChunk> make_chunks(const std::vector<Prepared>& reqs, double target, uint64_t unit,
                                    double* total_cost, double frac = 1.0) {
  struct C {
    QueueChunk c;
    double cost;
  };
  std::vector<C> v;
  double total = 0;
  for (uint32_t i = 0; i < reqs.size(); ++i) {
    const Prepared& p = reqs[i];
    uint64_t nw = p.args.nwalks;
    if (nw == 0) continue;
    if (frac < 1.0) nw = std::max<uint64_t>(1, (uint64_t)std::ceil((double)nw * frac));
    total += p.walk_cost * (double)nw;
    uint64_t cw = (uint64_t)std::max(1.0, std::floor(target / std::max(p.walk_cost, 1e-9)));
    const uint64_t u = p.args.path != (uint32_t)Path::kGeneric ? 64 : unit;
    cw = std::max<uint64_t>(u, (cw + u - 1) / u * u);
    for (uint64_t w0 = 0; w0 < nw; w0 += cw) {
      const uint64_t w1 = std::min(nw, w0 + cw);
      v.push_back({{i, 0, w0, w1}, p.walk_cost * (double)(w1 - w0)});
    }
  }
  std::stable_sort(v.begin(), v.end(), [](const C& a, const C& b) { return a.cost > b.cost; });
  std::vector<QueueChunk> out(v.size());
  for (size_t k = 0; k < v.size(); ++k) out[k] = v[k].c;
  if (total_cost) *total_cost = total;
  return out;
}

// Device memory whose last use is a kernel still in flight: freed once the
// recorded event has completed.
std::mutex g_defer_mu;  // guards g_deferred
std::vector<std::pair<hipEvent_t, void*>> g_deferred;

void reap_deferred(bool wait) {
  std::lock_guard<std::mutex> lk(g_defer_mu);
  for (size_t i = 0; i < g_deferred.size();) {
    hipEvent_t ev = g_deferred[i].first;
    if (wait) (void)hipEventSynchronize(ev);
    if (hipEventQuery(ev) == hipSuccess) {
      (void)hipFree(g_deferred[i].second);
      (void)hipEventDestroy(ev);
      g_deferred[i] = g_deferred.back();
      g_deferred.pop_back();
    } else {
      ++i;
    }
  }
}

int upload_tables(const std::vector<Prepared>& reqs, const std::vector<QueueChunk>& chunks, void** block,
                  WalkArgs** d_reqs, QueueChunk** d_chunks, uint32_t** d_head) {
  const size_t rb = reqs.size() * sizeof(WalkArgs);
  const size_t cb = chunks.size() * sizeof(QueueChunk);
  const size_t off_c = (rb + 255) / 256 * 256;
  const size_t off_h = off_c + (cb + 255) / 256 * 256;
  const size_t bytes = off_h + 256;
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail(N2V_ERR_NOMEM, "hipMalloc batch tables: %s", hipGetErrorString(e));
  std::vector<uint8_t> h(bytes, 0);
  for (size_t i = 0; i < reqs.size(); ++i) std::memcpy(h.data() + i * sizeof(WalkArgs), &reqs[i].args, sizeof(WalkArgs));
  if (cb) std::memcpy(h.data() + off_c, chunks.data(), cb);
  e = hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "upload batch tables");
  }
  *block = d;
  *d_reqs = (WalkArgs*)d;
  *d_chunks = (QueueChunk*)((uint8_t*)d + off_c);
  *d_head = (uint32_t*)((uint8_t*)d + off_h);
  return N2V_OK;
}

// Wavefronts of a shape resident on the whole device at once.
double resident_waves(const LaunchCfg& c, const DevInfo& di) {
  return (double)queue_grid_blocks(c, di, 1u << 30) * 4.0;
}

// Node2vec rows per chunk unit: one per walker group of a wavefront.
uint64_t group_unit(const LaunchCfg& c) { return (uint64_t)(64 / c.lanes_per_walker); }

// Chunk size (work units) giving about 16 chunks per resident wavefront: a
// queue with too few chunks leaves wavefronts idle (and a long tail).
double chunk_target(double total, const LaunchCfg& c, const DevInfo& di) {
  return std::max(total / (resident_waves(c, di) * 16.0), 1.0);
}

LaunchCfg shape_cfg(int lanes, int tile, int cap) {
  LaunchCfg c;
  c.lanes_per_walker = lanes;
  c.lds_tile = tile;
  c.list_cap = cap;
  return c;
}

// Default launch shape of a batch: 4-lane groups when every second-order
// request's graph keeps a stored common-neighbour list for every edge (a step
// is then a few short searches, and 16 walks per wavefront keep more loads in
// flight) and the batch has the walks to fill the device that way; one walk
// per wavefront otherwise (wide groups build long lists faster).
LaunchCfg batch_default_cfg(const std::vector<Prepared>& reqs, const DevInfo& di) {
  uint64_t gen = 0;
  bool lists = true;
  for (const Prepared& r : reqs) {
    if (r.args.path != (uint32_t)Path::kGeneric || r.args.nwalks == 0) continue;
    gen += r.args.nwalks;
    lists = lists && r.full_lists;
  }
  const uint64_t cus = di.cus > 0 ? (uint64_t)di.cus : 256;
  if (gen > 0 && lists && gen >= 96 * cus) return shape_cfg(4, 16, 32);
  return shape_cfg(64, 64, 576);
}

// ---------------------------------------------------------------------------
// Batch plans
// ---------------------------------------------------------------------------
struct BatchPlan {
  std::vector<Prepared> reqs;
  std::vector<QueueChunk> chunks;
  void* block = nullptr;
  WalkArgs* d_reqs = nullptr;
  QueueChunk* d_chunks = nullptr;
  uint32_t* d_head = nullptr;
  LaunchCfg cfg;
  DevInfo di;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double est = 0;
  uint64_t nwalks = 0;
};

std::mutex g_plan_mu;
std::unordered_map<uint64_t, BatchPlan*> g_plans;
uint64_t g_next_plan = 1;

void free_plan(BatchPlan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->block) (void)hipFree(p->block);
  delete p;
}

// Time candidate launch shapes on a sample of the batch: the first eighth of
// every request's rows, chunked for each shape as the full batch would be
// (16 chunks per resident group), so that a narrow shape's many groups are as
// busy in the sample as in the real launch.
int autotune(BatchPlan* p) {
  double total = 0;
  for (const Prepared& r : p->reqs) total += r.walk_cost * (double)r.args.nwalks;
  if (total <= 0) return N2V_OK;
  constexpr double kFrac = 0.125;
  hipStream_t st;
  hipEvent_t e0, e1;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int shapes[][3] = {{64, 64, 576}, {64, 128, 512}, {32, 64, 256}, {16, 32, 128}, {4, 16, 32}};
  float best = 1e30f;
  LaunchCfg best_cfg = p->cfg;
  hipError_t e = hipSuccess;
  int rc = N2V_OK;
  for (const auto& sh : shapes) {
    LaunchCfg c = shape_cfg(sh[0], sh[1], sh[2]);
    c.full = needs_full(p->reqs) ? 1 : 0;
    c.w32 = all_w32(p->reqs);
    c.lists = all_lists(p->reqs);
    if (block_lds_bytes(c.lanes_per_walker, c.lds_tile, c.list_cap) > p->di.lds_per_block_max) continue;
    const std::vector<QueueChunk> sample =
        make_chunks(p->reqs, chunk_target(total * kFrac, c, p->di), group_unit(c), nullptr, kFrac);
    void* blk = nullptr;
    WalkArgs* dr;
    QueueChunk* dc;
    uint32_t* dh;
    rc = upload_tables(p->reqs, sample, &blk, &dr, &dc, &dh);
    if (rc != N2V_OK) break;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = launch_queue(dr, dc, (uint32_t)sample.size(), dh, c, p->di, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) ms_min = std::min(ms_min, ms);
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(blk);
    if (e != hipSuccess) break;
    if (ms_min < best) {
      best = ms_min;
      best_cfg = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  if (rc != N2V_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "autotune");
  p->cfg = best_cfg;
  return N2V_OK;
}

// ---------------------------------------------------------------------------
// Server
// ---------------------------------------------------------------------------
enum class RState { kQueued, kActive, kDone, kFailed };

struct SrvReq {
  uint64_t id = 0;
  n2v_request_desc_t desc{};
  std::vector<int32_t> h_starts;
  GraphRec* gr = nullptr;
  uint64_t nwalks = 0, footprint = 0;
  uint64_t t_arrival = 0, t_admit = 0, t_start = 0, t_done = 0;
  RState state = RState::kQueued;
  int slot = -1;
  void* mem = nullptr;  // walks | lens | starts
  WalkArgs args{};
  double walk_cost = 0;
  uint64_t chunk_rows = 1;
  uint64_t next_row = 0;       // rows not yet given to a quantum start here
  uint64_t rows_done = 0;      // rows whose quantum has completed
  uint64_t steps = 0;
  int err = N2V_OK;
};

struct Quantum {
  hipEvent_t done = nullptr;
  void* block = nullptr;       // device tables
  size_t block_bytes = 0;
  uint8_t* h_stage = nullptr;  // pinned staging for the tables
  size_t stage_bytes = 0;
  uint64_t* h_steps = nullptr; // pinned copy of the per-slot step counters
  std::vector<std::pair<SrvReq*, uint64_t>> rows;  // rows of each request in this quantum
  double est = 0;
  uint64_t t_launch = 0;
  bool busy = false;
};

struct Server {
  uint64_t handle = 0;
  uint64_t budget = 0, in_use = 0;
  uint32_t max_slots = 0;
  std::vector<int> free_slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SrvReq*> fifo;
  std::vector<SrvReq*> active;  // admitted, not finished, in admission order
  std::unordered_map<uint64_t, SrvReq*> all;
  std::vector<GraphRec*> graphs;
  uint64_t next_req = 1;
  bool stop = false;
  std::thread th;
  hipStream_t st = nullptr;
  unsigned long long* d_steps = nullptr;  // one counter per slot
  Quantum q[2];
  LaunchCfg cfg;
  DevInfo di;
  int device = 0;
  size_t quantum_chunks = 0;  // chunks per quantum: eight per resident wavefront
  int fatal = N2V_OK;
};

std::mutex g_srv_mu;
std::unordered_map<uint64_t, Server*> g_servers;
uint64_t g_next_srv = 1;

Server* find_server(n2v_server h) {
  std::lock_guard<std::mutex> lk(g_srv_mu);
  auto it = g_servers.find(h);
  return it == g_servers.end() ? nullptr : it->second;
}

uint64_t footprint_of(uint64_t ns, uint64_t nw, uint32_t L) {
  const uint64_t walks = nw * L * 4, lens = nw * 4, starts = ns * 4;
  return (walks + 255) / 256 * 256 + (lens + 255) / 256 * 256 + (starts + 255) / 256 * 256;
}

// Admit queued requests in FIFO order while memory and slots allow (under mu).
void admit_locked(Server* s) {
  while (!s->fifo.empty() && !s->free_slots.empty()) {
    SrvReq* r = s->fifo.front();
    if (r->footprint > s->budget - s->in_use) break;  // FIFO: the head waits for memory
    s->fifo.pop_front();
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->in_use += r->footprint;
    r->t_admit = now_ns();
    const n2v_request_desc_t& d = r->desc;
    const uint64_t walks = r->nwalks * d.walk_len * 4, lens = r->nwalks * 4;
    const uint64_t off_l = (walks + 255) / 256 * 256, off_s = off_l + (lens + 255) / 256 * 256;
    hipError_t e = hipMallocAsync(&r->mem, std::max<uint64_t>(r->footprint, 256), s->st);
    if (e == hipSuccess && d.n_starts)
      e = hipMemcpyAsync((uint8_t*)r->mem + off_s, r->h_starts.data(), d.n_starts * 4, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_steps + r->slot, 0, sizeof(unsigned long long), s->st);
    Path path;
    int rc = e == hipSuccess ? N2V_OK : N2V_ERR_NOMEM;
    if (rc == N2V_OK)
      rc = prepare_request(*r->gr, d.kind, (const int32_t*)((uint8_t*)r->mem + off_s), d.n_starts,
                           d.walks_per_start, d.walk_len, d.p, d.q, d.seed, d.walk_id_base,
                           (int32_t*)r->mem, (int32_t*)((uint8_t*)r->mem + off_l), d.k_approx, &r->args, &path);
    if (rc != N2V_OK) {
      r->state = RState::kFailed;
      r->err = rc;
      r->t_done = now_ns();
      s->free_slots.push_back(r->slot);
      r->slot = -1;
      s->in_use -= r->footprint;
      if (r->mem) (void)hipFreeAsync(r->mem, s->st);
      r->mem = nullptr;
      continue;
    }
    r->args.steps = s->d_steps + r->slot;
    r->walk_cost = (double)(d.walk_len > 1 ? d.walk_len - 1 : 1) * step_cost(*r->gr, path);
    // the finest grain a wavefront can use: one walk per walker group on the
    // node2vec path, one walk per lane on the lane paths
    r->chunk_rows = path == Path::kGeneric ? (uint64_t)(64 / s->cfg.lanes_per_walker) : 64;
    r->state = RState::kActive;
    s->active.push_back(r);
  }
}

// Build the next quantum's chunk list (under mu): one chunk for every active
// request with rows left (so every admitted request progresses), then more
// chunks oldest-first until the quantum holds about eight chunks for every
// resident wavefront.
void build_quantum_locked(Server* s, Quantum* q, std::vector<WalkArgs>* reqs, std::vector<QueueChunk>* chunks) {
  q->rows.clear();
  q->est = 0;
  reqs->clear();
  chunks->clear();
  const size_t budget = s->quantum_chunks;
  std::unordered_map<SrvReq*, uint32_t> idx;
  auto take = [&](SrvReq* r) {
    const uint64_t w0 = r->next_row, w1 = std::min(r->nwalks, w0 + r->chunk_rows);
    auto it = idx.find(r);
    uint32_t k;
    if (it == idx.end()) {
      k = (uint32_t)reqs->size();
      idx[r] = k;
      reqs->push_back(r->args);
      q->rows.push_back({r, 0});
    } else {
      k = it->second;
    }
    chunks->push_back({k, 0, w0, w1});
    q->rows[k].second += w1 - w0;
    q->est += r->walk_cost * (double)(w1 - w0);
    r->next_row = w1;
  };
  for (SrvReq* r : s->active)
    if (r->next_row < r->nwalks && chunks->size() < budget) take(r);
  for (SrvReq* r : s->active)
    while (r->next_row < r->nwalks && chunks->size() < budget) take(r);
  // longest estimated chunks first, so the quantum's tail is short walks
  std::vector<double> cost(reqs->size());
  for (auto& kv : idx) cost[kv.second] = kv.first->walk_cost;
  std::stable_sort(chunks->begin(), chunks->end(), [&](const QueueChunk& a, const QueueChunk& b) {
    return cost[a.req] * (double)(a.w1 - a.w0) > cost[b.req] * (double)(b.w1 - b.w0);
  });
}

int launch_quantum(Server* s, Quantum* q, const std::vector<WalkArgs>& reqs, const std::vector<QueueChunk>& chunks) {
  const size_t rb = reqs.size() * sizeof(WalkArgs), cb = chunks.size() * sizeof(QueueChunk);
  const size_t off_c = (rb + 255) / 256 * 256, off_h = off_c + (cb + 255) / 256 * 256;
  const size_t bytes = off_h + 256;
  if (bytes > q->block_bytes) {
    if (q->block) (void)hipFree(q->block);
    if (q->h_stage) (void)hipHostFree(q->h_stage);
    q->block = nullptr;
    q->h_stage = nullptr;
    size_t cap = std::max<size_t>(bytes * 2, 1 << 20);
    if (hipMalloc(&q->block, cap) != hipSuccess) return N2V_ERR_NOMEM;
    if (hipHostMalloc((void**)&q->h_stage, cap, 0) != hipSuccess) return N2V_ERR_NOMEM;
    q->block_bytes = q->stage_bytes = cap;
  }
  std::memcpy(q->h_stage, reqs.data(), rb);
  std::memcpy(q->h_stage + off_c, chunks.data(), cb);
  hipError_t e = hipMemcpyAsync(q->block, q->h_stage, off_h, hipMemcpyHostToDevice, s->st);
  LaunchCfg cfg = s->cfg;
  cfg.full = 0;
  cfg.w32 = 1;
  for (const WalkArgs& r : reqs) {
    if (r.k_approx != 0) cfg.full = 1;
    if (!weighted32(r)) cfg.w32 = 0;
  }
  if (e == hipSuccess)
    e = launch_queue((WalkArgs*)q->block, (QueueChunk*)((uint8_t*)q->block + off_c), (uint32_t)chunks.size(),
                     (uint32_t*)((uint8_t*)q->block + off_h), cfg, s->di, s->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(q->h_steps, s->d_steps, sizeof(uint64_t) * s->max_slots, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipEventRecord(q->done, s->st);
  if (e != hipSuccess) return hip_fail(e, "server quantum");
  q->t_launch = now_ns();
  q->busy = true;
  return N2V_OK;
}

void dispatcher(Server* s) {
  (void)hipSetDevice(s->device);
  std::deque<Quantum*> inflight;
  std::vector<WalkArgs> reqs;
  std::vector<QueueChunk> chunks;
  int next_q = 0;
  while (true) {
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->fatal != N2V_OK && inflight.empty()) {
      // a launch failed: nothing more will run; fail what is admitted or queued
      for (SrvReq* r : s->active) {
        r->state = RState::kFailed;
        r->err = s->fatal;
        r->t_done = now_ns();
        s->free_slots.push_back(r->slot);
      }
      s->active.clear();
      for (SrvReq* r : s->fifo) {
        r->state = RState::kFailed;
        r->err = s->fatal;
      }
      s->fifo.clear();
      s->cv.notify_all();
      if (s->stop) break;
      s->cv.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    admit_locked(s);
    bool more = false;
    for (SrvReq* r : s->active) more |= r->next_row < r->nwalks;
    if (more && inflight.size() < 2 && s->fatal == N2V_OK) {
      Quantum* q = &s->q[next_q];
      next_q ^= 1;
      build_quantum_locked(s, q, &reqs, &chunks);
      const uint64_t t = now_ns();
      for (auto& pr : q->rows)
        if (!pr.first->t_start) pr.first->t_start = t;
      lk.unlock();
      int rc = launch_quantum(s, q, reqs, chunks);
      if (rc != N2V_OK) {
        std::lock_guard<std::mutex> g(s->mu);
        s->fatal = rc;
      } else {
        inflight.push_back(q);
      }
      continue;
    }
    if (!inflight.empty()) {
      Quantum* q = inflight.front();
      lk.unlock();
      hipError_t e = hipEventSynchronize(q->done);
      const uint64_t t = now_ns();
      lk.lock();
      inflight.pop_front();
      q->busy = false;
      if (e != hipSuccess) s->fatal = N2V_ERR_HIP;
      for (auto& pr : q->rows) {
        SrvReq* r = pr.first;
        r->rows_done += pr.second;
        if (r->rows_done == r->nwalks && r->state == RState::kActive) {
          r->state = s->fatal == N2V_OK ? RState::kDone : RState::kFailed;
          r->err = s->fatal;
          r->t_done = t;
          r->steps = q->h_steps[r->slot];
          s->free_slots.push_back(r->slot);
          s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        }
      }
      s->cv.notify_all();
      continue;
    }
    // requests with zero walks finish at admission
    for (size_t i = 0; i < s->active.size();) {
      SrvReq* r = s->active[i];
      if (r->nwalks == 0) {
        r->state = RState::kDone;
        r->t_start = r->t_done = now_ns();
        s->free_slots.push_back(r->slot);
        s->active.erase(s->active.begin() + i);
      } else {
        ++i;
      }
    }
    if (s->stop && s->active.empty()) break;
    s->cv.wait_for(lk, std::chrono::milliseconds(2));
  }
}

// ---------------------------------------------------------------------------
// Allocation-free batched launch: the request table, the chunk queue and its
// head counter live in a file-scope device array instead of a hipMalloc'd
// block.  Each device holds its own copy of the array; host code uses only
// the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr uint32_t kScratchMaxReqs = 4096;
static_assert((size_t)kScratchMaxReqs * sizeof(WalkArgs) + 1024 < kScratchBytes / 2,
              "request table must leave room for the chunk queue");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;  // guards g_scratch_ptr
std::unordered_map<int, void*> g_scratch_ptr;

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return N2V_OK;
}

}  // namespace
}  // namespace n2v

using namespace n2v;

extern "C" {

int n2v_walks_batched(const n2v_request_desc_t* reqs, uint32_t n_reqs, void* hip_stream) {
  if (n_reqs > 0 && !reqs) return fail(N2V_ERR_INVALID_ARG, "reqs is NULL");
  reap_deferred(false);
  std::vector<Prepared> pr;
  int rc = prepare_all(reqs, n_reqs, &pr);
  if (rc != N2V_OK) return rc;
  DevInfo di;
  rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  double total = 0;
  for (const Prepared& r : pr) total += r.walk_cost * (double)r.args.nwalks;
  LaunchCfg cfg = batch_default_cfg(pr, di);
  apply_tuning_override(&cfg, di);
  cfg.full = needs_full(pr) ? 1 : 0;
  cfg.w32 = all_w32(pr);
  cfg.lists = all_lists(pr);
  std::vector<QueueChunk> chunks = make_chunks(pr, chunk_target(total, cfg, di), group_unit(cfg), nullptr);
  if (chunks.empty()) return N2V_OK;
  if (chunks.size() > (1u << 30)) return fail(N2V_ERR_INVALID_ARG, "too many chunks");
  void* blk;
  WalkArgs* dr;
  QueueChunk* dc;
  uint32_t* dh;
  rc = upload_tables(pr, chunks, &blk, &dr, &dc, &dh);
  if (rc != N2V_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = launch_queue(dr, dc, (uint32_t)chunks.size(), dh, cfg, di, st);
  hipEvent_t ev;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, st);
  if (e != hipSuccess) {
    (void)hipDeviceSynchronize();
    (void)hipFree(blk);
    return hip_fail(e, "batched launch");
  }
  std::lock_guard<std::mutex> lk(g_defer_mu);
  g_deferred.push_back({ev, blk});
  return N2V_OK;
}

int n2v_walks_batched_noalloc(const n2v_request_desc_t* reqs, uint32_t n_reqs, void* hip_stream) {
  if (n_reqs > 0 && !reqs) return fail(N2V_ERR_INVALID_ARG, "reqs is NULL");
  if (n_reqs > kScratchMaxReqs)
    return fail(N2V_ERR_INVALID_ARG, "n_reqs %u exceeds the allocation-free limit of %u requests", n_reqs,
                kScratchMaxReqs);
  std::vector<Prepared> pr;
  int rc = prepare_all(reqs, n_reqs, &pr);
  if (rc != N2V_OK) return rc;
  DevInfo di;
  rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  double total = 0;
  for (const Prepared& r : pr) total += r.walk_cost * (double)r.args.nwalks;
  LaunchCfg cfg = batch_default_cfg(pr, di);
  apply_tuning_override(&cfg, di);
  cfg.full = needs_full(pr) ? 1 : 0;
  cfg.w32 = all_w32(pr);
  cfg.lists = all_lists(pr);
  // table layout as in upload_tables: requests | chunks | head counter
  const size_t rb = pr.size() * sizeof(WalkArgs);
  const size_t off_c = (rb + 255) / 256 * 256;
  const size_t max_chunks = (kScratchBytes - off_c - 512) / sizeof(QueueChunk);
  double target = chunk_target(total, cfg, di);
  std::vector<QueueChunk> chunks = make_chunks(pr, target, group_unit(cfg), nullptr);
  // coarser chunks until the queue fits (only the load balance changes; at
  // most one chunk per request in the limit, and n_reqs <= kScratchMaxReqs)
  while (chunks.size() > max_chunks) {
    target *= 2.0;
    chunks = make_chunks(pr, target, group_unit(cfg), nullptr);
  }
  if (chunks.empty()) return N2V_OK;
  const size_t cb = chunks.size() * sizeof(QueueChunk);
  const size_t off_h = off_c + (cb + 255) / 256 * 256;
  const size_t bytes = off_h + 256;
  void* base = nullptr;
  rc = scratch_address(&base);
  if (rc != N2V_OK) return rc;
  std::vector<uint8_t> h(bytes, 0);  // the head counter starts at zero
  for (size_t i = 0; i < pr.size(); ++i) std::memcpy(h.data() + i * sizeof(WalkArgs), &pr[i].args, sizeof(WalkArgs));
  std::memcpy(h.data() + off_c, chunks.data(), cb);
  hipStream_t st = (hipStream_t)hip_stream;
  // stream order: the copy waits for earlier work on st (an earlier call's
  // kernel still reading the array); the wait below makes the host buffer
  // free to go and the tables complete before the kernel is enqueued
  hipError_t e = hipMemcpyAsync(base, h.data(), bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "allocation-free batch tables");
  uint8_t* b = (uint8_t*)base;
  e = launch_queue((const WalkArgs*)b, (const QueueChunk*)(b + off_c), (uint32_t)chunks.size(), (uint32_t*)(b + off_h),
                   cfg, di, st);
  if (e != hipSuccess) return hip_fail(e, "allocation-free batched launch");
  return N2V_OK;
}

int n2v_batch_create(const n2v_request_desc_t* reqs, uint32_t n_reqs, uint32_t flags, n2v_batch* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  *out = 0;
  if (n_reqs > 0 && !reqs) return fail(N2V_ERR_INVALID_ARG, "reqs is NULL");
  if (flags & ~(uint32_t)N2V_BATCH_AUTOTUNE) return fail(N2V_ERR_INVALID_ARG, "unknown flags");
  BatchPlan* p = new BatchPlan();
  int rc = prepare_all(reqs, n_reqs, &p->reqs);
  if (rc == N2V_OK) rc = current_devinfo(&p->di);
  if (rc != N2V_OK) {
    delete p;
    return rc;
  }
  double total = 0;
  for (const Prepared& r : p->reqs) total += r.walk_cost * (double)r.args.nwalks;
  for (const Prepared& r : p->reqs) p->nwalks += r.args.nwalks;
  p->cfg = batch_default_cfg(p->reqs, p->di);
  p->cfg.full = needs_full(p->reqs) ? 1 : 0;
  p->cfg.w32 = all_w32(p->reqs);
  p->cfg.lists = all_lists(p->reqs);
  if (flags & N2V_BATCH_AUTOTUNE) rc = autotune(p);
  apply_tuning_override(&p->cfg, p->di);  // an explicit n2v_set_tuning wins
  // the final chunking follows the chosen shape
  if (rc == N2V_OK) {
    p->chunks = make_chunks(p->reqs, chunk_target(total, p->cfg, p->di), group_unit(p->cfg), &p->est);
    if (p->chunks.size() > (1u << 30)) rc = fail(N2V_ERR_INVALID_ARG, "too many chunks");
  }
  if (rc == N2V_OK) rc = upload_tables(p->reqs, p->chunks, &p->block, &p->d_reqs, &p->d_chunks, &p->d_head);
  if (rc == N2V_OK && !p->chunks.empty()) {
    p->cfg.grid_blocks = queue_grid_blocks(p->cfg, p->di, (uint32_t)p->chunks.size());
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = launch_queue(p->d_reqs, p->d_chunks, (uint32_t)p->chunks.size(), p->d_head, p->cfg, p->di, cs);
      e = hipStreamEndCapture(cs, &p->graph);
      if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) rc = hip_fail(e, "batch graph capture");
  }
  if (rc != N2V_OK) {
    free_plan(p);
    return rc;
  }
  std::lock_guard<std::mutex> lk(g_plan_mu);
  const uint64_t h = g_next_plan++;
  g_plans[h] = p;
  *out = h;
  return N2V_OK;
}

int n2v_batch_launch(n2v_batch b, void* hip_stream) {
  BatchPlan* p;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(b);
    if (it == g_plans.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown batch");
    p = it->second;
  }
  if (!p->exec) return N2V_OK;
  hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return N2V_OK;
}

int n2v_batch_info(n2v_batch b, n2v_batch_info_t* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(b);
  if (it == g_plans.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown batch");
  const BatchPlan* p = it->second;
  out->n_requests = (uint32_t)p->reqs.size();
  out->n_chunks = (uint32_t)p->chunks.size();
  out->lanes_per_walker = (uint32_t)p->cfg.lanes_per_walker;
  out->lds_tile = (uint32_t)p->cfg.lds_tile;
  out->list_cap = (uint32_t)p->cfg.list_cap;
  out->reserved = 0;
  out->n_walks = p->nwalks;
  out->est_cost = p->est;
  return N2V_OK;
}

int n2v_batch_destroy(n2v_batch b) {
  BatchPlan* p;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(b);
    if (it == g_plans.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown batch");
    p = it->second;
    g_plans.erase(it);
  }
  (void)hipDeviceSynchronize();  // a replay may still be running
  free_plan(p);
  return N2V_OK;
}

int n2v_server_create(uint64_t hbm_budget_bytes, uint32_t max_slots, const n2v_tuning_t* tuning, n2v_server* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  *out = 0;
  if (tuning) {
    const int trc = check_tuning(*tuning);
    if (trc != N2V_OK) return trc;
  }
  if (max_slots == 0 || max_slots > (1u << 16)) return fail(N2V_ERR_INVALID_ARG, "max_slots must be in [1, 65536]");
  if (hbm_budget_bytes == 0) return fail(N2V_ERR_INVALID_ARG, "budget must be > 0");
  Server* s = new Server();
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  for (int i = (int)max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  int rc = current_devinfo(&s->di);
  if (rc != N2V_OK) {
    delete s;
    return rc;
  }
  s->device = s->di.device;
  s->cfg = shape_cfg(64, 64, 576);
  apply_tuning_override(&s->cfg, s->di, tuning);
  hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&s->d_steps, sizeof(unsigned long long) * max_slots);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&s->q[i].done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->q[i].h_steps, sizeof(uint64_t) * max_slots, 0);
  }
  if (e == hipSuccess) e = hipMemset(s->d_steps, 0, sizeof(unsigned long long) * max_slots);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "server create");
  }
  s->cfg.grid_blocks = queue_grid_blocks(s->cfg, s->di, 1u << 30);
  s->quantum_chunks = (size_t)s->cfg.grid_blocks * 4 * 8;
  s->th = std::thread(dispatcher, s);
  std::lock_guard<std::mutex> lk(g_srv_mu);
  s->handle = g_next_srv++;
  g_servers[s->handle] = s;
  *out = s->handle;
  return N2V_OK;
}

int n2v_server_add_graph(n2v_server sh, n2v_graph g) {
  Server* s = find_server(sh);
  if (!s) return fail(N2V_ERR_BAD_HANDLE, "unknown server");
  GraphRec* gr = find_graph(g);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph");
  if (gr->storage != N2V_STORAGE_CSR) return fail(N2V_ERR_INVALID_ARG, "servers need a CSR graph");
  std::lock_guard<std::mutex> lk(s->mu);
  if (std::find(s->graphs.begin(), s->graphs.end(), gr) == s->graphs.end()) s->graphs.push_back(gr);
  return N2V_OK;
}

int n2v_request_submit(n2v_server sh, const n2v_request_desc_t* desc, uint64_t arrival_ns, n2v_request* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  *out = 0;
  if (!desc) return fail(N2V_ERR_INVALID_ARG, "desc is NULL");
  Server* s = find_server(sh);
  if (!s) return fail(N2V_ERR_BAD_HANDLE, "unknown server");
  GraphRec* gr = find_graph(desc->graph);
  if (!gr) return fail(N2V_ERR_BAD_HANDLE, "unknown graph");
  if (gr->storage != N2V_STORAGE_CSR) return fail(N2V_ERR_INVALID_ARG, "servers need a CSR graph");
  if (desc->n_starts > 0 && !desc->d_starts) return fail(N2V_ERR_INVALID_ARG, "starts is NULL");
  if (desc->walk_len == 0 || desc->walks_per_start == 0) return fail(N2V_ERR_INVALID_ARG, "empty walk shape");
  if ((unsigned __int128)desc->n_starts * desc->walks_per_start * desc->walk_len >= ((unsigned __int128)1 << 60))
    return fail(N2V_ERR_INVALID_ARG, "request too large");
  // validate p, q and overflow now (same rules as the plain calls)
  {
    WalkArgs a;
    Path path;
    int32_t dummy = 0;
    int rc = prepare_request(*gr, desc->kind, &dummy, 0, desc->walks_per_start, desc->walk_len, desc->p, desc->q,
                             desc->seed, desc->walk_id_base, &dummy, nullptr, desc->k_approx, &a, &path);
    if (rc != N2V_OK) return rc;
  }
  SrvReq* r = new SrvReq();
  r->desc = *desc;
  r->gr = gr;
  r->nwalks = desc->n_starts * (uint64_t)desc->walks_per_start;
  r->footprint = footprint_of(desc->n_starts, r->nwalks, desc->walk_len);
  r->t_arrival = arrival_ns ? arrival_ns : now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (std::find(s->graphs.begin(), s->graphs.end(), gr) == s->graphs.end()) {
    delete r;
    return fail(N2V_ERR_BAD_HANDLE, "graph not added to this server");
  }
  if (r->footprint > s->budget) {
    delete r;
    return fail(N2V_ERR_REJECTED, "request needs %llu bytes, budget is %llu", (unsigned long long)r->footprint,
                (unsigned long long)s->budget);
  }
  if (s->stop) {
    delete r;
    return fail(N2V_ERR_BAD_HANDLE, "server is shutting down");
  }
  r->h_starts.assign(desc->d_starts, desc->d_starts + desc->n_starts);
  r->id = s->next_req++;
  s->all[r->id] = r;
  s->fifo.push_back(r);
  s->cv.notify_all();
  *out = r->id;
  return N2V_OK;
}

int n2v_request_poll(n2v_server sh, n2v_request rq, n2v_result_t* out) {
  if (!out) return fail(N2V_ERR_INVALID_ARG, "out is NULL");
  Server* s = find_server(sh);
  if (!s) return fail(N2V_ERR_BAD_HANDLE, "unknown server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(rq);
  if (it == s->all.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown request");
  SrvReq* r = it->second;
  if (r->state == RState::kFailed) return fail(r->err ? r->err : N2V_ERR_HIP, "request failed");
  if (r->state != RState::kDone) {
    if (s->fatal != N2V_OK) return fail(s->fatal, "server failed");
    return N2V_PENDING;
  }
  const uint64_t walks = r->nwalks * r->desc.walk_len * 4;
  out->d_walks = (const int32_t*)r->mem;
  out->d_lens = (const int32_t*)((uint8_t*)r->mem + (walks + 255) / 256 * 256);
  out->n_walks = r->nwalks;
  out->steps = r->steps;
  out->t_arrival_ns = r->t_arrival;
  out->t_admit_ns = r->t_admit;
  out->t_start_ns = r->t_start;
  out->t_done_ns = r->t_done;
  return N2V_OK;
}

int n2v_request_release(n2v_server sh, n2v_request rq) {
  Server* s = find_server(sh);
  if (!s) return fail(N2V_ERR_BAD_HANDLE, "unknown server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(rq);
  if (it == s->all.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown request");
  SrvReq* r = it->second;
  if (r->state == RState::kQueued || r->state == RState::kActive)
    return fail(N2V_ERR_INVALID_ARG, "request still pending");
  if (r->mem) {
    (void)hipFreeAsync(r->mem, s->st);
    s->in_use -= r->footprint;  // memory is accounted exactly while mem is held
  }
  s->all.erase(it);
  delete r;
  s->cv.notify_all();
  return N2V_OK;
}

int n2v_server_destroy(n2v_server sh) {
  Server* s;
  {
    std::lock_guard<std::mutex> lk(g_srv_mu);
    auto it = g_servers.find(sh);
    if (it == g_servers.end()) return fail(N2V_ERR_BAD_HANDLE, "unknown server");
    s = it->second;
    g_servers.erase(it);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // queued requests that were never admitted are cancelled
    for (SrvReq* r : s->fifo) {
      r->state = RState::kFailed;
      r->err = N2V_ERR_BAD_HANDLE;
    }
    s->fifo.clear();
    s->cv.notify_all();
  }
  s->th.join();
  (void)hipStreamSynchronize(s->st);
  for (auto& kv : s->all) {
    if (kv.second->mem) (void)hipFreeAsync(kv.second->mem, s->st);
    delete kv.second;
  }
  (void)hipStreamSynchronize(s->st);
  for (int i = 0; i < 2; ++i) {
    if (s->q[i].block) (void)hipFree(s->q[i].block);
    if (s->q[i].h_stage) (void)hipHostFree(s->q[i].h_stage);
    if (s->q[i].h_steps) (void)hipHostFree(s->q[i].h_steps);
    if (s->q[i].done) (void)hipEventDestroy(s->q[i].done);
  }
  (void)hipFree(s->d_steps);
  (void)hipStreamDestroy(s->st);
  delete s;
  return N2V_OK;
}

}  // extern "C"
