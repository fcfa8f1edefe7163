// Host-runtime internals shared by the C-ABI translation units.
#pragma once

#include <stdint.h>

#include <string>

#include "n2v_internal.hpp"
#include "n2vwalk.h"

namespace n2v {

constexpr uint32_t kC16Host = 65536u;

struct GraphRec {
  uint64_t handle = 0;
  GraphDev dev;
  uint64_t n_nodes = 0, n_entries = 0;
  uint64_t max_degree = 0, max_row_wsum = 0, sum_deg_sq = 0;
  uint32_t weighted = 0;
  uint64_t owned_bytes = 0;
  int device = 0;
  int32_t* neg_guide = nullptr;  // built on the first negative-sampling call
  uint32_t neg_shift = 0;
  uint32_t storage = N2V_STORAGE_CSR;
  EFDev ef;                  // Elias-Fano store (storage == N2V_STORAGE_EF)
  void* ef_mem = nullptr;    // owned: H, L, S1, S0
  uint32_t ef_quantum = 0;
  uint64_t pair_lists = 0, pair_entries = 0;  // stored edge lists (n2v_pairs.hip)
  uint64_t hub_count = 0;                     // hub membership sets (dev.hub_sets)
};

extern thread_local std::string t_err;
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int q16_of(double x, uint32_t* out);
int current_devinfo(DevInfo* out);
GraphRec* find_graph(n2v_graph g);
LaunchCfg choose_cfg(const GraphRec& gr, const DevInfo& di);
// N2V_OK if every field of t is a valid setting (else INVALID_ARG with a message).
int check_tuning(const n2v_tuning_t& t);
// Apply a tuning to a batched / served launch shape: `fixed` when given (a
// server's own), else the n2v_set_tuning override, if any.
void apply_tuning_override(LaunchCfg* c, const DevInfo& di, const n2v_tuning_t* fixed = nullptr);
int prepare_request(const GraphRec& gr, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                    uint32_t walks_per_start, uint32_t walk_len, double p, double q, uint64_t seed,
                    uint64_t walk_id_base, int32_t* d_walks, int32_t* d_lens, uint32_t k_approx,
                    WalkArgs* a, Path* path);

}  // namespace n2v
