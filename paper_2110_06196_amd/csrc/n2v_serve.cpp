// Batched and served forms of the walk generator.
#include <hip/hip_runtime.h>

#include "n2v_runtime.hpp"

using namespace n2v;

extern "C" {

int n2v_walks_batched(const n2v_request_desc_t* reqs, uint32_t n_reqs, void* hip_stream) {
  if (n_reqs > 0 && !reqs) return fail(N2V_ERR_INVALID_ARG, "reqs is NULL");
  DevInfo di;
  int rc = current_devinfo(&di);
  if (rc != N2V_OK) return rc;
  for (uint32_t i = 0; i < n_reqs; ++i) {
    const n2v_request_desc_t& r = reqs[i];
    GraphRec* gr = find_graph(r.graph);
    if (!gr) return fail(N2V_ERR_BAD_HANDLE, "request %u: unknown graph", i);
    WalkArgs a;
    Path path;
    rc = prepare_request(*gr, r.kind, r.d_starts, r.n_starts, r.walks_per_start, r.walk_len, r.p,
                         r.q, r.seed, r.walk_id_base, r.d_walks, r.d_lens, &a, &path);
    if (rc != N2V_OK) return rc;
    hipError_t e = launch_walks(a, path, choose_cfg(*gr, di), di, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
  }
  return N2V_OK;
}

int n2v_server_create(uint64_t, uint32_t, void*, n2v_server* out) {
  if (out) *out = 0;
  return fail(N2V_ERR_INVALID_ARG, "server not available");
}
int n2v_server_add_graph(n2v_server, n2v_graph) { return fail(N2V_ERR_BAD_HANDLE, "no server"); }
int n2v_request_submit(n2v_server, const n2v_request_desc_t*, uint64_t, n2v_request* out) {
  if (out) *out = 0;
  return fail(N2V_ERR_BAD_HANDLE, "no server");
}
int n2v_request_poll(n2v_server, n2v_request, n2v_result_t*) { return fail(N2V_ERR_BAD_HANDLE, "no server"); }
int n2v_request_release(n2v_server, n2v_request) { return fail(N2V_ERR_BAD_HANDLE, "no server"); }
int n2v_server_destroy(n2v_server) { return fail(N2V_ERR_BAD_HANDLE, "no server"); }

}  // extern "C"
