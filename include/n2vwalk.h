/*
 * n2vwalk: exact first-order (DeepWalk) and second-order (node2vec) random-walk
 * generation over a sorted CSR graph on AMD Instinct MI355X (gfx950).
 *
 * The operation is the one defined in the paper's Methods, "First and
 * second-order RW-based embedding methods":
 *   - a first-order step from v picks x in N(v) with probability w_vx / sum_x w_vx;
 *   - a node2vec step from v, arrived at from t, picks x with probability
 *     proportional to pi_vx = alpha_pq(t,x) * w_vx, where alpha is 1/p if x == t,
 *     1 if x is a neighbour of t, and 1/q otherwise (Eq. 1, and its split into
 *     the return and in-out biases, Eq. 2-3);
 *   - sampling is done on the fly (section "Efficient sampling for Node2Vec
 *     RWs"): biased weights, their cumulative sum, a uniform value in
 *     [0, total), and the first index whose cumulative sum exceeds it.
 *
 * Exact integer arithmetic: weights are uint32, 1/p and 1/q are Q16 fixed
 * point (P16 = round-half-even(65536/p), Q16 likewise, C16 = 65536), running
 * sums are uint64, and the uniform value is floor(r64 * total / 2^64) with
 * r64 = out0 | out1 << 32 of Philox4x32-10 (Salmon et al., SC'11) under key
 * (seed lo, seed hi) and counter (step, walk id lo, walk id hi, 0).  The first
 * step of a node2vec walk, which has no previous node, is a first-order step.
 * Every walk is therefore a pure function of (graph, kind, start, walk length,
 * P16, Q16, seed, walk id), independent of stream, tuning and batch company.
 *
 * Conventions for every function:
 *   - returns an int32 status (N2V_OK or a negative N2V_ERR_*); never throws;
 *     n2v_last_error() gives a message for the calling thread's last failure;
 *   - "device pointer" means memory the GPU can read/write (hipMalloc, torch
 *     CUDA tensors); "host pointer" means ordinary CPU memory;
 *   - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *
 * Walk output layout: walks is int32[n_walks][walk_len] (1 <= walk_len <= 2^30),
 * row-major, 4-byte aligned (rows are stored in whole 64-byte lines where the
 * address allows), with
 * n_walks = walks_per_start * n_starts and row w = rep * n_starts + i using
 * start starts[i] and walk id walk_id_base + w.  Slot 0 holds the start; a walk
 * that reaches a node with no out-edge (or whose candidates all have weight
 * zero) stops there; unused slots hold -1.  lens[w] = number of slots written
 * (walk_len for a full walk, 0 for a start outside [0, n_nodes)).
 */
#ifndef N2VWALK_H
#define N2VWALK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  N2V_OK = 0,
  N2V_PENDING = 1,          /* n2v_request_poll: not finished yet (not an error) */
  N2V_ERR_INVALID_ARG = -1, /* NULL pointer, zero size where one is needed, walk_len == 0 or > 2^30,
                               walks_per_start == 0, p or q not finite and > 0, or their
                               Q16 value outside [1, 2^32-1] */
  N2V_ERR_UNSORTED = -2,    /* offsets[0] != 0, offsets not monotone, offsets[n] != n_entries,
                               a row not strictly increasing, or a destination outside [0,n) */
  N2V_ERR_OVERFLOW = -3,    /* max row weight sum * max(P16, 65536, Q16) >= 2^64 */
  N2V_ERR_NOMEM = -4,       /* device or host allocation failed */
  N2V_ERR_HIP = -5,         /* a HIP runtime call failed (message in n2v_last_error) */
  N2V_ERR_BAD_HANDLE = -6,  /* unknown or released handle */
  N2V_ERR_REJECTED = -7     /* request can never fit the server's memory budget */
};

enum { N2V_FIRST_ORDER = 0, N2V_NODE2VEC = 1 };

typedef uint64_t n2v_graph;   /* opaque, 0 = invalid */
typedef uint64_t n2v_server;  /* opaque, 0 = invalid */
typedef uint64_t n2v_request; /* opaque, 0 = invalid */

typedef struct {
  uint64_t n_nodes;
  uint64_t n_entries;
  uint64_t max_degree;
  uint64_t max_row_wsum;   /* max over rows of the sum of weights (degree if unweighted) */
  uint64_t sum_deg_sq;     /* sum over nodes of degree^2 (stationary mean degree = this / n_entries) */
  uint32_t weighted;       /* 1 if weights were given */
  uint32_t prefix_bytes;   /* 0 (unweighted), 4 or 8: width of the per-row weight prefix */
  uint64_t device_bytes;   /* library-owned device memory held by this graph */
  uint32_t storage;        /* N2V_STORAGE_CSR or N2V_STORAGE_EF */
  uint32_t ef_quantum;     /* quantum of the Elias-Fano indexes (0 for CSR) */
  uint64_t pair_lists;     /* edges whose common-neighbour list is stored (see n2v_graph_upload) */
  uint64_t pair_entries;   /* entries of those lists (16 bytes each) */
  uint64_t hub_sets;       /* rows that keep a membership set (see n2v_graph_upload) */
  uint64_t hub_min_degree; /* degree from which rows may keep one (0 when none is kept) */
} n2v_graph_info_t;

enum { N2V_STORAGE_CSR = 0, N2V_STORAGE_EF = 1 };

/* Launch tuning.  Zero fields mean "automatic".  Tuning never changes a walk:
 * every setting produces bit-identical output.  Automatic node2vec launches
 * use 4 lanes per walker on graphs whose edges all keep a stored
 * common-neighbour list when the launch has at least 96 walks per compute
 * unit, and 16 to 64 lanes (by the graph's degree spread) otherwise; batched
 * and served launches take 4, 16, 32 or 64 (8 runs as 16). */
typedef struct {
  uint32_t lanes_per_walker; /* node2vec (1/q != 1) path: 4, 8, 16, 32 or 64 lanes per walker */
  uint32_t lds_tile;         /* entries of the previous node's row staged in LDS per walker */
  uint32_t list_cap;         /* entries of the common-neighbour list kept in LDS per walker */
  uint32_t route;            /* N2V_ROUTE_*: how a node2vec step with 1/q != 1 classifies */
  uint32_t flags;            /* N2V_TUNE_* bits */
} n2v_tuning_t;

enum {
  N2V_ROUTE_AUTO = 0,     /* per step, the cheapest of PROBE, STREAM and MERGE by a latency estimate */
  N2V_ROUTE_TWO_PASS = 1, /* stream the biased weights of N(v) twice (block sums, then one block) */
  N2V_ROUTE_PROBE = 2,    /* bisect every node of N(t) into N(v) to list the common neighbours */
  N2V_ROUTE_STREAM = 3,   /* stream N(v) and test each candidate against N(t) */
  N2V_ROUTE_MERGE = 4,    /* merge the two sorted rows, a window of N(t) at a time in LDS */
  N2V_ROUTE_HUB_SETS = 5  /* on 64-lane groups: look candidates up in the membership set of v (keys
                             from N(t)) or of t (keys from N(v)) whenever one of them has a set;
                             other steps as AUTO.  AUTO weighs the sets by the same estimate */
};

enum { N2V_UPLOAD_NO_PAIR_LISTS = 1u, N2V_UPLOAD_NO_HUB_SETS = 2u };
/* Upload flag: rows of degree >= 2^k (k in [1, 31]) may keep a membership
 * set; without it the threshold is automatic (4096). */
#define N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(k) ((uint32_t)((k) & 31u) << 8)

enum {
  N2V_TUNE_GENERIC_ONLY = 1u  /* route every step through the G-lanes-per-walker kernel
                                 (no first-order / 1/q == 1 lane-per-walker specialisations) */
};

/* ---------------------------------------------------------------------------
 * Graph residency (once per graph).
 *
 * d_offsets: device uint64[n_nodes+1]; d_dst: device int32[n_entries]; each row
 * d_dst[offsets[v] .. offsets[v+1]) strictly increasing (the sorted neighbour
 * set of the paper's CSR store, Methods "Succinct data structures").
 * d_weights: device uint32[n_entries], or NULL for an unweighted graph
 * (every weight 1).  flags: 0, or any of N2V_UPLOAD_NO_PAIR_LISTS,
 * N2V_UPLOAD_NO_HUB_SETS and N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(k).
 * The three arrays are BORROWED: the caller keeps them alive and unchanged
 * until n2v_graph_release.  Derived arrays (per-row inclusive weight prefix,
 * statistics) are owned by the library.
 * For weighted graphs with row sums below 2^32 and at most 2^28 entries the
 * upload also stores, for every edge t -> v, the list a second-order step
 * from v after t builds: the positions in N(v) of the common neighbours
 * (x in N(t), x != t) with the prefix of their weights, and the position of
 * t in N(v).  All lists are kept when they fit min(32 GiB, 256 bytes per
 * graph entry), else the ones with the most saved work per stored entry;
 * n2v_graph_info reports them.  They change no walk, only how fast its steps
 * run, and cost upload time (about 0.1 s per 2e7 entries of a power-law
 * graph, all on the device) and temporary device memory to lay them out
 * (about 44 bytes per graph entry, 77 when not every list fits).  A graph
 * whose lists do not fit the device memory left is registered without them.
 * N2V_UPLOAD_NO_PAIR_LISTS skips them.
 * Graphs where some edge keeps no stored list also keep, for their longest
 * rows (degree >= 4096, or >= 2^k with N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(k);
 * longest first, within min(16 GiB, a quarter of the free device memory)),
 * a membership set: one bit per node id plus a running member count every
 * 480 ids (n / 480 * 64 bytes per row, e.g. 2.7 MB at 2e7 nodes), so that a
 * second-order step between such a row and another classifies a candidate
 * with one line read instead of a bisection (Methods, "Succinct data
 * structures": rank over a bitmap).  They change no walk.
 * N2V_UPLOAD_NO_HUB_SETS skips them.
 * Synchronous: validates on the device, builds the derived arrays on
 * hip_stream and waits for it.  Errors: INVALID_ARG, UNSORTED, NOMEM, HIP.
 * ------------------------------------------------------------------------- */
int n2v_graph_upload(const uint64_t* d_offsets, uint64_t n_nodes, const int32_t* d_dst,
                     uint64_t n_entries, const uint32_t* d_weights, uint32_t flags,
                     void* hip_stream, n2v_graph* out);
int n2v_graph_info(n2v_graph g, n2v_graph_info_t* out);
/* Frees the library-owned arrays.  The caller must make sure no walk on g is
 * still running (synchronise the streams first). */
int n2v_graph_release(n2v_graph g);

/* ---------------------------------------------------------------------------
 * Elias-Fano graph store (Methods, "Edge Encoding", "Operations on
 * Elias-Fano", "Efficient implementation of Elias-Fano").
 *
 * n2v_graph_upload_ef takes the same CSR arrays as n2v_graph_upload, builds on
 * the device the Elias-Fano list of the edge codes phi_k(a, b) = a 2^k + b
 * (k = ceil(log2 n_nodes), u = n_nodes 2^k): l = floor(log2(u / n_entries))
 * low bits per code in L (field i = bits [i l, (i + 1) l) of little-endian
 * 64-bit words), the high parts as inverted unary gaps in the bit vector H
 * (the one of code i is bit (code_i >> l) + i; ((u - 1) >> l) + 1 zeros), and
 * quantum indexes S1[j] / S0[j] = position of one / zero number j * quantum.
 * quantum: a power of two in [8, 65536], 0 for 256.  For weighted graphs the
 * per-row weight prefix is kept (weights are its differences).  The handle
 * owns everything: the CSR arrays are not referenced after the call returns
 * (synchronous), so the caller may free them.
 * Walks (n2v_walks_first_order, n2v_walks_node2vec) and negatives on such a
 * handle are the same as on the CSR handle of the same graph, bit for bit;
 * approximated walks, batches and servers need a CSR handle (INVALID_ARG).
 * Errors: as n2v_graph_upload; INVALID_ARG for n_nodes == 0 or a bad quantum.
 * ------------------------------------------------------------------------- */
int n2v_graph_upload_ef(const uint64_t* d_offsets, uint64_t n_nodes, const int32_t* d_dst,
                        uint64_t n_entries, const uint32_t* d_weights, uint32_t quantum,
                        void* hip_stream, n2v_graph* out);

typedef struct {
  uint32_t k, l, quantum, pad;
  uint64_t u, n_codes, n_zeros, h_bits;
  uint64_t h_words, l_words, s1_len, s0_len; /* lengths in uint64 of H, L, S1, S0 */
  const uint64_t* d_H;                       /* device arrays, owned by the graph */
  const uint64_t* d_L;
  const uint64_t* d_S1;
  const uint64_t* d_S0;
} n2v_ef_info_t;
/* INVALID_ARG unless g is an Elias-Fano handle. */
int n2v_ef_info(n2v_graph g, n2v_ef_info_t* out);
/* d_out[i] = select(d_idx[i]) (the code of rank d_idx[i]; UINT64_MAX when
 * d_idx[i] >= n_codes) and rank(d_x[i]) (codes strictly below d_x[i]); device
 * uint64 arrays of length count, enqueued on hip_stream. */
int n2v_ef_select(n2v_graph g, const uint64_t* d_idx, uint64_t count, uint64_t* d_out, void* hip_stream);
int n2v_ef_rank(n2v_graph g, const uint64_t* d_x, uint64_t count, uint64_t* d_out, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Plain walk generation (one launch per call).
 *
 * d_starts: device int32[n_starts]; d_walks: device int32[walks_per_start *
 * n_starts][walk_len]; d_lens: device int32[walks_per_start * n_starts] or NULL.
 * All caller-owned.  Arguments are validated synchronously, then the work is
 * enqueued on hip_stream; the outputs are valid once the stream has been
 * synchronised.  A start outside [0, n_nodes) yields a row of -1 with length 0
 * (not an error).  n_starts == 0 is a no-op.  Reentrant across streams and
 * threads.  The kernels hand walks out from a device counter of hip_stream:
 * the first call on a stream takes 8 bytes for it from a library-owned device
 * slab (hipMalloc of 4 KB per 512 streams, kept until the process ends); a
 * stream under graph capture gets no counter and the walks are split in fixed
 * shares instead (same output).
 * Errors: INVALID_ARG, BAD_HANDLE, OVERFLOW (node2vec), HIP.
 * ------------------------------------------------------------------------- */
int n2v_walks_first_order(n2v_graph g, const int32_t* d_starts, uint64_t n_starts,
                          uint32_t walks_per_start, uint32_t walk_len, uint64_t seed,
                          uint64_t walk_id_base, int32_t* d_walks, int32_t* d_lens,
                          void* hip_stream);
int n2v_walks_node2vec(n2v_graph g, const int32_t* d_starts, uint64_t n_starts,
                       uint32_t walks_per_start, uint32_t walk_len, double p, double q,
                       uint64_t seed, uint64_t walk_id_base, int32_t* d_walks,
                       int32_t* d_lens, void* hip_stream);

/* Approximated walks (Methods, "Approximated RWs"): a step from a node of
 * degree d > k considers only k of its neighbours, chosen by Sorted Unique
 * Sub-Sampling: [0, d) is cut into k buckets of length floor(d / k), the last
 * one also taking the remainder, and one position is drawn uniformly in each
 * bucket (bucket i uses the 64-bit word pair (2 (i mod 2), 2 (i mod 2) + 1) of
 * Philox4x32-10 with counter (step, walk id lo, walk id hi, 1 + floor(i / 2))).
 * The step then samples among the k candidates exactly as an exact step does
 * among all of N(v) (weights, search biases, cumulative sum, same draw).
 * Steps from nodes of degree <= k are exact, so k >= max degree reproduces
 * n2v_walks_first_order / n2v_walks_node2vec.  kind: N2V_FIRST_ORDER (p, q
 * ignored) or N2V_NODE2VEC.  k == 0 is INVALID_ARG; otherwise as the plain calls. */
int n2v_walks_approximated(n2v_graph g, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                           uint32_t walks_per_start, uint32_t walk_len, double p, double q,
                           uint32_t k, uint64_t seed, uint64_t walk_id_base, int32_t* d_walks,
                           int32_t* d_lens, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Training corpora from walks (the walks feed SkipGram / CBOW / GloVe models
 * trained on sliding windows, Methods "First and second-order RW-based
 * embedding methods"; Walklets uses skip distances).
 *
 * n2v_walk_contexts: d_walks int32[n_walks][walk_len] (as produced above, -1
 * padded); d_contexts int32[n_walks][walk_len][2 window] receives, for every
 * position i holding a node, the nodes at positions i + o * stride for
 * o = -window .. -1, 1 .. window (slot c <-> o = c - window for c < window,
 * c - window + 1 otherwise), or -1 outside the walk; positions without a node
 * get -1 everywhere.  stride 1: SkipGram / CBOW windows; window 1 and stride k:
 * the Walklets pairs of scale k.  Enqueued on hip_stream.
 *
 * n2v_negative_samples: d_negatives int32[n_walks][walk_len][n_neg]; for every
 * position i of walk row r holding a node, n_neg nodes drawn with probability
 * proportional to their out-degree ("scale-free negative sampling"): node v
 * with offsets[v] <= T < offsets[v+1], T = floor(r64 * n_entries / 2^64), r64
 * the word pair (2 (j mod 2), 2 (j mod 2) + 1) of Philox4x32-10 under key seed
 * and counter (i, wid lo, wid hi, 2^31 + floor(j / 2)) with wid =
 * walk_id_base + r.  Other slots get -1.  Enqueued on hip_stream.
 * ------------------------------------------------------------------------- */
int n2v_walk_contexts(const int32_t* d_walks, uint64_t n_walks, uint32_t walk_len, uint32_t window,
                      uint32_t stride, int32_t* d_contexts, void* hip_stream);
/* Fused walk -> contexts: the context slots n2v_walk_contexts would write
 * for the walks n2v_walks_first_order (kind N2V_FIRST_ORDER; p, q ignored) or
 * n2v_walks_node2vec (kind N2V_NODE2VEC) would produce with the same
 * arguments, written while the walks are taken, without the walk array: each
 * walker keeps its last 2 H + 1 positions (H = min(window * stride,
 * walk_len - 1)) in LDS and emits the slots of position s - H once position
 * s is drawn (and the rest when the walk ends).  d_contexts:
 * int32[walks_per_start * n_starts][walk_len][2 window]; d_lens as in the
 * walk calls (may be NULL).  window, stride >= 1 and H <= 1023
 * (INVALID_ARG otherwise: materialise the walks and call
 * n2v_walk_contexts).  Enqueued on hip_stream. */
int n2v_walks_contexts(n2v_graph g, uint32_t kind, const int32_t* d_starts, uint64_t n_starts,
                       uint32_t walks_per_start, uint32_t walk_len, double p, double q, uint64_t seed,
                       uint64_t walk_id_base, uint32_t window, uint32_t stride, int32_t* d_contexts,
                       int32_t* d_lens, void* hip_stream);
int n2v_negative_samples(n2v_graph g, const int32_t* d_walks, uint64_t n_walks, uint32_t walk_len,
                         uint32_t n_neg, uint64_t seed, uint64_t walk_id_base, int32_t* d_negatives,
                         void* hip_stream);

/* Process-wide tuning override (NULL restores automatic tuning).  Used to
 * show that every tuning point yields identical walks. */
int n2v_set_tuning(const n2v_tuning_t* tuning);

/* ---------------------------------------------------------------------------
 * Batched generation: many requests (different graphs, kinds, lengths, p, q,
 * seeds) in ONE persistent launch fed by a device work queue of walk chunks,
 * longest estimated work first.  Each request's output is bit-identical to the
 * plain call with the same arguments.  reqs is a host array; the pointers
 * inside are device pointers as in the plain calls.  Enqueued on hip_stream;
 * the host array may be reused as soon as the call returns.
 * ------------------------------------------------------------------------- */
typedef struct {
  n2v_graph graph;
  uint32_t kind;            /* N2V_FIRST_ORDER or N2V_NODE2VEC */
  uint32_t walks_per_start;
  uint32_t walk_len;
  uint32_t k_approx;        /* 0: exact walks; k: approximated walks (see n2v_walks_approximated) */
  double p, q;              /* ignored for first order */
  uint64_t seed;
  uint64_t walk_id_base;
  const int32_t* d_starts;
  uint64_t n_starts;
  int32_t* d_walks;
  int32_t* d_lens;          /* may be NULL */
} n2v_request_desc_t;

int n2v_walks_batched(const n2v_request_desc_t* reqs, uint32_t n_reqs, void* hip_stream);

/* Allocation-free form of n2v_walks_batched, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and the same walks, bit for bit.  The request table, the chunk
 * queue and its counter live in a fixed 8 MiB device array inside the library
 * (one per GPU, held until the process ends) instead of a per-call allocation:
 * at most 4096 requests (more: N2V_ERR_INVALID_ARG, before any device work),
 * and a batch whose chunk queue would not fit is cut into fewer, larger chunks
 * (the walks do not change).  The call copies the tables on hip_stream and
 * waits for that copy (so also for the stream's earlier work); the walk kernel
 * itself runs asynchronously.  Every call on one GPU shares the array: calls
 * whose kernels overlap in time (on different streams or host threads) race
 * and must be serialised by the caller; calls on one stream are ordered. */
int n2v_walks_batched_noalloc(const n2v_request_desc_t* reqs, uint32_t n_reqs, void* hip_stream);

/* Reusable batch plan: the request and chunk tables are uploaded once, the
 * launch shape (lanes per walker, LDS tile, list capacity) is chosen by timing
 * candidate shapes on a sample of the chunks (N2V_BATCH_AUTOTUNE; any shape
 * yields the same walks, so the sample's outputs are simply rewritten), and
 * the counter reset plus the persistent kernel are captured once into a
 * hipGraph that n2v_batch_launch replays on hip_stream.  The caller keeps the
 * graphs and the device buffers named in reqs alive until n2v_batch_destroy.
 * n2v_batch_create is synchronous (it may launch the autotuning samples on an
 * internal stream). */
typedef uint64_t n2v_batch; /* opaque, 0 = invalid */
enum { N2V_BATCH_AUTOTUNE = 1u };
typedef struct {
  uint32_t n_requests;
  uint32_t n_chunks;
  uint32_t lanes_per_walker; /* chosen launch shape */
  uint32_t lds_tile;
  uint32_t list_cap;
  uint32_t reserved;
  uint64_t n_walks;
  double est_cost;           /* estimated work units (walk steps x per-step cost factor) */
} n2v_batch_info_t;
int n2v_batch_create(const n2v_request_desc_t* reqs, uint32_t n_reqs, uint32_t flags, n2v_batch* out);
int n2v_batch_launch(n2v_batch b, void* hip_stream);
int n2v_batch_info(n2v_batch b, n2v_batch_info_t* out);
int n2v_batch_destroy(n2v_batch b);

/* ---------------------------------------------------------------------------
 * Serving: resident graphs, requests admitted by memory footprint, continuous
 * batching (requests that arrive while others run are started as slots and
 * memory free up; their walks overlap on the device).  Thread-safe.
 *
 * n2v_server_create: hbm_budget_bytes caps the device memory the server holds
 * for request inputs and results; max_slots caps requests in flight.
 * n2v_server_add_graph: makes g servable (g stays owned by the caller and must
 * outlive the server).
 * n2v_request_submit: desc as above but d_starts is a HOST pointer (copied at
 * submit) and d_walks / d_lens are ignored (the server allocates the results).
 * arrival_ns is the caller's timestamp (CLOCK_MONOTONIC; 0 = now) for latency
 * accounting: an argument of its own because the descriptor is shared with the
 * batched calls, where an arrival time means nothing.  Errors: REJECTED if the
 * request alone exceeds the budget.
 * n2v_request_poll: N2V_PENDING until done, then N2V_OK and *out filled;
 * results stay valid until n2v_request_release.
 * ------------------------------------------------------------------------- */
typedef struct {
  const int32_t* d_walks;   /* device int32[n_walks][walk_len], server-owned */
  const int32_t* d_lens;    /* device int32[n_walks], server-owned */
  uint64_t n_walks;
  uint64_t steps;           /* sum over walks of (len - 1), transitions taken */
  uint64_t t_arrival_ns, t_admit_ns, t_start_ns, t_done_ns; /* CLOCK_MONOTONIC */
} n2v_result_t;

/* n2v_server_create: tuning fixes the launch shape of the server's queue
 * kernel (lanes per walker, LDS tile, list capacity, route; zero fields keep
 * the automatic value); NULL = automatic (64 lanes per walker, or the
 * process-wide n2v_set_tuning override when one is set).  The shape never
 * changes a walk.  Work runs on an internal stream in bounded quanta: each
 * quantum is one launch of the persistent queue kernel over chunks of every
 * admitted request (about eight chunks per resident walker group), and newly
 * admitted requests join the next quantum.  No kernel ever waits on the host.
 * Errors: INVALID_ARG (budget 0, max_slots outside [1, 65536], an invalid
 * tuning field), HIP. */
int n2v_server_create(uint64_t hbm_budget_bytes, uint32_t max_slots, const n2v_tuning_t* tuning,
                      n2v_server* out);
int n2v_server_add_graph(n2v_server s, n2v_graph g);
int n2v_request_submit(n2v_server s, const n2v_request_desc_t* desc, uint64_t arrival_ns,
                       n2v_request* out);
int n2v_request_poll(n2v_server s, n2v_request r, n2v_result_t* out);
int n2v_request_release(n2v_server s, n2v_request r);
int n2v_server_destroy(n2v_server s);

/* Thread-local message describing the calling thread's last error ("" if none). */
const char* n2v_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* N2VWALK_H */
