/*
 * Plain single-threaded CPU oracle for exact first-order (DeepWalk) and
 * second-order (node2vec) random-walk generation over a sorted CSR graph.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * definition the GPU path is checked against.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no source with the GPU library.
 *
 * What it computes follows the paper's Methods, "First and second-order
 * RW-based embedding methods":
 *   - transition weight pi_vx = alpha_pq(t,x) * w_vx          (Eq. 1)
 *   - alpha = 1/p if x == t, 1 if x in N(t), 1/q otherwise   (Eq. 1-3 and the
 *     set-difference / return-bias reformulations that follow them)
 *   - sampling on the fly: biased weights, cumulative sum, a uniform value in
 *     [0, total), first index whose cumulative sum exceeds it   ("Efficient
 *     sampling for Node2Vec RWs", steps 1-4)
 * with 1/p and 1/q represented as Q16 fixed point so that the whole walk is
 * exact integer arithmetic, and the uniform value taken from Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",
 * SC'11) keyed by (seed) with counter (step, walk id).
 *
 * Parity with the paper: pinned by closed-form transition probabilities,
 * exact rational tables, brute-force walk enumeration and chi-square tests
 * (tests/test_oracle_*.py).  Which particular walk a seed produces is fixed by
 * this definition, not by the paper.
 */
#ifndef N2V_ORACLE_H
#define N2V_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  N2VO_OK = 0,
  N2VO_ERR_INVALID_ARG = -1,
  N2VO_ERR_UNSORTED = -2,
  N2VO_ERR_OVERFLOW = -3
};

enum { N2VO_FIRST_ORDER = 0, N2VO_NODE2VEC = 1 };

/* 65536/x rounded to nearest, ties to even, in IEEE double; the result must
 * lie in [1, 2^32-1].  Returns N2VO_OK or N2VO_ERR_INVALID_ARG. */
int n2vo_q16(double x, uint32_t* out);

/* Philox4x32 with 10 rounds: ctr[4], key[2] -> out[4]. */
void n2vo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The 64-bit uniform draw of step s of walk `wid`:
 * key = (seed lo, seed hi), counter = (s, wid lo, wid hi, 0),
 * r64 = out0 | out1 << 32. */
uint64_t n2vo_draw64(uint64_t seed, uint32_t step, uint64_t wid);

/* floor(r64 * total / 2^64): a uniform value in [0, total). */
uint64_t n2vo_scale(uint64_t r64, uint64_t total);

/* CSR validity: O[0]==0, O non-decreasing, O[n]==m, every row strictly
 * increasing, every destination in [0,n).  Returns N2VO_OK or
 * N2VO_ERR_UNSORTED. */
int n2vo_validate(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m);

/* Max degree and max row weight sum (weights NULL = all ones). */
void n2vo_stats(const uint64_t* O, int64_t n, const uint32_t* W,
                uint64_t* max_deg, uint64_t* max_row_wsum);

/* Biased weights of every candidate x in N(v) for one step from v whose
 * previous node is t (t < 0: no previous node, first step).
 * second_order == 0 or t < 0: a = 1; else a = P16 if x == t, 65536 if
 * x in N(t), Q16 otherwise.  b[j] = w_j * a_j.  Returns d_v. */
int64_t n2vo_step_weights(const uint64_t* O, const int32_t* D, const uint32_t* W,
                          int32_t t, int32_t v, int second_order,
                          uint32_t P16, uint32_t Q16, uint64_t* b);

/* First j with b[0]+...+b[j] > T (plain linear scan); d if none. */
int64_t n2vo_select(const uint64_t* b, int64_t d, uint64_t T);

/* Generate the walks whose row indices are listed in widx[0..nw).
 * Row w uses start S[w mod ns] and walk id walk_id_base + w.
 * Y is [nw][L] (row k belongs to walk widx[k]); lens is [nw] or NULL.
 * kind: N2VO_FIRST_ORDER or N2VO_NODE2VEC (p, q ignored for first order).
 * Returns N2VO_OK, N2VO_ERR_INVALID_ARG or N2VO_ERR_OVERFLOW. */
int n2vo_walks_subset(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
                      const uint32_t* W, const int32_t* S, int64_t ns,
                      uint32_t reps, uint32_t L, int kind, double p, double q,
                      uint64_t seed, uint64_t walk_id_base,
                      const int64_t* widx, int64_t nw, int32_t* Y, int32_t* lens);

/* Sorted Unique Sub-Sampling (Methods, "Approximated RWs"): k sorted, unique
 * positions in [0, d) for d > k.  The range is cut into k buckets of length
 * floor(d / k), the last one also taking the remainder; bucket i gets the
 * position start_i + floor(r64_i * len_i / 2^64), where r64_i is the 64-bit
 * word pair (2 (i mod 2), 2 (i mod 2) + 1) of Philox4x32-10 under key seed and
 * counter (step, wid lo, wid hi, 1 + floor(i / 2)). */
void n2vo_suss(uint64_t seed, uint32_t step, uint64_t wid, uint32_t d, uint32_t k, uint32_t* pos);

/* n2vo_walks_subset with approximated steps: a step from a node of degree
 * d > k_approx considers only the SUSS sub-sample of k_approx neighbours
 * (weights and search biases as in the exact step, normalised over the
 * sub-sample); k_approx == 0 or d <= k_approx gives the exact step. */
int n2vo_walks_approx_subset(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
                             const uint32_t* W, const int32_t* S, int64_t ns,
                             uint32_t reps, uint32_t L, int kind, double p, double q,
                             uint32_t k_approx, uint64_t seed, uint64_t walk_id_base,
                             const int64_t* widx, int64_t nw, int32_t* Y, int32_t* lens);

/* Training contexts of every walk position (Methods, "First and second-order
 * RW-based embedding methods": window-based SkipGram / CBOW corpora; with a
 * stride k the Walklets corpus of scale k).  For walk row r and centre i
 * (Y[r][i] >= 0), slot c in [0, 2 window) holds Y[r][i + o * stride] with
 * o = c - window for c < window and o = c - window + 1 otherwise, or -1 when
 * that position is outside the walk or unused (-1).  C is [nw][L][2 window]. */
void n2vo_contexts(const int32_t* Y, int64_t nw, uint32_t L, uint32_t window, uint32_t stride, int32_t* C);

/* Scale-free negatives: for walk row r (walk id walk_id_base + r) and centre i
 * with Y[r][i] >= 0, N[r][i][j] (j < n_neg) is the node v with
 * O[v] <= T < O[v+1], T = floor(r64 * m / 2^64), i.e. a node drawn with
 * probability proportional to its out-degree; r64 is the word pair
 * (2 (j mod 2), 2 (j mod 2) + 1) of Philox4x32-10 under key seed and counter
 * (i, wid lo, wid hi, 2^31 + floor(j / 2)).  Other slots hold -1. */
void n2vo_negatives(const uint64_t* O, int64_t n, const int32_t* Y, int64_t nw, uint32_t L, uint32_t n_neg,
                    uint64_t seed, uint64_t walk_id_base, int32_t* N);

/* ------------------------------------------------------------------------
 * Elias-Fano (Methods, "Memory Complexity", "Edge Encoding", "Operations on
 * Elias-Fano", "Efficient implementation of Elias-Fano").
 *
 * A non-decreasing list of m integers below u is stored with
 * l = floor(log2(u / m)) low bits each (l = 0 when m == 0 or u < 2m): the
 * low parts go to L, field i occupying bits [i l, (i + 1) l) of a stream of
 * 64-bit words, least significant bit first; the high parts h_i = y_i >> l go
 * to the bit vector H as the inverted unary codes of their gaps, so the one of
 * element i is bit h_i + i (bit p = bit p mod 64 of word p / 64), and H holds
 * n_zeros = ((u - 1) >> l) + 1 zeros, m + n_zeros bits in all.  The quantum
 * indexes hold S1[j] = position of one number j q and S0[j] = position of
 * zero number j q (numbers from 0).
 *
 * A graph on n nodes is the list of its edge codes phi_k(a, b) = a 2^k + b,
 * k = ceil(log2 n), in CSR order, with u = n 2^k.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t k;        /* bits of a node id in an edge code (graphs only) */
  uint32_t l;        /* low bits per element */
  uint64_t u;        /* every element is below u */
  uint64_t m;        /* elements */
  uint64_t n_zeros;  /* zeros of H */
  uint64_t h_bits;   /* m + n_zeros */
} n2vo_ef_shape;

/* Shape of an Elias-Fano list of m elements below u (u >= 1). */
void n2vo_ef_shape_of(uint64_t m, uint64_t u, n2vo_ef_shape* s);
/* Word counts of H, L, S1 and S0 for a shape and quantum q. */
void n2vo_ef_words(const n2vo_ef_shape* s, uint32_t q, uint64_t* h_words, uint64_t* l_words,
                   uint64_t* s1_len, uint64_t* s0_len);
/* Encode a non-decreasing list y[0..m) below u; the output arrays (sizes from
 * n2vo_ef_words) are overwritten.  Returns N2VO_OK or N2VO_ERR_INVALID_ARG. */
int n2vo_ef_encode(const uint64_t* y, uint64_t m, uint64_t u, uint32_t q, uint64_t* H, uint64_t* L,
                   uint64_t* S1, uint64_t* S0);
/* The edge list of a sorted CSR graph on n >= 1 nodes: shape (with k) and
 * encoding as above.  Returns N2VO_OK or N2VO_ERR_INVALID_ARG. */
int n2vo_ef_graph_shape(int64_t n, uint64_t m, n2vo_ef_shape* s);
int n2vo_ef_encode_graph(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m, uint32_t q, uint64_t* H,
                         uint64_t* L, uint64_t* S1, uint64_t* S0);
/* select(i): the i-th smallest element (i < m), by scanning H from bit 0. */
uint64_t n2vo_ef_select(const n2vo_ef_shape* s, const uint64_t* H, const uint64_t* L, uint64_t i);
/* rank(x): the number of elements strictly below x, by scanning H from bit 0. */
uint64_t n2vo_ef_rank(const n2vo_ef_shape* s, const uint64_t* H, const uint64_t* L, uint64_t x);

/* All reps*ns walks, row w = rep*ns + i. */
int n2vo_walks(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
               const uint32_t* W, const int32_t* S, int64_t ns,
               uint32_t reps, uint32_t L, int kind, double p, double q,
               uint64_t seed, uint64_t walk_id_base, int32_t* Y, int32_t* lens);

#ifdef __cplusplus
}
#endif
#endif
