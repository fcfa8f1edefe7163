/*
 * Plain single-threaded CPU oracle for exact DeepWalk / node2vec walks.
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library.  See n2v_oracle.h
 * for what each function computes and which passage of the paper it follows.
 */
#include "n2v_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>

/* ------------------------------------------------------------------------ */
/* Q16 fixed point for the search-bias constants 1/p and 1/q (Eq. 1).        */
/* ------------------------------------------------------------------------ */
int n2vo_q16(double x, uint32_t* out) {
  if (!(x > 0.0) || !isfinite(x)) return N2VO_ERR_INVALID_ARG;
  double r = nearbyint(65536.0 / x); /* default rounding: to nearest, ties to even */
  if (!(r >= 1.0) || !(r <= 4294967295.0)) return N2VO_ERR_INVALID_ARG;
  *out = (uint32_t)r;
  return N2VO_OK;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon et al. (SC'11): ten rounds of         */
/*   (x0,x1,x2,x3) -> (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1,   */
/*                     lo(M0*x0))                                            */
/* with the key bumped by the Weyl constants between rounds.                 */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void n2vo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint64_t n2vo_draw64(uint64_t seed, uint32_t step, uint64_t wid) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {step, (uint32_t)wid, (uint32_t)(wid >> 32), 0u};
  uint32_t out[4];
  n2vo_philox4x32_10(ctr, key, out);
  return (uint64_t)out[0] | ((uint64_t)out[1] << 32);
}

/* Step 3 of the on-the-fly sampler: a uniform value in [0, total). */
uint64_t n2vo_scale(uint64_t r64, uint64_t total) {
  unsigned __int128 prod = (unsigned __int128)r64 * (unsigned __int128)total;
  return (uint64_t)(prod >> 64);
}

/* ------------------------------------------------------------------------ */
/* CSR checks and statistics (Methods, "Succinct data structures": the     */
/* neighbours of a node form a sorted set).                                  */
/* ------------------------------------------------------------------------ */
int n2vo_validate(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m) {
  if (n < 0) return N2VO_ERR_INVALID_ARG;
  if (O[0] != 0) return N2VO_ERR_UNSORTED;
  if (O[n] != m) return N2VO_ERR_UNSORTED;
  for (int64_t v = 0; v < n; ++v) {
    if (O[v + 1] < O[v]) return N2VO_ERR_UNSORTED;
  }
  for (int64_t v = 0; v < n; ++v) {
    for (uint64_t e = O[v]; e < O[v + 1]; ++e) {
      if (D[e] < 0 || (int64_t)D[e] >= n) return N2VO_ERR_UNSORTED;
      if (e > O[v] && !(D[e - 1] < D[e])) return N2VO_ERR_UNSORTED;
    }
  }
  return N2VO_OK;
}

void n2vo_stats(const uint64_t* O, int64_t n, const uint32_t* W,
                uint64_t* max_deg, uint64_t* max_row_wsum) {
  uint64_t md = 0, ms = 0;
  for (int64_t v = 0; v < n; ++v) {
    uint64_t d = O[v + 1] - O[v];
    uint64_t s = 0;
    for (uint64_t e = O[v]; e < O[v + 1]; ++e) s += W ? (uint64_t)W[e] : 1u;
    if (d > md) md = d;
    if (s > ms) ms = s;
  }
  *max_deg = md;
  *max_row_wsum = ms;
}

/* Is x a member of N(t)?  Binary search over the sorted row of t. */
static int in_row(const uint64_t* O, const int32_t* D, int32_t t, int32_t x) {
  uint64_t lo = O[t], hi = O[t + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (D[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < O[t + 1] && D[lo] == x;
}

/* Step 1 of the sampler: un-normalised transition weights pi_vx = alpha * w_vx
 * (Eq. 1), alpha read with precedence return (x == t) > common neighbour
 * (x in N(t), distance 1) > far (distance 2). */
int64_t n2vo_step_weights(const uint64_t* O, const int32_t* D, const uint32_t* W,
                          int32_t t, int32_t v, int second_order,
                          uint32_t P16, uint32_t Q16, uint64_t* b) {
  int64_t d = (int64_t)(O[v + 1] - O[v]);
  for (int64_t j = 0; j < d; ++j) {
    int32_t x = D[O[v] + j];
    uint64_t w = W ? (uint64_t)W[O[v] + j] : 1u;
    uint64_t a;
    if (!second_order || t < 0) a = 1u;
    else if (x == t) a = P16;
    else if (in_row(O, D, t, x)) a = 65536u;
    else a = Q16;
    b[j] = w * a;
  }
  return d;
}

/* Step 4 of the sampler: first index whose cumulative sum exceeds T. */
int64_t n2vo_select(const uint64_t* b, int64_t d, uint64_t T) {
  uint64_t cum = 0;
  for (int64_t j = 0; j < d; ++j) {
    cum += b[j];
    if (cum > T) return j;
  }
  return d;
}

/* ------------------------------------------------------------------------ */
/* Sorted Unique Sub-Sampling (Methods, "Approximated RWs").                 */
/* ------------------------------------------------------------------------ */
void n2vo_suss(uint64_t seed, uint32_t step, uint64_t wid, uint32_t d, uint32_t k, uint32_t* pos) {
  uint32_t len = d / k;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (uint32_t i = 0; i < k; ++i) {
    uint32_t ctr[4] = {step, (uint32_t)wid, (uint32_t)(wid >> 32), 1u + i / 2u};
    uint32_t out[4];
    n2vo_philox4x32_10(ctr, key, out);
    uint64_t r = (uint64_t)out[2 * (i % 2)] | ((uint64_t)out[2 * (i % 2) + 1] << 32);
    uint32_t start = i * len;
    uint32_t blen = (i + 1 < k) ? len : d - start; /* the last bucket takes the remainder */
    pos[i] = start + (uint32_t)n2vo_scale(r, blen);
  }
}

/* Biased weights of the sub-sampled candidates N(v)[pos[i]], i < k. */
static void sub_weights(const uint64_t* O, const int32_t* D, const uint32_t* W, int32_t t, int32_t v,
                        int second_order, uint32_t P16, uint32_t Q16, const uint32_t* pos, uint32_t k,
                        uint64_t* b) {
  for (uint32_t i = 0; i < k; ++i) {
    uint64_t e = O[v] + pos[i];
    int32_t x = D[e];
    uint64_t w = W ? (uint64_t)W[e] : 1u;
    uint64_t a;
    if (!second_order || t < 0) a = 1u;
    else if (x == t) a = P16;
    else if (in_row(O, D, t, x)) a = 65536u;
    else a = Q16;
    b[i] = w * a;
  }
}

/* One walk, slots Y[0..L): start, then up to L-1 steps, then -1 padding.
 * k_approx > 0: steps from nodes of degree > k_approx use the SUSS sub-sample. */
static int32_t one_walk(const uint64_t* O, int64_t n, const int32_t* D, const uint32_t* W,
                        int32_t start, uint32_t L, int second_order,
                        uint32_t P16, uint32_t Q16, uint64_t seed, uint64_t wid, uint32_t k_approx,
                        uint32_t* pos, uint64_t* b, int32_t* Y) {
  for (uint32_t s = 0; s < L; ++s) Y[s] = -1;
  if (start < 0 || (int64_t)start >= n) return 0;
  Y[0] = start;
  int32_t len = 1;
  int32_t t = -1, v = start;
  for (uint32_t s = 1; s < L; ++s) {
    int64_t d = (int64_t)(O[v + 1] - O[v]);
    if (d == 0) break; /* dead end */
    int sub = k_approx > 0 && d > (int64_t)k_approx;
    int64_t nc;
    if (sub) {
      n2vo_suss(seed, s, wid, (uint32_t)d, k_approx, pos);
      sub_weights(O, D, W, t, v, second_order, P16, Q16, pos, k_approx, b);
      nc = k_approx;
    } else {
      nc = n2vo_step_weights(O, D, W, t, v, second_order, P16, Q16, b);
    }
    uint64_t total = 0;
    for (int64_t j = 0; j < nc; ++j) total += b[j];
    if (total == 0) break; /* every candidate has weight zero */
    uint64_t T = n2vo_scale(n2vo_draw64(seed, s, wid), total);
    int64_t j = n2vo_select(b, nc, T);
    int32_t x = D[O[v] + (sub ? (uint64_t)pos[j] : (uint64_t)j)];
    Y[s] = x;
    len = (int32_t)s + 1;
    t = v;
    v = x;
  }
  return len;
}

int n2vo_walks_approx_subset(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
                             const uint32_t* W, const int32_t* S, int64_t ns,
                             uint32_t reps, uint32_t L, int kind, double p, double q,
                             uint32_t k_approx, uint64_t seed, uint64_t walk_id_base,
                             const int64_t* widx, int64_t nw, int32_t* Y, int32_t* lens) {
  if (n < 0 || ns < 0 || nw < 0 || L == 0 || reps == 0) return N2VO_ERR_INVALID_ARG;
  for (int64_t k = 0; k < nw; ++k)
    if (widx[k] < 0 || widx[k] >= ns * (int64_t)reps) return N2VO_ERR_INVALID_ARG;
  if (kind != N2VO_FIRST_ORDER && kind != N2VO_NODE2VEC) return N2VO_ERR_INVALID_ARG;
  uint32_t P16 = 65536u, Q16 = 65536u;
  if (kind == N2VO_NODE2VEC) {
    if (n2vo_q16(p, &P16) != N2VO_OK) return N2VO_ERR_INVALID_ARG;
    if (n2vo_q16(q, &Q16) != N2VO_OK) return N2VO_ERR_INVALID_ARG;
  }
  /* Exactness precondition: every cumulative sum fits in 64 bits. */
  uint64_t amax = 1u;
  if (kind == N2VO_NODE2VEC) {
    amax = 65536u;
    if (P16 > amax) amax = P16;
    if (Q16 > amax) amax = Q16;
  }
  uint64_t max_deg = 0, max_sum = 0;
  n2vo_stats(O, n, W, &max_deg, &max_sum);
  if ((unsigned __int128)max_sum * amax > (unsigned __int128)UINT64_MAX) return N2VO_ERR_OVERFLOW;

  uint64_t* b = (uint64_t*)0;
  uint32_t* pos = (uint32_t*)malloc(sizeof(uint32_t) * (k_approx ? k_approx : 1));
  if (!pos) return N2VO_ERR_INVALID_ARG;
  if (max_deg > 0) {
    b = (uint64_t*)malloc(sizeof(uint64_t) * max_deg);
    if (!b) {
      free(pos);
      return N2VO_ERR_INVALID_ARG;
    }
  }
  (void)m;
  for (int64_t k = 0; k < nw; ++k) {
    int64_t w = widx[k];
    int32_t start = S[w % ns];
    int32_t len = one_walk(O, n, D, W, start, L, kind == N2VO_NODE2VEC, P16, Q16, seed,
                           walk_id_base + (uint64_t)w, k_approx, pos, b, Y + (size_t)k * L);
    if (lens) lens[k] = len;
  }
  free(b);
  free(pos);
  return N2VO_OK;
}

int n2vo_walks_subset(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
                      const uint32_t* W, const int32_t* S, int64_t ns,
                      uint32_t reps, uint32_t L, int kind, double p, double q,
                      uint64_t seed, uint64_t walk_id_base,
                      const int64_t* widx, int64_t nw, int32_t* Y, int32_t* lens) {
  return n2vo_walks_approx_subset(O, n, D, m, W, S, ns, reps, L, kind, p, q, 0u, seed, walk_id_base,
                                  widx, nw, Y, lens);
}

int n2vo_walks(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m,
               const uint32_t* W, const int32_t* S, int64_t ns,
               uint32_t reps, uint32_t L, int kind, double p, double q,
               uint64_t seed, uint64_t walk_id_base, int32_t* Y, int32_t* lens) {
  if (ns < 0 || reps == 0) return N2VO_ERR_INVALID_ARG;
  int64_t nw = ns * (int64_t)reps;
  int64_t* widx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nw > 0 ? nw : 1));
  if (!widx) return N2VO_ERR_INVALID_ARG;
  for (int64_t w = 0; w < nw; ++w) widx[w] = w;
  int rc = n2vo_walks_subset(O, n, D, m, W, S, ns, reps, L, kind, p, q, seed, walk_id_base,
                             widx, nw, Y, lens);
  free(widx);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Training contexts and scale-free negatives.                               */
/* ------------------------------------------------------------------------ */
void n2vo_contexts(const int32_t* Y, int64_t nw, uint32_t L, uint32_t window, uint32_t stride, int32_t* C) {
  for (int64_t r = 0; r < nw; ++r) {
    for (uint32_t i = 0; i < L; ++i) {
      int32_t* out = C + ((size_t)r * L + i) * 2 * window;
      for (uint32_t c = 0; c < 2 * window; ++c) {
        int64_t o = c < window ? (int64_t)c - (int64_t)window : (int64_t)c - (int64_t)window + 1;
        int64_t j = (int64_t)i + o * (int64_t)stride;
        int32_t v = -1;
        if (Y[(size_t)r * L + i] >= 0 && j >= 0 && j < (int64_t)L) v = Y[(size_t)r * L + j];
        out[c] = v;
      }
    }
  }
}

void n2vo_negatives(const uint64_t* O, int64_t n, const int32_t* Y, int64_t nw, uint32_t L, uint32_t n_neg,
                    uint64_t seed, uint64_t walk_id_base, int32_t* N) {
  uint64_t m = O[n];
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t r = 0; r < nw; ++r) {
    uint64_t wid = walk_id_base + (uint64_t)r;
    for (uint32_t i = 0; i < L; ++i) {
      int32_t* out = N + ((size_t)r * L + i) * n_neg;
      for (uint32_t j = 0; j < n_neg; ++j) {
        int32_t v = -1;
        if (Y[(size_t)r * L + i] >= 0 && m > 0) {
          uint32_t ctr[4] = {i, (uint32_t)wid, (uint32_t)(wid >> 32), 0x80000000u + j / 2u};
          uint32_t o[4];
          n2vo_philox4x32_10(ctr, key, o);
          uint64_t r64 = (uint64_t)o[2 * (j % 2)] | ((uint64_t)o[2 * (j % 2) + 1] << 32);
          uint64_t T = n2vo_scale(r64, m);
          /* the node whose range of entries [O[v], O[v+1]) holds T: plain scan */
          int64_t lo = 0, hi = n; /* O[lo] <= T < O[hi] */
          while (hi - lo > 1) {
            int64_t mid = lo + (hi - lo) / 2;
            if (O[mid] <= T) lo = mid;
            else hi = mid;
          }
          v = (int32_t)lo;
        }
        out[j] = v;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Elias-Fano list and the edge-code list of a graph (Methods, "Memory       */
/* Complexity", "Edge Encoding", "Efficient implementation of Elias-Fano"). */
/* ------------------------------------------------------------------------ */
void n2vo_ef_shape_of(uint64_t m, uint64_t u, n2vo_ef_shape* s) {
  s->k = 0;
  s->u = u;
  s->m = m;
  /* l = floor(log2(u / m)): the largest l with m 2^l <= u */
  uint32_t l = 0;
  if (m > 0) {
    uint64_t ratio = u / m; /* floor(log2(u/m)) == floor(log2(floor(u/m))) */
    while (l < 63 && (ratio >> (l + 1)) > 0) ++l;
  }
  s->l = l;
  s->n_zeros = ((u - 1) >> l) + 1;
  s->h_bits = m + s->n_zeros;
}

void n2vo_ef_words(const n2vo_ef_shape* s, uint32_t q, uint64_t* h_words, uint64_t* l_words,
                   uint64_t* s1_len, uint64_t* s0_len) {
  *h_words = (s->h_bits + 63) / 64;
  *l_words = (s->m * s->l + 63) / 64;
  *s1_len = (s->m + q - 1) / q;
  *s0_len = (s->n_zeros + q - 1) / q;
}

static int get_bit(const uint64_t* H, uint64_t p) { return (int)((H[p / 64] >> (p % 64)) & 1u); }

static uint64_t get_low(const uint64_t* L, uint32_t l, uint64_t i) {
  uint64_t v = 0;
  for (uint32_t b = 0; b < l; ++b) { /* bit by bit: plain */
    uint64_t p = i * l + b;
    v |= ((L[p / 64] >> (p % 64)) & 1u) << b;
  }
  return v;
}

int n2vo_ef_encode(const uint64_t* y, uint64_t m, uint64_t u, uint32_t q, uint64_t* H, uint64_t* L,
                   uint64_t* S1, uint64_t* S0) {
  if (u == 0 || q == 0) return N2VO_ERR_INVALID_ARG;
  for (uint64_t i = 0; i < m; ++i)
    if (y[i] >= u || (i > 0 && y[i] < y[i - 1])) return N2VO_ERR_INVALID_ARG;
  n2vo_ef_shape s;
  n2vo_ef_shape_of(m, u, &s);
  uint64_t hw, lw, n1, n0;
  n2vo_ef_words(&s, q, &hw, &lw, &n1, &n0);
  for (uint64_t w = 0; w < hw; ++w) H[w] = 0;
  for (uint64_t w = 0; w < lw; ++w) L[w] = 0;
  for (uint64_t i = 0; i < m; ++i) {
    uint64_t h = y[i] >> s.l;
    uint64_t p = h + i; /* h zeros and i ones precede this one */
    H[p / 64] |= 1ull << (p % 64);
    for (uint32_t b = 0; b < s.l; ++b) {
      uint64_t bit = (y[i] >> b) & 1u;
      uint64_t pl = i * s.l + b;
      L[pl / 64] |= bit << (pl % 64);
    }
  }
  /* the quantum indexes: one linear pass over H */
  uint64_t ones = 0, zeros = 0;
  for (uint64_t p = 0; p < s.h_bits; ++p) {
    if (get_bit(H, p)) {
      if (ones % q == 0) S1[ones / q] = p;
      ++ones;
    } else {
      if (zeros % q == 0) S0[zeros / q] = p;
      ++zeros;
    }
  }
  return (ones == m && zeros == s.n_zeros) ? N2VO_OK : N2VO_ERR_INVALID_ARG;
}

int n2vo_ef_graph_shape(int64_t n, uint64_t m, n2vo_ef_shape* s) {
  if (n < 1) return N2VO_ERR_INVALID_ARG;
  uint32_t k = 0;
  while ((1ll << k) < n) ++k; /* k = ceil(log2 n) */
  n2vo_ef_shape_of(m, (uint64_t)n << k, s);
  s->k = k;
  return N2VO_OK;
}

int n2vo_ef_encode_graph(const uint64_t* O, int64_t n, const int32_t* D, uint64_t m, uint32_t q, uint64_t* H,
                         uint64_t* L, uint64_t* S1, uint64_t* S0) {
  n2vo_ef_shape s;
  if (n2vo_ef_graph_shape(n, m, &s) != N2VO_OK) return N2VO_ERR_INVALID_ARG;
  if (n2vo_validate(O, n, D, m) != N2VO_OK) return N2VO_ERR_INVALID_ARG;
  uint64_t* y = (uint64_t*)malloc((m ? m : 1) * sizeof(uint64_t));
  if (!y) return N2VO_ERR_INVALID_ARG;
  for (int64_t a = 0; a < n; ++a)
    for (uint64_t i = O[a]; i < O[a + 1]; ++i) y[i] = ((uint64_t)a << s.k) | (uint64_t)D[i]; /* phi_k(a, b) */
  int rc = n2vo_ef_encode(y, m, s.u, q, H, L, S1, S0);
  free(y);
  return rc;
}

uint64_t n2vo_ef_select(const n2vo_ef_shape* s, const uint64_t* H, const uint64_t* L, uint64_t i) {
  uint64_t ones = 0;
  for (uint64_t p = 0; p < s->h_bits; ++p) {
    if (!get_bit(H, p)) continue;
    if (ones == i) return ((p - i) << s->l) | get_low(L, s->l, i);
    ++ones;
  }
  return ~0ull; /* i >= m */
}

uint64_t n2vo_ef_rank(const n2vo_ef_shape* s, const uint64_t* H, const uint64_t* L, uint64_t x) {
  uint64_t ones = 0;
  for (uint64_t p = 0; p < s->h_bits; ++p) {
    if (!get_bit(H, p)) continue;
    uint64_t y = ((p - ones) << s->l) | get_low(L, s->l, ones);
    if (y >= x) return ones; /* the list is non-decreasing */
    ++ones;
  }
  return ones;
}
