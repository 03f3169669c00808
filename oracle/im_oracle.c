/*
 * im_oracle.c -- plain, single-threaded CPU oracle for the GreediRIS hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product.  Written from the paper
 * (arXiv 2408.10982) and the published definitions it relies on; each routine
 * names the passage it follows.  Build: gcc -O2 -ffp-contract=off (no fast
 * math) so that its fp64 steps round exactly as written.
 *
 * Parity pins live in tests/test_oracle_*.py: Philox known-answer vectors,
 * closed forms (p = 1 reverse reachability, p = 0 singletons), exact
 * enumeration of live-edge worlds on tiny graphs, brute-force max-k-cover,
 * lazy == plain greedy, the streaming and truncation bounds, and the worked
 * approximation ratio printed in the paper.
 */
#include "im_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11).  Round: two 32x32->64 products of counter words 0 and 2 with  */
/* the two published multipliers; the high halves are mixed with the other   */
/* counter words and the key; the key advances by the two Weyl constants     */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL_A;
      k1 += PHILOX_WEYL_B;
    }
    uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
    uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
    uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
    uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
    uint32_t n0 = hi_b ^ c1 ^ k0;
    uint32_t n1 = lo_b;
    uint32_t n2 = hi_a ^ c3 ^ k1;
    uint32_t n3 = lo_a;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint32_t or_draw(uint64_t seed, uint32_t tag, uint32_t stream, uint32_t sample, uint32_t id) {
  uint32_t ctr[4] = {id >> 2, sample, tag, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  or_philox4x32_10(ctr, key, out);
  return out[id & 3u];
}

/* ------------------------------------------------------------------------ */
/* Graph ingest (IC and LT models, Sec. 2).                                  */
/* ------------------------------------------------------------------------ */
int or_ic_thresholds(int64_t num_edges, const float* p, uint32_t* q) {
  for (int64_t e = 0; e < num_edges; ++e) {
    float x = p[e];
    if (!(x >= 0.0f) || x > 1.0f) return -1; /* NaN or outside [0,1] */
    if (x >= 1.0f)
      q[e] = 0xFFFFFFFFu;
    else
      q[e] = (uint32_t)((double)x * 4294967296.0); /* exact: p * 2^32 < 2^32 */
  }
  return 0;
}

int or_lt_thresholds(int32_t n, const int32_t* in_off, const float* w, uint32_t* c) {
  for (int32_t v = 0; v < n; ++v) {
    uint64_t acc = 0;
    for (int32_t j = in_off[v]; j < in_off[v + 1]; ++j) {
      float x = w[j];
      if (!(x >= 0.0f) || isinf(x)) return -1;
      uint64_t q = (x >= 1.0f) ? 4294967296ull : (uint64_t)((double)x * 4294967296.0);
      acc += q;
      c[j] = acc >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)acc;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Run-length form of IC for vertices whose in-edges share one threshold.    */
/* The live in-edges of such a vertex form a Bernoulli(p) sequence over its  */
/* in-edge list, so the gap before the next live edge is Geometric(p):       */
/* G = floor(log(U) / log(1 - p)), U uniform on (0, 1].  log is evaluated by */
/* a fixed sequence of IEEE-754 basic operations (below) so that every       */
/* implementation of the method obtains the same bits.                      */
/* ------------------------------------------------------------------------ */
double or_log(double x) {
  /* x > 0, finite, normal.  x = m 2^e with m in [1, 2), folded into
   * [sqrt(1/2), sqrt(2)); log m = 2 atanh(s), s = (m - 1)/(m + 1), as the
   * odd series 2 (s + s^3/3 + ... + s^19/19). */
  uint64_t bits;
  memcpy(&bits, &x, sizeof bits);
  int32_t e = (int32_t)((bits >> 52) & 0x7FF) - 1023;
  uint64_t mb = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
  double m;
  memcpy(&m, &mb, sizeof m);
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  double s = (m - 1.0) / (m + 1.0);
  double z = s * s;
  double t = 2.0 / 19.0;
  t = t * z + 2.0 / 17.0;
  t = t * z + 2.0 / 15.0;
  t = t * z + 2.0 / 13.0;
  t = t * z + 2.0 / 11.0;
  t = t * z + 2.0 / 9.0;
  t = t * z + 2.0 / 7.0;
  t = t * z + 2.0 / 5.0;
  t = t * z + 2.0 / 3.0;
  t = t * z + 2.0;
  return (double)e * 0.6931471805599453 + s * t;
}

void or_ic_skip_table(int32_t n, const int32_t* in_off, const uint32_t* thr, double* skip) {
  for (int32_t v = 0; v < n; ++v) {
    int32_t a = in_off[v], b = in_off[v + 1];
    skip[v] = 0.0;
    if (b - a < 2) continue;
    uint32_t q = thr[a];
    if (q == 0u || q == 0xFFFFFFFFu) continue;
    int same = 1;
    for (int32_t e = a + 1; e < b; ++e)
      if (thr[e] != q) {
        same = 0;
        break;
      }
    if (!same) continue;
    skip[v] = or_rl_factor(q);
  }
}

double or_rl_factor(uint32_t q) {
  double keep = (4294967296.0 - (double)q) * 2.3283064365386963e-10; /* (2^32 - q) 2^-32 */
  return 1.0 / or_log(keep);
}

int64_t or_rl_gap(double u, double factor) {
  /* in-edges skipped before the next live one: floor(ln U / ln(1 - p)) */
  return (int64_t)floor(or_log(u) * factor);
}

double or_rl_uniform(uint64_t seed, uint32_t stream, uint32_t i, uint32_t v, uint32_t j) {
  uint32_t ctr[4] = {v, i, 0x80000000u | (j >> 1), stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  or_philox4x32_10(ctr, key, out);
  uint32_t hi = out[2 * (j & 1u)] >> 11, lo = out[2 * (j & 1u) + 1];
  double u = (double)(((uint64_t)hi << 32) | lo) + 1.0;
  return u * 1.1102230246251565e-16; /* 2^-53 */
}

int32_t or_root(uint64_t seed, uint32_t stream, uint32_t i, int32_t n) {
  uint32_t r = or_draw(seed, OR_TAG_ROOT, stream, 0u, i);
  return (int32_t)(((uint64_t)r * (uint64_t)(uint32_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* RRR sampling (Def. 2.3; Sec. 2.1 steps 1-2).                              */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static int32_t ceil_log2_plus1(int32_t deg) {
  /* ceil(log2(deg + 1)): probes a binary search over deg entries needs */
  int32_t r = 0;
  while (((int64_t)1 << r) < (int64_t)deg + 1) ++r;
  return r;
}

typedef struct {
  int32_t* buf;
  int64_t len, cap;
} i32vec;

static int vec_push_many(i32vec* v, const int32_t* src, int64_t cnt) {
  if (v->len + cnt > v->cap) {
    int64_t nc = v->cap ? v->cap : 1024;
    while (nc < v->len + cnt) nc *= 2;
    int32_t* nb = (int32_t*)realloc(v->buf, (size_t)nc * sizeof(int32_t));
    if (!nb) return -1;
    v->buf = nb;
    v->cap = nc;
  }
  memcpy(v->buf + v->len, src, (size_t)cnt * sizeof(int32_t));
  v->len += cnt;
  return 0;
}

/* IC: R(i) = vertices with a path to root_i in the live-edge world g_i.
 * Explored by BFS over in-edges; every in-edge carries its own coin, so the
 * set does not depend on the visiting order.  Returns the set size. */
static int32_t sample_ic_one(int32_t n, const int32_t* in_off, const int32_t* in_src,
                             const uint32_t* thr, const double* skip, uint64_t seed,
                             uint32_t stream, uint32_t i, uint32_t* mark, uint32_t stamp,
                             int32_t* queue, int64_t* examined, int64_t* live) {
  int32_t root = or_root(seed, stream, i, n);
  int32_t head = 0, tail = 0;
  queue[tail++] = root;
  mark[root] = stamp;
  while (head < tail) {
    int32_t v = queue[head++];
    if (skip && skip[v] != 0.0) {
      /* run-length form: live positions pos_j = pos_{j-1} + 1 + G_j */
      const int64_t deg = in_off[v + 1] - in_off[v];
      int64_t pos = -1;
      for (uint32_t j = 0;; ++j) {
        ++*examined;
        int64_t g = or_rl_gap(or_rl_uniform(seed, stream, i, (uint32_t)v, j), skip[v]);
        if (g >= deg - 1 - pos) break; /* past the last in-edge */
        pos += 1 + g;
        ++*live;
        int32_t u = in_src[in_off[v] + pos];
        if (mark[u] != stamp) {
          mark[u] = stamp;
          queue[tail++] = u;
        }
      }
      continue;
    }
    for (int32_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      ++*examined;
      uint32_t q = thr[e];
      int is_live = (q == 0xFFFFFFFFu) || (or_draw(seed, OR_TAG_EDGE, stream, i, (uint32_t)e) < q);
      if (!is_live) continue;
      ++*live;
      int32_t u = in_src[e];
      if (mark[u] != stamp) {
        mark[u] = stamp;
        queue[tail++] = u;
      }
    }
  }
  return tail;
}

/* LT: each vertex keeps at most one live in-edge; the reverse-reachable set
 * of the root is the backward chain root <- u1 <- u2 ... which ends at a
 * vertex that keeps no in-edge or at a vertex already in the chain. */
static int32_t sample_lt_one(int32_t n, const int32_t* in_off, const int32_t* in_src,
                             const uint32_t* cum, uint64_t seed, uint32_t stream, uint32_t i,
                             uint32_t* mark, uint32_t stamp, int32_t* queue,
                             int64_t* examined, int64_t* live) {
  int32_t v = or_root(seed, stream, i, n);
  int32_t len = 0;
  queue[len++] = v;
  mark[v] = stamp;
  for (;;) {
    int32_t a = in_off[v], b = in_off[v + 1];
    if (a == b) break;
    *examined += ceil_log2_plus1(b - a);
    uint32_t r = or_draw(seed, OR_TAG_VERT, stream, i, (uint32_t)v);
    int32_t pick = -1;
    for (int32_t j = a; j < b; ++j) { /* first in-edge whose prefix passes r */
      if (cum[j] > r || cum[j] == 0xFFFFFFFFu) {
        pick = j;
        break;
      }
    }
    if (pick < 0) break;
    ++*live;
    int32_t u = in_src[pick];
    if (mark[u] == stamp) break;
    mark[u] = stamp;
    queue[len++] = u;
    v = u;
  }
  return len;
}

int or_sample(int model, int32_t n, const int32_t* in_off, const int32_t* in_src,
              const uint32_t* thr, const double* skip, uint64_t seed, uint32_t stream,
              uint32_t first, int64_t count, or_rrr* out) {
  memset(out, 0, sizeof(*out));
  if (n <= 0 || count < 0 || (model != OR_IC && model != OR_LT)) return -1;
  uint32_t* mark = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
  int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* off = (int64_t*)malloc((size_t)(count + 1) * sizeof(int64_t));
  i32vec mem = {0, 0, 0};
  if (!mark || !queue || !off) goto fail;
  off[0] = 0;
  for (int64_t s = 0; s < count; ++s) {
    uint32_t i = first + (uint32_t)s;
    uint32_t stamp = (uint32_t)(s + 1);
    int32_t len;
    if (model == OR_IC)
      len = sample_ic_one(n, in_off, in_src, thr, skip, seed, stream, i, mark, stamp, queue,
                          &out->examined, &out->live);
    else
      len = sample_lt_one(n, in_off, in_src, thr, seed, stream, i, mark, stamp, queue,
                          &out->examined, &out->live);
    qsort(queue, (size_t)len, sizeof(int32_t), cmp_i32);
    if (vec_push_many(&mem, queue, len)) goto fail;
    off[s + 1] = off[s] + len;
  }
  free(mark);
  free(queue);
  out->count = count;
  out->total = off[count];
  out->off = off;
  out->mem = mem.buf;
  return 0;
fail:
  free(mark);
  free(queue);
  free(off);
  free(mem.buf);
  memset(out, 0, sizeof(*out));
  return -1;
}

void or_rrr_free(or_rrr* r) {
  free(r->off);
  free(r->mem);
  memset(r, 0, sizeof(*r));
}

/* ------------------------------------------------------------------------ */
/* Covering subsets and coverage (Sec. 3.2).                                 */
/* ------------------------------------------------------------------------ */
void or_incidence(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                  int64_t* inc_off, int32_t* inc_mem) {
  int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int32_t v = 0; v <= n; ++v) inc_off[v] = 0;
  for (int64_t t = 0; t < off[count]; ++t) inc_off[mem[t] + 1]++;
  for (int32_t v = 0; v < n; ++v) inc_off[v + 1] += inc_off[v];
  for (int32_t v = 0; v < n; ++v) fill[v] = inc_off[v];
  for (int64_t i = 0; i < count; ++i)          /* samples in increasing order, */
    for (int64_t t = off[i]; t < off[i + 1]; ++t) /* so every S(v) is ascending */
      inc_mem[fill[mem[t]]++] = (int32_t)i;
  free(fill);
}

int64_t or_coverage(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                    int32_t nseeds, const int32_t* seeds) {
  (void)n;
  uint8_t* cov = (uint8_t*)calloc((size_t)count + 1, 1);
  int64_t c = 0;
  for (int32_t s = 0; s < nseeds; ++s) {
    int32_t v = seeds[s];
    for (int64_t t = inc_off[v]; t < inc_off[v + 1]; ++t)
      if (!cov[inc_mem[t]]) {
        cov[inc_mem[t]] = 1;
        ++c;
      }
  }
  free(cov);
  return c;
}

/* ------------------------------------------------------------------------ */
/* Greedy max-k-cover (Sec. 3.2) and Algorithm 2.                            */
/* ------------------------------------------------------------------------ */
static int64_t marginal(const int64_t* inc_off, const int32_t* inc_mem, const uint8_t* cov,
                        int32_t v) {
  int64_t g = 0;
  for (int64_t t = inc_off[v]; t < inc_off[v + 1]; ++t) g += !cov[inc_mem[t]];
  return g;
}

static void cover_with(const int64_t* inc_off, const int32_t* inc_mem, uint8_t* cov, int32_t v) {
  for (int64_t t = inc_off[v]; t < inc_off[v + 1]; ++t) cov[inc_mem[t]] = 1;
}

typedef struct {
  int64_t key;
  int32_t id;
} heap_ent;

static int heap_above(heap_ent a, heap_ent b) { /* tuple order (key, -id) */
  return a.key > b.key || (a.key == b.key && a.id < b.id);
}

static void heap_sift_down(heap_ent* h, int64_t len, int64_t at) {
  for (;;) {
    int64_t l = 2 * at + 1, r = l + 1, top = at;
    if (l < len && heap_above(h[l], h[top])) top = l;
    if (r < len && heap_above(h[r], h[top])) top = r;
    if (top == at) return;
    heap_ent tmp = h[at];
    h[at] = h[top];
    h[top] = tmp;
    at = top;
  }
}

static void heap_sift_up(heap_ent* h, int64_t at) {
  while (at > 0) {
    int64_t p = (at - 1) / 2;
    if (!heap_above(h[at], h[p])) return;
    heap_ent tmp = h[at];
    h[at] = h[p];
    h[p] = tmp;
    at = p;
  }
}

/* Standard greedy over the candidate list cand[0..nc) (ascending ids): each
 * step recomputes every candidate's marginal gain and keeps the first
 * (lowest-id) maximum; cov flags the covered samples of the universe. */
static int32_t greedy_plain_on(const int32_t* cand, int32_t nc, const int64_t* inc_off,
                               const int32_t* inc_mem, uint8_t* cov, int32_t k,
                               int32_t* seeds, int64_t* gains) {
  int32_t t;
  for (t = 0; t < k; ++t) {
    int64_t best = 0;
    int32_t arg = -1;
    for (int32_t c = 0; c < nc; ++c) {
      int64_t g = marginal(inc_off, inc_mem, cov, cand[c]);
      if (g > best) { /* strict: the lowest id keeps a tie */
        best = g;
        arg = cand[c];
      }
    }
    if (arg < 0) break; /* every candidate has zero marginal gain */
    seeds[t] = arg;
    gains[t] = best;
    cover_with(inc_off, inc_mem, cov, arg);
  }
  return t;
}

/* Algorithm 2 over the same candidates: a max-heap keyed by (stale gain, -id);
 * the popped vertex is taken when its recomputed gain still tops the heap.
 * The loop condition of Alg. 2 is read as "|S| < k and Q not empty", and a
 * zero gain ends the selection, as in the standard greedy. */
static int32_t greedy_lazy_on(const int32_t* cand, int32_t nc, const int64_t* inc_off,
                              const int32_t* inc_mem, uint8_t* cov, int32_t k,
                              int32_t* seeds, int64_t* gains) {
  heap_ent* h = (heap_ent*)malloc(((size_t)nc + 1) * sizeof(heap_ent));
  int64_t len = 0;
  for (int32_t c = 0; c < nc; ++c) { /* key = |S(v)|, the gain on an empty solution */
    int32_t v = cand[c];
    h[len].key = marginal(inc_off, inc_mem, cov, v);
    h[len].id = v;
    heap_sift_up(h, len);
    ++len;
  }
  int32_t t = 0;
  while (t < k && len > 0) {
    heap_ent top = h[0];
    h[0] = h[--len];
    heap_sift_down(h, len, 0);
    int64_t g = marginal(inc_off, inc_mem, cov, top.id);
    heap_ent fresh = {g, top.id};
    if (len == 0 || !heap_above(h[0], fresh)) {
      if (g == 0) break; /* nothing left to cover */
      seeds[t] = top.id;
      gains[t] = g;
      ++t;
      cover_with(inc_off, inc_mem, cov, top.id);
    } else {
      h[len] = fresh;
      heap_sift_up(h, len);
      ++len;
    }
  }
  free(h);
  return t;
}

static void greedy_entry(int lazy, int32_t n, int64_t count, const int64_t* inc_off,
                         const int32_t* inc_mem, int32_t k, int32_t* seeds, int64_t* gains,
                         int32_t* nsel, int64_t* coverage) {
  uint8_t* cov = (uint8_t*)calloc((size_t)count + 1, 1);
  int32_t* cand = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  for (int32_t v = 0; v < n; ++v) cand[v] = v;
  int32_t t = lazy ? greedy_lazy_on(cand, n, inc_off, inc_mem, cov, k, seeds, gains)
                   : greedy_plain_on(cand, n, inc_off, inc_mem, cov, k, seeds, gains);
  int64_t c = 0;
  for (int32_t s = 0; s < t; ++s) c += gains[s];
  *nsel = t;
  *coverage = c;
  free(cand);
  free(cov);
}

void or_greedy(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
               int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel, int64_t* coverage) {
  greedy_entry(0, n, count, inc_off, inc_mem, k, seeds, gains, nsel, coverage);
}

void or_lazy_greedy(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                    int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel, int64_t* coverage) {
  greedy_entry(1, n, count, inc_off, inc_mem, k, seeds, gains, nsel, coverage);
}

/* ------------------------------------------------------------------------ */
/* RandGreedi (Alg. 3 partition step, Alg. 4).                               */
/* ------------------------------------------------------------------------ */
void or_partition(int32_t n, int32_t m, uint64_t pseed, uint8_t* part) {
  for (int32_t v = 0; v < n; ++v) {
    uint32_t r = or_draw(pseed, OR_TAG_PART, 0u, 0u, (uint32_t)v);
    part[v] = (uint8_t)(((uint64_t)r * (uint64_t)(uint32_t)m) >> 32);
  }
}

void or_local_greedy(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                     const uint8_t* part, int32_t m, int32_t k, int lazy,
                     int32_t* lseeds, int64_t* lgains, int32_t* lcount, int64_t* lcover) {
  uint8_t* cov = (uint8_t*)malloc((size_t)count + 1);
  int32_t* cand = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  for (int32_t p = 0; p < m; ++p) {
    int32_t nc = 0;
    for (int32_t v = 0; v < n; ++v)
      if (part[v] == (uint8_t)p) cand[nc++] = v;
    memset(cov, 0, (size_t)count + 1);
    int32_t* sp = lseeds + (int64_t)p * k;
    int64_t* gp = lgains + (int64_t)p * k;
    int32_t t = lazy ? greedy_lazy_on(cand, nc, inc_off, inc_mem, cov, k, sp, gp)
                     : greedy_plain_on(cand, nc, inc_off, inc_mem, cov, k, sp, gp);
    int64_t c = 0;
    for (int32_t s = 0; s < t; ++s) c += gp[s];
    lcount[p] = t;
    lcover[p] = c;
  }
  free(cand);
  free(cov);
}

/* ------------------------------------------------------------------------ */
/* Truncation (Sec. 3.3.2) and streaming max-k-cover (Alg. 5).               */
/* ------------------------------------------------------------------------ */
int32_t or_trunc_len(int32_t k, double alpha) {
  double x = ceil(alpha * (double)k);
  int32_t t = (int32_t)x;
  if (t < 1) t = 1;
  if (t > k) t = k;
  return t;
}

int32_t or_num_buckets(int32_t k, double delta) {
  double b = ceil(log((double)k) / log(1.0 + delta));
  int32_t B = (int32_t)b;
  return B < 1 ? 1 : B;
}

void or_bucket_thresholds(int64_t l, int32_t k, double delta, int32_t B, int64_t* thr) {
  double g = 1.0; /* (1 + delta)^b by repeated multiplication */
  for (int32_t b = 0; b < B; ++b) {
    thr[b] = (int64_t)ceil((double)l * g / (2.0 * (double)k));
    g = g * (1.0 + delta);
  }
}

void or_stream_cover(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                     int32_t m, int32_t k, const int32_t* lseeds, const int64_t* lgains,
                     const int32_t* lcount, double delta, double alpha,
                     int32_t* seeds, int32_t* nsel, int64_t* coverage, int32_t* bucket,
                     int32_t* nbuckets) {
  (void)n;
  (void)lgains;
  int32_t T = or_trunc_len(k, alpha);
  /* the stream: local picks in selection order, partitions in lockstep */
  int64_t slen = 0;
  int32_t* stream = (int32_t*)malloc((size_t)m * (size_t)T * sizeof(int32_t) + 4);
  for (int32_t t = 0; t < T; ++t)
    for (int32_t p = 0; p < m; ++p)
      if (t < lcount[p]) stream[slen++] = lseeds[(int64_t)p * k + t];
  int32_t B = or_num_buckets(k, delta);
  *nbuckets = B;
  int64_t l = 0; /* lower bound on OPT: the largest single covering subset */
  for (int64_t s = 0; s < slen; ++s) {
    int64_t sz = inc_off[stream[s] + 1] - inc_off[stream[s]];
    if (sz > l) l = sz;
  }
  if (slen == 0 || l == 0) {
    *nsel = 0;
    *coverage = 0;
    *bucket = 0;
    free(stream);
    return;
  }
  int64_t* thr = (int64_t*)malloc((size_t)B * sizeof(int64_t));
  or_bucket_thresholds(l, k, delta, B, thr);
  uint8_t* C = (uint8_t*)calloc((size_t)B * (size_t)(count + 1), 1); /* C_b */
  int32_t* S = (int32_t*)malloc((size_t)B * (size_t)k * sizeof(int32_t)); /* S_b */
  int32_t* ns = (int32_t*)calloc((size_t)B, sizeof(int32_t));
  int64_t* csz = (int64_t*)calloc((size_t)B, sizeof(int64_t));
  for (int64_t s = 0; s < slen; ++s) {
    int32_t x = stream[s];
    for (int32_t b = 0; b < B; ++b) {
      if (ns[b] >= k) continue;
      uint8_t* Cb = C + (size_t)b * (size_t)(count + 1);
      int64_t g = 0;
      for (int64_t t = inc_off[x]; t < inc_off[x + 1]; ++t) g += !Cb[inc_mem[t]];
      if (g >= thr[b]) {
        for (int64_t t = inc_off[x]; t < inc_off[x + 1]; ++t) Cb[inc_mem[t]] = 1;
        S[(int64_t)b * k + ns[b]++] = x;
        csz[b] += g;
      }
    }
  }
  int32_t bs = 0;
  for (int32_t b = 1; b < B; ++b)
    if (csz[b] > csz[bs]) bs = b;
  for (int32_t j = 0; j < ns[bs]; ++j) seeds[j] = S[(int64_t)bs * k + j];
  *nsel = ns[bs];
  *coverage = csz[bs];
  *bucket = bs;
  free(stream);
  free(thr);
  free(C);
  free(S);
  free(ns);
  free(csz);
}

void or_greedi_offline(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                       int32_t m, int32_t k, const int32_t* lseeds, const int32_t* lcount,
                       double alpha, int lazy, int32_t* gseeds, int64_t* ggains, int32_t* gsel,
                       int64_t* gcover) {
  (void)n;
  int32_t T = or_trunc_len(k, alpha);
  /* the union of the gathered local solutions, ascending ids */
  int32_t* cand = (int32_t*)malloc(((size_t)m * (size_t)T + 1) * sizeof(int32_t));
  int32_t nc = 0;
  for (int32_t p = 0; p < m; ++p)
    for (int32_t t = 0; t < T && t < lcount[p]; ++t) cand[nc++] = lseeds[(int64_t)p * k + t];
  qsort(cand, (size_t)nc, sizeof(int32_t), cmp_i32);
  int32_t u = 0; /* the parts are disjoint, so this only guards repeated input */
  for (int32_t c = 0; c < nc; ++c)
    if (u == 0 || cand[c] != cand[u - 1]) cand[u++] = cand[c];
  uint8_t* cov = (uint8_t*)calloc((size_t)count + 1, 1);
  int32_t t = lazy ? greedy_lazy_on(cand, u, inc_off, inc_mem, cov, k, gseeds, ggains)
                   : greedy_plain_on(cand, u, inc_off, inc_mem, cov, k, gseeds, ggains);
  int64_t c = 0;
  for (int32_t j = 0; j < t; ++j) c += ggains[j];
  for (int32_t j = t; j < k; ++j) {
    gseeds[j] = -1;
    ggains[j] = 0;
  }
  *gsel = t;
  *gcover = c;
  free(cov);
  free(cand);
}

int or_final_select(int32_t m, int32_t k, const int32_t* lseeds, const int32_t* lcount,
                    const int64_t* lcover, const int32_t* gseeds, int32_t gsel, int64_t gcover,
                    int32_t* seeds, int32_t* nsel, int64_t* coverage) {
  int32_t pl = 0;
  for (int32_t p = 1; p < m; ++p)
    if (lcover[p] > lcover[pl]) pl = p;
  if (gcover >= lcover[pl]) {
    for (int32_t j = 0; j < gsel; ++j) seeds[j] = gseeds[j];
    *nsel = gsel;
    *coverage = gcover;
    return 1;
  }
  for (int32_t j = 0; j < lcount[pl]; ++j) seeds[j] = lseeds[(int64_t)pl * k + j];
  *nsel = lcount[pl];
  *coverage = lcover[pl];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward influence simulation (the quality measure of Sec. 4.1).           */
/* ------------------------------------------------------------------------ */
/* LT: the in-edge v keeps in world r (-1 if none), by a linear scan of its
 * prefix sums */
static int32_t sim_kept_edge(const int32_t* in_off, const uint32_t* thr, uint64_t seed,
                             uint32_t stream, uint32_t r, int32_t v) {
  uint32_t x = or_draw(seed, OR_TAG_SIM_VERT, stream, r, (uint32_t)v);
  for (int32_t j = in_off[v]; j < in_off[v + 1]; ++j)
    if (thr[j] > x || thr[j] == 0xFFFFFFFFu) return j;
  return -1;
}

int or_influence(int model, int32_t n, const int32_t* in_off, const int32_t* in_src,
                 const uint32_t* thr, uint64_t seed, uint32_t stream, uint32_t first,
                 int64_t nsims, int32_t nseeds, const int32_t* seeds, int64_t* counts) {
  int64_t E = in_off[n];
  /* out-edges of every vertex: the in-edge ids grouped by their source */
  int32_t* out_off = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t* out_e = (int32_t*)malloc(((size_t)E + 1) * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc(((size_t)E + 1) * sizeof(int32_t));
  int32_t* fill = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  uint32_t* mark = (uint32_t*)calloc((size_t)n + 1, sizeof(uint32_t));
  int32_t* queue = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  /* LT: each vertex's kept edge, found once per simulation */
  uint32_t* kstamp = (uint32_t*)calloc((size_t)n + 1, sizeof(uint32_t));
  int32_t* kept = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  if (!out_off || !out_e || !dst || !fill || !mark || !queue || !kstamp || !kept) {
    free(out_off); free(out_e); free(dst); free(fill); free(mark); free(queue);
    free(kstamp); free(kept);
    return -1;
  }
  for (int32_t v = 0; v < n; ++v)
    for (int32_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      dst[e] = v;
      out_off[in_src[e] + 1]++;
    }
  for (int32_t u = 0; u < n; ++u) out_off[u + 1] += out_off[u];
  for (int32_t u = 0; u < n; ++u) fill[u] = out_off[u];
  for (int64_t e = 0; e < E; ++e) out_e[fill[in_src[e]]++] = (int32_t)e;
  for (int64_t s = 0; s < nsims; ++s) {
    uint32_t r = first + (uint32_t)s, stamp = (uint32_t)(s + 1);
    int32_t head = 0, tail = 0;
    for (int32_t j = 0; j < nseeds; ++j)
      if (mark[seeds[j]] != stamp) {
        mark[seeds[j]] = stamp;
        queue[tail++] = seeds[j];
      }
    while (head < tail) {
      int32_t u = queue[head++];
      for (int32_t j = out_off[u]; j < out_off[u + 1]; ++j) {
        int32_t e = out_e[j], v = dst[e];
        if (mark[v] == stamp) continue;
        int live;
        if (model == OR_IC) {
          uint32_t q = thr[e];
          live = q == 0xFFFFFFFFu || or_draw(seed, OR_TAG_SIM_EDGE, stream, r, (uint32_t)e) < q;
        } else {
          if (kstamp[v] != stamp) {
            kstamp[v] = stamp;
            kept[v] = sim_kept_edge(in_off, thr, seed, stream, r, v);
          }
          live = kept[v] == e;
        }
        if (!live) continue;
        mark[v] = stamp;
        queue[tail++] = v;
      }
    }
    counts[s] = tail;
  }
  free(out_off); free(out_e); free(dst); free(fill); free(mark); free(queue);
  free(kstamp); free(kept);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* IMM (Alg. 1; sample-size bounds of Tang, Shi and Xiao 2015, with the      */
/* fresh final sample of Chen 2018 that Alg. 1 writes as Sample(G, theta)).  */
/* ------------------------------------------------------------------------ */
void or_imm_parameters(int32_t n, int32_t k, double eps, or_imm_params* o) {
  double nd = (double)n;
  double ln_n = log(nd);
  o->ell = 1.0 * (1.0 + log(2.0) / ln_n);
  o->eps_prime = sqrt(2.0) * eps;
  double lb = 0.0; /* ln C(n, k) */
  for (int32_t i = 0; i < k; ++i) lb += log(nd - (double)i);
  for (int32_t i = 1; i <= k; ++i) lb -= log((double)i);
  o->log_binom = lb;
  double ep = o->eps_prime;
  o->lambda_prime = (2.0 + 2.0 * ep / 3.0) * (lb + o->ell * ln_n + log(log2(nd))) * nd / (ep * ep);
  double e1 = 1.0 - exp(-1.0);
  o->alpha_i = sqrt(o->ell * ln_n + log(2.0));
  o->beta_i = sqrt(e1 * (lb + o->ell * ln_n + log(2.0)));
  double s = e1 * o->alpha_i + o->beta_i;
  o->lambda_star = 2.0 * nd * s * s / (eps * eps);
  o->theta1 = (int64_t)ceil(o->lambda_prime / (nd / 2.0));
  int32_t lg = 0;
  while (((int64_t)1 << (lg + 1)) <= (int64_t)n) ++lg; /* floor(log2 n) */
  o->rounds = lg - 1;
}

/* growable RRR pool: sets for sample ids [0, count) of one stream */
typedef struct {
  int64_t count, total;
  int64_t* off;
  int32_t* mem;
} pool_t;

static int pool_extend(pool_t* P, int model, int32_t n, const int32_t* in_off,
                       const int32_t* in_src, const uint32_t* thr, const double* skip,
                       uint64_t seed, uint32_t stream, int64_t new_count) {
  if (new_count <= P->count) return 0;
  or_rrr add;
  if (or_sample(model, n, in_off, in_src, thr, skip, seed, stream, (uint32_t)P->count,
                new_count - P->count, &add))
    return -1;
  int64_t* noff = (int64_t*)realloc(P->off, (size_t)(new_count + 1) * sizeof(int64_t));
  int32_t* nmem = (int32_t*)realloc(P->mem, (size_t)(P->total + add.total + 1) * sizeof(int32_t));
  if (!noff || !nmem) return -1;
  P->off = noff;
  P->mem = nmem;
  if (P->count == 0) P->off[0] = 0;
  for (int64_t s = 0; s < add.count; ++s) P->off[P->count + s + 1] = P->total + add.off[s + 1];
  memcpy(P->mem + P->total, add.mem, (size_t)add.total * sizeof(int32_t));
  P->total += add.total;
  P->count = new_count;
  or_rrr_free(&add);
  return 0;
}

/* one SelectSeeds call on the pool; seeds receives up to k ids */
static void select_on(const pool_t* P, int32_t n, const or_imm_opts* opt, int32_t* seeds,
                      int32_t* nsel, int64_t* coverage, int32_t* bucket, int* gwon,
                      int32_t* slen) {
  int32_t k = opt->k;
  int64_t* inc_off = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  int32_t* inc_mem = (int32_t*)malloc((size_t)(P->total + 1) * sizeof(int32_t));
  or_incidence(n, P->count, P->off, P->mem, inc_off, inc_mem);
  int64_t* gains = (int64_t*)malloc((size_t)k * sizeof(int64_t));
  *bucket = -1;
  *gwon = -1;
  *slen = 0;
  if (opt->selector == OR_SEL_GREEDY) {
    greedy_entry(opt->lazy, n, P->count, inc_off, inc_mem, k, seeds, gains, nsel, coverage);
  } else {
    int32_t m = opt->m;
    uint8_t* part = (uint8_t*)malloc((size_t)n);
    int32_t* ls = (int32_t*)malloc((size_t)m * k * sizeof(int32_t));
    int64_t* lg = (int64_t*)malloc((size_t)m * k * sizeof(int64_t));
    int32_t* lc = (int32_t*)malloc((size_t)m * sizeof(int32_t));
    int64_t* lv = (int64_t*)malloc((size_t)m * sizeof(int64_t));
    int32_t* gs = (int32_t*)malloc((size_t)k * sizeof(int32_t));
    int32_t gsel, nb;
    int64_t gcov;
    or_partition(n, m, opt->part_seed, part);
    or_local_greedy(n, P->count, inc_off, inc_mem, part, m, k, opt->lazy, ls, lg, lc, lv);
    if (opt->selector == OR_SEL_RANDGREEDI) {
      int64_t* gg = (int64_t*)malloc((size_t)k * sizeof(int64_t));
      or_greedi_offline(n, P->count, inc_off, inc_mem, m, k, ls, lc, opt->alpha, opt->lazy, gs,
                        gg, &gsel, &gcov);
      free(gg);
    } else {
      or_stream_cover(n, P->count, inc_off, inc_mem, m, k, ls, lg, lc, opt->delta, opt->alpha,
                      gs, &gsel, &gcov, bucket, &nb);
    }
    *gwon = or_final_select(m, k, ls, lc, lv, gs, gsel, gcov, seeds, nsel, coverage);
    int32_t T = or_trunc_len(k, opt->alpha); /* the stream: first T picks of each part */
    for (int32_t p = 0; p < m; ++p) *slen += lc[p] < T ? lc[p] : T;
    free(part); free(ls); free(lg); free(lc); free(lv); free(gs);
  }
  free(gains);
  free(inc_off);
  free(inc_mem);
}

int or_imm(int32_t n, const int32_t* in_off, const int32_t* in_src, const uint32_t* thr,
           const double* skip, const or_imm_opts* opt, int32_t* seeds, or_imm_result* res) {
  memset(res, 0, sizeof(*res));
  or_imm_params prm;
  or_imm_parameters(n, opt->k, opt->eps, &prm);
  double nd = (double)n;
  double lb = 1.0;
  int32_t nsel = 0, bucket = -1, slen = 0;
  int64_t cov = 0;
  int gwon = -1;
  int64_t theta;
  if (opt->theta_override > 0) {
    theta = opt->theta_override;
  } else {
    pool_t P = {0, 0, NULL, NULL};
    int64_t th = prm.theta1;
    for (int32_t i = 1; i <= prm.rounds; ++i) {
      if (i > 1) th *= 2;
      if (pool_extend(&P, opt->model, n, in_off, in_src, thr, skip, opt->seed, 0u, th))
        return -1;
      select_on(&P, n, opt, seeds, &nsel, &cov, &bucket, &gwon, &slen);
      res->rounds_run = i;
      double x = nd / ldexp(1.0, i);
      if (nd * (double)cov / (double)th >= (1.0 + prm.eps_prime) * x) {
        lb = nd * (double)cov / ((double)th * (1.0 + prm.eps_prime));
        break;
      }
    }
    res->martingale_samples = P.count;
    free(P.off);
    free(P.mem);
    theta = (int64_t)ceil(prm.lambda_star / lb);
  }
  pool_t F = {0, 0, NULL, NULL};
  if (pool_extend(&F, opt->model, n, in_off, in_src, thr, skip, opt->seed, 1u, theta)) return -1;
  select_on(&F, n, opt, seeds, &nsel, &cov, &bucket, &gwon, &slen);
  free(F.off);
  free(F.mem);
  res->nsel = nsel;
  res->coverage = cov;
  res->theta = theta;
  res->lb = lb;
  res->bucket = bucket;
  res->global_won = gwon;
  res->stream_len = slen;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* OPIM (bounds of Tang, Tang, Xiao and Yuan 2018).                          */
/* ------------------------------------------------------------------------ */
static int cmp_i64_desc(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x < y) - (x > y);
}

/* sum of the k largest of v[0..n) (v is reordered) */
static int64_t top_k_sum(int64_t* v, int32_t n, int32_t k) {
  qsort(v, (size_t)n, sizeof(int64_t), cmp_i64_desc);
  int64_t s = 0;
  for (int32_t j = 0; j < k && j < n; ++j) s += v[j];
  return s;
}

int or_opim(int32_t n, const int32_t* in_off, const int32_t* in_src, const uint32_t* thr,
            const double* skip, const or_imm_opts* opt, double fail, int64_t theta_cap,
            int32_t* seeds, or_opim_result* res) {
  memset(res, 0, sizeof(*res));
  int32_t k = opt->k;
  double nd = (double)n, eps = opt->eps;
  double e1 = 1.0 - exp(-1.0);
  double lb = 0.0; /* ln C(n, k) */
  for (int32_t i = 0; i < k; ++i) lb += log(nd - (double)i);
  for (int32_t i = 1; i <= k; ++i) lb -= log((double)i);
  double l6 = log(6.0 / fail);
  double t = e1 * sqrt(l6) + sqrt(e1 * (lb + l6));
  double theta_max = 2.0 * nd * t * t / (eps * eps * (double)k);
  int64_t theta = (int64_t)ceil(theta_max * eps * eps * (double)k / nd);
  int32_t i_max = (int32_t)ceil(log2(theta_max / (double)theta));
  if (i_max < 1) i_max = 1;
  double a = log(3.0 * (double)i_max / fail);
  res->theta_max = theta_max;
  res->i_max = i_max;
  pool_t R1 = {0, 0, NULL, NULL}, R2 = {0, 0, NULL, NULL};
  int64_t* marg = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  int rc = 0;
  for (int32_t i = 1;; ++i) {
    if (pool_extend(&R1, opt->model, n, in_off, in_src, thr, skip, opt->seed, 0u, theta) ||
        pool_extend(&R2, opt->model, n, in_off, in_src, thr, skip, opt->seed, 1u, theta)) {
      rc = -1;
      break;
    }
    int32_t nsel = 0, bucket = -1, slen = 0;
    int64_t cov1 = 0;
    int gwon = -1;
    select_on(&R1, n, opt, seeds, &nsel, &cov1, &bucket, &gwon, &slen);
    /* upper bound on the optimum's coverage of R1 */
    int64_t* io1 = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* im1 = (int32_t*)malloc(((size_t)R1.total + 1) * sizeof(int32_t));
    or_incidence(n, R1.count, R1.off, R1.mem, io1, im1);
    for (int32_t v = 0; v < n; ++v) marg[v] = io1[v + 1] - io1[v];
    int64_t u0 = top_k_sum(marg, n, k);
    uint8_t* cov = (uint8_t*)calloc((size_t)R1.count + 1, 1);
    for (int32_t j = 0; j < nsel; ++j) cover_with(io1, im1, cov, seeds[j]);
    for (int32_t v = 0; v < n; ++v) marg[v] = marginal(io1, im1, cov, v);
    int64_t u1 = cov1 + top_k_sum(marg, n, k);
    int64_t up1 = u0 < u1 ? u0 : u1;
    free(cov);
    free(io1);
    free(im1);
    /* validation on R2 */
    int64_t* io2 = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t* im2 = (int32_t*)malloc(((size_t)R2.total + 1) * sizeof(int32_t));
    or_incidence(n, R2.count, R2.off, R2.mem, io2, im2);
    int64_t cov2 = or_coverage(n, R2.count, io2, im2, nsel, seeds);
    free(io2);
    free(im2);
    double th = (double)theta;
    double x = sqrt((double)cov2 + 2.0 * a / 9.0) - sqrt(a / 2.0);
    double lower = (x * x - a / 18.0) * nd / th;
    double y = sqrt((double)up1 + a / 2.0) + sqrt(a / 2.0);
    double upper = y * y * nd / th;
    double g = lower / upper;
    res->nsel = nsel;
    res->rounds = i;
    res->theta = theta;
    res->cover1 = cov1;
    res->cover2 = cov2;
    res->upper1 = up1;
    res->lower = lower;
    res->upper = upper;
    res->guarantee = g;
    if (g >= e1 - eps || i >= i_max || 2 * theta >= theta_cap) break;
    theta *= 2;
  }
  free(marg);
  free(R1.off);
  free(R1.mem);
  free(R2.off);
  free(R2.mem);
  return rc;
}
