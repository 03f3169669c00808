/*
 * im_oracle.h -- plain, single-threaded CPU oracle for the GreediRIS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its
 * Python binding) may include, link, call or execute this code.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header, table or constant generator with the GPU path.
 *
 * Every function restates a definition or algorithm of the paper
 * "GreediRIS: Scalable Influence Maximization using Distributed Streaming
 * Maximum Cover" (Barik et al., arXiv 2408.10982); the citation sits beside
 * each declaration.  Where the paper is silent or garbled the reading taken
 * is stated beside the function that takes it.
 *
 * Integer work is exact; the few floating-point steps (IMM's sample-size
 * bounds, the streaming thresholds) run in fp64 in a fixed operation order.
 */
#ifndef IM_ORACLE_H
#define IM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Draw domains: each random quantity of the method is keyed by its domain. */
enum { OR_TAG_ROOT = 0, OR_TAG_EDGE = 1, OR_TAG_VERT = 2, OR_TAG_PART = 3 };
enum { OR_IC = 0, OR_LT = 1 };
enum { OR_SEL_GREEDY = 0, OR_SEL_GREEDIRIS = 1 };

/* Philox4x32-10 of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of the
 * published round function with the published multipliers and key bumps. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* One uint32 of the method's random stream.  Counter = (id>>2, sample, tag,
 * stream), key = (seed lo, seed hi), word id&3.  Replaces the paper's
 * Leap-Frog generator (Sec. 3.2): every draw is a pure function of its ids,
 * so the result does not depend on how work is split. */
uint32_t or_draw(uint64_t seed, uint32_t tag, uint32_t stream, uint32_t sample, uint32_t id);

/* Graph ingest.  IC: per-edge probability p in [0,1] -> threshold
 * q = (p >= 1) ? 0xFFFFFFFF : floor(p * 2^32); the edge is live iff
 * q == 0xFFFFFFFF or draw < q (Sec. 2, IC model).  Returns 0, or -1 on a
 * NaN / out-of-range weight. */
int or_ic_thresholds(int64_t num_edges, const float* p, uint32_t* q);

/* LT: per-edge weight w >= 0 -> q = (w >= 1) ? 2^32 : floor(w * 2^32);
 * c_j = min(sum_{i<=j} q_i over v's in-edges in CSR order, 0xFFFFFFFF)
 * (Sec. 2, LT model, read as the live-edge process: each vertex keeps at most
 * one in-edge, edge j with probability w_j). */
int or_lt_thresholds(int32_t n, const int32_t* in_off, const float* w, uint32_t* c);

/* Root of sample i: floor(draw * n / 2^32), uniform over V (Sec. 2.1). */
int32_t or_root(uint64_t seed, uint32_t stream, uint32_t i, int32_t n);

/* A collection of RRR sets, sample-major, members ascending in each set. */
typedef struct {
  int64_t count;     /* number of sets */
  int64_t total;     /* sum of set sizes */
  int64_t* off;      /* count+1 offsets into mem */
  int32_t* mem;      /* total members */
  int64_t examined;  /* in-edges looked at (IC) / search probes (LT) */
  int64_t live;      /* live in-edges found (IC) / edges taken (LT) */
} or_rrr;

/* RRR sets for sample ids [first, first+count) of the given stream
 * (Def. 2.3 and the two-step sampler of Sec. 2.1).  In-CSR of the graph:
 * in_off[n+1], in_src[E]; thr from or_ic_thresholds / or_lt_thresholds.
 * Allocates out->off / out->mem (free with or_rrr_free).  Returns 0 or -1. */
int or_sample(int model, int32_t n, const int32_t* in_off, const int32_t* in_src,
              const uint32_t* thr, uint64_t seed, uint32_t stream, uint32_t first,
              int64_t count, or_rrr* out);
void or_rrr_free(or_rrr* r);

/* Covering subsets S(v) = {i : v in R(i)} (Sec. 3.2), ascending in i.
 * inc_off[n+1], inc_mem[total]. */
void or_incidence(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                  int64_t* inc_off, int32_t* inc_mem);

/* C(S) = |union of S(v), v in S| (Sec. 3.2). */
int64_t or_coverage(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                    int32_t nseeds, const int32_t* seeds);

/* Standard greedy max-k-cover (Sec. 3.2): k times take the vertex of largest
 * marginal coverage, lowest id on ties; stop early at zero gain. */
void or_greedy(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
               int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel, int64_t* coverage);

/* Algorithm 2 (lazy greedy) with heap keys (gain, -id). */
void or_lazy_greedy(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                    int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel, int64_t* coverage);

/* Uniform random vertex partition (Alg. 3, partition step):
 * part(v) = floor(draw(pseed, PART, 0, 0, v) * m / 2^32). */
void or_partition(int32_t n, int32_t m, uint64_t pseed, uint8_t* part);

/* Alg. 4 local step: greedy restricted to candidates V_p, universe all
 * samples; all k picks recorded (Sec. 3.4, S3).  lseeds/lgains are m*k, row p
 * for part p.  lazy != 0 evaluates with Algorithm 2 (same result). */
void or_local_greedy(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                     const uint8_t* part, int32_t m, int32_t k, int lazy,
                     int32_t* lseeds, int64_t* lgains, int32_t* lcount, int64_t* lcover);

/* Truncation length T = ceil(alpha * k) (Sec. 3.3.2), fp64. */
int32_t or_trunc_len(int32_t k, double alpha);

/* Number of buckets B = max(1, ceil(ln k / ln(1+delta))) and the integer
 * thresholds thr_b = ceil(l * (1+delta)^b / (2k)) (Alg. 5), fp64. */
int32_t or_num_buckets(int32_t k, double delta);
void or_bucket_thresholds(int64_t l, int32_t k, double delta, int32_t B, int64_t* thr);

/* Alg. 5 over the fixed stream order "round t, then partition p".  Returns
 * the best bucket's seeds (acceptance order), their coverage and the bucket. */
void or_stream_cover(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                     int32_t m, int32_t k, const int32_t* lseeds, const int64_t* lgains,
                     const int32_t* lcount, double delta, double alpha,
                     int32_t* seeds, int32_t* nsel, int64_t* coverage, int32_t* bucket,
                     int32_t* nbuckets);

/* Alg. 4 final step: S = S_g if C(S_g) >= C(S_l) else S_l, S_l the lowest
 * partition of largest local coverage.  Returns 1 if the global solution won. */
int or_final_select(int32_t m, int32_t k, const int32_t* lseeds, const int32_t* lcount,
                    const int64_t* lcover, const int32_t* gseeds, int32_t gsel, int64_t gcover,
                    int32_t* seeds, int32_t* nsel, int64_t* coverage);

/* IMM parameters (Alg. 1 with the bounds of Tang et al. 2015). */
typedef struct {
  double ell, eps_prime, log_binom, lambda_prime, lambda_star, alpha_i, beta_i;
  int64_t theta1;    /* first martingale sample count, ceil(lambda' * 2 / n) */
  int32_t rounds;    /* floor(log2 n) - 1 */
} or_imm_params;
void or_imm_parameters(int32_t n, int32_t k, double eps, or_imm_params* out);

typedef struct {
  int model, selector, lazy;  /* lazy != 0: greedy steps evaluated by Alg. 2 */
  int32_t k, m;
  double eps, delta, alpha;
  uint64_t seed, part_seed;
  int64_t theta_override;   /* > 0: skip the martingale loop, use this theta */
} or_imm_opts;

typedef struct {
  int32_t nsel;
  int64_t coverage;
  int64_t theta;
  int32_t rounds_run;
  double lb;
  int64_t martingale_samples;
  int32_t bucket;
  int global_won;
} or_imm_result;

/* Alg. 1: martingale rounds on stream 0, then theta fresh samples on stream 1
 * and the final selection.  seeds holds k entries. */
int or_imm(int32_t n, const int32_t* in_off, const int32_t* in_src, const uint32_t* thr,
           const or_imm_opts* opt, int32_t* seeds, or_imm_result* res);

#ifdef __cplusplus
}
#endif
#endif
