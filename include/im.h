/*
 * im.h -- C ABI of the MI355X influence-maximization hot path.
 *
 * Reverse influence sampling of random reverse-reachable (RRR) sets under the
 * Independent Cascade (IC) and Linear Threshold (LT) models, and seed
 * selection by maximum k-cover over them: standard greedy, the RandGreedi
 * split into per-partition local greedy plus a streaming threshold-bucket
 * cover with optional truncation, and the IMM driver around them.  The method
 * is that of "GreediRIS: Scalable Influence Maximization using Distributed
 * Streaming Maximum Cover" (Barik et al., arXiv 2408.10982); each entry point
 * names the passage that defines its operation.
 *
 * Conventions shared by every entry point
 *  - Pointers marked [device] are HIP device memory owned by the caller;
 *    pointers marked [host] are host memory owned by the caller.  The library
 *    never frees caller memory and allocates no device memory of its own
 *    (the one fixed array of im_greedy_cover_static aside).
 *  - Workspace: every entry point that needs device memory beyond its inputs
 *    and outputs takes (ws, ws_bytes), a [device] region owned by the caller
 *    and used on `stream` only for the duration of the call (its contents
 *    are undefined before and after).  im_workspace_size() gives the bytes to
 *    pass for a problem shape.  A workspace shorter than the call's minimum
 *    returns IM_ENOMEM before any device work or output write; one that runs
 *    out part way (the data-dependent sizes of the IMM and OPIM pools and of
 *    the sampling arena) returns IM_ENOMEM with outputs undefined.  In both
 *    cases im_workspace_need() then gives the bytes that call needed at
 *    least; repeating it with that many bytes gets further or succeeds.
 *    After any call it also gives the bytes that call could have used.
 *    Larger workspaces let sampling stage more sets per pass and run more
 *    large-set workers, and let the covering subsets be built in one round;
 *    results never depend on the size.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it; entry points that return a host-side value (sizes, counts)
 *    synchronise that stream before returning, and say so.
 *  - Errors are status codes; nothing is thrown across the ABI.  IM_EINVAL is
 *    returned before any device work is enqueued or any output is written.
 *  - Calls that share one stream run in order.  Calls on different streams
 *    may overlap when they are given different workspaces; they must not
 *    write the same caller buffers.  Their kernels run side by side only if
 *    the streams sit on different hardware queues: HIP gives a stream its
 *    queue on first use, and past GPU_MAX_HW_QUEUES queues (HIP's default 4)
 *    streams share them and run one after the other, so a process that
 *    overlaps solves sets that variable above its stream count before HIP
 *    starts.
 *  - All arithmetic on the device is integer.  The only floating-point steps
 *    (IMM sample-size bounds, streaming bucket thresholds) run on the host in
 *    fp64 with a fixed operation order.
 *
 * Random numbers.  Every random quantity is one 32-bit word of Philox4x32-10
 * (Salmon et al., SC'11) with key (seed lo, seed hi) and counter
 * (id >> 2, sample id, domain tag, stream tag), word id & 3.  Domain tags:
 * root 0, IC edge 1, LT vertex 2, partition 3, simulation edge 4, simulation
 * vertex 5.  A draw depends only on its
 * ids, so results do not depend on launch shape or on how samples are split
 * (the property the paper's Leap-Frog generator provides, Sec. 3.2).
 */
#ifndef IM_H
#define IM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IM_OK = 0,
  IM_EINVAL = -1,  /* invalid argument; nothing was enqueued or written */
  IM_ERANGE = -2,  /* output capacity too small; the needed size is returned */
  IM_ENOMEM = -3,  /* the workspace is too small (im_workspace_need() gives the bytes
                      needed), or a sampling arena stayed short after its retries
                      (the detail is in im_last_error()) */
  IM_EDEVICE = -4  /* a HIP call failed (the HIP error is in im_last_error()) */
} im_status;

typedef enum { IM_IC = 0, IM_LT = 1 } im_model;

typedef enum { IM_SEL_GREEDY = 0, IM_SEL_GREEDIRIS = 1, IM_SEL_RANDGREEDI = 2 } im_selector;

/* A graph prepared for sampling.  The in-edge CSR lists, for every vertex v,
 * the edges u -> v as in_src[in_off[v] .. in_off[v+1]); edge id e is the
 * position in that array.  thr[e] comes from im_prepare_graph. */
typedef struct {
  int32_t n;               /* vertices, 1 <= n < 2^31 */
  int64_t num_edges;       /* E, 0 <= E < 2^31 */
  const int32_t* in_off;   /* [device] n+1, non-decreasing, in_off[0]=0, in_off[n]=E */
  const int32_t* in_src;   /* [device] E, each in [0, n) */
  const uint32_t* thr;     /* [device] round_up(E, 4) entries from im_prepare_graph */
  int32_t model;           /* IM_IC or IM_LT, as given to im_prepare_graph */
  const double* skip;      /* [device] n entries from im_prepare_graph (IC), or NULL */
  const uint32_t* lt_index;  /* [device] im_lt_index_size(E) entries from im_prepare_graph
                                (LT), or NULL (the kept edge is then found by binary
                                search; the sets are the same either way) */
} im_graph;

/* Sampling statistics of one im_sample_rrr call.  The counts are exact and
 * deterministic; the times are device times of the three launches, taken
 * with HIP events on `stream` (only when statistics are requested). */
typedef struct {
  int64_t total;           /* sum of set sizes */
  int64_t examined;        /* IC: in-edges examined; LT: binary-search probes
                              charged as ceil(log2(indeg+1)) per expanded vertex */
  int64_t live;            /* IC: live in-edges found; LT: in-edges taken */
  int64_t large_sets;      /* sets finished by the large-set launch: those that
                              outgrew the main launch's LDS tier, and those not yet
                              started when its last batch was claimed (this part
                              depends on timing; the sets themselves do not) */
  int64_t large_total;     /* ... their summed sizes */
  int64_t large_examined;  /* ... their examined count */
  int64_t large_live;      /* ... their live count */
  int64_t redo_examined;   /* in-edges the main launch examined in rounds it
                              abandoned when handing a set to the large path */
  double ms_main;          /* main sampling launch (small IC sets, or LT walks) */
  double ms_large;         /* large-set launch (0 if none) */
  double ms_canon;         /* size scan + gather into the canonical CSR */
} im_sample_stats;

/* Library version string. */
const char* im_version(void);
/* Text of the calling thread's last error: a failed HIP call, a short
 * workspace or arena ("" if none). */
const char* im_last_error(void);
/* Waits for the current device and releases the calling thread's captured
 * cover graphs (IM_TUNE_GRAPH).  The caller must ensure no call is in flight. */
int im_release(void);

/* Entry points whose workspace im_workspace_size() reports. */
typedef enum {
  IM_WS_PREPARE_GRAPH = 0,  /* im_prepare_graph */
  IM_WS_SAMPLE = 1,         /* im_sample_rrr: n, model, count, total = capacity */
  IM_WS_INCIDENCE = 2,      /* im_build_incidence: n, total */
  IM_WS_GREEDY = 3,         /* im_greedy_cover: n, count, k */
  IM_WS_RANDGREEDI = 4,     /* im_randgreedi: n, count, total, k, m */
  IM_WS_STREAM = 5,         /* im_stream_cover: count, k, m, delta (alpha = 1 bound) */
  IM_WS_OFFLINE = 6,        /* im_greedi_offline: n, count, k, m */
  IM_WS_FORWARD = 7,        /* im_prepare_forward: n */
  IM_WS_INFLUENCE = 8,      /* im_influence: n, count = nsims, k = nseeds */
  IM_WS_SOLVE = 9,          /* im_solve: n, model, count = theta, total, k, selector, m, delta */
  IM_WS_OPIM = 10,          /* im_opim: as im_solve, count = samples per half */
  IM_WS_BATCH = 11          /* im_solve_batch: ntasks, n = sum of vertices, count = sum of
                               theta, total, k = largest k, model (LT if any) */
} im_ws_op;

/* A problem shape for im_workspace_size.  Fields an op does not list are
 * ignored.  total is the sum of set sizes; where it is not known yet (IMM,
 * OPIM, batches) an estimate, e.g. count times the mean set size of a small
 * sample.  full = 1 asks for room for the fastest launch shapes (every
 * large-set worker up to 16 GiB, one round of covering subsets); 0 for the
 * least the op runs in.  num_cus: compute units of the device the call will
 * run on, or 0 for the current device. */
typedef struct {
  int32_t n;
  int32_t model;
  int64_t count;
  int64_t total;
  int32_t k;
  int32_t m;
  double delta;
  int32_t selector;
  int32_t ntasks;
  int32_t full;
  int32_t num_cus;
} im_ws_shape;

/* Bytes of workspace to pass for `op` on `shape` (host only, except that
 * num_cus = 0 queries the current device).  For im_solve, im_opim and
 * im_solve_batch it is an estimate from shape->total; the calls report
 * IM_ENOMEM and im_workspace_need() when it falls short. */
int im_workspace_size(int32_t op, const im_ws_shape* shape, size_t* bytes);
/* For the calling thread's last call with a workspace: *need = the bytes it
 * needed at least if it returned IM_ENOMEM for its workspace (else 0);
 * *want = the bytes that would have let it take its fastest launch shapes
 * (at least what it used: more large-set workers, one round of covering
 * subsets).  Either pointer may be NULL, not both. */
int im_workspace_need(size_t* need, size_t* want);

/*
 * Launch-shape knobs (the batched and served paths' tile choices; the
 * autotuner in the Python package sets them from measurements).  No setting
 * changes any result: the sets, seeds, gains and coverage are the same bit
 * for bit, only the time differs.  Process-wide; read at each call.
 *   IM_TUNE_SAMPLE_BLOCKS  workgroups (4 wavefronts) per CU of the main IC
 *                          sampling launch, 1..64 (default 5: as many as are
 *                          resident at once, so none starts late)
 *   IM_TUNE_BIG_SHAPE      large-set launch: 1 one wavefront per set (24 per
 *                          CU), 2 256 threads per set (8 per CU), 0 automatic
 *                          (one wavefront unless more than 1/8 of the
 *                          launch's sets were handed off) (default 0)
 *   IM_TUNE_APPLY_BLOCKS   workgroups (1024 threads) per CU of the plain
 *                          greedy's aggregated apply, 1..16 (default 1)
 *   IM_TUNE_DENSE_RATIO    members per vertex above which the covering
 *                          subsets take the dense form, >= 0 (0: always
 *                          dense; default 256)
 *   IM_TUNE_LT_BLOCKS      workgroups (4 wavefronts, one walk per lane) per CU
 *                          of the LT sampling launch, 1..32 (default 2: half of
 *                          the four wavefronts per SIMD the walk kernel is
 *                          built for, so that work of other streams runs beside
 *                          it; each lane holds 4 KiB of walk list in the
 *                          workspace)
 *   IM_TUNE_GRAPH          1: a cover's 2k + 2 launches (greedy, RandGreedi local
 *                          step, offline aggregation, batch) are captured into a
 *                          hipGraph once per launch shape and replayed (updated
 *                          with each call's arguments) as one submission; 0:
 *                          launched one by one (default 0: measured no faster,
 *                          the launches already run back to back)
 *   IM_TUNE_LT_GRAB        sample ids an LT wavefront claims at once, 1..4096
 *                          (default 16: with 256 only ~1,250 wavefronts of a
 *                          320 K-walk launch get work; 16 spreads it over all)
 *   IM_TUNE_LISTS          1: the RandGreedi local step (partitions of at
 *                          most 2^18 positions on average) finds each pick
 *                          from a per-partition list of the highest counts,
 *                          one workgroup per partition, scanning a partition
 *                          only when its list can no longer decide; 0: every
 *                          pick scans all counts over the whole device
 *                          (default 1)
 * value -1 restores the default.  Returns IM_EINVAL for an unknown key or a
 * value outside its range (nothing changes then).  im_tune_get writes the
 * value in effect.
 */
typedef enum {
  IM_TUNE_SAMPLE_BLOCKS = 0,
  IM_TUNE_BIG_SHAPE = 1,
  IM_TUNE_APPLY_BLOCKS = 2,
  IM_TUNE_DENSE_RATIO = 3,
  IM_TUNE_LT_BLOCKS = 4,
  IM_TUNE_LT_GRAB = 5,
  IM_TUNE_GRAPH = 6,
  IM_TUNE_LISTS = 7
} im_tune_key;
int im_tune_set(int32_t key, int64_t value);
int im_tune_get(int32_t key, int64_t* value);

/*
 * Graph ingest (Sec. 2: the IC and LT diffusion models).
 * weight[e] is the IC probability p(u,v) in [0,1], or the LT weight w(u,v) >= 0
 * (the model assumes the in-weights of a vertex sum to 1).  Writes thr:
 *  IC: thr[e] = p >= 1 ? 0xFFFFFFFF : floor(p * 2^32); edge e of sample i is
 *      live iff thr[e] == 0xFFFFFFFF or draw(edge, i, e) < thr[e].
 *  LT: q_e = w >= 1 ? 2^32 : floor(w * 2^32); thr[e] = min(sum of q over the
 *      in-edges of v up to and including e, 0xFFFFFFFF) (live-edge reading of
 *      LT: v keeps in-edge e with probability w_e, none with 1 - sum w).
 *  thr[E .. round_up(E,4)) is written 0.
 *  LT search index (lt_index may be NULL): level k = 1..7 holds, for every
 *      window of 16^k consecutive edge ids, the threshold of its last edge
 *      (of edge E-1 for the final partial window), padded to whole groups of
 *      16 entries (64 bytes), levels one after the other.  The sampler finds
 *      the kept in-edge of v by a 16-ary search: one 64-byte group per level
 *      from the lowest level whose window holds all of v's in-edges, down to
 *      the edges themselves -- about log16(indeg) + 1 dependent loads instead
 *      of log2(indeg).
 *  IC run-length table (skip may be NULL: one coin per in-edge everywhere):
 *      skip[v] = 1 / log(1 - q/2^32) when v has >= 2 in-edges that all share
 *      one threshold q with 0 < q < 0xFFFFFFFF (weighted cascade gives every
 *      vertex this shape), else 0.  For such a vertex the sampler generates
 *      its live in-edges by geometric gaps G = floor(log(U) * skip[v]) (U on
 *      (0,1] from 53 bits of draw pair j of (sample, v): counter (v, i,
 *      2^31 | j/2, stream)) instead of one coin per in-edge -- the same
 *      Bernoulli(p) sequence in distribution.  log is a fixed sequence of
 *      IEEE basic operations (exponent split, fold into [sqrt(1/2),
 *      sqrt(2)), odd atanh series to s^19), so results are reproducible
 *      bit for bit.
 * in_off [device] n+1; in_src [device] E; weight [device] E fp32;
 * thr [device] round_up(E,4); skip [device] n fp64 or NULL (ignored for LT);
 * lt_index [device] im_lt_index_size(E) uint32 or NULL (ignored for IC);
 * ws [device] 256 bytes.  Synchronises `stream`; returns IM_EINVAL if
 * in_off is not a valid CSR offset array (nothing else is then read), or if a
 * source id is outside [0,n), or a weight is NaN, negative, infinite, or (IC)
 * above 1 (thr is then partly written and must not be used).
 */
int im_prepare_graph(int32_t n, int64_t num_edges, const int32_t* in_off, const int32_t* in_src,
                     const float* weight, int32_t model, uint32_t* thr, double* skip,
                     uint32_t* lt_index, void* ws, size_t ws_bytes, void* stream);
/* Entries of the LT search index for num_edges edges (host only):
 * sum over k = 1..7 of round_up(ceil(E / 16^k), 16). */
int im_lt_index_size(int64_t num_edges, int64_t* entries);

/*
 * RRR sampling (Def. 2.3 and Sec. 2.1; Alg. 1 Sample, Alg. 3 sampling step).
 * Generates the sets of sample ids [first, first+count) of (seed, stream_tag):
 *  root_i = floor(draw(root, i) * n / 2^32) (uniform over V);
 *  IC: R(i) = vertices with a path to root_i over edges live in sample i
 *      (coins per in-edge, or run-length gaps where g->skip marks a vertex);
 *  LT: R(i) = the chain root_i <- u1 <- u2 ... where each vertex keeps the
 *      first in-edge e with draw(vertex, i, v) < thr[e] (or thr[e] saturated),
 *      ending at a vertex that keeps none or at a repeated vertex.
 * Output (sample-major CSR, canonical): off [device] count+1 int64 with
 * off[0] = 0; mem [device] capacity int32, set j = sample first+j occupies
 * mem[off[j] .. off[j+1]) with members strictly ascending.
 * *total [host] receives the sum of set sizes.  If it exceeds capacity the
 * call returns IM_ERANGE, off is written, mem is left undefined, and a repeat
 * with capacity >= *total returns bit-identical output.  stats [host] may be
 * NULL.  first + count <= 2^32.  The workspace stages the sets before they
 * are placed (about 4.5 bytes per member of capacity plus 16 per set) and
 * holds the large-set workers (4.125 n bytes each, at least one).
 * Synchronises `stream`.
 */
int im_sample_rrr(const im_graph* g, uint64_t seed, uint32_t stream_tag, int64_t first,
                  int64_t count, int64_t* off, int32_t* mem, int64_t capacity, int64_t* total,
                  im_sample_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Covering subsets (Sec. 3.2; Alg. 3 per-vertex step): S(v) = {j : v in R(j)}
 * for the count sets in (off, mem), j local indices in [0, count).
 * inc_off [device] n+1 int64; inc_mem [device] off[count] int32.  The order of
 * the ids inside one S(v) is unspecified (S(v) is a set).  Members must lie in
 * [0, n) (the caller's contract; sets from im_sample_rrr do).  Collections of
 * at most 256 members per vertex (the environment variable
 * IM_INCIDENCE_DENSE_RATIO changes that bound) are transposed through LDS
 * histograms: the workspace holds 8 bytes per member of one round (at least
 * 2^24 members), and a collection larger than the workspace allows is
 * transposed in rounds of vertex-id ranges (IM_INCIDENCE_PAIR_BUDGET, a member
 * count, lowers that cap; the round split synchronises `stream` once).
 * Denser collections over at most 4 x 32768 vertex ids count and place
 * members in LDS tiles of 32768 ids (8 bytes of workspace per vertex;
 * IM_INCIDENCE_DENSE_TILES=0 turns that form off); wider ones take one global
 * atomic per member and pass.  Otherwise asynchronous.
 */
int im_build_incidence(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                       int64_t total, int64_t* inc_off, int32_t* inc_mem, void* ws,
                       size_t ws_bytes, void* stream);

/*
 * Standard greedy max-k-cover (Sec. 3.2): k times take the vertex v of largest
 * marginal coverage |S(v) minus covered|, the lowest id on ties; stop early
 * when the largest gain is 0.  Universe = the count samples.
 * Inputs from im_sample_rrr / im_build_incidence (total = off[count]).
 * seeds [device] k int32 (entries past nsel set to -1); gains [device] k int64
 * (0 past nsel); nsel [device] 1 int32; coverage [device] 1 int64 = C(S).
 * Workspace: 4n + count + 8k bytes and change.  Asynchronous.
 */
int im_greedy_cover(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                    int64_t total, const int64_t* inc_off, const int32_t* inc_mem, int32_t k,
                    int32_t* seeds, int64_t* gains, int32_t* nsel, int64_t* coverage,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * im_greedy_cover without a workspace, for callers that cannot allocate
 * device memory: code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments (no ws), operation and
 * outputs as im_greedy_cover (bit-identical results).  Its scratch -- 64 + 8*round_up(k,8)
 * + 4n + count bytes: argmax keys, per-vertex counts, covered flags -- lives
 * in a fixed 64 MiB device array that each GPU the library runs on holds
 * until the process ends; a call needing more returns IM_ENOMEM (the sizes
 * are in im_last_error()) before any device work.  The array is looked up
 * once per device (hipGetSymbolAddress) on the first call there.  Every call
 * on one GPU shares that GPU's array and reinitialises it on `stream`, so
 * calls that overlap on one GPU (different streams, or concurrent host
 * threads) race and must not be issued.  Asynchronous; no memset nodes.
 */
int im_greedy_cover_static(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                           int64_t total, const int64_t* inc_off, const int32_t* inc_mem,
                           int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel,
                           int64_t* coverage, void* stream);

/*
 * RandGreedi local step (Alg. 3 partition step; Alg. 4, local greedy step; Sec. 3.4 S3).
 * Partitions V uniformly at random into m parts, part(v) = floor(draw(part,
 * v) * m / 2^32) with key part_seed, and runs the standard greedy above on
 * every part p with candidates V_p and the full universe, all m in one
 * launch, recording all k picks.  part [device] n uint8 (written);
 * lseeds [device] m*k int32, row p = part p's picks in order, -1 past
 * lcount[p]; lgains [device] m*k int64; lcount [device] m int32;
 * lcover [device] m int64 = C(S_p).  1 <= m <= 256.  Workspace: 12n + m count
 * + 4 total + 8mk bytes and change (the count position of every member is
 * stored beside the members once, so the local steps' member walks find the
 * partition and the count without random lookups).  Asynchronous.
 */
int im_randgreedi(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                  int64_t total, const int64_t* inc_off, const int32_t* inc_mem, int32_t k,
                  int32_t m, uint64_t part_seed, uint8_t* part, int32_t* lseeds, int64_t* lgains,
                  int32_t* lcount, int64_t* lcover, void* ws, size_t ws_bytes, void* stream);

/*
 * Streaming max-k-cover at the receiver (Alg. 5), truncation (Sec. 3.3.2) and
 * the final choice of Alg. 4.
 *  Stream: T = ceil(alpha*k) (clamped to [1,k]); for t < T, for p < m, the
 *   item lseeds[p][t] if t < lcount[p], carrying the full S(x).
 *  Buckets: l = max |S(x)| over the stream; B = max(1, ceil(ln k / ln(1+delta)));
 *   thr_b = ceil(l * (1+delta)^b / (2k)); bucket b takes x iff it holds < k
 *   seeds and |S(x) minus C_b| >= thr_b; b* = lowest bucket of largest |C_b|.
 *  Final: S = S_b* if |C_b*| >= max_p lcover[p], else the lowest p of largest
 *   lcover.
 * seeds [device] k int32 (-1 past nsel); nsel [device] 1; coverage [device] 1
 * int64; info [device] 4 int32 = {b*, B, global solution chosen (1/0), stream
 * length}.  0 < delta < 1/2, 0 < alpha <= 1.  Workspace: the stream (20 bytes
 * per item) and the buckets' seeds, plus B count / 8 bytes of bucket bitmaps
 * when count exceeds what LDS holds (1,179,648 samples).  Asynchronous.
 */
int im_stream_cover(int32_t n, int64_t count, const int64_t* inc_off, const int32_t* inc_mem,
                    int32_t k, int32_t m, const int32_t* lseeds, const int32_t* lcount,
                    const int64_t* lcover, double delta, double alpha, int32_t* seeds,
                    int32_t* nsel, int64_t* coverage, int32_t* info, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * RandGreedi's global step without streaming, the offline GreeDI aggregation
 * (Alg. 4: the local solutions are gathered, Alg. 2 lazy greedy selects among
 * their union, then the final choice).  Gathered: the first T = ceil(alpha*k)
 * picks of every part (clamped to [1,k]; all k at alpha = 1), i.e. row p of
 * lseeds up to min(T, lcount[p]), from im_randgreedi.  The global solution
 * S_g is the standard greedy (lowest id on ties, stop at zero gain -- the
 * same picks as Alg. 2) with those vertices as candidates and all count
 * samples as universe.  Final: S = S_g if C(S_g) >= max_p lcover[p], else
 * the lowest p of largest lcover.
 * seeds [device] k int32 (-1 past nsel); nsel [device] 1; coverage [device] 1
 * int64; info [device] 4 int32 = {global solution chosen (1/0), vertices
 * gathered, |S_g|, best local partition}; gcover [device] 1 int64 = C(S_g),
 * or NULL.  0 < alpha <= 1, 1 <= m <= 256.  Workspace: 4n + count + 8mk
 * bytes and change.  Reads lcount back to size the launches (synchronises
 * `stream` once); otherwise asynchronous.
 */
int im_greedi_offline(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                      int64_t total, const int64_t* inc_off, const int32_t* inc_mem, int32_t k,
                      int32_t m, const int32_t* lseeds, const int32_t* lcount,
                      const int64_t* lcover, double alpha, int32_t* seeds, int32_t* nsel,
                      int64_t* coverage, int32_t* info, int64_t* gcover, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * Forward view of a graph for influence simulation: the in-edge ids grouped
 * by source.  out_off [device] n+1 int64 (out_off[u] .. out_off[u+1] index
 * out_eid); out_eid [device] E int32, the in-edge ids e with in_src[e] = u
 * (order inside a source unspecified); edge_dst [device] E int32, the
 * vertex whose in-edge list holds e.  Workspace: 8n bytes and change.
 * Synchronises `stream`.
 */
int im_prepare_forward(int32_t n, int64_t num_edges, const int32_t* in_off, const int32_t* in_src,
                       int64_t* out_off, int32_t* out_eid, int32_t* edge_dst, void* ws,
                       size_t ws_bytes, void* stream);

/*
 * Forward Monte-Carlo influence of a seed set -- the paper's quality measure
 * (Sec. 4.1: mean number of vertices the diffusion model activates from the
 * seeds over simulations).  Simulation r draws one live-edge world of the
 * model (the live-edge reading of Sec. 2's IC and LT models) from its own
 * domains, independent of the RRR samples:
 *  IC: in-edge e is live iff thr[e] == 0xFFFFFFFF or draw(sim edge 4, r, e) < thr[e];
 *  LT: vertex v keeps its first in-edge j with thr[j] > draw(sim vertex 5, r, v)
 *      or thr[j] saturated (none if no such j).
 * Activated = every vertex reachable from a seed over live edges, seeds
 * included (duplicates once).  counts [device] nsims int64: the activated
 * count of simulations r = first .. first+nsims-1 of (seed, stream_tag).
 * seeds [host] nseeds ids in [0, n) (else IM_EINVAL).  out_off / out_eid /
 * edge_dst from im_prepare_forward on the same graph.  first + nsims <= 2^32.
 * Workspace: 16 simulations at a time, 16.125 n bytes each.  Synchronises
 * `stream` (once per batch of 16 levels of the search).
 */
int im_influence(const im_graph* g, const int64_t* out_off, const int32_t* out_eid,
                 const int32_t* edge_dst, uint64_t seed, uint32_t stream_tag, int64_t first,
                 int64_t nsims, const int32_t* seeds, int32_t nseeds, int64_t* counts, void* ws,
                 size_t ws_bytes, void* stream);

/* IMM sample-size schedule (host values; see im_solve). */
typedef struct {
  double ell, eps_prime, log_binom, lambda_prime, lambda_star;
  int64_t theta1;   /* samples of the first martingale round */
  int32_t rounds;   /* floor(log2 n) - 1 */
} im_imm_plan_t;

/* The fp64 IMM bounds im_solve uses (Alg. 1 with Tang et al. 2015), so that a
 * caller driving the rounds itself (e.g. over resident sample pools) takes
 * exactly the same decisions.  Host only; 2 <= n, 1 <= k <= n, 0 < eps < 1. */
int im_imm_plan(int32_t n, int32_t k, double eps, im_imm_plan_t* out);

/* One martingale round's test of Alg. 1 (the bounds of im_solve): after
 * round x (1-based) selected seeds covering `coverage` of its theta_x
 * samples, stop = 1 and lb = n C / (theta_x (1 + eps')) when
 * n C / theta_x >= (1 + eps') n / 2^x; else stop = 0, lb = 1.  Host only. */
int im_imm_round(const im_imm_plan_t* plan, int32_t n, int32_t round, int64_t theta_x,
                 int64_t coverage, int32_t* stop, double* lb);
/* The final sample count of Alg. 1: theta = ceil(lambda_star / lb).  Host only. */
int im_imm_theta(const im_imm_plan_t* plan, double lb, int64_t* theta);

/* Options of im_solve. */
typedef struct {
  int32_t selector;      /* IM_SEL_GREEDY, IM_SEL_GREEDIRIS or IM_SEL_RANDGREEDI */
  int32_t m;             /* partitions (GreediRIS, RandGreedi), 1..256 */
  double delta;          /* bucket spacing (GreediRIS), 0 < delta < 1/2 */
  double alpha;          /* truncation fraction (GreediRIS: streamed picks per part;
                            RandGreedi: gathered picks per part), 0 < alpha <= 1 */
  uint64_t seed;         /* sampling seed */
  uint64_t part_seed;    /* partition seed (GreediRIS) */
  int64_t theta;         /* > 0: use this many samples and skip the IMM bound */
} im_solve_opts;

/* Result of im_solve (host). */
typedef struct {
  int32_t nsel;
  int64_t coverage;            /* C(S) over the final theta samples */
  int64_t theta;               /* final sample count */
  int32_t rounds;              /* martingale rounds run */
  double lower_bound;          /* LB of Alg. 1 (1.0 if never certified) */
  int64_t martingale_samples;  /* samples drawn in the martingale rounds */
  int32_t bucket;              /* b* of the last GreediRIS selection, else -1 */
  int32_t global_won;          /* 1 if the streamed solution won, 0 if local, -1 n/a */
  int32_t stream_len;          /* seeds streamed (GreediRIS) or gathered (RandGreedi) in
                                  the last selection, else 0 */
  int64_t final_total;         /* sum of set sizes of the final samples */
  /* Sampling and selection tally of the whole call (martingale rounds and
   * final samples).  Each pool extension samples its new sets once; the
   * counters are exact (as im_sample_stats), the times are device times of
   * the launches from HIP events on `stream`. */
  int32_t sample_launches;     /* sampling calls (pool extensions) */
  int32_t sample_passes;       /* main sampling launches (> launches only if a
                                  staging arena was short and a call sampled again) */
  int64_t sampled_sets, sampled_total, sampled_examined, sampled_live;
  double ms_sample_main;       /* main sampling launches (LT walks, or small IC sets) */
  double ms_sample_large;      /* large-set launches */
  double ms_sample_gather;     /* copies into the canonical pools */
  double ms_select;            /* covering subsets + selection, every round */
  double ms_incidence;         /* ... of which covering subsets */
  double ms_local;             /* ... standard greedy, or partition + local greedy */
  double ms_global;            /* ... streaming cover or offline aggregation + final choice */
  int64_t global_cover;        /* C(S_g) of the last RandGreedi selection, else -1 */
} im_solve_result;

/*
 * IMM (Alg. 1), with the sample-size bounds of Tang, Shi and Xiao (2015):
 * ell = 1 + ln2/ln n; eps' = sqrt(2) eps; lambda' = (2 + 2eps'/3)(ln C(n,k)
 * + ell ln n + ln log2 n) n / eps'^2; round x = 1 .. floor(log2 n) - 1 uses
 * theta_x = ceil(2 lambda'/n) * 2^(x-1) samples of stream 0 (earlier samples
 * kept, Sec. 3.2), selects S_x, and stops with LB = n C(S_x) / (theta_x
 * (1+eps')) once n C(S_x)/theta_x >= (1+eps') n / 2^x; then theta =
 * ceil(lambda_star / LB), lambda_star = 2n((1-1/e) a + b)^2/eps^2, a = sqrt(ell ln n +
 * ln 2), b = sqrt((1-1/e)(ln C(n,k) + ell ln n + ln 2)), and the final seeds
 * are selected on theta fresh samples of stream 1.  The selector is the
 * standard greedy, GreediRIS (im_randgreedi + im_stream_cover) or RandGreedi
 * with the offline global step (im_randgreedi + im_greedi_offline).
 * seeds [host] k int32; res [host].  The sample pools live in the workspace
 * (a pool, its covering subsets and the staging of its newest sets: about
 * 20 bytes per member at the final theta; IM_WS_SOLVE).  Synchronises `stream`.
 */
int im_solve(const im_graph* g, int32_t k, double eps, const im_solve_opts* opts,
             int32_t* seeds, im_solve_result* res, void* ws, size_t ws_bytes, void* stream);

/* Result of im_opim (host). */
typedef struct {
  int32_t nsel;
  int32_t rounds;
  int64_t theta;        /* samples per half (R1 and R2 each) in the last round */
  int64_t cover1;       /* C(S*) on R1 */
  int64_t cover2;       /* C(S*) on R2 */
  int64_t upper1;       /* upper bound on the optimum's coverage of R1 */
  double lower;         /* lower bound on sigma(S*) */
  double upper;         /* upper bound on sigma(OPT) */
  double guarantee;     /* lower / upper: the instance-wise approximation guarantee */
  double theta_max;
  int32_t i_max;
  int32_t bucket;       /* b* of the last GreediRIS selection, else -1 */
  int32_t global_won;   /* as in im_solve_result */
} im_opim_result;

/*
 * OPIM, the online RIS method the paper extends GreediRIS to (Sec. 3.3,
 * closing paragraph; Sec. 4.4), with the OPIM-C bounds of Tang, Tang, Xiao
 * and Yuan (2018).  Each round holds two independent halves of theta sets,
 * R1 (stream 0) and R2 (stream 1), doubled from round to round (earlier
 * samples kept); S* is selected on R1 by opts->selector (as in im_solve) and
 * validated on R2.  With a = ln(3 i_max / fail), in fp64:
 *   theta_max = 2n((1-1/e) sqrt(ln(6/fail)) + sqrt((1-1/e)(ln C(n,k) + ln(6/fail))))^2
 *               / (eps^2 k);   theta_1 = ceil(theta_max eps^2 k / n);
 *   i_max = max(1, ceil(log2(theta_max / theta_1)));
 *   U = min(sum of the k largest |S_R1(v)|, C_R1(S*) + sum of the k largest
 *       marginals |S_R1(v) minus covered|) -- an upper bound on the optimum's
 *       coverage of R1 for any selector, by submodularity;
 *   lower = ((sqrt(C_R2(S*) + 2a/9) - sqrt(a/2))^2 - a/18) n / theta;
 *   upper = (sqrt(U + a/2) + sqrt(a/2))^2 n / theta;  guarantee = lower / upper.
 * Stops when guarantee >= 1 - 1/e - eps, at round i_max, or once the two
 * halves together hold theta_cap samples or more (the paper's runs stop at
 * 2^20).  0 < eps < 1, 0 < fail < 1.  seeds [host] k int32 (-1 past nsel);
 * res [host].  opts->theta is ignored.  Both halves and their covering
 * subsets live in the workspace (IM_WS_OPIM).  Synchronises `stream`.
 */
int im_opim(const im_graph* g, int32_t k, double eps, double fail, int64_t theta_cap,
            const im_solve_opts* opts, int32_t* seeds, im_opim_result* res, void* ws,
            size_t ws_bytes, void* stream);

/* One task of a batch: theta samples [0, theta) of (seed, stream_tag) on a
 * prepared graph, then the standard greedy with k picks. */
typedef struct {
  im_graph graph;
  uint64_t seed;
  uint32_t stream_tag;
  int32_t k;
  int64_t theta;
} im_task;

/* Batch statistics (sums over the tasks; device times from HIP events). */
typedef struct {
  int64_t sets, total, examined, live;
  double ms_sample, ms_incidence, ms_cover;
} im_batch_stats;

/*
 * Batched sampling and greedy cover over many independent tasks (the same
 * operations as im_sample_rrr, im_build_incidence and im_greedy_cover of
 * Sec. 2.1 and 3.2, per task): all IC tasks share one sampling launch, all LT
 * tasks another, covering subsets of every task are built together, and the
 * greedy picks of every task run in the same launches.  Task t's results are
 * bit-identical to those three calls on task t alone.
 * tasks [host] ntasks; seeds [device] and gains [device] hold sum_t k_t
 * entries, task t's at offset sum_{u<t} k_u (-1 / 0 past its nsel);
 * nsel [device] ntasks int32; coverage [device] ntasks int64; stats [host]
 * may be NULL.  Tasks are processed 256 at a time, each group's sets,
 * covering subsets and counts in the workspace (IM_WS_BATCH).  Synchronises
 * `stream`.
 */
int im_solve_batch(const im_task* tasks, int32_t ntasks, int32_t* seeds, int64_t* gains,
                   int32_t* nsel, int64_t* coverage, im_batch_stats* stats, void* ws,
                   size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* IM_H */
