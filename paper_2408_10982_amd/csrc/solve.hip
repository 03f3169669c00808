// solve.hip -- the IMM driver (im_solve; Alg. 1 with the GreediRIS selector of
// Alg. 3/4/5 or the standard greedy).
//
// Host logic only: it grows a device-resident pool of RRR sets by sample-id
// range (earlier samples are kept across martingale rounds, Sec. 3.2),
// rebuilds the covering subsets, runs the selector on the device and reads
// back the coverage for the lower-bound test.  The fp64 bounds follow IMM
// (Tang, Shi and Xiao 2015); the final seeds come from theta fresh samples
// of a second stream (the Sample(G, theta) line of Alg. 1).
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "cover.h"
#include "incidence.h"
#include "sample.h"

namespace im {

__global__ void k_add_base(int64_t* __restrict__ off, int64_t n, int64_t base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) off[i] += base;
}

// A growable pool of RRR sets owned by one im_solve or im_opim call, held in
// two workspace slots (offsets and members) that are returned when the pool
// goes out of scope.
struct Pool {
  int32_t slot_off, slot_mem;
  int64_t count = 0, total = 0;
  int64_t cap_sets = 0, cap_mem = 0;
  int64_t* off = nullptr;
  int32_t* mem = nullptr;
  Pool(int32_t so, int32_t sm) : slot_off(so), slot_mem(sm) {}
  ~Pool() {
    scratch_release(slot_off);
    scratch_release(slot_mem);
  }
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
};

// Device times and exact counters of the sampling and selection calls of
// one im_solve.
struct SolveTally {
  int32_t launches = 0, passes = 0;
  int64_t sets = 0, total = 0, examined = 0, live = 0;
  double ms_main = 0.0, ms_large = 0.0, ms_gather = 0.0, ms_select = 0.0;
  double ms_inc = 0.0, ms_local = 0.0, ms_global = 0.0;
};

// Extends the pool to sets [0, want).  The new sets are sampled once into
// the staging arena; if the pool's member buffer is too small it grows and
// the sets are then copied in (sampling is never repeated for capacity).
static int pool_extend(Pool& P, const im_graph* g, uint64_t seed, uint32_t tag, int64_t want,
                       double mean_hint, SolveTally* tally, hipStream_t s) {
  if (want <= P.count) return IM_OK;
  if (want + 1 > P.cap_sets) {
    const int64_t nc = want + 1;
    void* p = nullptr;
    IM_TRY(scratch_grow(s, P.slot_off, P.count > 0 ? (size_t)(P.count + 1) * 8 : 0,
                        (size_t)nc * 8, &p));
    P.off = (int64_t*)p;
    P.cap_sets = nc;
  }
  if (P.count == 0) IM_HIP(hipMemsetAsync(P.off, 0, 8, s));
  const int64_t add = want - P.count;
  const TaskDesc T = task_of(g, seed, tag, P.count, add, 0);
  ArenaRun R;
  const int64_t expect = mean_hint > 0.0 ? (int64_t)(mean_hint * (double)add) : 0;
  IM_TRY(sample_to_arena(&T, 1, add, g->n, P.off + P.count, expect, 0, false, true, &R, s));
  if (P.cap_mem - P.total < R.total || !P.mem) {
    const int64_t nc = P.total + R.total;
    void* p = nullptr;
    IM_TRY(scratch_grow(s, P.slot_mem, (size_t)P.total * 4, (size_t)std::max<int64_t>(nc, 1) * 4,
                        &p));
    P.mem = (int32_t*)p;
    P.cap_mem = nc;
  }
  double ms_g = 0.0;
  IM_TRY(gather_arena(R, P.off + P.count, P.mem + P.total, &ms_g, s));
  if (P.total > 0) {
    k_add_base<<<dim3((unsigned)((add + 1 + 255) / 256)), dim3(256), 0, s>>>(P.off + P.count,
                                                                           add + 1, P.total);
    IM_HIP(hipGetLastError());
  }
  release_sampling();
  P.total += R.total;
  P.count = want;
  if (tally) {
    tally->launches += 1;
    tally->passes += R.passes;
    tally->sets += add;
    tally->total += R.total;
    tally->examined += R.examined;
    tally->live += R.live;
    tally->ms_main += R.ms_main;
    tally->ms_large += R.ms_large;
    tally->ms_gather += ms_g;
  }
  return IM_OK;
}

struct Selection {
  std::vector<int32_t> seeds;
  int32_t nsel = 0;
  int64_t coverage = 0;
  int32_t bucket = -1;
  int32_t global_won = -1;
  int32_t stream_len = 0;
  int64_t global_cover = -1;
};

static int select_on(const Pool& P, int32_t n, int32_t k, const im_solve_opts* o,
                     Selection* out, SolveTally* tally, hipStream_t s) {
  void *pio = nullptr, *pim = nullptr, *pout = nullptr;
  hipEvent_t ev[4];
  for (auto& e : ev) IM_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int j = 0; j < 4; ++j) (void)hipEventDestroy(e[j]);
    }
  } ev_guard{ev};
  IM_HIP(hipEventRecord(ev[0], s));
  IM_TRY(scratch(s, kSlotSolveIncOff, (size_t)(n + 1) * 8, &pio));
  IM_TRY(scratch(s, kSlotSolveInc, (size_t)std::max<int64_t>(P.total, 1) * 4, &pim));
  int64_t* inc_off = (int64_t*)pio;
  int32_t* inc_mem = (int32_t*)pim;
  IM_TRY(im_build_incidence(n, P.count, P.off, P.mem, P.total, inc_off, inc_mem, nullptr, 0, s));
  IM_HIP(hipEventRecord(ev[1], s));
  // outputs: seeds k, coverage, nsel, info 4, global cover
  IM_TRY(scratch(s, kSlotSolveOut, (size_t)k * 12 + 128, &pout));
  int32_t* d_seeds = (int32_t*)pout;
  int64_t* d_cov = (int64_t*)((char*)pout + ((size_t)k * 4 + 7) / 8 * 8);
  int32_t* d_nsel = (int32_t*)(d_cov + 1);
  int32_t* d_info = d_nsel + 2;
  int64_t* d_gcov = (int64_t*)(d_info + 4);
  out->seeds.assign(k, -1);
  if (o->selector == IM_SEL_GREEDY) {
    void* pg = nullptr;
    IM_TRY(scratch(s, kSlotSolveLocal, (size_t)k * 8, &pg));
    IM_TRY(im_greedy_cover(n, P.count, P.off, P.mem, P.total, inc_off, inc_mem, k, d_seeds,
                           (int64_t*)pg, d_nsel, d_cov, nullptr, 0, s));
    IM_HIP(hipEventRecord(ev[2], s));
  } else {
    const int32_t m = o->m;
    void* pl = nullptr;
    const size_t lbytes = (size_t)n + 64 + (size_t)m * k * 12 + (size_t)m * 12 + 64;
    IM_TRY(scratch(s, kSlotSolveLocal, lbytes, &pl));
    int64_t* lgains = (int64_t*)pl;
    int64_t* lcover = lgains + (size_t)m * k;
    int32_t* lseeds = (int32_t*)(lcover + m);
    int32_t* lcount = lseeds + (size_t)m * k;
    uint8_t* part = (uint8_t*)(lcount + m);
    IM_TRY(im_randgreedi(n, P.count, P.off, P.mem, P.total, inc_off, inc_mem, k, m, o->part_seed,
                         part, lseeds, lgains, lcount, lcover, nullptr, 0, s));
    IM_HIP(hipEventRecord(ev[2], s));
    if (o->selector == IM_SEL_GREEDIRIS)
      IM_TRY(im_stream_cover(n, P.count, inc_off, inc_mem, k, m, lseeds, lcount, lcover, o->delta,
                             o->alpha, d_seeds, d_nsel, d_cov, d_info, nullptr, 0, s));
    else
      IM_TRY(im_greedi_offline(n, P.count, P.off, P.mem, P.total, inc_off, inc_mem, k, m, lseeds,
                               lcount, lcover, o->alpha, d_seeds, d_nsel, d_cov, d_info, d_gcov,
                               nullptr, 0, s));
  }
  IM_HIP(hipEventRecord(ev[3], s));
  int32_t h_nsel = 0, h_info[4] = {-1, 0, -1, 0};
  int64_t h_cov = 0, h_gcov = -1;
  IM_HIP(hipMemcpyAsync(out->seeds.data(), d_seeds, (size_t)k * 4, hipMemcpyDeviceToHost, s));
  IM_HIP(hipMemcpyAsync(&h_nsel, d_nsel, 4, hipMemcpyDeviceToHost, s));
  IM_HIP(hipMemcpyAsync(&h_cov, d_cov, 8, hipMemcpyDeviceToHost, s));
  if (o->selector != IM_SEL_GREEDY)
    IM_HIP(hipMemcpyAsync(h_info, d_info, 16, hipMemcpyDeviceToHost, s));
  if (o->selector == IM_SEL_RANDGREEDI)
    IM_HIP(hipMemcpyAsync(&h_gcov, d_gcov, 8, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  float t_inc = 0.f, t_loc = 0.f, t_glob = 0.f;
  IM_HIP(hipEventElapsedTime(&t_inc, ev[0], ev[1]));
  IM_HIP(hipEventElapsedTime(&t_loc, ev[1], ev[2]));
  IM_HIP(hipEventElapsedTime(&t_glob, ev[2], ev[3]));
  if (tally) {
    tally->ms_select += (double)t_inc + t_loc + t_glob;
    tally->ms_inc += t_inc;
    tally->ms_local += t_loc;
    tally->ms_global += t_glob;
  }
  out->nsel = h_nsel;
  out->coverage = h_cov;
  out->bucket = -1;
  out->global_won = -1;
  out->stream_len = 0;
  out->global_cover = h_gcov;
  if (o->selector == IM_SEL_GREEDIRIS) {
    out->bucket = h_info[0];
    out->global_won = h_info[2];
    out->stream_len = h_info[3];
  } else if (o->selector == IM_SEL_RANDGREEDI) {
    out->global_won = h_info[0];
    out->stream_len = h_info[1];
  }
  return IM_OK;
}

// ------------------------------------------------------------------ OPIM
// Quantities of one OPIM round on a pool's covering subsets: the samples a
// seed set covers, the per-vertex marginals |S(v) minus covered| and sums of
// the k largest of them.
constexpr int kOpBlock = 256;

__global__ void k_op_fill_u8(uint8_t* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0;
}

// flags[i] = 1 for every sample i of S(s), s a seed (one workgroup per seed).
__global__ __launch_bounds__(kOpBlock) void k_op_mark(const int64_t* __restrict__ inc_off,
                                                      const int32_t* __restrict__ inc_mem,
                                                      const int32_t* __restrict__ seeds,
                                                      uint8_t* __restrict__ flags) {
  const int32_t v = seeds[blockIdx.x];
  for (int64_t t = inc_off[v] + threadIdx.x; t < inc_off[v + 1]; t += kOpBlock)
    flags[inc_mem[t]] = 1;
}

__global__ __launch_bounds__(kOpBlock) void k_op_count(const uint8_t* __restrict__ flags,
                                                       int64_t n,
                                                       unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[kOpBlock / kWave];
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kOpBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOpBlock)
    c += flags[i];
  c = wave_sum(c);
  if (lane_id() == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int q = 0; q < kOpBlock / kWave; ++q) s += red[q];
    if (s) atomicAdd(out, s);
  }
}

// marg[v] = |S(v)| minus the samples of S(v) flagged covered: a wavefront
// takes 64 vertices and walks their subsets end to end, 64 entries a step.
__global__ __launch_bounds__(kOpBlock) void k_op_marginals(int32_t n,
                                                           const int64_t* __restrict__ inc_off,
                                                           const int32_t* __restrict__ inc_mem,
                                                           const uint8_t* __restrict__ flags,
                                                           uint32_t* __restrict__ marg) {
  __shared__ int64_t wpre[kOpBlock / kWave][kWave];
  __shared__ uint32_t wcnt[kOpBlock / kWave][kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int64_t wid = ((int64_t)blockIdx.x * kOpBlock + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * kOpBlock / kWave;
  for (int64_t v0 = wid * kWave; v0 < n; v0 += nw * kWave) {  // wavefront-uniform
    const int64_t v = v0 + lane;
    int64_t a = 0, sz = 0;
    if (v < n) {
      a = inc_off[v];
      sz = inc_off[v + 1] - a;
    }
    const int64_t incl = wave_inclusive_scan(sz);
    const int64_t total = __shfl(incl, kWave - 1, kWave);
    const int64_t first = __shfl(a, 0, kWave);  // the 64 subsets are consecutive
    wpre[w][lane] = incl;
    wcnt[w][lane] = 0u;
    wave_sync();
    for (int64_t f = lane; f < total; f += kWave) {
      int lo = 0, hi = kWave - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (wpre[w][mid] > f)
          hi = mid;
        else
          lo = mid + 1;
      }
      if (!flags[inc_mem[first + f]]) atomicAdd(&wcnt[w][lo], 1u);
    }
    wave_sync();
    if (v < n) marg[v] = wcnt[w][lane];
    wave_sync();
  }
}

// Histogram of the digit (x >> shift) & dmask over the values whose bits
// above the digit equal `prefix` (mask selects those bits).
__global__ __launch_bounds__(kOpBlock) void k_op_hist(const uint32_t* __restrict__ x, int32_t n,
                                                      int shift, uint32_t dmask, uint32_t mask,
                                                      uint32_t prefix,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ uint32_t h[2048];
  for (int j = threadIdx.x; j < 2048; j += kOpBlock) h[j] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kOpBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOpBlock) {
    const uint32_t y = x[i];
    if ((y & mask) == prefix) atomicAdd(&h[(y >> shift) & dmask], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < 2048; j += kOpBlock)
    if (h[j]) atomicAdd(&hist[j], (unsigned long long)h[j]);
}

// Sum and count of the values above t.
__global__ __launch_bounds__(kOpBlock) void k_op_above(const uint32_t* __restrict__ x, int32_t n,
                                                       uint32_t t,
                                                       unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[2][kOpBlock / kWave];
  unsigned long long s = 0, c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kOpBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOpBlock) {
    const uint32_t y = x[i];
    if (y > t) {
      s += y;
      ++c;
    }
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = s;
    red[1][threadIdx.x / kWave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0;
    for (int q = 0; q < kOpBlock / kWave; ++q) {
      a += red[0][q];
      b += red[1][q];
    }
    if (a) atomicAdd(&out[0], a);
    if (b) atomicAdd(&out[1], b);
  }
}

// Sum of the k largest of x[0..n) (k <= n): the k-th largest value t by a
// three-digit radix select (11 + 11 + 10 bits, a histogram per digit), then
// the values above t plus t for the remaining places.
static int top_k_sum(const uint32_t* x, int32_t n, int32_t k, unsigned long long* dwork,
                     int64_t* out, hipStream_t s) {
  DeviceInfo di;
  IM_TRY(device_info(&di));
  const unsigned grid = (unsigned)di.num_cus * 4;
  std::vector<unsigned long long> h(2048);
  uint32_t prefix = 0, mask = 0;
  int64_t need = k;  // rank of t among the values matching the prefix
  const int shifts[3] = {21, 10, 0};
  const int widths[3] = {11, 11, 10};
  for (int d = 0; d < 3; ++d) {
    IM_HIP(hipMemsetAsync(dwork, 0, 2048 * 8, s));
    const uint32_t dmask = (1u << widths[d]) - 1u;
    k_op_hist<<<dim3(grid), dim3(kOpBlock), 0, s>>>(x, n, shifts[d], dmask, mask, prefix, dwork);
    IM_HIP(hipGetLastError());
    IM_HIP(hipMemcpyAsync(h.data(), dwork, 2048 * 8, hipMemcpyDeviceToHost, s));
    IM_HIP(hipStreamSynchronize(s));
    int b = (1 << widths[d]) - 1;
    for (; b > 0; --b) {
      if ((int64_t)h[b] >= need) break;
      need -= (int64_t)h[b];
    }
    prefix |= (uint32_t)b << shifts[d];
    mask |= (uint32_t)((1u << widths[d]) - 1u) << shifts[d];
  }
  const uint32_t t = prefix;
  IM_HIP(hipMemsetAsync(dwork, 0, 16, s));
  k_op_above<<<dim3(grid), dim3(kOpBlock), 0, s>>>(x, n, t, dwork);
  IM_HIP(hipGetLastError());
  unsigned long long sc[2] = {0, 0};
  IM_HIP(hipMemcpyAsync(sc, dwork, 16, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  *out = (int64_t)sc[0] + ((int64_t)k - (int64_t)sc[1]) * (int64_t)t;
  return IM_OK;
}

// Samples of a pool's covering subsets that a seed set covers, and (if
// marg is given) every vertex's marginal coverage given the set.
static int cover_and_marginals(int32_t n, int64_t count, const int64_t* inc_off,
                               const int32_t* inc_mem, const int32_t* d_seeds, int32_t nseeds,
                               uint8_t* flags, unsigned long long* dwork, int64_t* covered,
                               uint32_t* marg, hipStream_t s) {
  DeviceInfo di;
  IM_TRY(device_info(&di));
  const unsigned grid = (unsigned)di.num_cus * 4;
  k_op_fill_u8<<<dim3(grid), dim3(kOpBlock), 0, s>>>(flags, count);
  if (nseeds > 0) k_op_mark<<<dim3((unsigned)nseeds), dim3(kOpBlock), 0, s>>>(inc_off, inc_mem,
                                                                            d_seeds, flags);
  IM_HIP(hipMemsetAsync(dwork, 0, 8, s));
  k_op_count<<<dim3(grid), dim3(kOpBlock), 0, s>>>(flags, count, dwork);
  IM_HIP(hipGetLastError());
  if (marg) {
    k_op_marginals<<<dim3((unsigned)di.num_cus * 8), dim3(kOpBlock), 0, s>>>(n, inc_off, inc_mem,
                                                                            flags, marg);
    IM_HIP(hipGetLastError());
  }
  unsigned long long c = 0;
  IM_HIP(hipMemcpyAsync(&c, dwork, 8, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  *covered = (int64_t)c;
  return IM_OK;
}

// Workspace of the selection on a pool of `count` sets and `total` members:
// the covering subsets and their build, the outputs, the local step and the
// selector's own scratch.
static size_t ws_select(int32_t n, int64_t count, int64_t total, int32_t k, int32_t selector,
                        int32_t m, double delta, bool full) {
  size_t b = ws_align((size_t)(n + 1) * 8) + ws_align((size_t)std::max<int64_t>(total, 1) * 4) +
             ws_align((size_t)k * 12 + 128);
  size_t inner = ws_incidence(n, total, 0, full);
  if (selector == IM_SEL_GREEDY) {
    b += ws_align((size_t)k * 8);
    inner = std::max(inner, ws_greedy(n, count, k));
  } else {
    b += ws_align((size_t)n + 64 + (size_t)m * k * 12 + (size_t)m * 12 + 64);
    const size_t global = selector == IM_SEL_GREEDIRIS ? ws_stream(n, count, k, m, delta)
                                                       : ws_offline(n, count, k, m);
    // the local step's scratch stays while the global step runs
    inner = std::max(inner, ws_randgreedi(n, count, total, k, m) + global);
  }
  return b + inner;
}

// Workspace of a pool of `count` sets with `total` members.
static size_t ws_pool(int64_t count, int64_t total) {
  return ws_align((size_t)(count + 1) * 8) + ws_align((size_t)std::max<int64_t>(total, 1) * 4);
}

size_t ws_solve(int num_cus, int32_t n, int32_t model, int64_t count, int64_t total, int32_t k,
                int32_t selector, int32_t m, double delta, bool full) {
  const size_t pool = ws_pool(count, total);
  const size_t samp = ws_sample(num_cus, count, total, n, model, full);
  const size_t sel = ws_select(n, count, total, k, selector, m, delta, full);
  // one pool at a time; a grown pool is copied from its previous region
  return pool + pool / 2 + std::max(samp, sel) + ((size_t)1 << 20);
}

size_t ws_opim(int num_cus, int32_t n, int32_t model, int64_t count, int64_t total, int32_t k,
               int32_t selector, int32_t m, double delta, bool full) {
  const size_t pool = ws_pool(count, total);
  const size_t samp = ws_sample(num_cus, count, total, n, model, full);
  // both pools, R1's covering subsets kept while R2's are built, flags and marginals
  const size_t sel = ws_select(n, count, total, k, selector, m, delta, full) +
                     ws_align((size_t)(n + 1) * 8) + ws_align((size_t)std::max<int64_t>(total, 1) * 4) +
                     ws_align((size_t)count + 256) + ws_align((size_t)n * 4 + 2048 * 8 + (size_t)k * 4 + 256);
  return 2 * (pool + pool / 2) + std::max(samp, sel) + ((size_t)1 << 20);
}

}  // namespace im

extern "C" int im_imm_plan(int32_t n, int32_t k, double eps, im_imm_plan_t* out) {
  if (n <= 1 || k <= 0 || k > n || !(eps > 0.0 && eps < 1.0) || !out) return IM_EINVAL;
  // IMM bounds (fp64, fixed order)
  const double nd = (double)n;
  const double ln_n = log(nd);
  const double ell = 1.0 * (1.0 + log(2.0) / ln_n);
  const double eps_p = sqrt(2.0) * eps;
  double lbin = 0.0;
  for (int32_t i = 0; i < k; ++i) lbin += log(nd - (double)i);
  for (int32_t i = 1; i <= k; ++i) lbin -= log((double)i);
  const double lambda_p =
      (2.0 + 2.0 * eps_p / 3.0) * (lbin + ell * ln_n + log(log2(nd))) * nd / (eps_p * eps_p);
  const double e1 = 1.0 - exp(-1.0);
  const double a_i = sqrt(ell * ln_n + log(2.0));
  const double b_i = sqrt(e1 * (lbin + ell * ln_n + log(2.0)));
  const double sm = e1 * a_i + b_i;
  out->ell = ell;
  out->eps_prime = eps_p;
  out->log_binom = lbin;
  out->lambda_prime = lambda_p;
  out->lambda_star = 2.0 * nd * sm * sm / (eps * eps);
  out->theta1 = (int64_t)ceil(lambda_p / (nd / 2.0));
  int32_t lg = 0;
  while (((int64_t)1 << (lg + 1)) <= (int64_t)n) ++lg;
  out->rounds = lg - 1;
  return IM_OK;
}

extern "C" int im_imm_round(const im_imm_plan_t* plan, int32_t n, int32_t round, int64_t theta_x,
                            int64_t coverage, int32_t* stop, double* lb) {
  if (!plan || !stop || !lb || n <= 1 || round < 1 || theta_x <= 0 || coverage < 0)
    return IM_EINVAL;
  const double nd = (double)n;
  const double x = nd / ldexp(1.0, round);
  if (nd * (double)coverage / (double)theta_x >= (1.0 + plan->eps_prime) * x) {
    *stop = 1;
    *lb = nd * (double)coverage / ((double)theta_x * (1.0 + plan->eps_prime));
  } else {
    *stop = 0;
    *lb = 1.0;
  }
  return IM_OK;
}

extern "C" int im_imm_theta(const im_imm_plan_t* plan, double lb, int64_t* theta) {
  if (!plan || !theta || !(lb > 0.0)) return IM_EINVAL;
  *theta = (int64_t)ceil(plan->lambda_star / lb);
  return IM_OK;
}

extern "C" int im_solve(const im_graph* g, int32_t k, double eps, const im_solve_opts* o,
                        int32_t* seeds, im_solve_result* res, void* ws, size_t ws_bytes,
                        void* stream) {
  using namespace im;
  if (!g || !o || !seeds || !res || k <= 0 || g->n <= 1 || k > g->n || !(eps > 0.0 && eps < 1.0) ||
      (o->selector != IM_SEL_GREEDY && o->selector != IM_SEL_GREEDIRIS &&
       o->selector != IM_SEL_RANDGREEDI) ||
      o->theta < 0)
    return IM_EINVAL;
  if (o->selector != IM_SEL_GREEDY &&
      (o->m < 1 || o->m > 256 || !(o->alpha > 0.0 && o->alpha <= 1.0) ||
       (o->selector == IM_SEL_GREEDIRIS && !(o->delta > 0.0 && o->delta < 0.5))))
    return IM_EINVAL;
  if (g->model != IM_IC && g->model != IM_LT) return IM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int32_t n = g->n;
  im_imm_plan_t plan;
  IM_TRY(im_imm_plan(n, k, eps, &plan));
  const int32_t rounds = plan.rounds;
  DeviceInfo di;
  IM_TRY(device_info(&di));
  // at least the first round's pool with one member per set
  WsScope scope(ws, ws_bytes);
  const int64_t first = o->theta > 0 ? o->theta : plan.theta1;
  if (!scope.check(ws_solve(di.num_cus, n, g->model, first, first, k, o->selector, o->m, o->delta,
                            false)))
    return IM_ENOMEM;

  *res = im_solve_result{};
  res->bucket = -1;
  res->global_won = -1;
  double lb = 1.0;
  int64_t theta;
  Selection sel;
  SolveTally tally;
  double mean = 0.0;  // mean set size seen so far (sizes the next arena)
  if (o->theta > 0) {
    theta = o->theta;
  } else {
    Pool P(kSlotPoolOff0, kSlotPoolMem0);
    int64_t th = plan.theta1;
    for (int32_t i = 1; i <= rounds; ++i) {
      if (i > 1) th *= 2;
      if (th >= ((int64_t)1 << 31)) return IM_ERANGE;
      IM_TRY(pool_extend(P, g, o->seed, 0u, th, mean, &tally, s));
      mean = (double)P.total / (double)P.count;
      IM_TRY(select_on(P, n, k, o, &sel, &tally, s));
      res->rounds = i;
      int32_t stop = 0;
      double lbx = 1.0;
      IM_TRY(im_imm_round(&plan, n, i, th, sel.coverage, &stop, &lbx));
      if (stop) {
        lb = lbx;
        break;
      }
    }
    res->martingale_samples = P.count;
    IM_TRY(im_imm_theta(&plan, lb, &theta));
  }
  if (theta >= ((int64_t)1 << 31)) return IM_ERANGE;
  Pool F(kSlotPoolOff1, kSlotPoolMem1);
  IM_TRY(pool_extend(F, g, o->seed, 1u, theta, mean, &tally, s));
  IM_TRY(select_on(F, n, k, o, &sel, &tally, s));
  for (int32_t j = 0; j < k; ++j) seeds[j] = sel.seeds[j];
  res->nsel = sel.nsel;
  res->coverage = sel.coverage;
  res->theta = theta;
  res->lower_bound = lb;
  res->bucket = sel.bucket;
  res->global_won = sel.global_won;
  res->stream_len = sel.stream_len;
  res->final_total = F.total;
  res->sample_launches = tally.launches;
  res->sample_passes = tally.passes;
  res->sampled_sets = tally.sets;
  res->sampled_total = tally.total;
  res->sampled_examined = tally.examined;
  res->sampled_live = tally.live;
  res->ms_sample_main = tally.ms_main;
  res->ms_sample_large = tally.ms_large;
  res->ms_sample_gather = tally.ms_gather;
  res->ms_select = tally.ms_select;
  res->ms_incidence = tally.ms_inc;
  res->ms_local = tally.ms_local;
  res->ms_global = tally.ms_global;
  res->global_cover = sel.global_cover;
  return IM_OK;
}

extern "C" int im_opim(const im_graph* g, int32_t k, double eps, double fail, int64_t theta_cap,
                       const im_solve_opts* o, int32_t* seeds, im_opim_result* res, void* ws,
                       size_t ws_bytes, void* stream) {
  using namespace im;
  if (!g || !o || !seeds || !res || k <= 0 || g->n <= 1 || k > g->n ||
      !(eps > 0.0 && eps < 1.0) || !(fail > 0.0 && fail < 1.0) || theta_cap < 1 ||
      (o->selector != IM_SEL_GREEDY && o->selector != IM_SEL_GREEDIRIS &&
       o->selector != IM_SEL_RANDGREEDI))
    return IM_EINVAL;
  if (o->selector != IM_SEL_GREEDY &&
      (o->m < 1 || o->m > 256 || !(o->alpha > 0.0 && o->alpha <= 1.0) ||
       (o->selector == IM_SEL_GREEDIRIS && !(o->delta > 0.0 && o->delta < 0.5))))
    return IM_EINVAL;
  if (g->model != IM_IC && g->model != IM_LT) return IM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int32_t n = g->n;
  const double nd = (double)n;
  // the schedule and the confidence term (fp64, fixed order)
  const double e1 = 1.0 - exp(-1.0);
  double lbin = 0.0;
  for (int32_t i = 0; i < k; ++i) lbin += log(nd - (double)i);
  for (int32_t i = 1; i <= k; ++i) lbin -= log((double)i);
  const double l6 = log(6.0 / fail);
  const double tt = e1 * sqrt(l6) + sqrt(e1 * (lbin + l6));
  const double theta_max = 2.0 * nd * tt * tt / (eps * eps * (double)k);
  int64_t theta = (int64_t)ceil(theta_max * eps * eps * (double)k / nd);
  int32_t i_max = (int32_t)ceil(log2(theta_max / (double)theta));
  if (i_max < 1) i_max = 1;
  DeviceInfo di;
  IM_TRY(device_info(&di));
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_opim(di.num_cus, n, g->model, theta, theta, k, o->selector, o->m, o->delta,
                           false)))
    return IM_ENOMEM;
  const double a = log(3.0 * (double)i_max / fail);
  *res = im_opim_result{};
  res->theta_max = theta_max;
  res->i_max = i_max;
  res->bucket = -1;
  res->global_won = -1;
  Pool R1(kSlotPoolOff0, kSlotPoolMem0), R2(kSlotPoolOff1, kSlotPoolMem1);
  Selection sel;
  double mean = 0.0;
  for (int32_t i = 1;; ++i) {
    if (theta >= ((int64_t)1 << 31)) return IM_ERANGE;
    IM_TRY(pool_extend(R1, g, o->seed, 0u, theta, mean, nullptr, s));
    mean = (double)R1.total / (double)R1.count;
    IM_TRY(pool_extend(R2, g, o->seed, 1u, theta, mean, nullptr, s));
    IM_TRY(select_on(R1, n, k, o, &sel, nullptr, s));
    // select_on left R1's covering subsets in the stream's solve slots
    void *pio = nullptr, *pim = nullptr, *pw = nullptr;
    IM_TRY(scratch(s, kSlotSolveIncOff, (size_t)(n + 1) * 8, &pio));
    IM_TRY(scratch(s, kSlotSolveInc, (size_t)std::max<int64_t>(R1.total, 1) * 4, &pim));
    const int64_t* io1 = (const int64_t*)pio;
    const int32_t* im1 = (const int32_t*)pim;
    const size_t fl = ((size_t)std::max(R1.count, R2.count) + 256) / 256 * 256;
    const size_t wbytes = fl + (size_t)n * 4 + 2048 * 8 + (size_t)k * 4 + 256;
    IM_TRY(scratch(s, kSlotOpim, wbytes, &pw));
    uint8_t* flags = (uint8_t*)pw;
    uint32_t* marg = (uint32_t*)((char*)pw + fl);
    unsigned long long* dwork = (unsigned long long*)(marg + n);
    int32_t* d_seeds = (int32_t*)(dwork + 2048);
    IM_HIP(hipMemcpyAsync(d_seeds, sel.seeds.data(), (size_t)k * 4, hipMemcpyHostToDevice, s));
    // U = min(top-k |S(v)|, C_R1(S*) + top-k marginals given S*) on R1
    int64_t c0 = 0, u0 = 0, c1 = 0, u1 = 0;
    IM_TRY(cover_and_marginals(n, R1.count, io1, im1, d_seeds, 0, flags, dwork, &c0, marg, s));
    IM_TRY(top_k_sum(marg, n, k, dwork, &u0, s));
    IM_TRY(cover_and_marginals(n, R1.count, io1, im1, d_seeds, sel.nsel, flags, dwork, &c1, marg,
                               s));
    IM_TRY(top_k_sum(marg, n, k, dwork, &u1, s));
    const int64_t up1 = std::min(u0, sel.coverage + u1);
    // validation: the coverage of S* on R2
    void *pio2 = nullptr, *pim2 = nullptr;
    IM_TRY(scratch(s, kSlotOpimIncOff, (size_t)(n + 1) * 8, &pio2));
    IM_TRY(scratch(s, kSlotOpimInc, (size_t)std::max<int64_t>(R2.total, 1) * 4, &pim2));
    IM_TRY(im_build_incidence(n, R2.count, R2.off, R2.mem, R2.total, (int64_t*)pio2,
                              (int32_t*)pim2, nullptr, 0, s));
    int64_t c2 = 0;
    IM_TRY(cover_and_marginals(n, R2.count, (const int64_t*)pio2, (const int32_t*)pim2, d_seeds,
                               sel.nsel, flags, dwork, &c2, nullptr, s));
    const double th = (double)theta;
    const double x = sqrt((double)c2 + 2.0 * a / 9.0) - sqrt(a / 2.0);
    const double lower = (x * x - a / 18.0) * nd / th;
    const double y = sqrt((double)up1 + a / 2.0) + sqrt(a / 2.0);
    const double upper = y * y * nd / th;
    const double gq = lower / upper;
    res->nsel = sel.nsel;
    res->rounds = i;
    res->theta = theta;
    res->cover1 = sel.coverage;
    res->cover2 = c2;
    res->upper1 = up1;
    res->lower = lower;
    res->upper = upper;
    res->guarantee = gq;
    res->bucket = sel.bucket;
    res->global_won = sel.global_won;
    if (gq >= e1 - eps || i >= i_max || 2 * theta >= theta_cap) break;
    theta *= 2;
  }
  for (int32_t j = 0; j < k; ++j) seeds[j] = sel.seeds[j];
  return IM_OK;
}
