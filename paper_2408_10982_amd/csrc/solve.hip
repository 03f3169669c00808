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
#include "sample.h"

namespace im {

__global__ void k_add_base(int64_t* __restrict__ off, int64_t n, int64_t base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) off[i] += base;
}

// A growable device pool of RRR sets owned by one im_solve call.
struct Pool {
  int64_t count = 0, total = 0;
  int64_t cap_sets = 0, cap_mem = 0;
  int64_t* off = nullptr;
  int32_t* mem = nullptr;
  ~Pool() {
    if (off) (void)hipFree(off);
    if (mem) (void)hipFree(mem);
  }
};

static int grow(void** p, size_t old_bytes, size_t new_bytes, hipStream_t s) {
  void* q = nullptr;
  if (hipMalloc(&q, new_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return IM_ENOMEM;
  }
  if (*p) {
    if (old_bytes) IM_HIP(hipMemcpyAsync(q, *p, old_bytes, hipMemcpyDeviceToDevice, s));
    IM_HIP(hipStreamSynchronize(s));
    IM_HIP(hipFree(*p));
  }
  *p = q;
  return IM_OK;
}

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
    int64_t nc = std::max<int64_t>(want + 1, P.cap_sets * 2);
    IM_TRY(grow((void**)&P.off, (size_t)(P.count + 1) * 8, (size_t)nc * 8, s));
    P.cap_sets = nc;
  }
  if (P.count == 0) IM_HIP(hipMemsetAsync(P.off, 0, 8, s));
  const int64_t add = want - P.count;
  const TaskDesc T = task_of(g, seed, tag, P.count, add, 0);
  ArenaRun R;
  const int64_t expect = mean_hint > 0.0 ? (int64_t)(mean_hint * (double)add) : 0;
  IM_TRY(sample_to_arena(&T, 1, add, g->n, P.off + P.count, expect, false, true, &R, s));
  if (P.cap_mem - P.total < R.total) {
    const int64_t nc = std::max<int64_t>(P.total + R.total + R.total / 4, P.cap_mem * 2);
    IM_TRY(grow((void**)&P.mem, (size_t)P.total * 4, (size_t)std::max<int64_t>(nc, 1) * 4, s));
    P.cap_mem = nc;
  }
  double ms_g = 0.0;
  IM_TRY(gather_arena(R, P.off + P.count, P.mem + P.total, &ms_g, s));
  if (P.total > 0) {
    k_add_base<<<dim3((unsigned)((add + 1 + 255) / 256)), dim3(256), 0, s>>>(P.off + P.count,
                                                                           add + 1, P.total);
    IM_HIP(hipGetLastError());
  }
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
  IM_TRY(im_build_incidence(n, P.count, P.off, P.mem, P.total, inc_off, inc_mem, s));
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
                           (int64_t*)pg, d_nsel, d_cov, s));
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
                         part, lseeds, lgains, lcount, lcover, s));
    IM_HIP(hipEventRecord(ev[2], s));
    if (o->selector == IM_SEL_GREEDIRIS)
      IM_TRY(im_stream_cover(n, P.count, inc_off, inc_mem, k, m, lseeds, lcount, lcover, o->delta,
                             o->alpha, d_seeds, d_nsel, d_cov, d_info, s));
    else
      IM_TRY(im_greedi_offline(n, P.count, P.off, P.mem, P.total, inc_off, inc_mem, k, m, lseeds,
                               lcount, lcover, o->alpha, d_seeds, d_nsel, d_cov, d_info, d_gcov,
                               s));
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

extern "C" int im_solve(const im_graph* g, int32_t k, double eps, const im_solve_opts* o,
                        int32_t* seeds, im_solve_result* res, void* stream) {
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
  const double nd = (double)n;
  im_imm_plan_t plan;
  IM_TRY(im_imm_plan(n, k, eps, &plan));
  const double eps_p = plan.eps_prime;
  const double lambda_s = plan.lambda_star;
  const int32_t rounds = plan.rounds;

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
    Pool P;
    int64_t th = plan.theta1;
    for (int32_t i = 1; i <= rounds; ++i) {
      if (i > 1) th *= 2;
      if (th >= ((int64_t)1 << 31)) return IM_ERANGE;
      IM_TRY(pool_extend(P, g, o->seed, 0u, th, mean, &tally, s));
      mean = (double)P.total / (double)P.count;
      IM_TRY(select_on(P, n, k, o, &sel, &tally, s));
      res->rounds = i;
      const double x = nd / ldexp(1.0, i);
      if (nd * (double)sel.coverage / (double)th >= (1.0 + eps_p) * x) {
        lb = nd * (double)sel.coverage / ((double)th * (1.0 + eps_p));
        break;
      }
    }
    res->martingale_samples = P.count;
    theta = (int64_t)ceil(lambda_s / lb);
  }
  if (theta >= ((int64_t)1 << 31)) return IM_ERANGE;
  Pool F;
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
