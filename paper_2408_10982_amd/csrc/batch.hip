// batch.hip -- many independent (graph, seed, k, theta) tasks in one set of
// launches (im_solve_batch).
//
// The tasks' samples are laid out one after the other in one canonical CSR,
// their vertices one after the other in one count array, and every task
// becomes one partition of the greedy launches (own vertex range, own
// samples, own k).  All IC tasks are sampled by one launch and all LT tasks
// by another; covering subsets of all tasks are built by one transpose
// (vertices of task t at vbase[t] + id); the greedy runs max k picks for all
// tasks together.
// Each task's seeds are therefore exactly those of im_sample_rrr +
// im_build_incidence + im_greedy_cover on that task alone.
#include <algorithm>
#include <vector>

#include "common.h"
#include "cover.h"
#include "incidence.h"
#include "sample.h"

namespace im {

// Records that the whole call needs `bytes`, if the workspace is smaller
// (defined with the other workspace bookkeeping in runtime.hip).
void scratch_need_whole(size_t bytes);

// tables | off | inc_off | cnt | covered | gmax | done
static size_t batch_bytes(int32_t nt, int64_t S, int64_t V, int32_t max_k) {
  const size_t tab = (size_t)(nt + 1) * 16 + (size_t)nt * 12 + 256;
  return ws_align(tab + (size_t)(S + 1) * 8 + (size_t)(V + 1) * 8 + (size_t)V * 4 + (size_t)S +
                  (size_t)max_k * nt * 8 + 64 + 8 * 64);
}

static int batch_chunk(const im_task* tasks, int32_t nt, int64_t out_base, int32_t* seeds,
                       int64_t* gains, int32_t* nsel, int64_t* coverage, im_batch_stats* st,
                       hipStream_t s) {
  DeviceInfo di;
  IM_TRY(device_info(&di));
  std::vector<TaskDesc> td(nt);
  std::vector<int64_t> sb(nt + 1), vb(nt + 1), ko(nt);
  std::vector<int32_t> kp(nt);
  int64_t S = 0, V = 0, K = out_base;
  int32_t max_n = 1, max_k = 1, model = IM_IC;
  for (int t = 0; t < nt; ++t) {
    const im_task& q = tasks[t];
    sb[t] = S;
    vb[t] = V;
    ko[t] = K;
    kp[t] = q.k;
    td[t] = task_of(&q.graph, q.seed, q.stream_tag, 0, q.theta, S);
    S += q.theta;
    V += q.graph.n;
    K += q.k;
    max_n = std::max(max_n, q.graph.n);
    max_k = std::max(max_k, q.k);
    if (q.graph.model == IM_LT) model = IM_LT;
  }
  sb[nt] = S;
  vb[nt] = V;
  if (S >= ((int64_t)1 << 32) || V >= ((int64_t)1 << 31)) return IM_EINVAL;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotBatch, batch_bytes(nt, S, V, max_k), &p));
  char* c = (char*)p;
  auto take = [&](size_t b) {
    char* r = c;
    c += (b + 63) / 64 * 64;
    return r;
  };
  int64_t* d_sb = (int64_t*)take((size_t)(nt + 1) * 8);
  int64_t* d_vb = (int64_t*)take((size_t)(nt + 1) * 8);
  int64_t* d_ko = (int64_t*)take((size_t)nt * 8);
  int32_t* d_kp = (int32_t*)take((size_t)nt * 4);
  int64_t* off = (int64_t*)take((size_t)(S + 1) * 8);
  int64_t* inc_off = (int64_t*)take((size_t)(V + 1) * 8);
  uint32_t* cnt = (uint32_t*)take((size_t)V * 4);
  uint8_t* covered = (uint8_t*)take((size_t)S);
  unsigned long long* gmax = (unsigned long long*)take((size_t)max_k * nt * 8);
  int32_t* done = (int32_t*)take(64);
  IM_HIP(hipMemcpyAsync(d_sb, sb.data(), (size_t)(nt + 1) * 8, hipMemcpyHostToDevice, s));
  IM_HIP(hipMemcpyAsync(d_vb, vb.data(), (size_t)(nt + 1) * 8, hipMemcpyHostToDevice, s));
  IM_HIP(hipMemcpyAsync(d_ko, ko.data(), (size_t)nt * 8, hipMemcpyHostToDevice, s));
  IM_HIP(hipMemcpyAsync(d_kp, kp.data(), (size_t)nt * 4, hipMemcpyHostToDevice, s));

  hipEvent_t ev[4];
  for (auto& e : ev) IM_HIP(hipEventCreate(&e));
  struct G {
    hipEvent_t* e;
    ~G() {
      for (int j = 0; j < 4; ++j) (void)hipEventDestroy(e[j]);
    }
  } guard{ev};
  // sampling: the sets are staged in the arena, then gathered into a member
  // buffer of exactly their total.  The arena is sized from the member total
  // of this thread's previous batch (a short arena means sampling the batch
  // again; the total is kept as soon as it is counted, also when the call
  // then runs short of workspace and is repeated); results do not depend on it
  static thread_local int64_t last_total = 0;
  ArenaRun R;
  IM_HIP(hipEventRecord(ev[0], s));
  const int rc = sample_to_arena(td.data(), nt, S, max_n, off, last_total, 0, true, false, &R, s);
  if (R.total > 0) {
    last_total = R.total;
    // with the member total known, a workspace too small for the rest of the
    // call is reported with the size of the whole call, so that the caller
    // grows it once instead of once per stage (each growth repeats the call)
    scratch_need_whole(ws_batch(di.num_cus, nt, S, V, R.total, max_n, max_k, model, false));
  }
  IM_TRY(rc);
  const int64_t total = R.total;
  void* mp = nullptr;
  IM_TRY(scratch(s, kSlotBatchMem, (size_t)std::max<int64_t>(total, 1) * 4, &mp));
  int32_t* mem = (int32_t*)mp;
  IM_TRY(gather_arena(R, off, mem, nullptr, s));
  release_sampling();
  IM_HIP(hipEventRecord(ev[1], s));
  // covering subsets of every task, by global vertex position
  void* ip = nullptr;
  IM_TRY(scratch(s, kSlotBatchInc, (size_t)std::max<int64_t>(total, 1) * 4, &ip));
  int32_t* inc_mem = (int32_t*)ip;
  const IncSrc src{off, S, mem, total, d_sb, d_vb, nt, max_n};
  IM_TRY(build_incidence(src, (int32_t)V, inc_off, inc_mem, s));
  IM_HIP(hipEventRecord(ev[2], s));
  // greedy on every task at once
  CoverArgs A{};
  A.n = (int32_t)V;
  A.m = nt;
  A.count = S;
  A.k = max_k;
  A.off = off;
  A.mem = mem;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.pbase = d_vb;
  A.kpart = d_kp;
  A.koff = d_ko;
  A.sbase = d_sb;
  A.local_ids = 1;
  A.cnt = cnt;
  A.covered = covered;
  A.gmax = gmax;
  A.done = done;
  A.seeds = seeds;
  A.gains = gains;
  A.nsel = nsel;
  A.cover = coverage;
  IM_HIP(hipMemsetAsync(gains + out_base, 0, (size_t)(K - out_base) * 8, s));
  IM_TRY(launch_cover(A, s));
  IM_HIP(hipEventRecord(ev[3], s));
  IM_HIP(hipStreamSynchronize(s));
  if (st) {
    float a = 0.f, b = 0.f, c2 = 0.f;
    IM_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
    IM_HIP(hipEventElapsedTime(&b, ev[1], ev[2]));
    IM_HIP(hipEventElapsedTime(&c2, ev[2], ev[3]));
    st->sets += S;
    st->total += total;
    st->examined += R.examined;
    st->live += R.live;
    st->ms_sample += a;
    st->ms_incidence += b;
    st->ms_cover += c2;
  }
  return IM_OK;
}

size_t ws_batch(int num_cus, int32_t nt, int64_t S, int64_t V, int64_t total, int32_t max_n,
                int32_t max_k, int32_t model, bool full) {
  if (nt <= 0) return 0;
  const size_t own = batch_bytes(nt, S, V, max_k) + ws_align((size_t)std::max<int64_t>(total, 1) * 4);
  const size_t inc = ws_align((size_t)std::max<int64_t>(total, 1) * 4) +
                     ws_incidence((int32_t)std::min<int64_t>(V, INT32_MAX), total, nt, full);
  return own + std::max(ws_sample(num_cus, S, total, max_n, model, full), inc);
}

}  // namespace im

extern "C" int im_solve_batch(const im_task* tasks, int32_t ntasks, int32_t* seeds,
                              int64_t* gains, int32_t* nsel, int64_t* coverage,
                              im_batch_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  using namespace im;
  if (!tasks || ntasks <= 0 || !seeds || !gains || !nsel || !coverage) return IM_EINVAL;
  int64_t S = 0, V = 0;
  int32_t max_n = 1, max_k = 1, model = IM_IC;
  for (int32_t t = 0; t < ntasks; ++t) {
    const im_task& q = tasks[t];
    if (!graph_ok(&q.graph) || q.k <= 0 || q.theta < 0 || q.theta >= ((int64_t)1 << 32))
      return IM_EINVAL;
    if (t < kMaxParts) {  // the first chunk: a lower bound for the whole call
      S += q.theta;
      V += q.graph.n;
    }
    max_n = std::max(max_n, q.graph.n);
    max_k = std::max(max_k, q.k);
    if (q.graph.model == IM_LT) model = IM_LT;
  }
  DeviceInfo di;
  IM_TRY(device_info(&di));
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_batch(di.num_cus, std::min(ntasks, kMaxParts), S, V, S, max_n, max_k, model,
                            false)))
    return IM_ENOMEM;
  if (stats) *stats = im_batch_stats{};
  hipStream_t s = (hipStream_t)stream;
  int64_t out = 0;
  for (int32_t c0 = 0; c0 < ntasks; c0 += kMaxParts) {
    const int32_t nt = std::min<int32_t>(kMaxParts, ntasks - c0);
    IM_TRY(batch_chunk(tasks + c0, nt, out, seeds, gains, nsel + c0, coverage + c0, stats, s));
    for (int32_t t = 0; t < nt; ++t) out += tasks[c0 + t].k;
  }
  return IM_OK;
}
