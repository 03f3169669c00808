// influence.hip -- forward Monte-Carlo influence of a seed set
// (im_prepare_forward, im_influence): the quality measure of Sec. 4.1, the
// mean number of vertices the diffusion model activates from the seeds.
//
// Simulation r is one live-edge world of the model, drawn from its own
// domains so that it is independent of the RRR samples: IC in-edge e is live
// iff its threshold is saturated or draw(sim edge, r, e) < thr[e]; under LT a
// vertex keeps its first in-edge whose inclusive prefix exceeds draw(sim
// vertex, r, v).  The activated set is everything reachable from the seeds
// over live edges, found by a level-synchronous forward BFS over out-edges
// (in-edge ids grouped by source) with one visited bitmap per simulation.  A
// batch of simulations shares each level's launch; a level's frontier is
// spread over the lanes of each wavefront by a prefix sum of out-degrees.
// The count of a simulation is a pure function of (seed, stream, r, seeds),
// so any launch shape gives the same integers.
#include <algorithm>
#include <vector>

#include "common.h"

namespace im {

constexpr uint32_t kTagSimEdge = 4, kTagSimVert = 5;
constexpr int kFwdBlock = 256;
constexpr int kSimBatch = 16;         // simulations per batch of level launches
constexpr int kLevelsPerCheck = 16;   // level launches between host checks

// ----------------------------------------------------------- forward CSR
__global__ void k_fwd_degree(int64_t E, const int32_t* __restrict__ in_src,
                             uint32_t* __restrict__ deg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) atomicAdd(&deg[in_src[e]], 1u);
}

__global__ void k_fwd_scatter(int64_t E, const int32_t* __restrict__ in_src,
                              const int64_t* __restrict__ out_off, uint32_t* __restrict__ fill,
                              int32_t* __restrict__ out_eid) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int32_t u = in_src[e];
  const uint32_t at = atomicAdd(&fill[u], 1u);
  out_eid[out_off[u] + at] = (int32_t)e;
}

// edge_dst[e] = v for the in-edges e of v (a wavefront per vertex group)
__global__ void k_fwd_dst(int32_t n, const int32_t* __restrict__ in_off,
                          int32_t* __restrict__ edge_dst) {
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  const int lane = lane_id();
  for (int64_t v = gw; v < n; v += nw)
    for (int32_t e = in_off[v] + lane; e < in_off[v + 1]; e += kWave) edge_dst[e] = (int32_t)v;
}

// ----------------------------------------------------------- simulation
struct FwdArgs {
  const int32_t* __restrict__ in_off;
  const uint32_t* __restrict__ thr;
  const int64_t* __restrict__ out_off;
  const int32_t* __restrict__ out_eid;
  const int32_t* __restrict__ edge_dst;
  int32_t n, model, nb;
  uint32_t seed_lo, seed_hi, stream, first;  // simulation ids first .. first+nb-1
  int64_t words;                             // bitmap words per simulation
  uint32_t* __restrict__ bits;               // nb bitmaps
  const uint64_t* __restrict__ cur;          // frontier: (sim << 32) | vertex
  uint64_t* __restrict__ next;
  unsigned long long* __restrict__ lvl;      // entries of the frontier of each level
  int32_t level;
};

__device__ __forceinline__ bool sim_live(const FwdArgs& A, uint32_t r, int32_t v, int32_t e) {
  if (A.model == IM_IC) {
    const uint32_t q = A.thr[e];
    if (q == 0xFFFFFFFFu) return true;
    const uint64_t seed = ((uint64_t)A.seed_hi << 32) | A.seed_lo;
    return draw1(seed, kTagSimEdge, A.stream, r, (uint32_t)e) < q;
  }
  const uint64_t seed = ((uint64_t)A.seed_hi << 32) | A.seed_lo;
  const uint32_t x = draw1(seed, kTagSimVert, A.stream, r, (uint32_t)v);
  int32_t lo = A.in_off[v], hi = A.in_off[v + 1];
  const int32_t end = hi;
  while (lo < hi) {  // first in-edge whose prefix passes x (or is saturated)
    const int32_t mid = lo + ((hi - lo) >> 1);
    const uint32_t c = A.thr[mid];
    if (c > x || c == 0xFFFFFFFFu)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo < end && lo == e;
}

// Marks v in simulation b; true if this call set the bit.
__device__ __forceinline__ bool mark(const FwdArgs& A, uint32_t b, int32_t v) {
  uint32_t* w = A.bits + (int64_t)b * A.words + ((uint32_t)v >> 5);
  const uint32_t bit = 1u << ((uint32_t)v & 31u);
  if (*w & bit) return false;  // bits are only ever set: a set bit is final
  return (atomicOr(w, bit) & bit) == 0u;
}

// Appends the lanes' new entries to the next frontier (one atomic per wave).
__device__ __forceinline__ void push(const FwdArgs& A, bool have, uint64_t entry) {
  const unsigned long long m = __ballot(have);
  if (!m) return;
  const int lane = lane_id();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&A.lvl[A.level + 1], (unsigned long long)__popcll(m));
  base = __shfl(base, 0, kWave);
  if (have) A.next[base + __popcll(m & ((1ull << lane) - 1ull))] = entry;
}

// The seeds of every simulation of the batch form level 0.
__global__ void k_fwd_seed(FwdArgs A, const int32_t* __restrict__ seeds, int32_t nseeds) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool have = false;
  uint64_t entry = 0;
  if (t < (int64_t)A.nb * nseeds) {
    const uint32_t b = (uint32_t)(t / nseeds);
    const int32_t s = seeds[t % nseeds];
    if (mark(A, b, s)) {
      have = true;
      entry = ((uint64_t)b << 32) | (uint32_t)s;
    }
  }
  push(A, have, entry);
}

// One BFS level for every simulation of the batch: a wavefront takes 64
// frontier entries, lays their out-edges end to end, and tests 64 at a time.
// Each lane's entry (out-edge base, simulation) and the inclusive prefix of
// the out-degrees sit in the wavefront's LDS rows, where any lane reads them.
__global__ __launch_bounds__(kFwdBlock) void k_fwd_level(FwdArgs A) {
  __shared__ int32_t wpre[kFwdBlock / kWave][kWave];
  __shared__ int64_t wbase[kFwdBlock / kWave][kWave];
  __shared__ uint32_t wsim[kFwdBlock / kWave][kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint64_t ncur = A.lvl[A.level];
  const int64_t wid = ((int64_t)blockIdx.x * kFwdBlock + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * kFwdBlock / kWave;
  for (int64_t c0 = wid * kWave; c0 < (int64_t)ncur; c0 += nw * kWave) {  // wavefront-uniform
    const int64_t idx = c0 + lane;
    uint32_t b = 0;
    int64_t a = 0;
    int32_t deg = 0;
    if (idx < (int64_t)ncur) {
      const uint64_t en = A.cur[idx];
      const int32_t u = (int32_t)(uint32_t)en;
      b = (uint32_t)(en >> 32);
      a = A.out_off[u];
      deg = (int32_t)(A.out_off[u + 1] - a);
    }
    const int32_t incl = wave_inclusive_scan(deg);
    const int32_t total = __shfl(incl, kWave - 1, kWave);
    wpre[w][lane] = incl;
    wbase[w][lane] = a;
    wsim[w][lane] = b;
    wave_sync();
    for (int32_t f0 = 0; f0 < total; f0 += kWave) {
      const int32_t f = f0 + lane;
      bool have = false;
      uint64_t entry = 0;
      if (f < total) {
        int lo = 0, hi = kWave - 1;  // first lane whose inclusive prefix exceeds f
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (wpre[w][mid] > f)
            hi = mid;
          else
            lo = mid + 1;
        }
        const int32_t before = lo ? wpre[w][lo - 1] : 0;
        const uint32_t bo = wsim[w][lo];
        const int32_t e = A.out_eid[wbase[w][lo] + (f - before)];
        const int32_t v = A.edge_dst[e];
        const uint32_t* wv = A.bits + (int64_t)bo * A.words + ((uint32_t)v >> 5);
        if (!(*wv & (1u << ((uint32_t)v & 31u))) && sim_live(A, A.first + bo, v, e) &&
            mark(A, bo, v)) {
          have = true;
          entry = ((uint64_t)bo << 32) | (uint32_t)v;
        }
      }
      push(A, have, entry);
    }
    wave_sync();  // the rows are rewritten for the next 64 entries
  }
}

// counts[b] = activated vertices of simulation b (popcount of its bitmap).
__global__ __launch_bounds__(kFwdBlock) void k_fwd_count(const uint32_t* __restrict__ bits,
                                                         int64_t words,
                                                         unsigned long long* __restrict__ cnt) {
  __shared__ unsigned long long red[kFwdBlock / kWave];
  const int b = blockIdx.y;
  const uint32_t* bm = bits + (int64_t)b * words;
  unsigned long long c = 0;
  for (int64_t j = (int64_t)blockIdx.x * kFwdBlock + threadIdx.x; j < words;
       j += (int64_t)gridDim.x * kFwdBlock)
    c += (unsigned long long)__popc(bm[j]);
  c = wave_sum(c);
  if (lane_id() == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int q = 0; q < kFwdBlock / kWave; ++q) s += red[q];
    atomicAdd(&cnt[b], s);
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ x, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0ull;
}

__global__ void k_counts_out(const unsigned long long* __restrict__ cnt, int32_t nb,
                             int64_t* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) out[b] = (int64_t)cnt[b];
}

constexpr int kMaxLevelsBuf = 1 << 16;

// Scratch of a simulation batch of nb_max cascades: visited bits, two level
// queues of (simulation, vertex) entries, per-level counts, per-simulation
// counts and the seeds.
static size_t influence_bytes(int32_t n, int32_t nb_max, int32_t nseeds) {
  const int64_t words = ((int64_t)n + 31) / 32;
  const int64_t qcap = (int64_t)nb_max * n;  // a simulation reaches each vertex once
  return ws_align((size_t)nb_max * words * 4) + 2 * ws_align((size_t)qcap * 8) +
         ws_align((size_t)kMaxLevelsBuf * 8) + ws_align((size_t)nb_max * 8) +
         ws_align((size_t)std::max(nseeds, 1) * 4);
}

size_t ws_forward(int32_t n) {
  return ws_align((size_t)n * 8 + 64) + ws_align((size_t)(n / 8192 + 2) * 8);
}

size_t ws_influence(int32_t n, int64_t nsims, int32_t nseeds) {
  if (nsims <= 0) return 0;
  return influence_bytes(n, (int32_t)std::min<int64_t>(nsims, kSimBatch), nseeds);
}

}  // namespace im

using namespace im;

extern "C" int im_prepare_forward(int32_t n, int64_t num_edges, const int32_t* in_off,
                                  const int32_t* in_src, int64_t* out_off, int32_t* out_eid,
                                  int32_t* edge_dst, void* ws, size_t ws_bytes, void* stream) {
  if (n <= 0 || num_edges < 0 || num_edges >= (int64_t)0x7FFFFFFF || !in_off || !out_off ||
      (num_edges > 0 && (!in_src || !out_eid || !edge_dst)))
    return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_forward(n))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotForward, (size_t)n * 8 + 64, &p));
  uint32_t* deg = (uint32_t*)p;
  uint32_t* fill = deg + n;
  const unsigned fb = (unsigned)std::min<int64_t>(((int64_t)n * 2 + 255) / 256, 65535);
  k_fill_u32<<<dim3(fb), dim3(256), 0, s>>>(deg, (int64_t)n * 2, 0u);
  IM_HIP(hipGetLastError());
  if (num_edges > 0) {
    const unsigned eb = (unsigned)((num_edges + 255) / 256);
    k_fwd_degree<<<dim3(eb), dim3(256), 0, s>>>(num_edges, in_src, deg);
    IM_HIP(hipGetLastError());
    IM_TRY(exclusive_scan_u32_to_i64(deg, n, out_off, s));
    k_fwd_scatter<<<dim3(eb), dim3(256), 0, s>>>(num_edges, in_src, out_off, fill, out_eid);
    IM_HIP(hipGetLastError());
    DeviceInfo di;
    IM_TRY(device_info(&di));
    k_fwd_dst<<<dim3((unsigned)di.num_cus * 8), dim3(256), 0, s>>>(n, in_off, edge_dst);
    IM_HIP(hipGetLastError());
  } else {
    IM_TRY(exclusive_scan_u32_to_i64(deg, n, out_off, s));
  }
  IM_HIP(hipStreamSynchronize(s));
  return IM_OK;
}

extern "C" int im_influence(const im_graph* g, const int64_t* out_off, const int32_t* out_eid,
                            const int32_t* edge_dst, uint64_t seed, uint32_t stream_tag,
                            int64_t first, int64_t nsims, const int32_t* seeds, int32_t nseeds,
                            int64_t* counts, void* ws, size_t ws_bytes, void* stream) {
  if (!g || g->n <= 0 || !g->in_off || !out_off || (g->num_edges > 0 && (!out_eid || !edge_dst ||
                                                                         !g->thr)) ||
      (g->model != IM_IC && g->model != IM_LT) || first < 0 || nsims < 0 ||
      first + nsims > ((int64_t)1 << 32) || nseeds < 0 || (nseeds > 0 && !seeds) ||
      (nsims > 0 && !counts))
    return IM_EINVAL;
  for (int32_t j = 0; j < nseeds; ++j)
    if (seeds[j] < 0 || seeds[j] >= g->n) return IM_EINVAL;
  if (nsims == 0) return IM_OK;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_influence(g->n, nsims, nseeds))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  DeviceInfo di;
  IM_TRY(device_info(&di));
  const int32_t n = g->n;
  const int64_t words = ((int64_t)n + 31) / 32;
  const int32_t nb_max = (int32_t)std::min<int64_t>(nsims, kSimBatch);
  const int64_t qcap = (int64_t)nb_max * n;  // a simulation reaches each vertex once
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotForward, influence_bytes(n, nb_max, nseeds), &p));
  char* c = (char*)p;
  auto take = [&](size_t b) {
    char* r = c;
    c += up(b);
    return r;
  };
  uint32_t* bits = (uint32_t*)take((size_t)nb_max * words * 4);
  uint64_t* q0 = (uint64_t*)take((size_t)qcap * 8);
  uint64_t* q1 = (uint64_t*)take((size_t)qcap * 8);
  unsigned long long* lvl = (unsigned long long*)take((size_t)kMaxLevelsBuf * 8);
  unsigned long long* cnt = (unsigned long long*)take((size_t)nb_max * 8);
  int32_t* d_seeds = (int32_t*)take((size_t)std::max(nseeds, 1) * 4);
  if (nseeds > 0)
    IM_HIP(hipMemcpyAsync(d_seeds, seeds, (size_t)nseeds * 4, hipMemcpyHostToDevice, s));
  const unsigned grid = (unsigned)di.num_cus * 8;
  for (int64_t b0 = 0; b0 < nsims; b0 += nb_max) {
    const int32_t nb = (int32_t)std::min<int64_t>(nb_max, nsims - b0);
    FwdArgs A{};
    A.in_off = g->in_off;
    A.thr = g->thr;
    A.out_off = out_off;
    A.out_eid = out_eid;
    A.edge_dst = edge_dst;
    A.n = n;
    A.model = g->model;
    A.nb = nb;
    A.seed_lo = (uint32_t)seed;
    A.seed_hi = (uint32_t)(seed >> 32);
    A.stream = stream_tag;
    A.first = (uint32_t)(first + b0);
    A.words = words;
    A.bits = bits;
    A.lvl = lvl;
    k_fill_u32<<<dim3(grid), dim3(256), 0, s>>>(bits, (int64_t)nb * words, 0u);
    k_fill_u64<<<dim3(grid), dim3(256), 0, s>>>(lvl, kMaxLevelsBuf);
    k_fill_u64<<<1, 64, 0, s>>>(cnt, nb);
    IM_HIP(hipGetLastError());
    // level L reads queue L % 2 (lvl[L] entries) and appends to queue
    // (L + 1) % 2, counting in lvl[L + 1]; the seeds are level 0, appended
    // as if by a level -1
    FwdArgs S = A;
    S.cur = nullptr;
    S.next = q0;
    S.level = -1;
    if (nseeds > 0) {
      const int64_t t = (int64_t)nb * nseeds;
      k_fwd_seed<<<dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s>>>(S, d_seeds, nseeds);
      IM_HIP(hipGetLastError());
    }
    int32_t level = 0;
    for (;;) {
      for (int q = 0; q < kLevelsPerCheck; ++q, ++level) {
        if (level + 1 >= kMaxLevelsBuf) {
          set_error_text("im_influence: more than 65535 BFS levels");
          return IM_ENOMEM;
        }
        A.level = level;
        A.cur = (level & 1) ? q1 : q0;
        A.next = (level & 1) ? q0 : q1;
        k_fwd_level<<<dim3(grid), dim3(kFwdBlock), 0, s>>>(A);
        IM_HIP(hipGetLastError());
      }
      unsigned long long h = 0;
      IM_HIP(hipMemcpyAsync(&h, lvl + level, 8, hipMemcpyDeviceToHost, s));
      IM_HIP(hipStreamSynchronize(s));
      if (h == 0) break;
    }
    const unsigned cb = (unsigned)std::min<int64_t>((words + kFwdBlock - 1) / kFwdBlock, 64);
    k_fwd_count<<<dim3(std::max(cb, 1u), (unsigned)nb), dim3(kFwdBlock), 0, s>>>(bits, words,
                                                                                 cnt);
    k_counts_out<<<1, 64, 0, s>>>(cnt, nb, counts + b0);
    IM_HIP(hipGetLastError());
  }
  IM_HIP(hipStreamSynchronize(s));
  return IM_OK;
}
