// offline.hip -- RandGreedi's global step without streaming: the offline
// GreeDI aggregation of Alg. 4 (im_greedi_offline).
//
// The local solutions of the m partitions (the first T = ceil(alpha k) picks
// of each, all k at alpha = 1) are gathered and the standard greedy -- which
// selects exactly what Alg. 2's lazy greedy selects, lowest id on ties --
// picks at most k seeds among their union over the full universe of samples
// (Alg. 4, global step).  Then Alg. 4's final choice keeps the better of that
// global solution and the best local one.  The greedy runs on the cover
// kernels of greedy.hip with the gathered vertices as its candidate
// positions; the partitions are disjoint, so the union is the concatenation
// of the local solutions.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "cover.h"

namespace im {

__global__ void k_fill_i32(int32_t* __restrict__ x, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// Candidate position of the t-th pick of partition p: the picks of the
// partitions before p, then t (one workgroup; m <= kMaxParts).
__global__ __launch_bounds__(kMaxParts) void k_offline_gather(int32_t m, int32_t k, int32_t T,
                                                              const int32_t* __restrict__ lseeds,
                                                              const int32_t* __restrict__ lcount,
                                                              int32_t* __restrict__ order,
                                                              int32_t* __restrict__ pos_of) {
  __shared__ int32_t base[kMaxParts + 1];
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int p = 0; p < m; ++p) {
      base[p] = acc;
      acc += min(T, lcount[p]);
    }
    base[m] = acc;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < m; p += blockDim.x) {
    const int32_t c = min(T, lcount[p]);
    for (int32_t t = 0; t < c; ++t) {
      const int32_t x = lseeds[(int64_t)p * k + t];
      order[base[p] + t] = x;
      pos_of[x] = base[p] + t;
    }
  }
}

// Alg. 4's final choice: the global solution unless the lowest partition of
// largest local cover covers strictly more.
__global__ __launch_bounds__(256) void k_offline_final(int32_t m, int32_t k, int32_t nc,
                                                       const int32_t* __restrict__ lseeds,
                                                       const int32_t* __restrict__ lcount,
                                                       const int64_t* __restrict__ lcover,
                                                       const int32_t* __restrict__ gseeds,
                                                       const int32_t* __restrict__ gnsel,
                                                       const int64_t* __restrict__ gcov,
                                                       int32_t* __restrict__ seeds,
                                                       int32_t* __restrict__ nsel,
                                                       int64_t* __restrict__ coverage,
                                                       int32_t* __restrict__ info,
                                                       int64_t* __restrict__ gcover_out) {
  __shared__ int s_pl;
  if (threadIdx.x == 0) {
    int pl = 0;
    for (int p = 1; p < m; ++p)
      if (lcover[p] > lcover[pl]) pl = p;
    s_pl = pl;
  }
  __syncthreads();
  const int pl = s_pl;
  const bool global = *gcov >= lcover[pl];
  const int32_t c = global ? *gnsel : lcount[pl];
  for (int j = threadIdx.x; j < k; j += blockDim.x)
    seeds[j] = j < c ? (global ? gseeds[j] : lseeds[(int64_t)pl * k + j]) : -1;
  if (threadIdx.x == 0) {
    *nsel = c;
    *coverage = global ? *gcov : lcover[pl];
    info[0] = global ? 1 : 0;
    info[1] = nc;
    info[2] = *gnsel;
    info[3] = pl;
    if (gcover_out) *gcover_out = *gcov;
  }
}

// Scratch of one call gathering nc local seeds: order, pos_of, cnt, covered,
// the greedy's gmax, seeds and gains, and three flags.
static size_t offline_bytes(int32_t n, int64_t count, int32_t k, int64_t nc) {
  const size_t c = (size_t)std::max<int64_t>(nc, 1) * 4;
  return ws_align(c) + ws_align((size_t)n * 4) + ws_align(c) + ws_align((size_t)count + 1) +
         ws_align((size_t)k * 8) * 3 + ws_align(64) * 3;
}

size_t ws_offline(int32_t n, int64_t count, int32_t k, int32_t m) {
  return offline_bytes(n, count, k, (int64_t)k * m);
}

}  // namespace im

using namespace im;

extern "C" int im_greedi_offline(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                                 int64_t total, const int64_t* inc_off, const int32_t* inc_mem,
                                 int32_t k, int32_t m, const int32_t* lseeds, const int32_t* lcount,
                                 const int64_t* lcover, double alpha, int32_t* seeds,
                                 int32_t* nsel, int64_t* coverage, int32_t* info,
                                 int64_t* gcover, void* ws, size_t ws_bytes, void* stream) {
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || total < 0 || k <= 0 || m < 1 ||
      m > kMaxParts || !off || !inc_off || !lseeds || !lcount || !lcover || !seeds || !nsel ||
      !coverage || !info || (total > 0 && (!mem || !inc_mem)) || !(alpha > 0.0 && alpha <= 1.0))
    return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_offline(n, count, k, m))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  int32_t T = (int32_t)ceil(alpha * (double)k);
  T = std::max(1, std::min(T, k));
  // the number of gathered seeds sizes the greedy's launches
  std::vector<int32_t> lc(m);
  IM_HIP(hipMemcpyAsync(lc.data(), lcount, (size_t)m * 4, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  int64_t nc = 0;
  for (int p = 0; p < m; ++p) nc += std::max(0, std::min(T, lc[p]));
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotOffline, offline_bytes(n, count, k, nc), &p));
  char* c = (char*)p;
  auto take = [&](size_t b) {
    char* r = c;
    c += up(b);
    return r;
  };
  int32_t* order = (int32_t*)take((size_t)std::max<int64_t>(nc, 1) * 4);
  int32_t* pos_of = (int32_t*)take((size_t)n * 4);
  uint32_t* cnt = (uint32_t*)take((size_t)std::max<int64_t>(nc, 1) * 4);
  uint8_t* covered = (uint8_t*)take((size_t)count + 1);
  unsigned long long* gmax = (unsigned long long*)take((size_t)k * 8);
  int32_t* gseeds = (int32_t*)take((size_t)k * 8);
  int64_t* ggains = (int64_t*)take((size_t)k * 8);
  int32_t* done = (int32_t*)take(64);
  int32_t* gnsel = (int32_t*)take(64);
  int64_t* gcov = (int64_t*)take(64);
  k_fill_i32<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(pos_of, n, -1);
  IM_HIP(hipGetLastError());
  k_offline_gather<<<1, kMaxParts, 0, s>>>(m, k, T, lseeds, lcount, order, pos_of);
  IM_HIP(hipGetLastError());
  CoverArgs A{};
  A.n = (int32_t)nc;
  A.m = 1;
  A.count = count;
  A.k = k;
  A.off = off;
  A.mem = mem;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.order = order;
  A.pos_of = pos_of;
  A.cnt = cnt;
  A.covered = covered;
  A.gmax = gmax;
  A.done = done;
  A.seeds = gseeds;
  A.gains = ggains;
  A.nsel = gnsel;
  A.cover = gcov;
  IM_HIP(hipMemsetAsync(ggains, 0, (size_t)k * 8, s));
  IM_TRY(launch_cover(A, s));
  k_offline_final<<<1, 256, 0, s>>>(m, k, (int32_t)nc, lseeds, lcount, lcover, gseeds, gnsel, gcov,
                                    seeds, nsel, coverage, info, gcover);
  IM_HIP(hipGetLastError());
  return IM_OK;
}
