// ingest.hip -- graph ingest: edge weights -> integer thresholds (im_prepare_graph).
//
// IC (Sec. 2): an edge with probability p is live in a sample iff its 32-bit
// draw is below floor(p * 2^32) (p = 1 saturates to "always").  LT (Sec. 2):
// read as the live-edge process, each vertex keeps in-edge e with probability
// w_e; the inclusive integer prefix of floor(w * 2^32) over v's in-edges lets
// the sampler pick the kept edge with one draw and a search.
#include <algorithm>

#include "common.h"

namespace im {

enum { kBadOffsets = 1, kBadSource = 2, kBadWeight = 4 };

__global__ void k_check_csr(int32_t n, int64_t E, const int32_t* __restrict__ in_off,
                            uint32_t* __restrict__ flags) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  int32_t o = in_off[v];
  bool bad = (v == 0 && o != 0) || (v == n && (int64_t)o != E) || o < 0 || (int64_t)o > E;
  if (v < n && in_off[v + 1] < o) bad = true;
  if (bad) atomicOr(flags, (uint32_t)kBadOffsets);
}

__global__ void k_ic_thresholds(int64_t E, int64_t E4, const int32_t* __restrict__ in_src,
                                int32_t n, const float* __restrict__ w,
                                uint32_t* __restrict__ thr, uint32_t* __restrict__ flags) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E4;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e >= E) {
      thr[e] = 0u;
      continue;
    }
    float p = w[e];
    int32_t s = in_src[e];
    if (s < 0 || s >= n) atomicOr(flags, (uint32_t)kBadSource);
    if (!(p >= 0.0f) || p > 1.0f) {
      atomicOr(flags, (uint32_t)kBadWeight);
      thr[e] = 0u;
      continue;
    }
    // p * 2^32 is exact in fp32 (power-of-two scale); p < 1 keeps it below 2^32.
    thr[e] = p >= 1.0f ? 0xFFFFFFFFu : (uint32_t)(p * 4294967296.0f);
  }
}

// One thread per vertex walks its in-edges (ingest runs once per graph).
__global__ void k_lt_thresholds(int32_t n, int64_t E, int64_t E4,
                                const int32_t* __restrict__ in_off,
                                const int32_t* __restrict__ in_src, const float* __restrict__ w,
                                uint32_t* __restrict__ thr, uint32_t* __restrict__ flags) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) {
    for (int64_t e = E; e < E4; ++e) thr[e] = 0u;
  }
  if (v >= n) return;
  uint64_t acc = 0;
  const int32_t a = in_off[v], b = in_off[v + 1];
  for (int32_t e = a; e < b; ++e) {
    float x = w[e];
    int32_t s = in_src[e];
    if (s < 0 || s >= n) atomicOr(flags, (uint32_t)kBadSource);
    if (!(x >= 0.0f) || __builtin_isinf(x)) {
      atomicOr(flags, (uint32_t)kBadWeight);
      x = 0.0f;
    }
    uint64_t q = x >= 1.0f ? 4294967296ull : (uint64_t)(x * 4294967296.0f);
    acc += q;
    thr[e] = acc >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)acc;
  }
}

// Run-length table: 1/log(1 - q/2^32) for vertices whose >= 2 in-edges share
// one threshold strictly between 0 and 0xFFFFFFFF; 0 elsewhere.
__global__ __launch_bounds__(256) void k_ic_skip(int32_t n, const int32_t* __restrict__ in_off,
                                                 const uint32_t* __restrict__ thr,
                                                 double* __restrict__ skip) {
  constexpr int kShort = 16;  // lists up to this length are checked by their own lane
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  int32_t a = 0, b = 0;
  uint32_t q = 0;
  bool same = false;
  if (v < n) {
    a = in_off[v];
    b = in_off[v + 1];
    if (b - a >= 2) {
      q = thr[a];
      same = q != 0u && q != 0xFFFFFFFFu;
    }
  }
  if (same && b - a <= kShort)
    for (int32_t e = a + 1; same && e < b; ++e) same = thr[e] == q;
  // long lists: the whole wavefront compares one list at a time
  unsigned long long todo = __ballot(same && b - a > kShort);
  while (todo) {
    const int src = __ffsll(todo) - 1;
    todo &= todo - 1;
    const int32_t sa = __shfl(a, src, kWave), sb = __shfl(b, src, kWave);
    const uint32_t sq = (uint32_t)__shfl((int)q, src, kWave);
    bool ok = true;
    for (int32_t e = sa + 1 + lane; e < sb; e += kWave) ok = ok && thr[e] == sq;
    const bool all = __ballot(!ok) == 0ull;
    if (lane == src) same = all;
  }
  if (v >= n) return;
  double out = 0.0;
  if (same) {
    const double keep = (4294967296.0 - (double)q) * 2.3283064365386963e-10;  // (2^32-q) 2^-32
    out = 1.0 / im_log(keep);
  }
  skip[v] = out;
}

// LT search index, level k: entry w = threshold of the last edge of window w
// (16^k edge ids), clamped to edge E-1; padding entries 0.
__global__ void k_lt_index(const uint32_t* __restrict__ thr, int64_t E, int k, int64_t nw,
                           int64_t nw_pad, uint32_t* __restrict__ out) {
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw_pad;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t last = ((w + 1) << (4 * k)) - 1;
    out[w] = w < nw ? thr[last < E ? last : E - 1] : 0u;
  }
}

int64_t lt_index_entries(int64_t E) {
  int64_t t = 0;
  for (int k = 1; k <= kLtLevels; ++k) {
    const int64_t nw = (E + ((int64_t)1 << (4 * k)) - 1) >> (4 * k);
    t += (nw + 15) & ~(int64_t)15;
  }
  return t;
}

}  // namespace im

extern "C" int im_lt_index_size(int64_t num_edges, int64_t* entries) {
  if (num_edges < 0 || !entries) return IM_EINVAL;
  *entries = im::lt_index_entries(num_edges);
  return IM_OK;
}

extern "C" int im_prepare_graph(int32_t n, int64_t num_edges, const int32_t* in_off,
                                const int32_t* in_src, const float* weight, int32_t model,
                                uint32_t* thr, double* skip, uint32_t* lt_index, void* ws,
                                size_t ws_bytes, void* stream) {
  using namespace im;
  if (n <= 0 || num_edges < 0 || num_edges >= (int64_t)0x7FFFFFFF || !in_off || !thr ||
      (num_edges > 0 && (!weight || !in_src)) || (model != IM_IC && model != IM_LT))
    return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_align(64))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotScan, 64, &p));
  uint32_t* flags = (uint32_t*)p;
  IM_HIP(hipMemsetAsync(flags, 0, sizeof(uint32_t), s));
  const int64_t E = num_edges, E4 = (num_edges + 3) & ~(int64_t)3;
  k_check_csr<<<dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s>>>(n, E, in_off, flags);
  IM_HIP(hipGetLastError());
  uint32_t hf = 0;
  IM_HIP(hipMemcpyAsync(&hf, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  if (hf) return IM_EINVAL;  // offsets unusable: never index with them
  if (model == IM_IC) {
    int64_t blocks = (E4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    k_ic_thresholds<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(E, E4, in_src, n, weight, thr,
                                                                 flags);
  } else {
    k_lt_thresholds<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, E, E4, in_off,
                                                                           in_src, weight, thr,
                                                                           flags);
  }
  IM_HIP(hipGetLastError());
  if (model == IM_IC && skip) {
    k_ic_skip<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, in_off, thr, skip);
    IM_HIP(hipGetLastError());
  }
  if (model == IM_LT && lt_index && E > 0) {
    int64_t base = 0;
    for (int k = 1; k <= kLtLevels; ++k) {
      const int64_t nw = (E + ((int64_t)1 << (4 * k)) - 1) >> (4 * k);
      const int64_t nw_pad = (nw + 15) & ~(int64_t)15;
      const int64_t blocks = std::min<int64_t>((nw_pad + 255) / 256, 65536);
      k_lt_index<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(thr, E, k, nw, nw_pad,
                                                             lt_index + base);
      IM_HIP(hipGetLastError());
      base += nw_pad;
    }
  }
  IM_HIP(hipMemcpyAsync(&hf, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  return hf ? IM_EINVAL : IM_OK;
}
