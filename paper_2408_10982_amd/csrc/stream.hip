// stream.hip -- streaming max-k-cover at the receiver with truncation, and the
// final choice between the streamed and the best local solution
// (im_stream_cover; Alg. 5, Sec. 3.3.2, Alg. 4, final choice).
//
// Alg. 5's buckets are independent once the stream is fixed: bucket b's test
// reads only its own seeds S_b and cover C_b.  So every bucket is one
// workgroup on its own CU, keeping C_b as a bitmap over the samples (in LDS
// when it fits, else in HBM), and all buckets walk the same stream at once.
// A bucket changes only when it accepts a set, so a workgroup evaluates a
// window of consecutive stream entries together -- one per wavefront, each
// counting |S(x) minus C_b| with LDS bit tests -- and takes the first entry
// that passes; the entries after it are evaluated again from the new state.
// A set with |S(x)| below the bucket's threshold cannot pass and is rejected
// without counting.  The decisions are exactly those of one pass in stream
// order.
//
// Launches (all asynchronous, no host round trip):
//   k_stream_build   one workgroup: the stream in its fixed order (compacted),
//                    the ranges of its S(x), l = max |S(x)|, the length, and
//                    the B integer thresholds (fp64, the same operations as
//                    the definition: (1+delta)^b by repeated products);
//   k_stream_bucket  one workgroup per bucket;
//   k_stream_final   b* and the final choice of Alg. 4.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace im {

constexpr int kSBlock = 1024;
constexpr int kWin = kSBlock / kWave;         // stream entries evaluated together
constexpr int64_t kLdsWords = 36864;          // 144 KB: C_b in LDS up to 1,179,648 samples
constexpr int kMaxStreamBuckets = 4096;
constexpr int kBuildBlock = 1024;

struct StreamArgs {
  int64_t count;                         // samples (universe)
  int32_t k, m, T, B;
  double delta;
  const int64_t* __restrict__ inc_off;
  const int32_t* __restrict__ inc_mem;
  const int32_t* __restrict__ lseeds;
  const int32_t* __restrict__ lcount;
  const int64_t* __restrict__ lcover;
  // stream (k_stream_build): vertex, S(x) = inc_mem[sa .. sb), length and l
  int32_t* __restrict__ sx;
  int64_t* __restrict__ sa;
  int64_t* __restrict__ sb;
  int64_t* __restrict__ hdr;             // [0] l, [1] stream length
  int64_t* __restrict__ thr;             // B thresholds
  uint32_t* __restrict__ gbits;          // B bitmaps of `words` words (HBM form only)
  int64_t words;
  int32_t* __restrict__ bseeds;          // B * k
  int32_t* __restrict__ bcount;          // B
  int64_t* __restrict__ bcover;          // B
  int32_t* __restrict__ seeds;
  int32_t* __restrict__ nsel;
  int64_t* __restrict__ coverage;
  int32_t* __restrict__ info;
};

// The stream in round-major order (position t of every partition p in turn:
// entry t*m + p, present iff t < lcount[p]), compacted, with the ranges of
// S(x); then l, the length and the thresholds thr_b = ceil(l g_b / (2k)),
// g_0 = 1, g_{b+1} = g_b (1 + delta).
__global__ __launch_bounds__(kBuildBlock) void k_stream_build(StreamArgs A) {
  __shared__ int32_t wsum[kBuildBlock / kWave];
  __shared__ unsigned long long s_l;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  if (tid == 0) s_l = 0ull;
  const int64_t n_entries = (int64_t)A.T * A.m;
  int32_t carry = 0;
  unsigned long long lmax = 0ull;
  for (int64_t j0 = 0; j0 < n_entries; j0 += kBuildBlock) {
    const int64_t j = j0 + tid;
    int32_t x = -1;
    if (j < n_entries) {
      const int t = (int)(j / A.m), p = (int)(j % A.m);
      if (t < A.lcount[p]) x = A.lseeds[(int64_t)p * A.k + t];
    }
    const int32_t have = x >= 0 ? 1 : 0;
    const int32_t inc = wave_inclusive_scan(have);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int32_t before = carry;
    for (int q = 0; q < w; ++q) before += wsum[q];
    int32_t tot = 0;
    for (int q = 0; q < kBuildBlock / kWave; ++q) tot += wsum[q];
    if (have) {
      const int32_t at = before + inc - 1;
      const int64_t a = A.inc_off[x], b = A.inc_off[x + 1];
      A.sx[at] = x;
      A.sa[at] = a;
      A.sb[at] = b;
      const unsigned long long sz = (unsigned long long)(b - a);
      lmax = sz > lmax ? sz : lmax;
    }
    carry += tot;
    __syncthreads();
  }
  atomicMax(&s_l, lmax);
  __syncthreads();
  const int64_t l = (int64_t)s_l;
  if (tid == 0) {
    A.hdr[0] = l;
    A.hdr[1] = carry;
  }
  for (int b = tid; b < A.B; b += kBuildBlock) {
    double g = 1.0;
    for (int q = 0; q < b; ++q) g = g * (1.0 + A.delta);
    A.thr[b] = (int64_t)ceil((double)l * g / (2.0 * (double)A.k));
  }
}

template <bool kLds>
__device__ __forceinline__ uint32_t bitmap_word(const uint32_t* bits, uint32_t i) {
  if constexpr (kLds)
    return bits[i >> 5];
  else  // other wavefronts' atomics land in L2: read past the CU's L1
    return __hip_atomic_load(&bits[i >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One bucket per workgroup: walk the stream, kWin entries per round.
template <bool kLds>
__global__ __launch_bounds__(kSBlock) void k_stream_bucket(StreamArgs A) {
  __shared__ uint32_t lbits[kLds ? kLdsWords : 1];
  __shared__ int32_t s_gain[kWin];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  uint32_t* bits = kLds ? lbits : A.gbits + (int64_t)b * A.words;
  for (int64_t j = tid; j < A.words; j += kSBlock) bits[j] = 0u;
  const int64_t thr = A.thr[b];
  const int32_t L = A.hdr[0] > 0 ? (int32_t)A.hdr[1] : 0;  // l = 0: nothing can pass
  int32_t* out = A.bseeds + (int64_t)b * A.k;
  __syncthreads();
  int32_t ns = 0;
  int64_t csz = 0;
  int32_t pos = 0;
  while (pos < L && ns < A.k) {  // uniform over the workgroup
    const int32_t j = pos + w;
    int32_t g = -1;
    if (j < L) {
      const int64_t a = A.sa[j], e = A.sb[j];
      if (e - a >= thr) {
        int32_t c = 0;
        constexpr int kU = 8;  // ids loaded together, then their bits tested
        for (int64_t q0 = a + lane; q0 < e; q0 += kU * kWave) {
          uint32_t ids[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int64_t q = q0 + (int64_t)u * kWave;
            ids[u] = q < e ? (uint32_t)A.inc_mem[q] : 0xFFFFFFFFu;
          }
#pragma unroll
          for (int u = 0; u < kU; ++u)
            if (ids[u] != 0xFFFFFFFFu)
              c += (int32_t)(((bitmap_word<kLds>(bits, ids[u]) >> (ids[u] & 31u)) & 1u) ^ 1u);
        }
        c = wave_sum(c);
        g = (int64_t)c >= thr ? c : -1;
      }
    }
    if (lane == 0) s_gain[w] = g;
    __syncthreads();
    int first = -1;
    for (int q = 0; q < kWin; ++q)
      if (s_gain[q] >= 0) {
        first = q;
        break;
      }
    if (first >= 0) {
      const int32_t ja = pos + first;
      const int64_t a = A.sa[ja], e = A.sb[ja];
      if (tid == 0) out[ns] = A.sx[ja];
      ns += 1;
      csz += s_gain[first];
      for (int64_t q = a + tid; q < e; q += kSBlock) {
        const uint32_t i = (uint32_t)A.inc_mem[q];
        atomicOr(&bits[i >> 5], 1u << (i & 31u));
      }
      pos = ja + 1;
    } else {
      pos += kWin;
    }
    __syncthreads();  // bits and s_gain settled before the next round
  }
  if (tid == 0) {
    A.bcount[b] = ns;
    A.bcover[b] = csz;
  }
}

// b* = lowest bucket of largest cover; then Alg. 4's final choice against the
// lowest partition of largest local cover (ties go to the streamed solution).
__global__ __launch_bounds__(256) void k_stream_final(StreamArgs A) {
  __shared__ int s_bs, s_pl;
  __shared__ bool s_global;
  if (threadIdx.x == 0) {
    int bs = 0;
    for (int q = 1; q < A.B; ++q)
      if (A.bcover[q] > A.bcover[bs]) bs = q;
    int pl = 0;
    for (int p = 1; p < A.m; ++p)
      if (A.lcover[p] > A.lcover[pl]) pl = p;
    s_bs = bs;
    s_pl = pl;
    s_global = A.bcover[bs] >= A.lcover[pl];
  }
  __syncthreads();
  const int bs = s_bs, pl = s_pl;
  const bool global = s_global;
  const int32_t c = global ? A.bcount[bs] : A.lcount[pl];
  for (int j = threadIdx.x; j < A.k; j += blockDim.x)
    A.seeds[j] = j < c ? (global ? A.bseeds[(int64_t)bs * A.k + j] : A.lseeds[(int64_t)pl * A.k + j])
                       : -1;
  if (threadIdx.x == 0) {
    *A.nsel = c;
    *A.coverage = global ? A.bcover[bs] : A.lcover[pl];
    A.info[0] = bs;
    A.info[1] = A.B;
    A.info[2] = global ? 1 : 0;
    A.info[3] = (int32_t)A.hdr[1];
  }
}

// Truncation length T, bucket count B and scratch bytes of one call:
// stream (x, a, b per entry) | header | thresholds | bucket seeds, counts and
// covers | bucket bitmaps when they do not fit in LDS.
static size_t stream_layout(int64_t count, int32_t k, int32_t m, double delta, double alpha,
                            int32_t* T_out, int32_t* B_out) {
  int32_t T = (int32_t)ceil(alpha * (double)k);
  T = std::max(1, std::min(T, k));
  int32_t B = (int32_t)ceil(log((double)k) / log(1.0 + delta));
  if (B < 1) B = 1;
  *T_out = T;
  *B_out = B;
  const int64_t L = (int64_t)T * m;  // longest possible stream
  const int64_t words = (count + 31) / 32;
  const bool lds = words <= kLdsWords;
  return ws_align((size_t)L * 4) + ws_align((size_t)L * 8) * 2 + ws_align(16) +
         ws_align((size_t)B * 8) + ws_align((size_t)B * k * 4) + ws_align((size_t)B * 4) +
         ws_align((size_t)B * 8) + (lds ? 0 : (size_t)B * (size_t)words * 4);
}

size_t ws_stream(int32_t, int64_t count, int32_t k, int32_t m, double delta) {
  int32_t T = 0, B = 0;
  const size_t b = stream_layout(count, k, m, delta, 1.0, &T, &B);
  return B > kMaxStreamBuckets ? 0 : ws_align(b);
}

}  // namespace im

extern "C" int im_stream_cover(int32_t n, int64_t count, const int64_t* inc_off,
                               const int32_t* inc_mem, int32_t k, int32_t m,
                               const int32_t* lseeds, const int32_t* lcount,
                               const int64_t* lcover, double delta, double alpha,
                               int32_t* seeds, int32_t* nsel, int64_t* coverage, int32_t* info,
                               void* ws, size_t ws_bytes, void* stream) {
  using namespace im;
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || k <= 0 || m < 1 || m > 256 ||
      !inc_off || !lseeds || !lcount || !lcover || !seeds || !nsel || !coverage || !info ||
      !(delta > 0.0 && delta < 0.5) || !(alpha > 0.0 && alpha <= 1.0))
    return IM_EINVAL;
  // truncation length and bucket count (fp64 on the host)
  int32_t T = 0, B = 0;
  const size_t bytes = stream_layout(count, k, m, delta, alpha, &T, &B);
  if (B > kMaxStreamBuckets) return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_align(bytes))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const int64_t L = (int64_t)T * m;  // longest possible stream
  const int64_t words = (count + 31) / 32;
  const bool lds = words <= kLdsWords;
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotStream, bytes, &p));
  char* c = (char*)p;
  auto take = [&](size_t b) {
    char* r = c;
    c += up(b);
    return r;
  };
  StreamArgs A;
  A.count = count;
  A.k = k;
  A.m = m;
  A.T = T;
  A.B = B;
  A.delta = delta;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.lseeds = lseeds;
  A.lcount = lcount;
  A.lcover = lcover;
  A.sx = (int32_t*)take((size_t)L * 4);
  A.sa = (int64_t*)take((size_t)L * 8);
  A.sb = (int64_t*)take((size_t)L * 8);
  A.hdr = (int64_t*)take(16);
  A.thr = (int64_t*)take((size_t)B * 8);
  A.bseeds = (int32_t*)take((size_t)B * k * 4);
  A.bcount = (int32_t*)take((size_t)B * 4);
  A.bcover = (int64_t*)take((size_t)B * 8);
  A.gbits = lds ? nullptr : (uint32_t*)c;
  A.words = words;
  A.seeds = seeds;
  A.nsel = nsel;
  A.coverage = coverage;
  A.info = info;
  k_stream_build<<<1, kBuildBlock, 0, s>>>(A);
  IM_HIP(hipGetLastError());
  if (lds)
    k_stream_bucket<true><<<dim3((unsigned)B), dim3(kSBlock), 0, s>>>(A);
  else
    k_stream_bucket<false><<<dim3((unsigned)B), dim3(kSBlock), 0, s>>>(A);
  IM_HIP(hipGetLastError());
  k_stream_final<<<1, 256, 0, s>>>(A);
  IM_HIP(hipGetLastError());
  return IM_OK;
}
