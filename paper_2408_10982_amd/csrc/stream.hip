// stream.hip -- streaming max-k-cover at the receiver with truncation, and the
// final choice between the streamed and the best local solution
// (im_stream_cover; Alg. 5, Sec. 3.3.2, Alg. 4, final choice).
//
// Alg. 5's buckets are independent once the stream is fixed: bucket b's test
// reads only its own seeds S_b and cover C_b.  So every bucket is one
// workgroup on its own CU, keeping C_b as a bitmap over the samples (in LDS
// when it fits, else in HBM), and all buckets walk the same stream at once.
// A bucket changes only when it accepts a set, so a workgroup counts
// |S(x) minus C_b| for a window of consecutive stream entries together (their
// ids spread evenly over the threads, LDS bit tests) and takes the first entry
// that passes; the entries after it are counted again from the ids still in
// registers, and so on until no entry of the window passes.  A set with
// |S(x)| below the bucket's threshold cannot pass and is rejected without
// counting, and a set that fails once never passes later (its gain only
// falls).  The decisions are exactly those of one pass in stream order.
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
constexpr int64_t kLdsWords = 36864;          // 144 KB: C_b in LDS up to 1,179,648 samples
constexpr int kMaxStreamBuckets = 4096;
constexpr int kBuildBlock = 1024;
// dynamic LDS of k_stream_bucket: 160 KB less the static part and a margin
constexpr size_t kStreamLds = 160 * 1024 - 4096;

// Lets a kernel take `bytes` of dynamic LDS (above the default limit).
static int allow_dynamic_lds(const void* kernel, size_t bytes) {
  IM_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return IM_OK;
}

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
  int32_t cache;                         // stream entries whose ranges k_stream_bucket
                                         // keeps in LDS
  int32_t vec;                           // inc_mem is 16-byte aligned
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

// Four ids of S(x) = inc_mem[a .. e) at positions q0 .. q0 + 3 (q0 a multiple
// of 4), 0xFFFFFFFF for positions outside [a, e): one vector load when all
// four lie before e (so never past the array), else one load per id.
__device__ __forceinline__ int4 load_group(const int32_t* __restrict__ mem, bool vec, int64_t q0,
                                           int64_t a, int64_t e) {
  int4 x;
  if (vec && q0 + 3 < e && q0 >= a) {
    x = *reinterpret_cast<const int4*>(mem + q0);
  } else {
    x.x = q0 >= a && q0 < e ? mem[q0] : -1;
    x.y = q0 + 1 >= a && q0 + 1 < e ? mem[q0 + 1] : -1;
    x.z = q0 + 2 >= a && q0 + 2 < e ? mem[q0 + 2] : -1;
    x.w = q0 + 3 >= a && q0 + 3 < e ? mem[q0 + 3] : -1;
  }
  return x;
}

// The ids of S(x) = inc_mem[a .. e), four at a time from 16-byte aligned
// positions: f(id) for each.  Position q0 (a multiple of 4) covers ids
// q0 .. q0 + 3; a vector load is used only when all four lie before e (so
// never past the array), the rest of a partial group is loaded one by one.
template <typename F>
__device__ __forceinline__ void for_group(const int32_t* __restrict__ mem, bool vec, int64_t q0,
                                          int64_t a, int64_t e, F f) {
  if (vec && q0 + 3 < e) {
    const int4 x = *reinterpret_cast<const int4*>(mem + q0);
    if (q0 >= a) f((uint32_t)x.x);
    if (q0 + 1 >= a) f((uint32_t)x.y);
    if (q0 + 2 >= a) f((uint32_t)x.z);
    f((uint32_t)x.w);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q0 + u >= a && q0 + u < e) f((uint32_t)mem[q0 + u]);
  }
}

// One bucket per workgroup: walk the stream a window at a time.  A window is
// up to 64 consecutive entries, as many as hold kRoundGroups groups of 4 ids
// of the sets that can still pass (|S(x)| >= thr; at least one entry).  The
// window's ids are spread evenly over the workgroup, each thread loading up
// to kGroupsPer groups before testing any bit, and the counts are summed per
// entry in LDS; the first entry that passes is taken (its bits set by the
// threads that hold its ids) and the next window starts right after it.  The
// stream's ranges are cached in LDS as far as they fit beside the bitmap.
constexpr int kGroupsPer = 8;
constexpr int kRoundGroups = kSBlock * kGroupsPer;

template <bool kLds>
__global__ __launch_bounds__(kSBlock) void k_stream_bucket(StreamArgs A) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ int64_t w_q[kWave];   // first group position of each window entry
  __shared__ int64_t w_a[kWave], w_e[kWave];
  __shared__ int32_t w_gp[kWave + 1];  // exclusive prefix of the entries' groups
  __shared__ int32_t w_cnt[kWave];
  __shared__ int32_t s_W, s_first;
  uint32_t* lbits = reinterpret_cast<uint32_t*>(dyn);
  const int64_t bm_bytes = kLds ? (A.words * 4 + 15) / 16 * 16 : 0;
  int64_t* s_a = reinterpret_cast<int64_t*>(dyn + bm_bytes);
  int32_t* s_n = reinterpret_cast<int32_t*>(dyn + bm_bytes + (int64_t)A.cache * 8);
  int32_t* s_x = s_n + A.cache;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  uint32_t* bits = kLds ? lbits : A.gbits + (int64_t)b * A.words;
  for (int64_t j = tid; j < A.words; j += kSBlock) bits[j] = 0u;
  const int64_t thr = A.thr[b];
  const int32_t L = A.hdr[0] > 0 ? (int32_t)A.hdr[1] : 0;  // l = 0: nothing can pass
  const int32_t nc = min(L, A.cache);
  for (int32_t j = tid; j < nc; j += kSBlock) {
    const int64_t a = A.sa[j];
    s_a[j] = a;
    s_n[j] = (int32_t)(A.sb[j] - a);
    s_x[j] = A.sx[j];
  }
  int32_t* out = A.bseeds + (int64_t)b * A.k;
  const bool vec = A.vec != 0;
  const int32_t* __restrict__ mem = A.inc_mem;
  __syncthreads();
  int32_t ns = 0;
  int64_t csz = 0;
  int32_t pos = 0;
  while (pos < L && ns < A.k) {  // uniform over the workgroup
    if (w == 0) {  // the window: entries pos + lane
      const int32_t j = pos + lane;
      int64_t a = 0, e = 0;
      if (j < L) {
        a = j < nc ? s_a[j] : A.sa[j];
        e = a + (j < nc ? (int64_t)s_n[j] : A.sb[j] - a);
      }
      const bool elig = j < L && e - a >= thr;
      const int64_t q = a & ~(int64_t)3;
      const int32_t ng = elig ? (int32_t)((e - q + 3) >> 2) : 0;
      const int32_t inc = wave_inclusive_scan(ng);
      // entries while the groups fit the round (the first one always)
      const bool in = j < L && (lane == 0 || inc <= kRoundGroups);
      const int32_t W = (int32_t)__popcll(__ballot(in));
      w_q[lane] = q;
      w_a[lane] = a;
      w_e[lane] = e;
      w_gp[lane] = inc - ng;
      w_cnt[lane] = elig ? 0 : -1;
      if (lane == W - 1) w_gp[W] = inc;
      if (lane == 0) s_W = W;
    }
    __syncthreads();
    const int32_t W = s_W, G = w_gp[W];
    // count: groups g = tid + r * kSBlock of each batch
    int4 x[kGroupsPer];
    int32_t je[kGroupsPer];
#pragma unroll
    for (int r = 0; r < kGroupsPer; ++r) {
      je[r] = -1;
      x[r] = make_int4(-1, -1, -1, -1);
    }
    for (int32_t gb = 0; gb < G; gb += kRoundGroups) {
#pragma unroll
      for (int r = 0; r < kGroupsPer; ++r) {
        const int32_t g = gb + tid + r * kSBlock;
        je[r] = -1;
        x[r] = make_int4(-1, -1, -1, -1);
        if (g < G) {
          int lo = 0, hi = W - 1;  // entry holding group g
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (w_gp[mid] <= g)
              lo = mid;
            else
              hi = mid - 1;
          }
          je[r] = lo;
          x[r] = load_group(mem, vec, w_q[lo] + 4 * (int64_t)(g - w_gp[lo]), w_a[lo], w_e[lo]);
        }
      }
#pragma unroll
      for (int r = 0; r < kGroupsPer; ++r) {
        int32_t c = 0;
        const uint32_t id4[4] = {(uint32_t)x[r].x, (uint32_t)x[r].y, (uint32_t)x[r].z,
                                 (uint32_t)x[r].w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (id4[u] != 0xFFFFFFFFu)
            c += (int32_t)(((bitmap_word<kLds>(bits, id4[u]) >> (id4[u] & 31u)) & 1u) ^ 1u);
        // one atomic per wavefront when all its lanes count for one entry
        const int32_t j0 = __shfl(je[r], 0, kWave);
        if (__all(je[r] == j0)) {
          c = wave_sum(c);
          if (lane == 0 && j0 >= 0 && c) atomicAdd(&w_cnt[j0], c);
        } else if (je[r] >= 0 && c) {
          atomicAdd(&w_cnt[je[r]], c);
        }
      }
    }
    __syncthreads();
    // take the first entry that passes; when the whole window's ids are in
    // registers, recount the entries after it from them and go on taking in
    // the same window (an entry that fails never passes later: its gain only
    // falls), so the window is done when nothing more passes
    const bool held = G <= kRoundGroups;
    int after = -1;  // entries up to here are decided
    for (;;) {
      if (w == 0) {
        const bool pass =
            lane > after && lane < W && w_cnt[lane] >= 0 && (int64_t)w_cnt[lane] >= thr;
        const unsigned long long pm = __ballot(pass);
        if (lane == 0) s_first = pm ? __ffsll((long long)pm) - 1 : -1;
      }
      __syncthreads();
      const int first = s_first;
      if (first < 0) {
        pos += W;
        break;
      }
      const int32_t ja = pos + first;
      if (tid == 0) out[ns] = ja < nc ? s_x[ja] : A.sx[ja];
      ns += 1;
      csz += w_cnt[first];
      if (held) {
#pragma unroll
        for (int r = 0; r < kGroupsPer; ++r)
          if (je[r] == first) {
            const uint32_t id4[4] = {(uint32_t)x[r].x, (uint32_t)x[r].y, (uint32_t)x[r].z,
                                     (uint32_t)x[r].w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (id4[u] != 0xFFFFFFFFu) atomicOr(&bits[id4[u] >> 5], 1u << (id4[u] & 31u));
          }
      } else {
        const int64_t a = w_a[first], e = w_e[first];
        for (int64_t q0 = w_q[first] + 4 * tid; q0 < e; q0 += 4 * kSBlock)
          for_group(mem, vec, q0, a, e,
                    [&](uint32_t id) { atomicOr(&bits[id >> 5], 1u << (id & 31u)); });
      }
      if (!held || ns >= A.k || first == W - 1) {
        pos = ja + 1;
        break;
      }
      after = first;
      if (w == 0 && lane > after && lane < W && w_cnt[lane] >= 0) w_cnt[lane] = 0;
      __syncthreads();  // the new bits and the cleared counts
#pragma unroll
      for (int r = 0; r < kGroupsPer; ++r) {
        int32_t c = 0;
        const bool mine = je[r] > after;
        const uint32_t id4[4] = {(uint32_t)x[r].x, (uint32_t)x[r].y, (uint32_t)x[r].z,
                                 (uint32_t)x[r].w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (mine && id4[u] != 0xFFFFFFFFu)
            c += (int32_t)(((bitmap_word<kLds>(bits, id4[u]) >> (id4[u] & 31u)) & 1u) ^ 1u);
        const int32_t jr = mine ? je[r] : -1;
        const int32_t j0 = __shfl(jr, 0, kWave);
        if (__all(jr == j0)) {
          c = wave_sum(c);
          if (lane == 0 && j0 >= 0 && c) atomicAdd(&w_cnt[j0], c);
        } else if (jr >= 0 && c) {
          atomicAdd(&w_cnt[jr], c);
        }
      }
      __syncthreads();
    }
    __syncthreads();  // bits and the window settled before the next round
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
  A.vec = ((uintptr_t)inc_mem & 15u) == 0 ? 1 : 0;
  // LDS: the bitmap (in-LDS form), then the ranges and vertices of as many
  // stream entries as fit (16 bytes each)
  const size_t bm_bytes = lds ? ((size_t)words * 4 + 15) / 16 * 16 : 0;
  const size_t room = kStreamLds > bm_bytes ? kStreamLds - bm_bytes : 0;
  A.cache = (int32_t)std::min<int64_t>(L, (int64_t)(room / 16));
  const size_t dyn = bm_bytes + (size_t)A.cache * 16;
  k_stream_build<<<1, kBuildBlock, 0, s>>>(A);
  IM_HIP(hipGetLastError());
  if (lds) {
    IM_TRY(allow_dynamic_lds((const void*)k_stream_bucket<true>, dyn));
    k_stream_bucket<true><<<dim3((unsigned)B), dim3(kSBlock), dyn, s>>>(A);
  } else {
    IM_TRY(allow_dynamic_lds((const void*)k_stream_bucket<false>, dyn));
    k_stream_bucket<false><<<dim3((unsigned)B), dim3(kSBlock), dyn, s>>>(A);
  }
  IM_HIP(hipGetLastError());
  k_stream_final<<<1, 256, 0, s>>>(A);
  IM_HIP(hipGetLastError());
  return IM_OK;
}
