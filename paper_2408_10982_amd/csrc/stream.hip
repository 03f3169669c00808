// stream.hip -- streaming max-k-cover at the receiver with truncation, and the
// final choice between the streamed and the best local solution
// (im_stream_cover; Alg. 5, Sec. 3.3.2, Alg. 4, final choice).
//
// Bucket state is bit-sliced: one 64-bit word per sample whose bit b says
// "covered in bucket b", so every streamed set is read once for all buckets.
// For each streamed vertex x the workgroup gathers the words of S(x); the
// uncovered counts of all buckets come from wavefront ballots (bit b of the
// 64 lanes' uncovered masks) and popcounts; the accept decision of every
// bucket is a threshold test; accepted buckets OR their bit into the words of
// S(x).  The stream is processed in its fixed order by one workgroup: each
// set's decision depends on every earlier one.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace im {

constexpr int kSBlock = 1024;
constexpr int kMaxBuckets = 64;

struct StreamArgs {
  int64_t count;
  int32_t k, m, T, B;
  int32_t empty;  // every streamed S(x) is empty (l = 0): no bucket takes anything
  const int64_t* __restrict__ inc_off;
  const int32_t* __restrict__ inc_mem;
  const int32_t* __restrict__ lseeds;
  const int32_t* __restrict__ lcount;
  const int64_t* __restrict__ lcover;
  const int64_t* __restrict__ thr;  // B thresholds
  uint64_t* __restrict__ masks;     // count words
  int32_t* __restrict__ bseeds;     // B*k
  int32_t* __restrict__ seeds;
  int32_t* __restrict__ nsel;
  int64_t* __restrict__ coverage;
  int32_t* __restrict__ info;
};

// l = largest |S(x)| over the stream, and the stream length.
__global__ __launch_bounds__(256) void k_stream_scan(const int64_t* __restrict__ inc_off,
                                                     const int32_t* __restrict__ lseeds,
                                                     const int32_t* __restrict__ lcount, int32_t k,
                                                     int32_t m, int32_t T,
                                                     unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[2];
  if (threadIdx.x == 0) red[0] = red[1] = 0;
  __syncthreads();
  unsigned long long l = 0, len = 0;
  for (int64_t j = threadIdx.x; j < (int64_t)m * T; j += blockDim.x) {
    const int p = (int)(j % m), t = (int)(j / m);
    if (t < lcount[p]) {
      const int32_t x = lseeds[(int64_t)p * k + t];
      const unsigned long long sz = (unsigned long long)(inc_off[x + 1] - inc_off[x]);
      l = sz > l ? sz : l;
      ++len;
    }
  }
  atomicMax(&red[0], l);
  atomicAdd(&red[1], len);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = red[0];
    out[1] = red[1];
  }
}

__global__ __launch_bounds__(kSBlock) void k_stream(StreamArgs A) {
  __shared__ int32_t ns[kMaxBuckets];
  __shared__ long long csz[kMaxBuckets];
  __shared__ unsigned long long gain[kMaxBuckets];
  __shared__ long long s_thr[kMaxBuckets];
  __shared__ unsigned long long s_accept;
  __shared__ int32_t s_live;
  __shared__ int32_t px[kSBlock];  // the next kSBlock stream entries: vertex,
  __shared__ int64_t pa[kSBlock];  // and the range of S(x) (pb = -1: no entry,
  __shared__ int64_t pb[kSBlock];  // past that partition's local count)
  const int tid = threadIdx.x, lane = lane_id();
  for (int64_t j = tid; j < A.count; j += kSBlock) A.masks[j] = 0ull;
  if (tid < kMaxBuckets) {
    ns[tid] = 0;
    csz[tid] = 0;
    gain[tid] = 0;
    s_thr[tid] = tid < A.B ? A.thr[tid] : 0;
  }
  if (tid == 0) s_live = A.B > 0 && !A.empty;
  const uint64_t all = A.B >= 64 ? ~0ull : ((1ull << A.B) - 1ull);
  __syncthreads();
  int32_t slen = 0;
  // stream order: position t of every partition p in turn, entry j = t * m + p;
  // each chunk of kSBlock entries is looked up by the whole block at once
  const int64_t n_entries = (int64_t)A.T * A.m;
  for (int64_t j0 = 0; j0 < n_entries; j0 += kSBlock) {
    {
      const int64_t j = j0 + tid;
      int32_t x = -1;
      int64_t a = 0, b = -1;
      if (j < n_entries) {
        const int t = (int)(j / A.m), p = (int)(j % A.m);
        if (t < A.lcount[p]) {
          x = A.lseeds[(int64_t)p * A.k + t];
          a = A.inc_off[x];
          b = A.inc_off[x + 1];
        }
      }
      px[tid] = x;
      pa[tid] = a;
      pb[tid] = b;
    }
    __syncthreads();
    const int n_in = (int)min((int64_t)kSBlock, n_entries - j0);
    for (int jj = 0; jj < n_in; ++jj) {
      if (pb[jj] < 0) continue;  // uniform
      ++slen;
      const int32_t x = px[jj];
      const int64_t a = pa[jj], b = pb[jj];
      // s_live: some bucket still open (set at the last decision, read after
      // the barrier that ended it)
      if (!s_live) continue;  // every bucket is full: nothing can change
      unsigned long long acc = 0;  // lane q: uncovered count of bucket q in this wave
      for (int64_t base = a; base < b; base += kSBlock) {
        const int64_t e = base + tid;
        const uint64_t unc = e < b ? (~A.masks[A.inc_mem[e]] & all) : 0ull;
        if (__any(unc != 0)) {
#pragma unroll 8
          for (int q = 0; q < kMaxBuckets; ++q) {
            const unsigned long long bal = __ballot((unc >> q) & 1ull);
            if (lane == q) acc += (unsigned long long)__popcll(bal);
          }
        }
      }
      if (acc) atomicAdd(&gain[lane], acc);
      __syncthreads();
      if (tid < kWave) {  // wavefront 0, lane q decides bucket q (buckets are independent)
        const int q = tid;
        const bool take = q < A.B && ns[q] < A.k && (long long)gain[q] >= s_thr[q];
        if (take) {
          A.bseeds[(int64_t)q * A.k + ns[q]] = x;
          ns[q] += 1;
          csz[q] += (long long)gain[q];
        }
        gain[q] = 0;  // for the next set
        const unsigned long long acc_mask = __ballot(take);
        const unsigned long long open = __ballot(q < A.B && ns[q] < A.k);
        if (tid == 0) {
          s_accept = acc_mask;
          s_live = open != 0ull;
        }
      }
      __syncthreads();
      const uint64_t acc_mask = s_accept;
      if (acc_mask)
        for (int64_t e = a + tid; e < b; e += kSBlock) A.masks[A.inc_mem[e]] |= acc_mask;
      __syncthreads();
    }
    __syncthreads();  // every entry of the chunk read before the next chunk
  }
  if (tid == 0) {
    int bs = 0;
    for (int q = 1; q < A.B; ++q)
      if (csz[q] > csz[bs]) bs = q;
    int pl = 0;
    for (int p = 1; p < A.m; ++p)
      if (A.lcover[p] > A.lcover[pl]) pl = p;
    const bool global = csz[bs] >= A.lcover[pl];
    const int32_t c = global ? ns[bs] : A.lcount[pl];
    for (int j = 0; j < A.k; ++j)
      A.seeds[j] = j < c ? (global ? A.bseeds[(int64_t)bs * A.k + j]
                                   : A.lseeds[(int64_t)pl * A.k + j])
                         : -1;
    *A.nsel = c;
    *A.coverage = global ? csz[bs] : A.lcover[pl];
    A.info[0] = bs;
    A.info[1] = A.B;
    A.info[2] = global ? 1 : 0;
    A.info[3] = slen;
  }
}

}  // namespace im

extern "C" int im_stream_cover(int32_t n, int64_t count, const int64_t* inc_off,
                               const int32_t* inc_mem, int32_t k, int32_t m,
                               const int32_t* lseeds, const int32_t* lcount,
                               const int64_t* lcover, double delta, double alpha,
                               int32_t* seeds, int32_t* nsel, int64_t* coverage, int32_t* info,
                               void* stream) {
  using namespace im;
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || k <= 0 || m < 1 || m > 256 ||
      !inc_off || !lseeds || !lcount || !lcover || !seeds || !nsel || !coverage || !info ||
      !(delta > 0.0 && delta < 0.5) || !(alpha > 0.0 && alpha <= 1.0))
    return IM_EINVAL;
  // truncation length and bucket count (fp64 on the host)
  int32_t T = (int32_t)ceil(alpha * (double)k);
  T = std::max(1, std::min(T, k));
  int32_t B = (int32_t)ceil(log((double)k) / log(1.0 + delta));
  if (B < 1) B = 1;
  if (B > kMaxBuckets) return IM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = 64 + (size_t)kMaxBuckets * 8 + (size_t)B * k * 4 + (size_t)count * 8 + 64;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotStream, bytes, &p));
  unsigned long long* lz = (unsigned long long*)p;
  int64_t* thr = (int64_t*)((char*)p + 64);
  uint64_t* masks = (uint64_t*)(thr + kMaxBuckets);
  int32_t* bseeds = (int32_t*)(masks + count);
  k_stream_scan<<<1, 256, 0, s>>>(inc_off, lseeds, lcount, k, m, T, lz);
  IM_HIP(hipGetLastError());
  unsigned long long hl[2] = {0, 0};
  IM_HIP(hipMemcpyAsync(hl, lz, sizeof(hl), hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  // thresholds ceil(l (1+delta)^b / (2k)), (1+delta)^b by repeated products
  int64_t ht[kMaxBuckets];
  double gpow = 1.0;
  for (int b = 0; b < B; ++b) {
    ht[b] = (int64_t)ceil((double)(int64_t)hl[0] * gpow / (2.0 * (double)k));
    gpow = gpow * (1.0 + delta);
  }
  IM_HIP(hipMemcpyAsync(thr, ht, (size_t)B * 8, hipMemcpyHostToDevice, s));
  StreamArgs A;
  A.count = count;
  A.k = k;
  A.m = m;
  A.T = T;
  A.B = B;
  A.empty = hl[0] == 0 ? 1 : 0;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.lseeds = lseeds;
  A.lcount = lcount;
  A.lcover = lcover;
  A.thr = thr;
  A.masks = masks;
  A.bseeds = bseeds;
  A.seeds = seeds;
  A.nsel = nsel;
  A.coverage = coverage;
  A.info = info;
  k_stream<<<1, kSBlock, 0, s>>>(A);
  IM_HIP(hipGetLastError());
  // the host copy of ht must outlive the async copy
  IM_HIP(hipStreamSynchronize(s));
  return IM_OK;
}
