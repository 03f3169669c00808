// greedy.hip -- standard greedy max-k-cover (im_greedy_cover) and the
// RandGreedi local step over m vertex partitions (im_randgreedi).
//
// Sec. 3.2: k times, take the vertex of largest marginal coverage (lowest id
// on ties).  The marginal coverage of every vertex is kept exactly as a count
// of its still-uncovered samples: when a sample becomes covered, every member
// of that sample loses one.  Two launches per pick:
//   A. every workgroup scans a tile of the counts for the argmax key
//      (count << 32 | ~v) and folds it into a global atomic max;
//   B. the samples of S(v*) are spread over the wavefronts; each newly
//      covered sample is walked by a whole wavefront, decrementing counts.
// A device-wide barrier inside one persistent kernel would need agent-scope
// fences, which on this multi-die part write back and invalidate the L2 of
// every wavefront's die; a kernel boundary does that once.
// The RandGreedi form runs all m partitions in the same launch: counts are
// laid out partition by partition, each partition keeps its own covered flags
// over the full universe of samples, and a covered sample only decrements the
// members of the partition that covered it (Alg. 4, local greedy step; Sec. 3.4 S3).
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "cover.h"

namespace im {

constexpr int kGBlock = 1024;
constexpr int kArgTile = kGBlock * 8;  // positions per workgroup in the argmax pass
constexpr int kApplyBlock = 256;
static_assert(kMaxParts <= kApplyBlock, "one apply thread per partition");
constexpr int kRecountBlock = 256;
constexpr int kRecountUnroll = 4;  // elements per lane per step of the recount
constexpr int kRecountPicks = 2;   // picks that may rebuild the counts
// Entries of S(v*) per wavefront chunk in the apply pass: a newly covered
// sample is walked by the whole wavefront, so small chunks spread the walks of
// a pick over many wavefronts.
#ifndef IM_APPLY_ENTRIES
#define IM_APPLY_ENTRIES 4
#endif
constexpr int kApplyEntries = IM_APPLY_ENTRIES;
// Workgroups per CU of the apply pass: the first picks' subsets hold most of
// the samples, and 8 per CU (all resident at its 38 VGPRs) walk them with
// twice the wavefronts of 4 (local greedy at m = 64 over 2^22 vertices: 7.9
// against 9.5 ms for 300 picks; 12 and 16 per CU no faster).
constexpr int kApplyPerCu = 8;

__device__ __forceinline__ int64_t part_lo(const CoverArgs& A, int p) {
  return A.pbase ? A.pbase[p] : 0;
}
__device__ __forceinline__ int64_t part_hi(const CoverArgs& A, int p) {
  return A.pbase ? A.pbase[p + 1] : (int64_t)A.n;
}
__device__ __forceinline__ int32_t part_k(const CoverArgs& A, int p) {
  return A.kpart ? A.kpart[p] : A.k;
}
__device__ __forceinline__ int64_t part_out(const CoverArgs& A, int p) {
  return A.koff ? A.koff[p] : (int64_t)p * A.k;
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long x,
                                                            unsigned long long* lds) {
  x = wave_max_u64(x);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = x;
  __syncthreads();
  unsigned long long r = 0;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) r = lds[j] > r ? lds[j] : r;
  __syncthreads();
  return r;
}

// Counts start at |S(v)|; nothing is covered; no argmax yet.
__global__ __launch_bounds__(kGBlock) void k_cover_init(CoverArgs A) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t pos = gtid; pos < A.n; pos += gthreads) {
    const int32_t v = A.order ? A.order[pos] : (int32_t)pos;
    A.cnt[pos] = (uint32_t)(A.inc_off[v + 1] - A.inc_off[v]);
  }
  const int64_t ncov = A.sbase ? A.count : (int64_t)A.m * A.count;
  for (int64_t j = gtid; j < ncov; j += gthreads) A.covered[j] = 0;
  for (int64_t j = gtid; j < (int64_t)A.m * A.k; j += gthreads) A.gmax[j] = 0ull;
  if (A.cand)
    for (int64_t j = gtid; j < A.m; j += gthreads) {
      A.cand_n[j] = 0;  // an empty list: the first pick scans the partition
      A.tau[j] = 0u;
    }
  if (gtid == 0) *A.done = 0;
}

// Pick `it`, step 1: every workgroup reduces one tile of positions to the
// argmax key (count << 32 | ~v) of each partition it overlaps.
__global__ __launch_bounds__(kGBlock) void k_cover_argmax(CoverArgs A, int it) {
  __shared__ unsigned long long red[kGBlock / kWave];
  __shared__ int64_t s_pb[kMaxParts + 1];  // partition bounds
  __shared__ int32_t s_k[kMaxParts];       // picks per partition
  constexpr int kQ = kArgTile / kGBlock;
  const int32_t done = *A.done;  // uniform; checked only before the atomic, so the
                                 // count loads do not wait for it
  const int64_t b0 = (int64_t)blockIdx.x * kArgTile;
  const int64_t b1 = min((int64_t)A.n, b0 + kArgTile);
  // the tile's counts (and ids) first: they do not depend on the partitions
  uint32_t c[kQ];
  int32_t vv[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int64_t pos = b0 + threadIdx.x + (int64_t)q * kGBlock;
    c[q] = 0u;
    vv[q] = 0;
    if (pos < b1) {
      c[q] = A.cnt[pos];
      vv[q] = A.order && !A.pos_keys ? A.order[pos] : (int32_t)pos;
    }
  }
  const int m = A.m;
  for (int j = threadIdx.x; j <= m; j += kGBlock) {
    s_pb[j] = A.pbase ? A.pbase[j] : (j == 0 ? 0 : (int64_t)A.n);
    if (j < m) s_k[j] = A.kpart ? A.kpart[j] : A.k;
  }
  __syncthreads();
  int p = 0;  // first partition overlapping the tile
  {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pb[mid] <= b0)
        lo = mid;
      else
        hi = mid - 1;
    }
    p = lo;
  }
  for (; p < m; ++p) {
    const int64_t lo = max(b0, s_pb[p]), hi = min(b1, s_pb[p + 1]);
    if (lo >= b1) break;
    if (it >= s_k[p]) continue;  // this partition has made all its picks (uniform)
    unsigned long long best = 0ull;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t pos = b0 + threadIdx.x + (int64_t)q * kGBlock;
      if (pos >= lo && pos < hi) {
        const unsigned long long key = argmax_key(c[q], (uint32_t)vv[q]);
        best = key > best ? key : best;
      }
    }
    best = block_max_u64(best, red);
    if (threadIdx.x == 0 && best && !done) atomicMax(&A.gmax[(int64_t)it * A.m + p], best);
  }
}

// Pick `it`, step 1, with candidate lists (RandGreedi): one workgroup per
// partition.  A partition's list holds every position whose count exceeded
// tau[p] when the list was built; counts only fall, so a position outside the
// list stays at or below tau[p], and a list entry above tau[p] with the best
// key is the partition's argmax (a strictly larger count than any outside).
// Otherwise the workgroup scans the partition's counts: their argmax is the
// pick, and the list is rebuilt from a histogram of the counts (the highest
// bins that together hold at most kListCap positions).  A partition whose
// counts are all 0 is marked exhausted (tau = ~0).  Same picks as the full
// argmax pass.
// Threads of a list workgroup (each holds kListCap / kListBlock entries):
// 256, 512 and 1024 measured within noise with four solves in flight, 512
// fastest on one stream (local greedy 7.66 against 7.84-7.86 ms).
#ifndef IM_LIST_BLOCK
#define IM_LIST_BLOCK 512
#endif
constexpr int kListBlock = IM_LIST_BLOCK;
constexpr int kListBins = kListCap;  // histogram bins of a rebuild
constexpr int kListPer = kListCap / kListBlock;  // list entries per thread
constexpr int kBinsPer = kListBins / kListBlock;  // bins per thread
static_assert(kListCap % kListBlock == 0 && kListBlock % kWave == 0, "list block shape");
constexpr uint32_t kListExhausted = 0xFFFFFFFFu;
constexpr int kListUnroll = 8;

__global__ __launch_bounds__(kListBlock) void k_cover_pick_list(CoverArgs A, int it) {
  __shared__ unsigned long long red[kListBlock / kWave];
  __shared__ uint32_t hist[kListBins];
  __shared__ uint32_t wsum[kListBlock / kWave];
  __shared__ int32_t csum[kListBlock / kWave];
  __shared__ int32_t s_n;
  const int p = blockIdx.x, tid = threadIdx.x;
  const uint32_t tau = A.tau[p];
  // uniform: the row of gmax stays 0 (no pick)
  if (*A.done || it >= part_k(A, p) || tau == kListExhausted) return;
  int32_t* L = A.cand + (int64_t)p * kListCap;
  const int32_t ln = A.cand_n[p];
  unsigned long long best = 0ull;
  {
    int32_t pos[kListPer];
    uint32_t cv[kListPer];
#pragma unroll
    for (int r = 0; r < kListPer; ++r) {
      const int j = tid + r * kListBlock;
      pos[r] = j < ln ? L[j] : -1;
    }
#pragma unroll
    for (int r = 0; r < kListPer; ++r) cv[r] = pos[r] >= 0 ? A.cnt[pos[r]] : 0u;
#pragma unroll
    for (int r = 0; r < kListPer; ++r) {
      const unsigned long long key = pos[r] >= 0 ? argmax_key(cv[r], (uint32_t)pos[r]) : 0ull;
      best = key > best ? key : best;
    }
  }
  best = block_max_u64(best, red);
  if (key_count(best) > tau) {
    if (tid == 0) A.gmax[(int64_t)it * A.m + p] = best;
    return;
  }
  const int64_t lo = part_lo(A, p), hi = part_hi(A, p);
  constexpr int64_t kStep = (int64_t)kListBlock * kListUnroll;
  best = 0ull;
  for (int64_t b = lo; b < hi; b += kStep) {
    uint32_t c[kListUnroll];
#pragma unroll
    for (int q = 0; q < kListUnroll; ++q) {
      const int64_t pos = b + tid + (int64_t)q * kListBlock;
      c[q] = pos < hi ? A.cnt[pos] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kListUnroll; ++q) {
      const int64_t pos = b + tid + (int64_t)q * kListBlock;
      const unsigned long long key = pos < hi ? argmax_key(c[q], (uint32_t)pos) : 0ull;
      best = key > best ? key : best;
    }
  }
  best = block_max_u64(best, red);
  const uint32_t mx = key_count(best);
  if (mx == 0) {  // nothing left to gain here, now or later
    if (tid == 0) {
      A.cand_n[p] = 0;
      A.tau[p] = kListExhausted;
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < kBinsPer; ++r) hist[tid + r * kListBlock] = 0u;
  if (tid == 0) s_n = 0;
  __syncthreads();
  // bin of a count c in [1, mx]: floor(c * kListBins / (mx + 1))
  for (int64_t b = lo; b < hi; b += kStep) {
    uint32_t c[kListUnroll];
#pragma unroll
    for (int q = 0; q < kListUnroll; ++q) {
      const int64_t pos = b + tid + (int64_t)q * kListBlock;
      c[q] = pos < hi ? A.cnt[pos] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kListUnroll; ++q)
      if (c[q] > 0u)
        atomicAdd(&hist[(uint32_t)(((uint64_t)c[q] * kListBins) / ((uint64_t)mx + 1))], 1u);
  }
  __syncthreads();
  // suffix sums of the bins (the sum over a bin and all above it), highest
  // bin first, thread t holding kBinsPer consecutive ones; cut = number of
  // bins whose suffix exceeds the cap
  const int w = tid / kWave;
  uint32_t hv[kBinsPer];
  uint32_t tsum = 0;
#pragma unroll
  for (int r = 0; r < kBinsPer; ++r) {
    hv[r] = hist[kListBins - 1 - (kBinsPer * tid + r)];
    tsum += hv[r];
  }
  const uint32_t incl = wave_inclusive_scan(tsum);
  if (lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - tsum;
  for (int q = 0; q < w; ++q) run += wsum[q];
  int32_t over = 0;
#pragma unroll
  for (int r = 0; r < kBinsPer; ++r) {
    run += hv[r];
    over += run > (uint32_t)kListCap ? 1 : 0;
  }
  over = wave_sum(over);
  if (lane_id() == 0) csum[w] = over;
  __syncthreads();
  int cut = 0;
  for (int q = 0; q < kListBlock / kWave; ++q) cut += csum[q];
  // the bins whose suffix exceeds the cap are bins 0 .. cut-1; the list
  // keeps bins >= cut, and a count is in a bin >= cut exactly when it is at
  // least cmin
  const uint64_t cmin = ((uint64_t)cut * ((uint64_t)mx + 1) + kListBins - 1) / kListBins;
  const uint32_t tau2 = cmin > 0 ? (uint32_t)(cmin - 1) : 0u;
  for (int64_t b = lo; b < hi; b += kStep) {
    uint32_t c[kListUnroll];
#pragma unroll
    for (int q = 0; q < kListUnroll; ++q) {
      const int64_t pos = b + tid + (int64_t)q * kListBlock;
      c[q] = pos < hi ? A.cnt[pos] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kListUnroll; ++q)
      if (c[q] > tau2) L[atomicAdd(&s_n, 1)] = (int32_t)(b + tid + (int64_t)q * kListBlock);
  }
  __syncthreads();
  if (tid == 0) {
    A.cand_n[p] = s_n;
    A.tau[p] = tau2;
    A.gmax[(int64_t)it * A.m + p] = best;
  }
}

// Pick `it`, step 2: record the picks, cover their covering subsets, and
// decrement the counts of the members of every newly covered sample.  Each
// wavefront takes kApplyEntries consecutive entries of the picks' subsets; a
// newly covered sample is then walked by the whole wavefront (one sample
// after another: walking the fresh samples of a chunk together, each lane
// finding its sample by a search over the prefix sums of their sizes,
// measured slower).
// One of the first kRecountPicks picks whose gain reaches recount_min
// (one-partition covers only): mark its samples covered and zero every count;
// k_cover_recount, launched for exactly those picks, then rebuilds them.
__device__ __forceinline__ bool recount_pick(const CoverArgs& A, int it) {
  return A.recount_min > 0 && it < kRecountPicks &&
         (int64_t)key_count(A.gmax[it]) >= A.recount_min;
}


__global__ __launch_bounds__(kApplyBlock) void k_cover_apply(CoverArgs A, int it) {
  __shared__ unsigned long long pbest[kMaxParts];
  __shared__ int64_t pre[kMaxParts + 1];
  __shared__ int64_t part_scan[kApplyBlock / kWave + 1];
  __shared__ int64_t ppos[kMaxParts];    // count position of each partition's pick
  __shared__ int64_t pstart[kMaxParts];  // where its covering subset starts
  __shared__ int64_t plo[kMaxParts], phi[kMaxParts];  // the partition's positions
  __shared__ uint32_t pvert[kMaxParts];  // its vertex
  const int tid = threadIdx.x, lane = lane_id();
  const int m = A.m;
  const unsigned long long* gm = A.gmax + (int64_t)it * m;
  const int32_t done = *A.done;  // uniform; loaded together with the picks
  // one thread per partition: its pick and the size of the pick's S(v)
  // (m <= kMaxParts = kApplyBlock)
  int64_t sz = 0;
  if (tid < m) {
    const unsigned long long b = it < part_k(A, tid) ? gm[tid] : 0ull;
    plo[tid] = part_lo(A, tid);
    phi[tid] = part_hi(A, tid);
    pbest[tid] = b;
    ppos[tid] = -1;
    pstart[tid] = 0;
    pvert[tid] = 0u;
    if (key_count(b) > 0) {
      const uint32_t x = key_vertex(b);
      const uint32_t v = A.pos_keys ? (uint32_t)A.order[x] : x;
      const int64_t s0 = A.inc_off[v];
      sz = A.inc_off[v + 1] - s0;
      pstart[tid] = s0;
      ppos[tid] = A.pos_keys ? (int64_t)x : (A.pos_of ? (int64_t)A.pos_of[v] : (int64_t)v);
      pvert[tid] = v;
    }
  }
  {  // pre = exclusive prefix of the sizes, pre[m] = total
    const int w = tid / kWave;
    const int64_t inc = wave_inclusive_scan(sz);
    if (lane == kWave - 1) part_scan[w] = inc;
    __syncthreads();
    if (tid == 0) {
      int64_t acc = 0;
      for (int j = 0; j < kApplyBlock / kWave; ++j) {
        const int64_t x = part_scan[j];
        part_scan[j] = acc;
        acc += x;
      }
      part_scan[kApplyBlock / kWave] = acc;
    }
    __syncthreads();
    if (tid < m) pre[tid] = part_scan[w] + inc - sz;
    if (tid == 0) pre[m] = done ? 0 : part_scan[kApplyBlock / kWave];
  }
  __syncthreads();
  const int64_t tot = pre[m];
  if (tot == 0) {  // no partition has anything left to gain
    if (blockIdx.x == 0 && tid == 0) *A.done = 1;
    return;
  }
  const bool decrement = !recount_pick(A, it);
  if (blockIdx.x == 0) {
    for (int p = tid; p < m; p += kApplyBlock) {
      const unsigned long long b = pbest[p];
      if (key_count(b) > 0) {
        const int64_t v = pvert[p];
        A.seeds[part_out(A, p) + it] = (int32_t)(A.local_ids ? v - plo[p] : v);
        A.gains[part_out(A, p) + it] = (int64_t)key_count(b);
        // every sample of S(v*) ends up covered, so the pick's own count
        // becomes 0; it is stored once here and skipped in the member walks
        // (one atomic per covered sample on that one address otherwise)
        if (decrement) A.cnt[ppos[p]] = 0u;
      }
    }
  }
  const int64_t gtid = (int64_t)blockIdx.x * kApplyBlock + tid;
  if (!decrement)
    for (int64_t pos = gtid; pos < A.n; pos += (int64_t)gridDim.x * kApplyBlock) A.cnt[pos] = 0u;
  const int64_t wid = gtid / kWave, nw = (int64_t)gridDim.x * kApplyBlock / kWave;
  const int64_t nchunks = (tot + kApplyEntries - 1) / kApplyEntries;
  for (int64_t c = wid; c < nchunks; c += nw) {
    const int64_t f = c * kApplyEntries + lane;
    int p = 0;
    bool fresh = false;
    int64_t ma = 0, mb = 0;  // the sample's member range, loaded with its flag
    if (lane < kApplyEntries && f < tot) {
      int lo = 0, hi = m - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= f)
          lo = mid;
        else
          hi = mid - 1;
      }
      p = lo;
      const int32_t smp = A.inc_mem[pstart[p] + (f - pre[p])];
      // flag index: a global sample position when each partition owns its
      // own samples, else one flag array per partition over all samples
      const int64_t fi = A.sbase ? A.sbase[p] + smp : (int64_t)p * A.count + smp;
      const int64_t gs = A.sbase ? A.sbase[p] + smp : (int64_t)smp;
      const uint8_t was = A.covered[fi];
      if (decrement) {
        ma = A.off[gs];
        mb = A.off[gs + 1];
      }
      if (!was) {  // each sample occurs once in S(v), so no race
        A.covered[fi] = 1;
        fresh = true;
      }
    }
    // each newly covered sample is walked by the whole wavefront
    unsigned long long todo = decrement ? __ballot(fresh) : 0ull;
    while (todo) {
      const int src = __ffsll(todo) - 1;
      todo &= todo - 1;
      const int q = __shfl(p, src, kWave);
      const int64_t a = __shfl(ma, src, kWave), b = __shfl(mb, src, kWave);
      for (int64_t t = a + lane; t < b; t += kWave) {
        // RandGreedi: only members of the covering partition lose a count;
        // their count positions, stored beside the members, say which
        if (A.mpos) {
          const int64_t pos = A.mpos[t];
          if (pos >= plo[q] && pos < phi[q] && pos != ppos[q]) atomicSub(&A.cnt[pos], 1u);
          continue;
        }
        const int32_t u = A.mem[t];
        if (A.part && A.part[u] != (uint8_t)q) continue;
        const int64_t pos = A.local_ids ? plo[q] + u : (A.pos_of ? A.pos_of[u] : u);
        if (pos >= plo[q] && pos < phi[q] && pos != ppos[q]) atomicSub(&A.cnt[pos], 1u);
      }
    }
  }
}

// Pick `it`, step 2, for a plain one-partition cover (positions = vertices).
// The members of newly covered samples repeat heavily (a high-count vertex
// sits in thousands of the samples one pick covers), and device atomics on
// one cache line serialize, so each workgroup takes a contiguous slice of
// S(v*), folds the decrements of its fresh samples into an LDS hash table
// (vertex -> amount) and then applies one atomic per distinct vertex.  A
// vertex that finds no slot within kAggProbe probes is decremented directly.
// The counts reached are the same as with one atomic per member.
#ifndef IM_AGG_BLOCK
#define IM_AGG_BLOCK 1024
#endif
#ifndef IM_AGG_BITS
#define IM_AGG_BITS 12
#endif
constexpr int kAggBlock = IM_AGG_BLOCK;
constexpr int kAggBits = IM_AGG_BITS;  // 2^12 slots: 32 KB of LDS
constexpr int kAggSlots = 1 << kAggBits;
constexpr int kAggProbe = 8;
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ void agg_decrement(uint32_t* hkey, uint32_t* hval, uint32_t* cnt,
                                              uint32_t u) {
  uint32_t h = (u * 0x9E3779B1u) >> (32 - kAggBits);
  for (int q = 0; q < kAggProbe; ++q) {
    const uint32_t old = atomicCAS(&hkey[h], kAggEmpty, u);
    if (old == kAggEmpty || old == u) {
      atomicAdd(&hval[h], 1u);
      return;
    }
    h = (h + 1) & (kAggSlots - 1);
  }
  atomicSub(&cnt[u], 1u);
}

__global__ __launch_bounds__(kAggBlock) void k_cover_apply_one(CoverArgs A, int it) {
  __shared__ uint32_t hkey[kAggSlots];
  __shared__ uint32_t hval[kAggSlots];
  const int tid = threadIdx.x, lane = lane_id();
  const unsigned long long key = A.gmax[it];
  if (*A.done || key_count(key) == 0) {  // nothing left to gain (uniform)
    if (blockIdx.x == 0 && tid == 0) *A.done = 1;
    return;
  }
  const uint32_t v = key_vertex(key);
  if (blockIdx.x == 0 && tid == 0) {
    A.seeds[it] = (int32_t)v;
    A.gains[it] = (int64_t)key_count(key);
  }
  const int64_t base = A.inc_off[v], tot = A.inc_off[v + 1] - base;
  const bool decrement = !recount_pick(A, it);
  if (!decrement) {  // mark only; k_cover_recount rebuilds the counts
    const int64_t gtid = (int64_t)blockIdx.x * kAggBlock + tid;
    const int64_t gthreads = (int64_t)gridDim.x * kAggBlock;
    for (int64_t pos = gtid; pos < A.n; pos += gthreads) A.cnt[pos] = 0u;
    for (int64_t f = gtid; f < tot; f += gthreads) A.covered[A.inc_mem[base + f]] = 1;
    return;
  }
  const int64_t per = (tot + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = min(tot, (int64_t)blockIdx.x * per), e1 = min(tot, e0 + per);
  if (e0 >= e1) return;  // uniform over the block
  for (int j = tid; j < kAggSlots; j += kAggBlock) {
    hkey[j] = kAggEmpty;
    hval[j] = 0u;
  }
  __syncthreads();
  const int wv = tid / kWave;
  const int64_t nchunks = (e1 - e0 + kApplyEntries - 1) / kApplyEntries;
  for (int64_t c = wv; c < nchunks; c += kAggBlock / kWave) {
    const int64_t f = e0 + c * kApplyEntries + lane;
    bool fresh = false;
    int64_t ma = 0, mb = 0;
    if (lane < kApplyEntries && f < e1) {
      const int32_t smp = A.inc_mem[base + f];
      const uint8_t was = A.covered[smp];
      ma = A.off[smp];
      mb = A.off[smp + 1];
      if (!was) {  // each sample occurs once in S(v), so no race
        A.covered[smp] = 1;
        fresh = true;
      }
    }
    unsigned long long todo = __ballot(fresh);
    while (todo) {
      const int src = __ffsll(todo) - 1;
      todo &= todo - 1;
      const int64_t a = __shfl(ma, src, kWave), b = __shfl(mb, src, kWave);
      for (int64_t t = a + lane; t < b; t += kWave) agg_decrement(hkey, hval, A.cnt, (uint32_t)A.mem[t]);
    }
  }
  __syncthreads();
  for (int j = tid; j < kAggSlots; j += kAggBlock) {
    const uint32_t d = hval[j];
    if (d) atomicSub(&A.cnt[hkey[j]], d);
  }
}

// One-partition cover after its first pick: cnt[v] = |S(v) minus covered| for
// every v, without per-member atomics.  Each wavefront takes an equal slice of
// the covering-subset elements and walks it 64 vertices at a time (their
// element ranges, clipped to the slice, are consecutive: coalesced loads,
// owner by binary search over 64 prefix sums), counting uncovered samples per
// vertex in LDS.  A vertex whose S(v) lies inside the slice is stored; a
// vertex cut by a slice boundary is added atomically (counts were zeroed).
__global__ __launch_bounds__(kRecountBlock) void k_cover_recount(CoverArgs A, int it) {
  __shared__ int64_t wpre[kRecountBlock / kWave][kWave];
  __shared__ uint32_t wcnt[kRecountBlock / kWave][kWave];
  if (*A.done || !recount_pick(A, it)) return;
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  const int64_t n = A.n;
  const int64_t E = A.inc_off[n];
  const int64_t nwaves = (int64_t)gridDim.x * (kRecountBlock / kWave);
  const int64_t per = (E + nwaves - 1) / nwaves;
  const int64_t e0 = min(E, ((int64_t)blockIdx.x * (kRecountBlock / kWave) + wv) * per);
  const int64_t e1 = min(E, e0 + per);
  if (e0 >= e1) return;  // this wavefront only; the kernel has no block barrier
  int64_t lo = 0, hi = n - 1;  // last vertex with inc_off[v] <= e0
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (A.inc_off[mid] <= e0)
      lo = mid;
    else
      hi = mid - 1;
  }
  int64_t vg = lo;
  for (;;) {
    const int64_t v = vg + lane;
    int64_t a = E, b = E;
    if (v < n) {
      a = A.inc_off[v];
      b = A.inc_off[v + 1];
    }
    const int64_t ca = max(a, e0), cb = min(b, e1);
    const int64_t sz = cb > ca ? cb - ca : 0;
    const int64_t incl = wave_inclusive_scan(sz);
    const int64_t all = __shfl(incl, kWave - 1, kWave);
    const int64_t first = __shfl(ca, 0, kWave);
    wpre[wv][lane] = incl;
    wcnt[wv][lane] = 0u;
    wave_sync();
    // kRecountUnroll elements per lane per step, in three phases so that each
    // phase's loads are in flight together
    for (int64_t x0 = lane; x0 < all; x0 += kWave * kRecountUnroll) {
      int own[kRecountUnroll];
      int32_t smp[kRecountUnroll];
      uint8_t cov[kRecountUnroll];
#pragma unroll
      for (int q = 0; q < kRecountUnroll; ++q) {
        const int64_t x = x0 + q * kWave;
        own[q] = -1;
        smp[q] = 0;
        if (x < all) {
          int o_lo = 0, o_hi = kWave - 1;  // first lane whose inclusive prefix exceeds x
          while (o_lo < o_hi) {
            const int mid = (o_lo + o_hi) >> 1;
            if (wpre[wv][mid] > x)
              o_hi = mid;
            else
              o_lo = mid + 1;
          }
          own[q] = o_lo;
          smp[q] = A.inc_mem[first + x];
        }
      }
#pragma unroll
      for (int q = 0; q < kRecountUnroll; ++q) cov[q] = own[q] >= 0 ? A.covered[smp[q]] : 1;
#pragma unroll
      for (int q = 0; q < kRecountUnroll; ++q)
        if (!cov[q]) atomicAdd(&wcnt[wv][own[q]], 1u);
    }
    wave_sync();
    if (v < n) {
      const uint32_t c = wcnt[wv][lane];
      if (a >= e0 && b <= e1)
        A.cnt[v] = c;  // all of S(v) is in this slice
      else if (c)
        atomicAdd(&A.cnt[v], c);
    }
    const int64_t last_end = __shfl(b, kWave - 1, kWave);
    wave_sync();
    if (vg + kWave >= n || last_end >= e1) break;
    vg += kWave;
  }
}

// Per partition: the picks with a positive gain, their count and coverage.
__global__ void k_cover_finish(CoverArgs A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.m) return;
  int32_t c = 0;
  int64_t s = 0;
  const int32_t kp = part_k(A, p);
  const int64_t o = part_out(A, p);
  for (int it = 0; it < kp; ++it) {
    const int64_t g = A.gains[o + it];
    if (g <= 0) break;
    ++c;
    s += g;
  }
  for (int it = c; it < kp; ++it) {
    A.seeds[o + it] = -1;
    A.gains[o + it] = 0;
  }
  A.nsel[p] = c;
  A.cover[p] = s;
}

// Partition draw: part(v) = floor(draw(part_seed, PART, 0, 0, v) * m / 2^32).
__global__ void k_partition(int32_t n, int32_t m, uint32_t s_lo, uint32_t s_hi,
                            uint8_t* __restrict__ part) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint4 r = philox4x32_10(make_uint4((uint32_t)v >> 2, 0u, kTagPart, 0u), s_lo, s_hi);
  part[v] = (uint8_t)scale_draw(pick_word(r, (uint32_t)v & 3u), (uint32_t)m);
}

// Counting sort of vertices by partition (stable in v): order, tile tables.
// The vertices of every partition in ascending id, by a stable counting
// sort over chunks of kPartChunk vertices: count (a partition-major matrix
// M[p][chunk] and the per-partition totals), an exclusive scan of M (the
// place of each (partition, chunk) run), and a scatter that ranks each
// vertex among the earlier ones of its chunk in the same partition.
constexpr int kPartChunk = 8192;
constexpr int kPartBlock = 256;

__global__ __launch_bounds__(kPartBlock) void k_part_count(int32_t n, int32_t m,
                                                           const uint8_t* __restrict__ part,
                                                           int64_t nchunks,
                                                           uint32_t* __restrict__ M,
                                                           uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kMaxParts];
  const int64_t c = blockIdx.x;
  for (int q = threadIdx.x; q < m; q += kPartBlock) h[q] = 0u;
  __syncthreads();
  const int64_t v0 = c * kPartChunk, v1 = min((int64_t)n, v0 + kPartChunk);
  for (int64_t v = v0 + threadIdx.x; v < v1; v += kPartBlock) atomicAdd(&h[part[v]], 1u);
  __syncthreads();
  for (int q = threadIdx.x; q < m; q += kPartBlock) {
    const uint32_t x = h[q];
    M[(int64_t)q * nchunks + c] = x;
    if (x) atomicAdd(&hist[q], x);
  }
}

// One block per chunk, kPartBlock vertices per round in id order.  Lanes of a
// wavefront with equal partition ids are found by one ballot per bit of the
// id; a vertex's place is its run's start (Moff), the chunk's earlier rounds
// (cur), the earlier wavefronts of this round (wc) and its rank among the
// lanes below it.
__global__ __launch_bounds__(kPartBlock) void k_part_scatter(int32_t n, int32_t m,
                                                             const uint8_t* __restrict__ part,
                                                             int64_t nchunks,
                                                             const int64_t* __restrict__ Moff,
                                                             int32_t* __restrict__ order) {
  constexpr int kNW = kPartBlock / kWave;
  __shared__ uint32_t cur[kMaxParts];
  __shared__ uint32_t wc[kNW][kMaxParts];
  const int64_t c = blockIdx.x;
  const int t = threadIdx.x, w = t / kWave, lane = lane_id();
  for (int q = t; q < kMaxParts; q += kPartBlock) cur[q] = 0u;
  const int64_t v0 = c * kPartChunk, v1 = min((int64_t)n, v0 + kPartChunk);
  for (int64_t vb = v0; vb < v1; vb += kPartBlock) {
    for (int q = lane; q < kMaxParts; q += kWave) wc[w][q] = 0u;
    __syncthreads();
    const int64_t v = vb + t;
    const bool valid = v < v1;
    const uint32_t p = valid ? (uint32_t)part[v] : 0u;
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long ones = __ballot(valid && ((p >> b) & 1u));
      same &= ((p >> b) & 1u) ? ones : ~ones;
    }
    const uint32_t rank = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    if (valid && rank == 0u) wc[w][p] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t before = cur[p];
      for (int j = 0; j < w; ++j) before += wc[j][p];
      order[Moff[(int64_t)p * nchunks + c] + before + rank] = (int32_t)v;
    }
    __syncthreads();
    for (int q = t; q < m; q += kPartBlock) {
      uint32_t add = 0u;
      for (int j = 0; j < kNW; ++j) add += wc[j][q];
      cur[q] += add;
    }
    __syncthreads();
  }
}

// The count position of every member of the sample collection, beside the
// members (its partition is the range the position falls in).
__global__ void k_member_pos(const int32_t* __restrict__ mem, int64_t total,
                             const int32_t* __restrict__ pos_of, int32_t* __restrict__ mpos) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    mpos[t] = pos_of[mem[t]];
}

__global__ void k_pos_of(int32_t n, const int32_t* __restrict__ order,
                         int32_t* __restrict__ pos_of) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos < n) pos_of[order[pos]] = (int32_t)pos;
}

// The launch sequence of one cover: init, then per pick argmax + apply (+ a
// recount for a heavy early pick), then finish.  Kernel boundaries make each
// pass's writes visible device-wide (one cache flush per launch rather than
// per wave).
struct CoverPlan {
  unsigned init_blocks, arg_blocks, apply_blocks, agg_blocks, recount_blocks, finish_blocks;
  bool can_recount, lists;
};

static void enqueue_cover(const CoverArgs& A, const CoverPlan& P, hipStream_t s) {
  k_cover_init<<<dim3(P.init_blocks), dim3(kGBlock), 0, s>>>(A);
  for (int it = 0; it < A.k; ++it) {
    if (P.lists)
      k_cover_pick_list<<<dim3((unsigned)A.m), dim3(kListBlock), 0, s>>>(A, it);
    else
      k_cover_argmax<<<dim3(P.arg_blocks), dim3(kGBlock), 0, s>>>(A, it);
    if (P.can_recount)
      k_cover_apply_one<<<dim3(P.agg_blocks), dim3(kAggBlock), 0, s>>>(A, it);
    else
      k_cover_apply<<<dim3(P.apply_blocks), dim3(kApplyBlock), 0, s>>>(A, it);
    if (P.can_recount && it < kRecountPicks)
      k_cover_recount<<<dim3(P.recount_blocks), dim3(kRecountBlock), 0, s>>>(A, it);
  }
  k_cover_finish<<<dim3(P.finish_blocks), dim3(256), 0, s>>>(A);
}

// Captured form: the sequence is recorded on a private stream of the calling
// thread into a hipGraph, instantiated once per launch shape (k, grids, form)
// and afterwards updated in place with the new arguments, then launched on
// the caller's stream as one submission.  Handles are plain values (no
// destructor runs HIP at thread or process exit); im_release destroys the
// calling thread's executables.
namespace {
struct PlanKey {
  int dev, k, m;
  unsigned init_blocks, arg_blocks, apply_blocks, agg_blocks, recount_blocks, finish_blocks;
  bool can_recount, lists;
  bool operator<(const PlanKey& o) const {
    return std::tie(dev, k, m, init_blocks, arg_blocks, apply_blocks, agg_blocks, recount_blocks,
                    finish_blocks, can_recount, lists) <
           std::tie(o.dev, o.k, o.m, o.init_blocks, o.arg_blocks, o.apply_blocks, o.agg_blocks,
                    o.recount_blocks, o.finish_blocks, o.can_recount, o.lists);
  }
};
thread_local std::map<PlanKey, hipGraphExec_t>* t_execs = nullptr;
thread_local hipStream_t t_capture[64] = {};
}  // namespace

void release_cover_graphs() {
  if (!t_execs) return;
  for (auto& kv : *t_execs) (void)hipGraphExecDestroy(kv.second);
  t_execs->clear();
}

static int launch_captured(const CoverArgs& A, const CoverPlan& P, int dev, hipStream_t s) {
  if (dev < 0 || dev >= 64) return IM_EDEVICE;
  if (!t_capture[dev]) IM_HIP(hipStreamCreateWithFlags(&t_capture[dev], hipStreamNonBlocking));
  const hipStream_t cap = t_capture[dev];
  IM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  enqueue_cover(A, P, cap);
  const hipError_t le = hipGetLastError();
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(cap, &graph);
  if (le != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_error(le != hipSuccess ? le : ee, "capture of the cover launches");
    return IM_EDEVICE;
  }
  if (!t_execs) t_execs = new std::map<PlanKey, hipGraphExec_t>();
  const PlanKey key{dev, A.k, A.m, P.init_blocks, P.arg_blocks, P.apply_blocks, P.agg_blocks,
                    P.recount_blocks, P.finish_blocks, P.can_recount, P.lists};
  auto it = t_execs->find(key);
  if (it != t_execs->end()) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult ur;
    if (hipGraphExecUpdate(it->second, graph, &err_node, &ur) != hipSuccess ||
        ur != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(it->second);
      t_execs->erase(it);
      it = t_execs->end();
    }
  }
  if (it == t_execs->end()) {
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      set_error(ie, "hipGraphInstantiate(cover)");
      return IM_EDEVICE;
    }
    it = t_execs->emplace(key, ex).first;
  }
  (void)hipGraphDestroy(graph);
  IM_HIP(hipGraphLaunch(it->second, s));
  return IM_OK;
}

// k picks: 2k + 2 launches (plus a recount per heavy early pick), enqueued
// directly or as one captured graph (IM_TUNE_GRAPH).
int launch_cover(CoverArgs& A, hipStream_t s) {
  DeviceInfo di;
  IM_TRY(device_info(&di));
  CoverPlan P;
  P.init_blocks = (unsigned)std::min<int64_t>(
      std::max<int64_t>(((int64_t)A.n + kGBlock - 1) / kGBlock, 1), (int64_t)di.num_cus * 4);
  P.arg_blocks = (unsigned)std::max<int64_t>(((int64_t)A.n + kArgTile - 1) / kArgTile, 1);
  P.apply_blocks = (unsigned)di.num_cus * kApplyPerCu;
  P.agg_blocks = (unsigned)(di.num_cus * tune(IM_TUNE_APPLY_BLOCKS));
  P.recount_blocks = (unsigned)di.num_cus * 8;
  P.finish_blocks = (unsigned)((A.m + 255) / 256);
  // A plain one-partition cover rebuilds all counts after one of its first
  // kRecountPicks picks if that pick covers at least count / 64 samples (at
  // 2^20 weighted-cascade sets the first pick newly covers 41 K samples
  // holding 12 M members, the second 7 K holding 0.9 M; a recount is one pass
  // over the covering subsets, 0.1 ms); the decision is taken on the device
  // from the pick's gain.  Its other picks use the aggregated apply.
  P.can_recount = A.m == 1 && !A.order && !A.pos_of && !A.sbase && !A.local_ids;
  P.lists = A.cand != nullptr;
  A.recount_min = P.can_recount ? std::max<int64_t>(1, A.count / 64) : 0;
  bool graph = tune(IM_TUNE_GRAPH) != 0;
  if (graph) {  // a stream the caller is capturing gets the launches themselves
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    IM_HIP(hipStreamIsCapturing(s, &cs));
    graph = cs == hipStreamCaptureStatusNone;
  }
  int rc = IM_OK;
  if (graph) {
    rc = launch_captured(A, P, di.device, s);
  } else {
    enqueue_cover(A, P, s);
    if (hipGetLastError() != hipSuccess) rc = IM_EDEVICE;
  }
  A.recount_min = 0;
  return rc;
}

// Scratch of one standard greedy: done | gmax (k) | cnt (n) | covered (count).
static size_t greedy_bytes(int32_t n, int64_t count, int32_t k) {
  return 64 + (size_t)k * 8 + 64 + (size_t)n * 4 + (size_t)count + 64;
}

// Scratch of one RandGreedi local step: gmax (k m) | done | pbase (m + 1) |
// hist (m) | order, pos_of, cnt (n each) | covered (m count) | M, Moff (the
// partition counts per chunk of kPartChunk vertices and their scan) | member
// positions (total) | candidate lists (m kListCap) and their sizes and
// thresholds (m each).
static size_t randgreedi_bytes(int32_t n, int64_t count, int64_t total, int32_t k, int32_t m) {
  const int64_t nch = ((int64_t)n + kPartChunk - 1) / kPartChunk;
  const size_t cells = (size_t)m * (size_t)nch;
  return (size_t)m * k * 8 + 64 + 64 + (size_t)(m + 1) * 8 + (size_t)m * 4 + 64 +
         (size_t)n * 12 + (size_t)m * (size_t)count + 256 + (cells * 4 + 64) / 64 * 64 +
         (cells + 1) * 8 + 64 + (size_t)total * 4 + 64 + (size_t)m * kListCap * 4 +
         (size_t)m * 8 + 128;
}

size_t ws_greedy(int32_t n, int64_t count, int32_t k) {
  return ws_align(greedy_bytes(n, count, k));
}

size_t ws_randgreedi(int32_t n, int64_t count, int64_t total, int32_t k, int32_t m) {
  const int64_t nch = ((int64_t)n + kPartChunk - 1) / kPartChunk;
  return ws_align(randgreedi_bytes(n, count, total, k, m)) +
         ws_align((size_t)(((int64_t)m * nch) / 8192 + 2) * 8);
}

}  // namespace im

using namespace im;

extern "C" int im_greedy_cover(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                               int64_t total, const int64_t* inc_off, const int32_t* inc_mem,
                               int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel,
                               int64_t* coverage, void* ws, size_t ws_bytes, void* stream) {
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || total < 0 || k <= 0 || !off ||
      !inc_off || !seeds || !gains || !nsel || !coverage || (total > 0 && (!mem || !inc_mem)))
    return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_greedy(n, count, k))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = greedy_bytes(n, count, k);
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotGreedy, bytes, &p));
  char* c = (char*)p;
  CoverArgs A{};
  A.n = n;
  A.m = 1;
  A.count = count;
  A.k = k;
  A.off = off;
  A.mem = mem;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.done = (int32_t*)c;
  c += 64;
  A.gmax = (unsigned long long*)c;
  c += ((size_t)k * 8 + 63) / 64 * 64;
  A.cnt = (uint32_t*)c;
  c += (size_t)n * 4;
  A.covered = (uint8_t*)c;
  A.seeds = seeds;
  A.gains = gains;
  A.nsel = nsel;
  A.cover = coverage;
  IM_HIP(hipMemsetAsync(gains, 0, (size_t)k * 8, s));
  return launch_cover(A, s);
}

extern "C" int im_randgreedi(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                             int64_t total, const int64_t* inc_off, const int32_t* inc_mem,
                             int32_t k, int32_t m, uint64_t part_seed, uint8_t* part,
                             int32_t* lseeds, int64_t* lgains, int32_t* lcount, int64_t* lcover,
                             void* ws, size_t ws_bytes, void* stream) {
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || total < 0 || k <= 0 || m < 1 ||
      m > kMaxParts || !off || !inc_off || !part || !lseeds || !lgains || !lcount || !lcover ||
      (total > 0 && (!mem || !inc_mem)))
    return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_randgreedi(n, count, total, k, m))) return IM_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  k_partition<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
      n, m, (uint32_t)part_seed, (uint32_t)(part_seed >> 32), part);
  IM_HIP(hipGetLastError());
  // scratch: gmax(k*m) | done | pbase(m+1) | hist(m) | order(n) | pos_of(n) | cnt(n) |
  // covered(m*count) | M(m*nch) | Moff(m*nch+1)
  const int64_t nch = ((int64_t)n + kPartChunk - 1) / kPartChunk;
  const size_t cells = (size_t)m * (size_t)nch;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotLocal, randgreedi_bytes(n, count, total, k, m), &p));
  char* c = (char*)p;
  unsigned long long* gmax = (unsigned long long*)c;
  c += ((size_t)m * k * 8 + 63) / 64 * 64;
  int32_t* done = (int32_t*)c;
  c += 64;
  int64_t* pbase = (int64_t*)c;
  c += (size_t)(m + 1) * 8;
  uint32_t* hist = (uint32_t*)c;
  c += ((size_t)m * 4 + 63) / 64 * 64;
  int32_t* order = (int32_t*)c;
  c += (size_t)n * 4;
  int32_t* pos_of = (int32_t*)c;
  c += (size_t)n * 4;
  uint32_t* cnt = (uint32_t*)c;
  c += (size_t)n * 4;
  uint8_t* covered = (uint8_t*)c;
  c += (size_t)m * (size_t)count;
  c = (char*)(((uintptr_t)c + 63) / 64 * 64);
  uint32_t* M = (uint32_t*)c;
  c += (cells * 4 + 63) / 64 * 64;
  int64_t* Moff = (int64_t*)c;
  c += (cells + 1) * 8;
  c = (char*)(((uintptr_t)c + 63) / 64 * 64);
  int32_t* mpos = (int32_t*)c;
  c += (size_t)total * 4;
  c = (char*)(((uintptr_t)c + 63) / 64 * 64);
  int32_t* cand = (int32_t*)c;
  c += (size_t)m * kListCap * 4;
  int32_t* cand_n = (int32_t*)c;
  c += ((size_t)m * 4 + 63) / 64 * 64;
  uint32_t* tau = (uint32_t*)c;
  IM_HIP(hipMemsetAsync(hist, 0, (size_t)m * 4, s));
  k_part_count<<<dim3((unsigned)nch), dim3(kPartBlock), 0, s>>>(n, m, part, nch, M, hist);
  IM_HIP(hipGetLastError());
  IM_TRY(exclusive_scan_u32_to_i64(M, (int64_t)cells, Moff, s));
  std::vector<uint32_t> hh(m);
  IM_HIP(hipMemcpyAsync(hh.data(), hist, (size_t)m * 4, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> hb(m + 1);
  hb[0] = 0;
  for (int q = 0; q < m; ++q) hb[q + 1] = hb[q] + hh[q];
  IM_HIP(hipMemcpyAsync(pbase, hb.data(), (size_t)(m + 1) * 8, hipMemcpyHostToDevice, s));
  k_part_scatter<<<dim3((unsigned)nch), dim3(kPartBlock), 0, s>>>(n, m, part, nch, Moff, order);
  IM_HIP(hipGetLastError());
  k_pos_of<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, order, pos_of);
  IM_HIP(hipGetLastError());
  if (total > 0) {
    DeviceInfo di;
    IM_TRY(device_info(&di));
    const int64_t mb = std::min<int64_t>((total + 255) / 256, (int64_t)di.num_cus * 16);
    k_member_pos<<<dim3((unsigned)mb), dim3(256), 0, s>>>(mem, total, pos_of, mpos);
    IM_HIP(hipGetLastError());
  }
  CoverArgs A{};
  A.n = n;
  A.m = m;
  A.count = count;
  A.k = k;
  A.off = off;
  A.mem = mem;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.order = order;
  A.pos_of = pos_of;
  A.pos_keys = 1;  // the partition scatter keeps each partition in ascending id order
  A.part = part;
  A.mpos = total > 0 ? mpos : nullptr;
  if (tune(IM_TUNE_LISTS) != 0 && (int64_t)n <= (int64_t)m * kListMaxPart) {
    A.cand = cand;
    A.cand_n = cand_n;
    A.tau = tau;
  }
  A.pbase = pbase;
  A.cnt = cnt;
  A.covered = covered;
  A.gmax = gmax;
  A.done = done;
  A.seeds = lseeds;
  A.gains = lgains;
  A.nsel = lcount;
  A.cover = lcover;
  IM_HIP(hipMemsetAsync(lgains, 0, (size_t)m * k * 8, s));
  int st = launch_cover(A, s);
  if (st != IM_OK) return st;
  // the host copy of hb must outlive the async copy
  IM_HIP(hipStreamSynchronize(s));
  return IM_OK;
}

// ----------------------------------------------------------------------------
// The same standard greedy with its scratch in a fixed device array, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops).  Every device holds its own copy of the array for the
// life of the process; its device address is looked up once per device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// file scope, outside namespace im (whose scratch() is the per-stream buffer)
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace im {

constexpr int kMaxStaticDevices = 64;
static std::mutex g_static_mu;
static void* g_static_ptr[kMaxStaticDevices] = {};

static int static_scratch(void** out) {
  int dev = 0;
  IM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxStaticDevices) {
    set_error_text("im_greedy_cover_static: device ordinal " + std::to_string(dev) +
                   " beyond the table of " + std::to_string(kMaxStaticDevices));
    return IM_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    // the array's name is a host-side stand-in; kernels get this address
    IM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return IM_OK;
}

__global__ void k_fill_i64(int64_t* __restrict__ x, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace im

extern "C" int im_greedy_cover_static(int32_t n, int64_t count, const int64_t* off,
                                      const int32_t* mem, int64_t total, const int64_t* inc_off,
                                      const int32_t* inc_mem, int32_t k, int32_t* seeds,
                                      int64_t* gains, int32_t* nsel, int64_t* coverage,
                                      void* stream) {
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || total < 0 || k <= 0 || !off ||
      !inc_off || !seeds || !gains || !nsel || !coverage || (total > 0 && (!mem || !inc_mem)))
    return IM_EINVAL;
  // same layout as im_greedy_cover: done | gmax (k) | cnt (n) | covered (count)
  const size_t gbytes = ((size_t)k * 8 + 63) / 64 * 64;
  const size_t bytes = 64 + gbytes + (size_t)n * 4 + (size_t)count;
  if (bytes > kStaticScratchBytes) {
    set_error_text("im_greedy_cover_static: n = " + std::to_string(n) + ", count = " +
                   std::to_string(count) + ", k = " + std::to_string(k) + " need " +
                   std::to_string(bytes) + " bytes of scratch; the fixed buffer holds " +
                   std::to_string(kStaticScratchBytes));
    return IM_ENOMEM;
  }
  void* p = nullptr;
  IM_TRY(static_scratch(&p));
  hipStream_t s = (hipStream_t)stream;
  char* c = (char*)p;
  CoverArgs A{};
  A.n = n;
  A.m = 1;
  A.count = count;
  A.k = k;
  A.off = off;
  A.mem = mem;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.done = (int32_t*)c;
  c += 64;
  A.gmax = (unsigned long long*)c;
  c += gbytes;
  A.cnt = (uint32_t*)c;
  c += (size_t)n * 4;
  A.covered = (uint8_t*)c;
  A.seeds = seeds;
  A.gains = gains;
  A.nsel = nsel;
  A.cover = coverage;
  // gains start at zero (a fill kernel: no memset node if the caller captures)
  k_fill_i64<<<dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s>>>(gains, k, 0);
  IM_HIP(hipGetLastError());
  return launch_cover(A, s);
}
