// incidence.hip -- covering subsets S(v) = {j : v in R(j)} (im_build_incidence).
//
// Sec. 3.2 / Alg. 3 per-vertex step: the transpose of the sample-major RRR
// collection.  Two forms, chosen by members per vertex:
//
// Sparse collections (the usual RRR sets: a few dozen members per vertex) are
// transposed without global atomics -- device-scope atomics retire at a
// fraction of the rate of plain stores on this part, and a histogram plus a
// scatter would take two per member.  Vertex ids are cut into buckets of 2^b
// consecutive ids (b >= 12, at most 4096 buckets):
//   1. count: each workgroup histograms the bucket ids of one chunk of
//      members in LDS and writes one column of a bucket-major count matrix;
//   2. an exclusive scan of the matrix places every (bucket, chunk) run;
//   3. partition: the chunk is walked again, now knowing the sample that owns
//      each member, and (vertex, sample) pairs are written bucket by bucket;
//   4. bucket: one workgroup per bucket counts its vertices' degrees in LDS
//      and scans them -- the offsets of S(v) are the bucket's start plus this
//      local scan, since buckets are consecutive id ranges -- then scatters
//      the sample ids with LDS cursors.
// A collection whose pairs do not fit the pair budget is transposed in rounds
// of consecutive buckets.
//
// Dense collections (hundreds of members per vertex, where one workgroup per
// bucket would leave most of the chip idle) use a degree histogram and a
// scatter: counted in LDS tiles of vertex ids when every task spans a few
// tiles at most, else with one global atomic per member each.
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "incidence.h"

namespace im {

constexpr int kIncBlock = 512;
constexpr int64_t kMinChunk = 8192;  // members per workgroup pass, at least
constexpr int kMinBucketBits = 12;
constexpr int32_t kMaxBuckets = 4096;
constexpr int kBktBlock = 1024;
constexpr int kSub = 4 * kBktBlock;            // vertices per LDS pass of the bucket kernel

__device__ __forceinline__ int64_t last_leq(const int64_t* a, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n - 1;  // last index i < n with a[i] <= x
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (a[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t first_lane_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Per-wavefront LDS of the member walk.
struct WalkLds {
  int64_t pre[kWave];  // inclusive prefix of the group's clipped set sizes
  int64_t vb[kWave];   // vertex offset of the task of each lane's sample
  int64_t sb[kWave];   // sample offset of that task
};

// Calls f(vertex, sample) for every member in [a, b), the whole wavefront
// together.  It takes 64 consecutive samples at a time; their member ranges,
// clipped to [a, b), are consecutive in memory, so after one scan of their
// sizes the lanes read the members coalesced and find each member's sample
// by binary search over the 64 prefix sums.
template <bool kTasks, typename Lds, typename F>
__device__ __forceinline__ void walk_wave(const IncSrc& S, int64_t a, int64_t b, Lds& W, F&& f) {
  if (a >= b) return;
  const int lane = lane_id();
  int64_t jg = first_lane_i64(last_leq(S.off, S.count, a));
  for (;;) {
    const int64_t j = jg + lane;
    int64_t s0 = S.total, s1 = S.total;
    if (j < S.count) {
      s0 = S.off[j];
      s1 = S.off[j + 1];
    }
    const int64_t c0 = max(s0, a), c1 = min(s1, b);
    const int64_t sz = c1 > c0 ? c1 - c0 : 0;
    const int64_t incl = wave_inclusive_scan(sz);
    const int64_t all = __shfl(incl, kWave - 1, kWave);
    const int64_t first = __shfl(c0, 0, kWave);
    W.pre[lane] = incl;
    if constexpr (kTasks) {
      int64_t vbl = 0, sbl = 0;
      if (j < S.count) {
        const int64_t t = last_leq(S.sbase, S.ntasks, j);
        vbl = S.vbase[t];
        sbl = S.sbase[t];
      }
      W.vb[lane] = vbl;
      W.sb[lane] = sbl;
    }
    wave_sync();
    for (int64_t x = lane; x < all; x += kWave) {
      int lo = 0, hi = kWave - 1;  // first lane whose inclusive prefix exceeds x
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (W.pre[mid] > x)
          hi = mid;
        else
          lo = mid + 1;
      }
      if constexpr (kTasks)
        f(W.vb[lo] + (int64_t)S.mem[first + x], jg + lo - W.sb[lo]);
      else
        f((int64_t)S.mem[first + x], jg + lo);
    }
    const int64_t last_end = __shfl(s1, kWave - 1, kWave);
    wave_sync();
    if (jg + kWave >= S.count || last_end >= b) break;
    jg += kWave;
  }
}

// The members of chunk c: [c * chunk, min((c + 1) * chunk, total)), split
// evenly over the block's wavefronts for the walk.
__device__ __forceinline__ void wave_range(int64_t c, int64_t chunk, int64_t total, int64_t* a,
                                           int64_t* b) {
  const int64_t c0 = c * chunk, c1 = min(c0 + chunk, total);
  const int64_t per = (c1 - c0 + kIncBlock / kWave - 1) / (kIncBlock / kWave);
  const int w = threadIdx.x / kWave;
  *a = min(c1, c0 + w * per);
  *b = min(c1, *a + per);
}

template <bool kTasks>
__global__ __launch_bounds__(kIncBlock) void k_inc_count(IncSrc S, int32_t nv, int bits,
                                                         int32_t nb, int64_t chunk,
                                                         int64_t nchunks,
                                                         uint32_t* __restrict__ M) {
  __shared__ uint32_t hist[kMaxBuckets];
  __shared__ WalkLds walk[kIncBlock / kWave];
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    for (int b = threadIdx.x; b < nb; b += kIncBlock) hist[b] = 0u;
    __syncthreads();
    if (!kTasks) {  // no owners needed: read the chunk coalesced
      const int64_t c1 = min((c + 1) * chunk, S.total);
      for (int64_t t = c * chunk + threadIdx.x; t < c1; t += kIncBlock) {
        const uint32_t v = (uint32_t)S.mem[t];
        if (v < (uint32_t)nv) atomicAdd(&hist[v >> bits], 1u);
      }
    } else {
      int64_t a, b;
      wave_range(c, chunk, S.total, &a, &b);
      walk_wave<true>(S, a, b, walk[threadIdx.x / kWave], [&](int64_t v, int64_t) {
        if (v >= 0 && v < nv) atomicAdd(&hist[(uint32_t)v >> bits], 1u);
      });
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kIncBlock) M[(int64_t)b * nchunks + c] = hist[b];
    __syncthreads();
  }
}

// Writes the pairs of buckets [b0, b1) only, at their place minus rs (the
// place of bucket b0's first pair).
template <bool kTasks>
__global__ __launch_bounds__(kIncBlock) void k_inc_partition(IncSrc S, int32_t nv, int bits,
                                                             int32_t b0, int32_t b1,
                                                             int64_t chunk, int64_t nchunks,
                                                             int64_t rs,
                                                             const int64_t* __restrict__ Moff,
                                                             int32_t* __restrict__ pv,
                                                             int32_t* __restrict__ pj) {
  __shared__ int64_t base[kMaxBuckets];
  __shared__ uint32_t cur[kMaxBuckets];
  __shared__ WalkLds walk[kIncBlock / kWave];
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    for (int b = b0 + threadIdx.x; b < b1; b += kIncBlock) {
      base[b] = Moff[(int64_t)b * nchunks + c] - rs;
      cur[b] = 0u;
    }
    __syncthreads();
    int64_t a, e;
    wave_range(c, chunk, S.total, &a, &e);
    walk_wave<kTasks>(S, a, e, walk[threadIdx.x / kWave], [&](int64_t v, int64_t j) {
      if (v >= 0 && v < nv) {
        const int32_t b = (int32_t)((uint32_t)v >> bits);
        if (b >= b0 && b < b1) {
          const int64_t idx = base[b] + atomicAdd(&cur[b], 1u);
          pv[idx] = (int32_t)v;
          pj[idx] = (int32_t)j;
        }
      }
    });
    __syncthreads();
  }
}

__device__ __forceinline__ int64_t bkt_exclusive_scan(int64_t x, int64_t* lds, int64_t* total) {
  // lds: kBktBlock / kWave + 1 entries; every thread of the block must call
  const int t = threadIdx.x, l = lane_id(), w = t / kWave;
  const int64_t inc = wave_inclusive_scan(x);
  if (l == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    const int64_t v = l < kBktBlock / kWave ? lds[l] : 0;
    const int64_t vi = wave_inclusive_scan(v);
    if (l < kBktBlock / kWave) lds[l] = vi - v;
    if (l == kWave - 1) lds[kBktBlock / kWave] = vi;
  }
  __syncthreads();
  const int64_t r = lds[w] + inc - x;
  *total = lds[kBktBlock / kWave];
  __syncthreads();
  return r;
}

// Bucket b0 + blockIdx.x; its pairs sit at [Moff[bk * nchunks] - rs, ...).
__global__ __launch_bounds__(kBktBlock) void k_inc_bucket(int32_t n, int bits, int32_t b0,
                                                          int64_t nchunks, int64_t rs,
                                                          const int64_t* __restrict__ Moff,
                                                          const int32_t* __restrict__ pv,
                                                          const int32_t* __restrict__ pj,
                                                          int64_t* __restrict__ inc_off,
                                                          int32_t* __restrict__ inc_mem) {
  __shared__ uint32_t cnt[kSub];
  __shared__ int64_t obase[kSub];
  __shared__ int64_t lds[kBktBlock / kWave + 1];
  const int tid = threadIdx.x;
  const int64_t bk = (int64_t)b0 + blockIdx.x;
  const int64_t a0 = Moff[bk * nchunks], a1 = Moff[(bk + 1) * nchunks];
  const int64_t i0 = a0 - rs, i1 = a1 - rs;  // pair indices
  const int64_t v0 = bk << bits;
  const int64_t v1 = min((int64_t)n, v0 + ((int64_t)1 << bits));
  int64_t run = a0;  // members of the vertices before the current sub-range
  for (int64_t s0 = v0; s0 < v1; s0 += kSub) {
    const int64_t w = min((int64_t)kSub, v1 - s0);
    for (int x = tid; x < kSub; x += kBktBlock) cnt[x] = 0u;
    __syncthreads();
    for (int64_t idx = i0 + tid; idx < i1; idx += kBktBlock) {
      const int64_t d = (int64_t)pv[idx] - s0;
      if (d >= 0 && d < w) atomicAdd(&cnt[d], 1u);
    }
    __syncthreads();
    uint32_t c4[4];
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c4[q] = cnt[tid * 4 + q];
      sum += c4[q];
    }
    int64_t tot;
    int64_t ex = bkt_exclusive_scan(sum, lds, &tot) + run;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int x = tid * 4 + q;
      obase[x] = ex;
      if (x < w) inc_off[s0 + x] = ex;
      ex += c4[q];
      cnt[x] = 0u;  // becomes the scatter cursor
    }
    run += tot;
    __syncthreads();
    for (int64_t idx = i0 + tid; idx < i1; idx += kBktBlock) {
      const int64_t d = (int64_t)pv[idx] - s0;
      if (d >= 0 && d < w) inc_mem[obase[d] + atomicAdd(&cnt[d], 1u)] = pj[idx];
    }
    __syncthreads();
  }
  if (v1 == (int64_t)n && tid == 0) inc_off[n] = run;
}

// ---- dense collections: one global atomic per member and pass
constexpr int kAtomBlock = 256;
constexpr int kAtomRun = 16;  // members per thread in the scatter

__global__ __launch_bounds__(kAtomBlock) void k_degree(const int32_t* __restrict__ mem,
                                                       int64_t total, uint32_t* __restrict__ deg) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&deg[mem[t]], 1u);
}

__global__ __launch_bounds__(kAtomBlock) void k_scatter(int64_t count,
                                                        const int64_t* __restrict__ off,
                                                        const int32_t* __restrict__ mem,
                                                        int64_t total,
                                                        const int64_t* __restrict__ inc_off,
                                                        uint32_t* __restrict__ fill,
                                                        int32_t* __restrict__ inc_mem) {
  const int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kAtomRun;
  if (t0 >= total) return;
  // owner of member t0: the last j with off[j] <= t0
  int64_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t0)
      lo = mid;
    else
      hi = mid - 1;
  }
  int64_t j = lo;
  int64_t end_j = off[j + 1];
  const int64_t t1 = min(t0 + kAtomRun, total);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= end_j) {
      ++j;
      end_j = off[j + 1];
    }
    const int32_t v = mem[t];
    const uint32_t slot = atomicAdd(&fill[v], 1u);
    inc_mem[inc_off[v] + slot] = (int32_t)j;
  }
}

// The same for a task collection: each thread walks kAtomRun consecutive
// members, tracking the sample and the task that own them.  kScatter = false:
// degree histogram; true: scatter.
template <bool kScatter>
__global__ __launch_bounds__(kAtomBlock) void k_task_incidence(IncSrc S,
                                                               uint32_t* __restrict__ deg,
                                                               uint32_t* __restrict__ fill,
                                                               const int64_t* __restrict__ inc_off,
                                                               int32_t* __restrict__ inc_mem) {
  const int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kAtomRun;
  if (t0 >= S.total) return;
  int64_t j = last_leq(S.off, S.count, t0);
  int64_t end_j = S.off[j + 1];
  int task = (int)last_leq(S.sbase, S.ntasks, j);
  int64_t task_end = S.sbase[task + 1];
  const int64_t t1 = min(t0 + kAtomRun, S.total);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= end_j) {
      ++j;
      end_j = S.off[j + 1];
    }
    while (j >= task_end) {
      ++task;
      task_end = S.sbase[task + 1];
    }
    const int64_t gv = S.vbase[task] + S.mem[t];
    if (!kScatter) {
      atomicAdd(&deg[gv], 1u);
    } else {
      const uint32_t slot = atomicAdd(&fill[gv], 1u);
      inc_mem[inc_off[gv] + slot] = (int32_t)(j - S.sbase[task]);
    }
  }
}

// ---- dense collections over small vertex ranges: LDS tiles
// When no task spans more than a few tiles of kTileV consecutive vertex ids,
// both passes count in LDS instead.  A work item is (task, slice of the
// task's samples holding about L members, tile); items are numbered task by
// task with the tile fastest, so the items that read one slice run at about
// the same time and share its members in the caches.
//   degree: the item counts the slice's members that fall in its tile with
//     LDS atomics, then adds each nonzero count to deg: one device atomic per
//     (item, vertex) instead of one per member;
//   scatter: the item counts again, reserves a run of S(v) for each of its
//     vertices with one device atomic, and walks the slice's samples placing
//     their ids with LDS cursors.
// The cursors are 32-bit offsets from the tile's first S(v); a tile whose
// covering subsets hold 2^32 entries or more takes device atomics per member.
constexpr int kTileBlock = 1024;
constexpr int32_t kTileV = 32768;                  // vertices per tile: 128 KB of counters
constexpr int kMaxTiles = 4;                       // tiles per task, at most, for this form
constexpr int64_t kTileMembers = (int64_t)1 << 22; // members per slice, at least
constexpr int64_t kMaxSlices = 4096;               // slices per collection, about

struct TileItem {
  int64_t s0;      // first sample of the task (sample ids in S(v) are task-local)
  int64_t j0, j1;  // samples of the slice
  int64_t v;       // first vertex of the tile, global
  uint32_t lo;     // first vertex of the tile, task-local (the id the members hold)
  uint32_t width;  // vertices in the tile
};

struct TileWalk {
  int64_t pre[kWave];
};

__device__ __forceinline__ int64_t first_geq(const int64_t* a, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {  // first i in [lo, hi) with a[i] >= x, else hi
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] >= x)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ void task_bounds(const IncSrc& S, int32_t nv, int64_t t, int64_t* s0,
                                            int64_t* s1, int64_t* v0, int64_t* v1) {
  if (S.ntasks == 0) {
    *s0 = 0;
    *s1 = S.count;
    *v0 = 0;
    *v1 = nv;
  } else {
    *s0 = S.sbase[t];
    *s1 = S.sbase[t + 1];
    *v0 = S.vbase[t];
    *v1 = S.vbase[t + 1];
  }
}

// itm[t + 1] - itm[t] = items of task t (slices x tiles); one wavefront.
__global__ __launch_bounds__(kWave) void k_tile_items(IncSrc S, int32_t nv, int64_t L,
                                                      int64_t* __restrict__ itm) {
  const int nt = S.ntasks > 0 ? S.ntasks : 1, lane = lane_id();
  int64_t carry = 0;
  for (int base = 0; base < nt; base += kWave) {
    const int t = base + lane;
    int64_t c = 0;
    if (t < nt) {
      int64_t s0, s1, v0, v1;
      task_bounds(S, nv, t, &s0, &s1, &v0, &v1);
      const int64_t m = S.off[s1] - S.off[s0];
      c = ((m + L - 1) / L) * ((v1 - v0 + kTileV - 1) / kTileV);
    }
    const int64_t incl = wave_inclusive_scan(c);
    if (t < nt) itm[t + 1] = carry + incl;
    carry += __shfl(incl, kWave - 1, kWave);
  }
  if (lane == 0) itm[0] = 0;
}

__device__ __forceinline__ TileItem tile_item(const IncSrc& S, int32_t nv, int64_t L,
                                              const int64_t* __restrict__ itm, int nt, int64_t i) {
  const int64_t t = last_leq(itm, nt, i);
  int64_t s0, s1, v0, v1;
  task_bounds(S, nv, t, &s0, &s1, &v0, &v1);
  const int64_t ntl = (v1 - v0 + kTileV - 1) / kTileV;
  const int64_t r = i - itm[t], sl = r / ntl, tl = r - sl * ntl;
  const int64_t m0 = S.off[s0], m1 = S.off[s1];
  const int64_t nsl = (m1 - m0 + L - 1) / L;
  TileItem it;
  it.s0 = s0;
  // sample j belongs to the slice that holds its first member
  it.j0 = sl == 0 ? s0 : first_geq(S.off, s0, s1, m0 + sl * L);
  it.j1 = sl == nsl - 1 ? s1 : first_geq(S.off, s0, s1, m0 + (sl + 1) * L);
  it.lo = (uint32_t)(tl * kTileV);
  it.v = v0 + it.lo;
  it.width = (uint32_t)(v1 - it.v < kTileV ? v1 - it.v : kTileV);
  return it;
}

// h[u] = members of the item's slice equal to lo + u, u < width.  Ends synchronised.
__device__ __forceinline__ void tile_count(const IncSrc& S, const TileItem& it,
                                           uint32_t* __restrict__ h) {
  for (uint32_t k = threadIdx.x; k < it.width; k += kTileBlock) h[k] = 0;
  __syncthreads();
  const int64_t a = S.off[it.j0], b = S.off[it.j1];
  auto add = [&](int32_t x) {
    const uint32_t u = (uint32_t)x - it.lo;
    if (u < it.width) atomicAdd(&h[u], 1u);
  };
  // 16-byte loads over the aligned middle, two per thread in flight
  const int64_t q0 = (a + 3) >> 2, q1 = b >> 2;
  if (q0 >= q1 || ((uintptr_t)S.mem & 15) != 0) {
    for (int64_t m = a + threadIdx.x; m < b; m += kTileBlock) add(S.mem[m]);
  } else {
    for (int64_t m = a + threadIdx.x; m < q0 * 4; m += kTileBlock) add(S.mem[m]);
    for (int64_t m = q1 * 4 + threadIdx.x; m < b; m += kTileBlock) add(S.mem[m]);
    const int4* __restrict__ m4 = (const int4*)S.mem;
    int64_t q = q0 + threadIdx.x;
    for (; q + kTileBlock < q1; q += 2 * kTileBlock) {
      const int4 x = m4[q], y = m4[q + kTileBlock];
      add(x.x), add(x.y), add(x.z), add(x.w);
      add(y.x), add(y.y), add(y.z), add(y.w);
    }
    if (q < q1) {
      const int4 x = m4[q];
      add(x.x), add(x.y), add(x.z), add(x.w);
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kTileBlock) void k_tile_degree(IncSrc S, int32_t nv, int64_t L,
                                                            const int64_t* __restrict__ itm,
                                                            uint32_t* __restrict__ deg) {
  __shared__ uint32_t h[kTileV];
  const int nt = S.ntasks > 0 ? S.ntasks : 1;
  const int64_t n_items = itm[nt];
  for (int64_t i = blockIdx.x; i < n_items; i += gridDim.x) {
    const TileItem it = tile_item(S, nv, L, itm, nt, i);
    tile_count(S, it, h);
    for (uint32_t k = threadIdx.x; k < it.width; k += kTileBlock) {
      const uint32_t c = h[k];
      if (c) atomicAdd(&deg[it.v + k], c);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kTileBlock) void k_tile_scatter(IncSrc S, int32_t nv, int64_t L,
                                                             const int64_t* __restrict__ itm,
                                                             uint32_t* __restrict__ fill,
                                                             const int64_t* __restrict__ inc_off,
                                                             int32_t* __restrict__ inc_mem) {
  __shared__ uint32_t h[kTileV];
  __shared__ TileWalk walk[kTileBlock / kWave];
  const int nt = S.ntasks > 0 ? S.ntasks : 1;
  const int64_t n_items = itm[nt];
  const int nw = kTileBlock / kWave, w = threadIdx.x / kWave;
  for (int64_t i = blockIdx.x; i < n_items; i += gridDim.x) {
    const TileItem it = tile_item(S, nv, L, itm, nt, i);
    tile_count(S, it, h);
    const int64_t cbase = inc_off[it.v];
    const bool cursors = inc_off[it.v + it.width] - cbase < ((int64_t)1 << 32);
    if (cursors) {
      for (uint32_t k = threadIdx.x; k < it.width; k += kTileBlock) {
        const uint32_t c = h[k];
        if (c) {
          const uint32_t pos = atomicAdd(&fill[it.v + k], c);
          h[k] = (uint32_t)(inc_off[it.v + k] - cbase) + pos;
        }
      }
      __syncthreads();
    }
    // each wavefront walks an equal share of the slice's members
    const int64_t a = S.off[it.j0], len = S.off[it.j1] - a;
    walk_wave<false>(S, a + len * w / nw, a + len * (w + 1) / nw, walk[w],
                     [&](int64_t x, int64_t j) {
                       const uint32_t u = (uint32_t)x - it.lo;
                       if (u >= it.width) return;
                       const int32_t id = (int32_t)(j - it.s0);
                       if (cursors) {
                         inc_mem[cbase + atomicAdd(&h[u], 1u)] = id;
                       } else {
                         const int64_t gv = it.v + u;
                         inc_mem[inc_off[gv] + atomicAdd(&fill[gv], 1u)] = id;
                       }
                     });
    __syncthreads();
  }
}

static int64_t tile_limit() {  // IM_INCIDENCE_DENSE_TILES: tiles per task, at most (0: never)
  if (const char* env = getenv("IM_INCIDENCE_DENSE_TILES")) return atoll(env);
  return kMaxTiles;
}

static int build_incidence_tiled(const IncSrc& S, int32_t nv, int64_t* inc_off, int32_t* inc_mem,
                                 hipStream_t s) {
  const int nt = S.ntasks > 0 ? S.ntasks : 1;
  const size_t bDeg = ((size_t)nv * 8 + 255) / 256 * 256;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotIncidence, bDeg + (size_t)(nt + 1) * 8, &p));
  uint32_t* deg = (uint32_t*)p;
  uint32_t* fill = deg + nv;
  int64_t* itm = (int64_t*)((char*)p + bDeg);
  IM_HIP(hipMemsetAsync(deg, 0, (size_t)nv * 8, s));
  // IM_INCIDENCE_TILE_MEMBERS (>= 1) sets the slice length, to exercise many slices
  int64_t L = std::max<int64_t>(kTileMembers, (S.total + kMaxSlices - 1) / kMaxSlices);
  if (const char* env = getenv("IM_INCIDENCE_TILE_MEMBERS"))
    if (atoll(env) >= 1) L = atoll(env);
  DeviceInfo di;
  IM_TRY(device_info(&di));
  const unsigned grid = (unsigned)di.num_cus;  // one 128 KB workgroup per CU
  k_tile_items<<<dim3(1), dim3(kWave), 0, s>>>(S, nv, L, itm);
  IM_HIP(hipGetLastError());
  k_tile_degree<<<dim3(grid), dim3(kTileBlock), 0, s>>>(S, nv, L, itm, deg);
  IM_HIP(hipGetLastError());
  IM_TRY(exclusive_scan_u32_to_i64(deg, nv, inc_off, s));
  k_tile_scatter<<<dim3(grid), dim3(kTileBlock), 0, s>>>(S, nv, L, itm, fill, inc_off, inc_mem);
  IM_HIP(hipGetLastError());
  return IM_OK;
}

static int build_incidence_dense(const IncSrc& S, int32_t nv, int64_t* inc_off,
                                 int32_t* inc_mem, hipStream_t s) {
  if (S.vspan > 0 && (S.vspan + kTileV - 1) / kTileV <= tile_limit())
    return build_incidence_tiled(S, nv, inc_off, inc_mem, s);
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotIncidence, (size_t)nv * 8, &p));
  uint32_t* deg = (uint32_t*)p;
  uint32_t* fill = deg + nv;
  IM_HIP(hipMemsetAsync(deg, 0, (size_t)nv * 8, s));
  DeviceInfo di;
  IM_TRY(device_info(&di));
  const int64_t runs = (S.total + kAtomRun - 1) / kAtomRun;
  const unsigned rblocks = (unsigned)((runs + kAtomBlock - 1) / kAtomBlock);
  if (S.ntasks > 0) {
    k_task_incidence<false><<<dim3(rblocks), dim3(kAtomBlock), 0, s>>>(S, deg, fill, inc_off,
                                                                        inc_mem);
  } else {
    const int64_t blocks = std::min<int64_t>((S.total + kAtomBlock - 1) / kAtomBlock,
                                             (int64_t)di.num_cus * 16);
    k_degree<<<dim3((unsigned)blocks), dim3(kAtomBlock), 0, s>>>(S.mem, S.total, deg);
  }
  IM_HIP(hipGetLastError());
  IM_TRY(exclusive_scan_u32_to_i64(deg, nv, inc_off, s));
  if (S.ntasks > 0)
    k_task_incidence<true><<<dim3(rblocks), dim3(kAtomBlock), 0, s>>>(S, deg, fill, inc_off,
                                                                       inc_mem);
  else
    k_scatter<<<dim3(rblocks), dim3(kAtomBlock), 0, s>>>(S.count, S.off, S.mem, S.total, inc_off,
                                                         fill, inc_mem);
  IM_HIP(hipGetLastError());
  return IM_OK;
}

// Pair budget: the (vertex, sample) pairs of one round of buckets, as many as
// the workspace holds beside the scan of `cells` counts (at least 2^24, or
// the total when smaller).  A collection whose pairs exceed it is transposed
// in rounds of consecutive buckets, each round re-walking the members once.
// IM_INCIDENCE_PAIR_BUDGET (pairs, >= 1) overrides it, to exercise the rounds.
static int64_t pair_budget(int64_t total, int64_t cells) {
  if (const char* env = getenv("IM_INCIDENCE_PAIR_BUDGET")) {
    const long long b = atoll(env);
    if (b >= 1) return std::min<int64_t>(total, (int64_t)b);
  }
  const size_t scan = ws_align((size_t)(cells / 8192 + 2) * 8) + 512;
  const size_t room = scratch_largest();
  const int64_t fit = room > scan ? (int64_t)((room - scan) / 8) : 0;
  return std::max<int64_t>(std::min<int64_t>(total, (int64_t)1 << 24),
                           std::min<int64_t>(total, fit));
}

// Members per vertex above which a collection takes the dense form
// (IM_TUNE_DENSE_RATIO); IM_INCIDENCE_DENSE_RATIO overrides it (0: always
// dense), for the tests.
static int64_t dense_ratio() {
  if (const char* env = getenv("IM_INCIDENCE_DENSE_RATIO")) return atoll(env);
  return tune(IM_TUNE_DENSE_RATIO);
}

int build_incidence(const IncSrc& S, int32_t nv, int64_t* inc_off, int32_t* inc_mem,
                    hipStream_t s) {
  if (S.total == 0) {
    IM_HIP(hipMemsetAsync(inc_off, 0, (size_t)(nv + 1) * 8, s));
    return IM_OK;
  }
  if (S.total > dense_ratio() * (int64_t)nv) return build_incidence_dense(S, nv, inc_off, inc_mem, s);
  int bits = kMinBucketBits;
  while ((((int64_t)nv - 1) >> bits) + 1 > kMaxBuckets) ++bits;
  const int32_t nb = (int32_t)((((int64_t)nv - 1) >> bits) + 1);
  // chunks of at least 64 * nb members keep the count matrix at most total / 64 cells
  const int64_t chunk = std::max<int64_t>(kMinChunk, (int64_t)64 * nb);
  const int64_t nchunks = (S.total + chunk - 1) / chunk;
  const int64_t cells = (int64_t)nb * nchunks;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t bM = up((size_t)cells * 4), bMoff = up((size_t)(cells + 1) * 8);
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotIncidence, bM + bMoff, &p));
  const int64_t budget = pair_budget(S.total, cells);
  if (budget < S.total)  // one round would have been enough with room for every pair
    scratch_wish(2 * ws_align((size_t)S.total * 4) + ws_align((size_t)(cells / 8192 + 2) * 8));
  uint32_t* M = (uint32_t*)p;
  int64_t* Moff = (int64_t*)((char*)p + bM);
  int32_t *pv = nullptr, *pj = nullptr;
  auto pairs = [&](int64_t n_pairs) -> int {  // its own slot: growing it keeps M and Moff
    const size_t bP = up((size_t)n_pairs * 4);
    void* q = nullptr;
    IM_TRY(scratch(s, kSlotIncPairs, 2 * bP, &q));
    pv = (int32_t*)q;
    pj = (int32_t*)((char*)q + bP);
    return IM_OK;
  };
  IM_TRY(pairs(budget));
  DeviceInfo di;
  IM_TRY(device_info(&di));
  const unsigned blocks = (unsigned)std::min<int64_t>(nchunks, (int64_t)di.num_cus * 4);
  if (S.ntasks > 0)
    k_inc_count<true><<<dim3(blocks), dim3(kIncBlock), 0, s>>>(S, nv, bits, nb, chunk,
                                                               nchunks, M);
  else
    k_inc_count<false><<<dim3(blocks), dim3(kIncBlock), 0, s>>>(S, nv, bits, nb, chunk,
                                                                nchunks, M);
  IM_HIP(hipGetLastError());
  IM_TRY(exclusive_scan_u32_to_i64(M, cells, Moff, s));
  auto round = [&](int32_t b0, int32_t b1, int64_t rs) -> int {
    if (S.ntasks > 0)
      k_inc_partition<true><<<dim3(blocks), dim3(kIncBlock), 0, s>>>(S, nv, bits, b0, b1, chunk,
                                                                     nchunks, rs, Moff, pv, pj);
    else
      k_inc_partition<false><<<dim3(blocks), dim3(kIncBlock), 0, s>>>(S, nv, bits, b0, b1, chunk,
                                                                      nchunks, rs, Moff, pv, pj);
    IM_HIP(hipGetLastError());
    k_inc_bucket<<<dim3((unsigned)(b1 - b0)), dim3(kBktBlock), 0, s>>>(nv, bits, b0, nchunks, rs,
                                                                      Moff, pv, pj, inc_off,
                                                                      inc_mem);
    IM_HIP(hipGetLastError());
    return IM_OK;
  };
  if (budget >= S.total) return round(0, nb, 0);
  // rounds: bucket starts on the host, then greedy groups of whole buckets
  std::vector<int64_t> bs(nb + 1);
  IM_HIP(hipMemcpy2DAsync(bs.data(), 8, Moff, (size_t)nchunks * 8, 8, (size_t)nb,
                          hipMemcpyDeviceToHost, s));
  IM_HIP(hipMemcpyAsync(&bs[nb], Moff + cells, 8, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  for (int32_t b0 = 0; b0 < nb;) {
    int32_t b1 = b0 + 1;  // a bucket larger than the budget gets a round of its own
    while (b1 < nb && bs[b1 + 1] - bs[b0] <= budget) ++b1;
    if (bs[b1] - bs[b0] > budget) IM_TRY(pairs(bs[b1] - bs[b0]));  // one oversized bucket
    IM_TRY(round(b0, b1, bs[b0]));
    b0 = b1;
  }
  return IM_OK;
}

static size_t ws_scan(int64_t n) { return ws_align((size_t)(n / 8192 + 2) * 8); }

size_t ws_incidence(int32_t nv, int64_t total, int32_t ntasks, bool full) {
  if (total <= 0) return 0;
  if (total > dense_ratio() * (int64_t)nv)  // either dense form
    return ws_align((size_t)nv * 8) + ws_align((size_t)(std::max(ntasks, 1) + 1) * 8) +
           ws_align((size_t)nv * 8) + ws_scan(nv);
  int bits = kMinBucketBits;
  while ((((int64_t)nv - 1) >> bits) + 1 > kMaxBuckets) ++bits;
  const int64_t nb = (((int64_t)nv - 1) >> bits) + 1;
  const int64_t chunk = std::max<int64_t>(kMinChunk, (int64_t)64 * nb);
  const int64_t cells = nb * ((total + chunk - 1) / chunk);
  const int64_t pairs = full ? total : std::min<int64_t>(total, (int64_t)1 << 24);
  return ws_align((size_t)cells * 4) + ws_align((size_t)(cells + 1) * 8) +
         2 * ws_align((size_t)pairs * 4) + ws_scan(cells) + 1024;
}

}  // namespace im

extern "C" int im_build_incidence(int32_t n, int64_t count, const int64_t* off,
                                  const int32_t* mem, int64_t total, int64_t* inc_off,
                                  int32_t* inc_mem, void* ws, size_t ws_bytes, void* stream) {
  using namespace im;
  if (n <= 0 || count < 0 || total < 0 || !off || !inc_off || (total > 0 && (!mem || !inc_mem)) ||
      count >= ((int64_t)1 << 31) || (total > 0 && count == 0))
    return IM_EINVAL;
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_incidence(n, total, 0, false))) return IM_ENOMEM;
  const IncSrc S{off, count, mem, total, nullptr, nullptr, 0, n};
  return build_incidence(S, n, inc_off, inc_mem, (hipStream_t)stream);
}
