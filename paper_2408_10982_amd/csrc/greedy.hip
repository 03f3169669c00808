// greedy.hip -- standard greedy max-k-cover (im_greedy_cover) and the
// RandGreedi local step over m vertex partitions (im_randgreedi).
//
// Sec. 3.2: k times, take the vertex of largest marginal coverage (lowest id
// on ties).  The marginal coverage of every vertex is kept exactly as a count
// of its still-uncovered samples: when a sample becomes covered, every member
// of that sample loses one.  Both steps run in one persistent cooperative
// launch with two grid barriers per pick:
//   A. every workgroup reduces the per-tile maxima (redundantly, no barrier
//      needed) to the argmax key (count << 32 | ~v);
//   B. the samples of S(v*) are spread over the grid; newly covered samples
//      decrement their members' counts and mark the members' tiles dirty;
//   C. dirty tiles recompute their maxima.
// The RandGreedi form runs all m partitions in the same launch: vertices are
// laid out partition by partition, tiles never straddle partitions, and a
// covered sample only decrements members of the partition that covered it
// (Alg. 4 lines 1-2 with the full universe of samples, Sec. 3.4 S3).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace cg = cooperative_groups;

namespace im {

constexpr int kGBlock = 256;
constexpr int kTile = 1024;  // vertices per tile (4 per thread)
constexpr int kMaxParts = 256;

struct CoverArgs {
  int32_t n;
  int32_t m;                 // partitions (1 for the standard greedy)
  int64_t count;             // samples
  int32_t k;
  const int64_t* __restrict__ off;
  const int32_t* __restrict__ mem;
  const int64_t* __restrict__ inc_off;
  const int32_t* __restrict__ inc_mem;
  const uint8_t* __restrict__ part;      // n (nullptr when m == 1)
  const int32_t* __restrict__ order;     // n: vertices partition by partition (nullptr: identity)
  const int32_t* __restrict__ tile_of;   // n: tile of each vertex (nullptr: v / kTile)
  const int32_t* __restrict__ tile_lo;   // ntiles: first position in `order`
  const int32_t* __restrict__ tile_hi;   // ntiles: end position
  const int32_t* __restrict__ part_tile; // m+1: tiles of partition p
  int32_t ntiles;
  uint32_t* __restrict__ cnt;            // n
  uint8_t* __restrict__ covered;         // m * count
  uint64_t* __restrict__ tile_max;       // ntiles
  uint32_t* __restrict__ dirty;          // ntiles
  int64_t* __restrict__ slice_pre;       // m+1 (scratch for the flattened slices)
  int32_t* __restrict__ seeds;           // m*k
  int64_t* __restrict__ gains;           // m*k
  int32_t* __restrict__ nsel;            // m
  int64_t* __restrict__ cover;           // m
};

__device__ __forceinline__ uint64_t block_max_u64(uint64_t x, uint64_t* lds) {
  x = wave_max_u64(x);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = x;
  __syncthreads();
  uint64_t r = 0;
  for (int j = 0; j < kGBlock / kWave; ++j) r = lds[j] > r ? lds[j] : r;
  __syncthreads();
  return r;
}

__device__ __forceinline__ uint64_t tile_reduce(const CoverArgs& A, int tile, uint64_t* lds) {
  const int32_t lo = A.tile_lo ? A.tile_lo[tile] : tile * kTile;
  const int32_t hi = A.tile_hi ? A.tile_hi[tile] : min((tile + 1) * kTile, A.n);
  uint64_t best = 0;
  for (int32_t pos = lo + threadIdx.x; pos < hi; pos += kGBlock) {
    const int32_t v = A.order ? A.order[pos] : pos;
    const uint64_t key = argmax_key(A.cnt[v], (uint32_t)v);
    best = key > best ? key : best;
  }
  return block_max_u64(best, lds);
}

__global__ __launch_bounds__(kGBlock) void k_cover(CoverArgs A) {
  cg::grid_group grid = cg::this_grid();
  __shared__ uint64_t red[kGBlock / kWave];
  __shared__ uint64_t pbest[kMaxParts];
  __shared__ int64_t pre[kMaxParts + 1];
  const int64_t gtid = (int64_t)blockIdx.x * kGBlock + threadIdx.x;
  const int64_t gthreads = (int64_t)gridDim.x * kGBlock;

  // init: counts = |S(v)|, nothing covered, all tiles fresh
  for (int64_t v = gtid; v < A.n; v += gthreads)
    A.cnt[v] = (uint32_t)(A.inc_off[v + 1] - A.inc_off[v]);
  for (int64_t j = gtid; j < (int64_t)A.m * A.count; j += gthreads) A.covered[j] = 0;
  grid.sync();
  for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
    const uint64_t b = tile_reduce(A, t, red);
    if (threadIdx.x == 0) {
      A.tile_max[t] = b;
      A.dirty[t] = 0;
    }
  }
  grid.sync();

  int32_t picks = 0;
  for (int it = 0; it < A.k; ++it) {
    // A: per-partition argmax over tile maxima (every block, same result)
    for (int p = threadIdx.x; p < A.m; p += kGBlock) pbest[p] = 0;
    __syncthreads();
    for (int p = 0; p < A.m; ++p) {
      const int t0 = A.part_tile ? A.part_tile[p] : 0;
      const int t1 = A.part_tile ? A.part_tile[p + 1] : A.ntiles;
      uint64_t b = 0;
      for (int t = t0 + threadIdx.x; t < t1; t += kGBlock) {
        const uint64_t x = A.tile_max[t];
        b = x > b ? x : b;
      }
      b = block_max_u64(b, red);
      if (threadIdx.x == 0) pbest[p] = b;
    }
    __syncthreads();
    // flattened slices of the picks with a positive gain
    if (threadIdx.x == 0) {
      int64_t acc = 0;
      for (int p = 0; p < A.m; ++p) {
        pre[p] = acc;
        const uint64_t b = pbest[p];
        if (key_count(b) > 0) {
          const uint32_t v = key_vertex(b);
          acc += A.inc_off[v + 1] - A.inc_off[v];
        }
      }
      pre[A.m] = acc;
    }
    __syncthreads();
    if (pre[A.m] == 0) break;  // no partition has anything left to gain
    if (blockIdx.x == 0) {
      for (int p = threadIdx.x; p < A.m; p += kGBlock) {
        const uint64_t b = pbest[p];
        if (key_count(b) > 0) {
          A.seeds[(int64_t)p * A.k + it] = (int32_t)key_vertex(b);
          A.gains[(int64_t)p * A.k + it] = (int64_t)key_count(b);
        }
      }
    }
    ++picks;
    // B: cover S(v*_p) for every partition
    const int64_t tot = pre[A.m];
    for (int64_t f = gtid; f < tot; f += gthreads) {
      int lo = 0, hi = A.m - 1;  // partition owning flat index f
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= f)
          lo = mid;
        else
          hi = mid - 1;
      }
      const int p = lo;
      const uint32_t v = key_vertex(pbest[p]);
      const int32_t smp = A.inc_mem[A.inc_off[v] + (f - pre[p])];
      uint8_t* cov = A.covered + (int64_t)p * A.count;
      if (cov[smp]) continue;
      cov[smp] = 1;
      for (int64_t t = A.off[smp]; t < A.off[smp + 1]; ++t) {
        const int32_t u = A.mem[t];
        if (A.part && A.part[u] != (uint8_t)p) continue;
        atomicSub(&A.cnt[u], 1u);
        const int32_t tile = A.tile_of ? A.tile_of[u] : u / kTile;
        if (!A.dirty[tile]) A.dirty[tile] = 1;
      }
    }
    grid.sync();
    // C: refresh dirty tiles
    for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
      if (!A.dirty[t]) continue;  // uniform per block
      const uint64_t b = tile_reduce(A, t, red);
      if (threadIdx.x == 0) {
        A.tile_max[t] = b;
        A.dirty[t] = 0;
      }
    }
    grid.sync();
  }
  // outputs: per partition, picks with positive gain
  if (blockIdx.x == 0) {
    for (int p = threadIdx.x; p < A.m; p += kGBlock) {
      int32_t c = 0;
      int64_t s = 0;
      for (int it = 0; it < picks; ++it) {
        const int64_t g = A.gains[(int64_t)p * A.k + it];
        if (g <= 0) break;
        ++c;
        s += g;
      }
      for (int it = c; it < A.k; ++it) {
        A.seeds[(int64_t)p * A.k + it] = -1;
        A.gains[(int64_t)p * A.k + it] = 0;
      }
      A.nsel[p] = c;
      A.cover[p] = s;
    }
  }
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
__global__ void k_part_hist(int32_t n, const uint8_t* __restrict__ part,
                            uint32_t* __restrict__ hist) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicAdd(&hist[part[v]], 1u);
}

// One block per partition scans the vertex range in order, writing the
// partition's vertices in ascending id (stable).
__global__ __launch_bounds__(kGBlock) void k_part_order(int32_t n, const uint8_t* __restrict__ part,
                                                        const int64_t* __restrict__ pbase,
                                                        int32_t* __restrict__ order) {
  __shared__ int64_t lds[kGBlock / kWave + 1];
  const int p = blockIdx.x;
  int64_t base = pbase[p];
  for (int64_t v0 = 0; v0 < n; v0 += kGBlock) {
    const int64_t v = v0 + threadIdx.x;
    const int flag = (v < n && part[v] == (uint8_t)p) ? 1 : 0;
    // block exclusive scan of flag
    const int l = lane_id(), w = threadIdx.x / kWave;
    int inc = wave_inclusive_scan(flag);
    if (l == kWave - 1) lds[w] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int j = 0; j < kGBlock / kWave; ++j) {
      if (j < w) before += lds[j];
      tot += lds[j];
    }
    if (flag) order[base + before + inc - 1] = (int32_t)v;
    base += tot;
    __syncthreads();
  }
}

__global__ void k_tile_of(int32_t n, const int32_t* __restrict__ order,
                          const uint8_t* __restrict__ part, const int64_t* __restrict__ pbase,
                          const int32_t* __restrict__ part_tile, int32_t* __restrict__ tile_of) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const int32_t v = order[pos];
  const int q = part[v];
  tile_of[v] = part_tile[q] + (int32_t)((pos - pbase[q]) / kTile);
}

static int launch_cover(CoverArgs& A, hipStream_t s) {
  DeviceInfo di;
  IM_TRY(device_info(&di));
  int per_cu = 0;
  IM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_cover, kGBlock, 0));
  if (per_cu < 1) per_cu = 1;
  int64_t want = std::max<int64_t>(A.ntiles, 1);
  int64_t blocks = std::min<int64_t>((int64_t)per_cu * di.num_cus, std::max<int64_t>(want, di.num_cus));
  void* args[] = {&A};
  IM_HIP(hipLaunchCooperativeKernel((const void*)k_cover, dim3((unsigned)blocks), dim3(kGBlock),
                                    args, 0, s));
  return IM_OK;
}

}  // namespace im

using namespace im;

extern "C" int im_greedy_cover(int32_t n, int64_t count, const int64_t* off, const int32_t* mem,
                               int64_t total, const int64_t* inc_off, const int32_t* inc_mem,
                               int32_t k, int32_t* seeds, int64_t* gains, int32_t* nsel,
                               int64_t* coverage, void* stream) {
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || total < 0 || k <= 0 || !off ||
      !inc_off || !seeds || !gains || !nsel || !coverage || (total > 0 && (!mem || !inc_mem)))
    return IM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int32_t ntiles = (int32_t)(((int64_t)n + kTile - 1) / kTile);
  const size_t bytes = (size_t)n * 4 + (size_t)count + 16 + (size_t)ntiles * 12 + 64;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotGreedy, bytes + 64, &p));
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
  A.ntiles = ntiles;
  A.tile_max = (uint64_t*)c;
  c += (size_t)ntiles * 8;
  A.cnt = (uint32_t*)c;
  c += (size_t)n * 4;
  A.dirty = (uint32_t*)c;
  c += (size_t)ntiles * 4;
  A.slice_pre = nullptr;
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
                             void* stream) {
  if (n <= 0 || count < 0 || count >= ((int64_t)1 << 31) || total < 0 || k <= 0 || m < 1 ||
      m > kMaxParts || !off || !inc_off || !part || !lseeds || !lgains || !lcount || !lcover ||
      (total > 0 && (!mem || !inc_mem)))
    return IM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // partition, then lay vertices out partition by partition
  k_partition<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
      n, m, (uint32_t)part_seed, (uint32_t)(part_seed >> 32), part);
  IM_HIP(hipGetLastError());
  // scratch: hist(m u32) pbase(m+1 i64) order(n) tile_of(n) cnt(n) tiles... covered(m*count)
  const int64_t max_tiles = ((int64_t)n + kTile - 1) / kTile + m;
  const size_t bytes = (size_t)m * 4 + (size_t)(m + 1) * 8 + (size_t)n * 12 +
                       (size_t)max_tiles * (8 + 4 + 4 + 4) + (size_t)(m + 1) * 4 +
                       (size_t)m * (size_t)count + 256;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotLocal, bytes, &p));
  char* c = (char*)p;
  uint64_t* tile_max = (uint64_t*)c;
  c += (size_t)max_tiles * 8;
  int64_t* pbase = (int64_t*)c;
  c += (size_t)(m + 1) * 8;
  uint32_t* hist = (uint32_t*)c;
  c += (size_t)m * 4;
  int32_t* order = (int32_t*)c;
  c += (size_t)n * 4;
  int32_t* tile_of = (int32_t*)c;
  c += (size_t)n * 4;
  uint32_t* cnt = (uint32_t*)c;
  c += (size_t)n * 4;
  int32_t* tile_lo = (int32_t*)c;
  c += (size_t)max_tiles * 4;
  int32_t* tile_hi = (int32_t*)c;
  c += (size_t)max_tiles * 4;
  uint32_t* dirty = (uint32_t*)c;
  c += (size_t)max_tiles * 4;
  int32_t* part_tile = (int32_t*)c;
  c += (size_t)(m + 1) * 4;
  uint8_t* covered = (uint8_t*)c;
  IM_HIP(hipMemsetAsync(hist, 0, (size_t)m * 4, s));
  k_part_hist<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, part, hist);
  IM_HIP(hipGetLastError());
  std::vector<uint32_t> hh(m);
  IM_HIP(hipMemcpyAsync(hh.data(), hist, (size_t)m * 4, hipMemcpyDeviceToHost, s));
  IM_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> hb(m + 1);
  std::vector<int32_t> hpt(m + 1), htlo, hthi;
  hb[0] = 0;
  for (int q = 0; q < m; ++q) hb[q + 1] = hb[q] + hh[q];
  int32_t nt = 0;
  for (int q = 0; q < m; ++q) {
    hpt[q] = nt;
    for (int64_t lo = hb[q]; lo < hb[q + 1]; lo += kTile) {
      htlo.push_back((int32_t)lo);
      hthi.push_back((int32_t)std::min<int64_t>(lo + kTile, hb[q + 1]));
      ++nt;
    }
  }
  hpt[m] = nt;
  IM_HIP(hipMemcpyAsync(pbase, hb.data(), (size_t)(m + 1) * 8, hipMemcpyHostToDevice, s));
  IM_HIP(hipMemcpyAsync(part_tile, hpt.data(), (size_t)(m + 1) * 4, hipMemcpyHostToDevice, s));
  if (nt > 0) {
    IM_HIP(hipMemcpyAsync(tile_lo, htlo.data(), (size_t)nt * 4, hipMemcpyHostToDevice, s));
    IM_HIP(hipMemcpyAsync(tile_hi, hthi.data(), (size_t)nt * 4, hipMemcpyHostToDevice, s));
  }
  k_part_order<<<dim3(m), dim3(kGBlock), 0, s>>>(n, part, pbase, order);
  IM_HIP(hipGetLastError());
  k_tile_of<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, order, part, pbase,
                                                                   part_tile, tile_of);
  IM_HIP(hipGetLastError());
  CoverArgs A{};
  A.n = n;
  A.m = m;
  A.count = count;
  A.k = k;
  A.off = off;
  A.mem = mem;
  A.inc_off = inc_off;
  A.inc_mem = inc_mem;
  A.part = part;
  A.order = order;
  A.tile_of = tile_of;
  A.tile_lo = tile_lo;
  A.tile_hi = tile_hi;
  A.part_tile = part_tile;
  A.ntiles = nt;
  A.cnt = cnt;
  A.covered = covered;
  A.tile_max = tile_max;
  A.dirty = dirty;
  A.seeds = lseeds;
  A.gains = lgains;
  A.nsel = lcount;
  A.cover = lcover;
  IM_HIP(hipMemsetAsync(lgains, 0, (size_t)m * k * 8, s));
  return launch_cover(A, s);
}
