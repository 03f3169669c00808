// sample.hip -- RRR sampling under IC and LT (im_sample_rrr).
//
// Definition 2.3 and Sec. 2.1: a sample picks its root uniformly at random
// and collects every vertex that reaches the root over the edges live in that
// sample.  IC: every in-edge flips its own coin; the set is explored by a
// reverse BFS.  LT: every vertex keeps at most one in-edge, so the set is the
// backward chain from the root.  Draws are keyed by (seed, sample, edge or
// vertex), so a set does not depend on who computes it or in which order.
//
// Work split (MI355X):
//  * IC small path: one wavefront per sample, persistent over a work counter.
//    Frontier vertices are expanded 64 at a time; their in-edge lists are cut
//    into aligned groups of 4 edges (one 16-byte threshold load and one
//    Philox call per group) and the groups are spread over the lanes.  The
//    visited set is an open-addressing hash in LDS; the member list doubles
//    as the BFS queue and is sorted in LDS before it is written.
//  * A set that outgrows the LDS table is handed, by sample id, to the large
//    path: one workgroup per sample with a private visited bitmap and queue in
//    HBM; members come out sorted from the bitmap.
//  * LT: one lane per walk (walks are sequential chains), lanes refill from
//    the work counter independently; the visited check is a per-lane Bloom
//    filter in registers backed by the walk's member list; the kept edge is
//    found by binary search over the inclusive integer prefix of the
//    in-weights.
//  * Sets are first written to a staging arena (atomic cursor), then an
//    exclusive scan of the sizes gives the canonical CSR offsets and a gather
//    copies (and, for LT, sorts) each set into place.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "common.h"
#include "sample.h"

namespace im {

constexpr int kSmallBlock = 256;            // 4 waves, each its own sample
constexpr int kSmallH = 512;                // LDS hash slots per wave
#ifndef IM_TINY
#define IM_TINY 16                          // members of a lane-pass set
#endif
constexpr int kSmallCap = 256;              // members before handing off
constexpr int kStage = 128;                 // staged live in-edges per wave
// Large sets: two shapes of the large-set kernel, chosen per launch.
// A large set's frontier usually holds a few dozen vertices per level, so one
// wavefront per set with many sets in flight hides more of each level's
// dependent loads (2^20 weighted-cascade sets: 1.57 ms against 2.18 ms for
// 256 threads); when most sets are handed off (supercritical cascades with
// thousands of members) a 256-thread workgroup per set is used instead.
template <int kBlockT, int kBitsT, int kPerCuT>
struct BigCfg {
  static constexpr int kBlock = kBlockT;             // threads per set
  static constexpr int kStage = kBlockT >= 256 ? 960 : 4 * kBlockT;  // staged live edges
  static constexpr int kBits = kBitsT;               // LDS tier: hash slots 2^kBits,
  static constexpr int kH = 1 << kBitsT;             // members kH / 2
  static constexpr int kCap = kH / 2;
  static constexpr int kPerCu = kPerCuT;             // workers per CU
  // LDS pool of the hash, member list and stage; once a set is complete it
  // holds the sort of up to kSortCap members (the 256-thread shape keeps its
  // pool within the 20 KB that 8 workgroups per CU allow)
  static constexpr int kSortCap = kBlockT >= 256 ? kH : (2 * kH < 2048 ? 2 * kH : 2048);
  static constexpr int kPool =
      kH + kCap + kStage > kSortCap ? kH + kCap + kStage : kSortCap;
  // LDS bitmap tier: a set that outgrows the hash marks its members in a
  // bitmap over the hash and member-list words when the graph has at most
  // kBitsN vertices (the stage stays where it is)
  static constexpr int kBitsN = (kH + kCap) * 32;
};
#ifndef IM_NARROW_BITS
#define IM_NARROW_BITS 10
#endif
using BigNarrow = BigCfg<64, IM_NARROW_BITS, 24>;
using BigWide = BigCfg<256, 11, 8>;
constexpr uint32_t kMaxHandoff = 1u << 16;  // large sets that resume from a snapshot
constexpr int kLtCap = 1024;                // per-lane walk length before handing off
constexpr int kLtBlock = 256;
constexpr int kGatherSortCap = kLtCap;      // LT sets sorted by the gather kernel
constexpr int32_t kEmpty = -1;

struct SampleArgs {
  const TaskDesc* __restrict__ tasks;
  int32_t ntasks;
  // this launch's work: segment j covers work items [seg_base[j], seg_base[j+1])
  // of task seg_task[j]
  const int64_t* __restrict__ seg_base;
  const int32_t* __restrict__ seg_task;
  int32_t nseg;
  uint64_t count;                // work items of this launch
  uint32_t lt_grab;              // LT: sample ids a wavefront claims at once
  int32_t* __restrict__ arena;
  uint64_t arena_cap;
  int64_t* __restrict__ start;   // per output position: arena position
  int32_t* __restrict__ len;     // per output position: size (-1 while on the large path)
  uint32_t* __restrict__ big_list;       // output positions handed to the large path
  struct Handoff* __restrict__ handoff;  // kMaxHandoff snapshots (IC)
  unsigned long long* __restrict__ ctr;  // [0] IC work, [1] cursor, [2] big count,
                                         // [3] examined, [4] live, [5] big work,
                                         // [6] big examined, [7] big live, [8] big total,
                                         // [9] examined in abandoned rounds,
                                         // [10] sum of set sizes, [11] LT work;
                                         // [16] (own cache line) every IC item claimed
};

// The graph and random stream of one task, as the kernels use them.
struct GView {
  const int32_t* in_off;
  const int32_t* in_src;
  const uint32_t* thr;
  const double* skip;
  const uint32_t* lt_index;
  int64_t ne;  // edges
  uint32_t n, seed_lo, seed_hi, stream;
};

__device__ __forceinline__ GView view_of(const TaskDesc& T) {
  GView g;
  g.in_off = T.in_off;
  g.in_src = T.in_src;
  g.thr = T.thr;
  g.skip = T.model == IM_IC ? T.skip : nullptr;
  g.lt_index = T.model == IM_LT ? T.lt_index : nullptr;
  g.ne = T.num_edges;
  g.n = (uint32_t)T.n;
  g.seed_lo = T.seed_lo;
  g.seed_hi = T.seed_hi;
  g.stream = T.stream;
  return g;
}

// Work item w of this launch -> (task, sample id, output position).
__device__ __forceinline__ void locate_work(const SampleArgs& A, uint64_t w, int* task,
                                            uint32_t* sample, int64_t* pos) {
  int lo = 0, hi = A.nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint64_t)A.seg_base[mid] <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int t = A.seg_task[lo];
  const int64_t local = (int64_t)w - A.seg_base[lo];
  *task = t;
  *sample = A.tasks[t].first + (uint32_t)local;
  *pos = A.tasks[t].sample_base + local;
}

// Output position -> task.
__device__ __forceinline__ int task_of_pos(const SampleArgs& A, int64_t pos) {
  int lo = 0, hi = A.ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.tasks[mid].sample_base <= pos)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t hash_slot(int32_t v, int bits) {
  return ((uint32_t)v * 2654435761u) >> (32 - bits);
}

// Index of the frontier slot owning flat group gi: the first slot whose
// inclusive group prefix exceeds gi (pre has NF entries, non-decreasing).
template <int NF>
__device__ __forceinline__ int owner_of(const int32_t* pre, int32_t gi) {
  int lo = 0, hi = NF - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] > gi)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// Tuning knobs (compile-time): groups per lane per iteration, and an
// occupancy hint for the two IC kernels.
// Measured on MI355X (R-MAT 2^20, IC weighted cascade, 2^20 sets): two groups
// per lane beat four by 22% on coin-drawn graphs (with run-length walks one and
// two are even); with the lane pass and the wavefront-parallel walks, the
// small-set kernel runs best at 5 waves per SIMD (2.55-2.67 ms against 2.66
// at 6, 2.78 at 4 and 2.99 at 7), with 4 draws per vertex per pass (2: 2.98,
// 8: 2.71).
// HBM per stream for the large-set workers' bitmaps and queues (GiB)
#ifndef IM_BIG_BUDGET_GIB
#define IM_BIG_BUDGET_GIB 16
#endif
#ifndef IM_UNROLL
#define IM_UNROLL 2
#endif
#ifndef IM_IC_WAVES_PER_EU
#define IM_IC_WAVES_PER_EU 5
#endif
#ifndef IM_BIG_WAVES_PER_EU
#define IM_BIG_WAVES_PER_EU 8
#endif
#define IM_IC_ATTR __attribute__((amdgpu_waves_per_eu(IM_IC_WAVES_PER_EU)))

#define IM_BIG_ATTR __attribute__((amdgpu_waves_per_eu(IM_BIG_WAVES_PER_EU)))
constexpr int kUnroll = IM_UNROLL;  // 4-edge groups per lane per iteration

// Same-address atomics serialise at one coherence point, so work and arena
// space are claimed in batches: 64 sample ids per IC wavefront (a launch
// knob for LT) and kChunk arena entries per atomic.

constexpr unsigned long long kChunk = 1024;

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long x, int src) {
  const uint32_t lo = __shfl((uint32_t)x, src, kWave);
  const uint32_t hi = __shfl((uint32_t)(x >> 32), src, kWave);
  return ((unsigned long long)hi << 32) | lo;
}

// A value every lane holds alike, moved to scalar registers (the compiler
// cannot prove that a value read back from one lane is wave-uniform).
__device__ __forceinline__ unsigned long long first_lane_u64(unsigned long long x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int64_t shfl_i64(int64_t x, int src) {
  return (int64_t)shfl_u64((unsigned long long)x, src);
}

// Run-length walks of the vertices held by a wavefront's lanes, with the
// draws of each vertex spread over lanes: kWalkD draws per vertex per pass on
// kWalkD lanes, a segmented prefix sum of (1 + gap) gives the in-edge
// positions, and a vertex goes on to its next kWalkD draws only if all were
// live.  Draws of a vertex are consumed in order, so the live edges and the
// counts (draws up to the one that ends the walk, live edges) equal those of
// walking each vertex alone; the critical path is one draw per pass instead
// of one per draw.  rl: this lane holds a run-length vertex v with in-edges
// [a, a + deg) and table entry sk.  owner_map: kWave ints of LDS.  Every lane
// of the wavefront must call; push(e) is called for each live in-edge e.
#ifndef IM_WALK_D
#define IM_WALK_D 4
#endif
constexpr int kWalkD = IM_WALK_D;

template <class Push>
__device__ __forceinline__ void rl_walks(bool rl, uint32_t v, int32_t a, int32_t deg, double sk,
                                         uint32_t seed_lo, uint32_t seed_hi, uint32_t stream,
                                         uint32_t i, int32_t* owner_map, uint32_t* ex,
                                         uint32_t* lv, Push&& push) {
  constexpr int D = kWalkD;
  const int lane = lane_id();
  int64_t pos = -1;
  uint32_t jb = 0;
  bool more = rl;
  for (;;) {
    const unsigned long long mm = __ballot(more);
    if (!mm) break;
    const int nm = __popcll(mm);
    const int my_rank = __popcll(mm & ((1ull << lane) - 1ull));
    if (more) owner_map[my_rank] = lane;
    wave_sync();
    for (int f0 = 0; f0 < nm; f0 += kWave / D) {
      const int r = f0 + lane / D, sub = lane % D;
      const bool act = r < nm;
      const int ol = act ? owner_map[r] : lane;
      const uint32_t vo = (uint32_t)__shfl((int)v, ol, kWave);
      const int32_t ao = __shfl(a, ol, kWave), dego = __shfl(deg, ol, kWave);
      const double sko = __shfl(sk, ol, kWave);
      const uint32_t jbo = (uint32_t)__shfl((int)jb, ol, kWave);
      const int64_t poso = shfl_i64(pos, ol);
      int64_t step = 0;
      if (act) {
        const double g =
            floor(im_log(skip_uniform(seed_lo, seed_hi, stream, i, vo, jbo + (uint32_t)sub)) * sko);
        step = 1 + (int64_t)fmin(g, (double)dego);  // any gap >= deg ends the walk alike
      }
      int64_t incl = step;  // inclusive prefix within the D lanes of a vertex
      static_assert(D <= 16, "a vertex's draws stay inside one row of 16 lanes");
      if constexpr (D > 1) {  // DPP row shifts: the D lanes never span two rows
        const int64_t y = dpp_move<0x111, 0xF>(incl);
        if (sub >= 1) incl += y;
      }
      if constexpr (D > 2) {
        const int64_t y = dpp_move<0x112, 0xF>(incl);
        if (sub >= 2) incl += y;
      }
      if constexpr (D > 4) {
        const int64_t y = dpp_move<0x114, 0xF>(incl);
        if (sub >= 4) incl += y;
      }
      if constexpr (D > 8) {
        const int64_t y = dpp_move<0x118, 0xF>(incl);
        if (sub >= 8) incl += y;
      }
      const int64_t p = poso + incl;
      const bool live = act && p <= (int64_t)dego - 1;
      if (live) push(ao + (int32_t)p);
      const unsigned long long lm = __ballot(live), tm = __ballot(act && !live);
      // the owners of this pass take their vertex's outcome
      const int grp = my_rank - f0;
      const bool mine = more && grp >= 0 && grp < kWave / D;
      const int64_t plast = shfl_i64(p, mine ? grp * D + D - 1 : lane);
      if (mine) {
        const unsigned long long gm = (1ull << D) - 1ull;
        const uint32_t nl = (uint32_t)__popcll((lm >> (grp * D)) & gm);
        const bool term = ((tm >> (grp * D)) & gm) != 0ull;
        *ex += nl + (term ? 1u : 0u);
        *lv += nl;
        if (term) {
          more = false;
        } else {
          pos = plast;
          jb += D;
        }
      }
    }
    wave_sync();
  }
}

__device__ __forceinline__ uint32_t ceil_log2_plus1(int32_t d) {
  // ceil(log2(d + 1)) for d >= 1
  return 32u - (uint32_t)__clz((uint32_t)d);
}

// ----------------------------------------------------------- LT kept edge
// Vertex v keeps its first in-edge e (in [a, b)) with thr[e] > r or thr[e]
// saturated; thr is non-decreasing over [a, b), so "taken" is false on a
// prefix and true after it.
__device__ __forceinline__ bool lt_taken(uint32_t c, uint32_t r) {
  return c > r || c == 0xFFFFFFFFu;
}

__device__ __forceinline__ uint32_t u4_at(const uint4 (&g)[4], int q) {
  const uint4 x = g[q >> 2];
  return (q & 3) == 0 ? x.x : (q & 3) == 1 ? x.y : (q & 3) == 2 ? x.z : x.w;
}

// Entries of the 16-entry group g at positions [lo, hi) that are not taken.
__device__ __forceinline__ int not_taken16(const uint4 (&g)[4], int lo, int hi, uint32_t r) {
  int c = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) c += (q >= lo && q < hi && !lt_taken(u4_at(g, q), r)) ? 1 : 0;
  return c;
}

__device__ __forceinline__ int64_t lt_level_base(int64_t E, int k) {
  int64_t base = 0;
  for (int j = 1; j < k; ++j) {
    const int64_t nw = (E + ((int64_t)1 << (4 * j)) - 1) >> (4 * j);
    base += (nw + 15) & ~(int64_t)15;
  }
  return base;
}

// The kept in-edge of a vertex with in-edges [a, b) (a < b) under draw r:
// its id, or b if none; *src = its source.  With the graph's search index,
// a 16-ary descent: the top level is the lowest whose aligned group of 16
// windows holds all of [a, b); at each level the windows before the first
// whose last edge is taken are counted in one 64-byte group (the windows
// entirely inside [a, b) only: the one holding b - 1 is where the search
// ends if no earlier one is taken); the last group holds the edges
// themselves, loaded with their sources.  Without the index (or with
// kIndex false, where the registers the descent holds would cost occupancy),
// a binary search.
template <bool kIndex = true>
__device__ __forceinline__ int32_t lt_pick(const GView& G, int32_t a, int32_t b, uint32_t r,
                                           int32_t* src) {
  if (!kIndex || !G.lt_index) {
    int32_t lo = a, hi = b;
    while (lo < hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      if (lt_taken(G.thr[mid], r))
        hi = mid;
      else
        lo = mid + 1;
    }
    if (lo < b) *src = G.in_src[lo];
    return lo;
  }
  const int64_t A = a, Bm = (int64_t)b - 1;
  int K = 0;
  while (K < kLtLevels && (A >> (4 * (K + 1))) != (Bm >> (4 * (K + 1)))) ++K;
  int64_t w = A >> 4;  // group of edges searched last (a level-1 window)
  if (K > 0) {
    int64_t base = lt_level_base(G.ne, K);
    {  // top level: windows [wa, wb) of one group
      const int64_t wa = A >> (4 * K), wb = Bm >> (4 * K), g = wa >> 4;
      const uint4* p = reinterpret_cast<const uint4*>(G.lt_index + base + 16 * g);
      const uint4 q[4] = {p[0], p[1], p[2], p[3]};
      w = wa + not_taken16(q, (int)(wa - 16 * g), (int)(wb - 16 * g), r);
    }
    for (int k = K - 1; k >= 1; --k) {
      base -= ((((G.ne + ((int64_t)1 << (4 * k)) - 1) >> (4 * k)) + 15) & ~(int64_t)15);
      const int64_t wa = A >> (4 * k), wb = Bm >> (4 * k);
      const int64_t lo = max(16 * w, wa), hi = min(16 * w + 16, wb);
      const uint4* p = reinterpret_cast<const uint4*>(G.lt_index + base + 16 * w);
      const uint4 q[4] = {p[0], p[1], p[2], p[3]};
      w = lo + not_taken16(q, (int)(lo - 16 * w), (int)(hi - 16 * w), r);
    }
  }
  // the edges: group w within [a, b)
  const int64_t e0 = 16 * w;
  const int lo = (int)(max(e0, A) - e0), hi = (int)(min(e0 + 16, (int64_t)b) - e0);
  const int64_t e4 = (G.ne + 3) & ~(int64_t)3;  // thr holds round_up(E, 4) entries
  const uint4* pt = reinterpret_cast<const uint4*>(G.thr + e0);
  uint4 t[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = e0 + 4 * q < e4 ? pt[q] : make_uint4(0u, 0u, 0u, 0u);
  const bool vec_src = e0 + 16 <= G.ne && ((uintptr_t)G.in_src & 15u) == 0;
  int4 sv[4] = {};
  if (vec_src) {
    const int4* ps = reinterpret_cast<const int4*>(G.in_src + e0);
#pragma unroll
    for (int q = 0; q < 4; ++q) sv[q] = ps[q];
  }
  const int idx = lo + not_taken16(t, lo, hi, r);
  if (idx >= hi) return b;
  if (vec_src) {
    int32_t u = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int4 x = sv[q >> 2];
      const int32_t y = (q & 3) == 0 ? x.x : (q & 3) == 1 ? x.y : (q & 3) == 2 ? x.z : x.w;
      u = q == idx ? y : u;
    }
    *src = u;
  } else {
    *src = G.in_src[e0 + idx];
  }
  return (int32_t)(e0 + idx);
}

// A set handed from the small to the large path resumes from the state it had
// at the start of the round that overflowed: members [0, tail), of which
// [0, head) are expanded, and the exact counters of those expansions.
struct Handoff {
  int32_t mem[kSmallCap];
  int32_t head, tail;
  unsigned long long ex, lv;
};

// ------------------------------------------------------------------ IC small
struct __align__(16) WaveLds {
  // the wavefront path's hash (kSmallH slots); the lane pass's lists
  int32_t hash[kSmallH > kWave * IM_TINY ? kSmallH : kWave * IM_TINY];
  int32_t queue[kSmallCap];
  int32_t pre[kWave];    // inclusive prefix of 4-edge group counts
  int32_t gbase[kWave];  // group id of a lane's first group minus its prefix start
  int32_t ea[kWave];     // in-edge range of each frontier vertex
  int32_t eb[kWave];
  int32_t stage[kStage];  // live in-edges whose sources are still to be loaded
  int32_t tail;
  int32_t nst;            // entries pushed to stage (may exceed kStage)
  int32_t pad[2];
};

// Inserts u; returns true if it was new.  Gives up (sets *over) once the
// member count reaches kSmallCap: the hash then holds at most kSmallCap + 63
// keys, so probing always finds a free slot.
__device__ __forceinline__ void lds_insert(WaveLds& L, int32_t u, bool* over) {
  uint32_t h = hash_slot(u, 9);
  for (;;) {
    int32_t cur = L.hash[h];
    if (cur == u) return;
    if (cur == kEmpty) {
      if (__atomic_load_n(&L.tail, __ATOMIC_RELAXED) >= kSmallCap) {
        *over = true;
        return;
      }
      int32_t old = atomicCAS(&L.hash[h], kEmpty, u);
      if (old == kEmpty) {
        int32_t pos = atomicAdd(&L.tail, 1);
        if (pos < kSmallCap)
          L.queue[pos] = u;
        else
          *over = true;
        return;
      }
      if (old == u) return;
    }
    h = (h + 1) & (kSmallH - 1);
  }
}

// Live in-edges are staged by edge index and their sources loaded together,
// one load per lane, so a BFS level waits for one round trip to in_src
// instead of one per live edge of its busiest lane.  An edge that finds the
// stage full is loaded and inserted at once.
__device__ __forceinline__ void stage_push(WaveLds& L, const int32_t* __restrict__ in_src,
                                           int32_t e, bool* over) {
  const int32_t k = atomicAdd(&L.nst, 1);
  if (k < kStage)
    L.stage[k] = e;
  else
    lds_insert(L, in_src[e], over);
}

__device__ __forceinline__ void stage_flush(WaveLds& L, const int32_t* __restrict__ in_src,
                                            int lane, bool* over) {
  wave_sync();
  const int32_t ns = min(L.nst, kStage);
  for (int32_t k = lane; k < ns; k += kWave) lds_insert(L, in_src[L.stage[k]], over);
  wave_sync();
  if (lane == 0) L.nst = 0;
  wave_sync();
}

// Lane pass: one lane per sample, for sets of at most kTiny members (most
// sets: 86% of the weighted-cascade sets at R-MAT scale 20).  The lane keeps
// its members in a list of kTiny entries and expands them one by one with the
// same draws as the wavefront path; a set that grows past kTiny members, or
// reaches a coin-drawn vertex with more than kTinyDeg in-edges, is left to the
// wavefront path, which starts it over.
constexpr int kTiny = IM_TINY;  // members per lane list; a wave's lists share its hash area
constexpr int32_t kTinyDeg = 16;

// Adds u to the lane's list unless present; false if the list is full.
// seen: bit (u mod 64) of every member, so most new members skip the scan.
__device__ __forceinline__ bool tiny_add(int32_t* list, int32_t* n, unsigned long long* seen,
                                         int32_t u) {
  const unsigned long long bit = 1ull << (u & 63);
  if (*seen & bit)
    for (int32_t k = 0; k < *n; ++k)
      if (list[k] == u) return true;
  if (*n == kTiny) return false;
  list[(*n)++] = u;
  *seen |= bit;
  return true;
}

// Grows the set of sample i from root; true if it completed within kTiny
// members (then list[0, *cnt) holds them and *ex, *lv its counters).
#ifdef IM_TINY_NOINLINE
__attribute__((noinline))
#endif
__device__ bool tiny_set(const GView& G, uint32_t i, int32_t root, int32_t* list, int32_t* cnt,
                         uint32_t* ex, uint32_t* lv) {
  list[0] = root;
  unsigned long long seen = 1ull << (root & 63);
  int32_t n = 1, h = 0;
  uint32_t e_ = 0, l_ = 0;
  while (h < n) {
    const int32_t v = list[h++];
    const int32_t a = G.in_off[v], b = G.in_off[v + 1];
    const double sk = G.skip ? G.skip[v] : 0.0;
    if (sk != 0.0) {  // run-length vertex
      const int64_t deg = b - a;
      int64_t pos = -1;
      uint4 blk;
      for (uint32_t j = 0;; ++j) {
        ++e_;
        const double gap = floor(
            im_log(skip_uniform_seq(G.seed_lo, G.seed_hi, G.stream, i, (uint32_t)v, j, &blk)) * sk);
        if (gap >= (double)(deg - 1 - pos)) break;
        pos += 1 + (int64_t)gap;
        ++l_;
        if (!tiny_add(list, &n, &seen, G.in_src[a + pos])) return false;
      }
    } else if (a < b) {  // coins, 4-edge groups as in the wavefront path
      if (b - a > kTinyDeg) return false;
      e_ += (uint32_t)(b - a);
      for (int32_t g = a >> 2; g <= (b - 1) >> 2; ++g) {
        const uint4 q = reinterpret_cast<const uint4*>(G.thr)[g];
        const uint4 r =
            philox4x32_10(make_uint4((uint32_t)g, i, kTagEdge, G.stream), G.seed_lo, G.seed_hi);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int32_t e = (g << 2) + w;
          const uint32_t qw = pick_word(q, w), rw = pick_word(r, w);
          if (e >= a && e < b && (qw == 0xFFFFFFFFu || rw < qw)) {
            ++l_;
            if (!tiny_add(list, &n, &seen, G.in_src[e])) return false;
          }
        }
      }
    }
  }
  // ascending, as every set is stored
  for (int32_t k = 1; k < n; ++k) {
    const int32_t x = list[k];
    int32_t j = k - 1;
    while (j >= 0 && list[j] > x) {
      list[j + 1] = list[j];
      --j;
    }
    list[j + 1] = x;
  }
  *cnt = n;
  *ex = e_;
  *lv = l_;
  return true;
}

// The lane pass over work items [b, b + 64): every lane grows one set alone
// (tiny_set).  Finished sets go to the arena; returns the mask of lanes whose
// set is left to the wavefront path.
__device__ __forceinline__ unsigned long long lane_pass(const SampleArgs& A, WaveLds& L, unsigned long long b,
                                          unsigned long long* cpos, unsigned long long* cend,
                                          unsigned long long* w_tot, unsigned long long* w_ex,
                                          unsigned long long* w_lv) {
  const int lane = lane_id();
  const unsigned long long my = b + (unsigned long long)lane;
  const bool have = my < A.count;
  int32_t* list = L.hash + lane * kTiny;  // the hash is cleared per set below
  bool done = false;
  int32_t n = 0;
  uint32_t t_ex = 0, t_lv = 0;
  int64_t il = 0;
  if (have) {
    int tk;
    uint32_t i;
    locate_work(A, my, &tk, &i, &il);
    const GView G = view_of(A.tasks[tk]);
    const int32_t root = (int32_t)scale_draw(
        draw1(((uint64_t)G.seed_hi << 32) | G.seed_lo, kTagRoot, G.stream, 0u, i), G.n);
    done = tiny_set(G, i, root, list, &n, &t_ex, &t_lv);
  }
  const int32_t sz = done ? n : 0;
  const int32_t incl = wave_inclusive_scan(sz);
  const unsigned long long tot = (unsigned long long)__shfl(incl, kWave - 1, kWave);
  if (tot > 0) {
    if (*cpos + tot > *cend) {
      const unsigned long long want = max(tot, kChunk);
      unsigned long long c = 0;
      if (lane == 0) c = atomicAdd(&A.ctr[1], want);
      *cpos = first_lane_u64(shfl_u64(c, 0));
      *cend = *cpos + want;
    }
    const unsigned long long pos = *cpos;
    *cpos += tot;
    *w_tot += tot;
    if (done) {
      const unsigned long long mine = pos + (unsigned long long)(incl - sz);
      if (pos + tot <= A.arena_cap)
        for (int32_t k = 0; k < n; ++k) A.arena[mine + k] = list[k];
      A.start[il] = (int64_t)mine;
      A.len[il] = n;
      *w_ex += t_ex;
      *w_lv += t_lv;
    }
  }
  return __ballot(have && !done);
}

// Per-wavefront counter sums of finished sets into the launch totals.
__device__ __forceinline__ void flush_counts(const SampleArgs& A, unsigned long long w_ex,
                                             unsigned long long w_lv, unsigned long long w_tot) {
  w_ex = wave_sum(w_ex);
  w_lv = wave_sum(w_lv);
  if (lane_id() == 0) {
    if (w_ex) atomicAdd(&A.ctr[3], w_ex);
    if (w_lv) atomicAdd(&A.ctr[4], w_lv);
    if (w_tot) atomicAdd(&A.ctr[10], w_tot);
  }
}


// The wavefront path for one set (work item `item`): the whole wavefront
// grows it with its visited set in LDS (kSmallH slots, kSmallCap members);
// a set that outgrows it is handed to the large-set launch with a snapshot of
// its state at the start of the overflowing round.
// cpos/cend: the wavefront's reserved arena chunk; w_*: its running sums.
__device__ __forceinline__ void wave_path(const SampleArgs& A, WaveLds& L,
                                          unsigned long long item, unsigned long long& cpos,
                                          unsigned long long& cend, unsigned long long& w_tot,
                                          unsigned long long& w_ex, unsigned long long& w_lv) {
  const int lane = lane_id();
  int tk;
  uint32_t i;
  int64_t il;
  locate_work(A, item, &tk, &i, &il);
  const GView G = view_of(A.tasks[tk]);
  const int32_t root =
      (int32_t)scale_draw(draw1(((uint64_t)G.seed_hi << 32) | G.seed_lo, kTagRoot, G.stream,
                                0u, i),
                          G.n);
  for (int j = lane; j < kSmallH; j += kWave) L.hash[j] = kEmpty;
  wave_sync();
  if (lane == 0) {
    L.hash[hash_slot(root, 9)] = root;
    L.queue[0] = root;
    L.tail = 1;
    L.nst = 0;
  }
  wave_sync();
  int32_t head = 0, tail = 1;
  bool over = false;
  uint32_t s_ex = 0, s_lv = 0;  // this set's draws / live edges, per lane
  int32_t head0 = 0, tail0 = 1;
  uint32_t ex0 = 0, lv0 = 0;
  while (head < tail) {
    head0 = head;  // snapshot for a hand-off
    tail0 = tail;
    ex0 = s_ex;
    lv0 = s_lv;
    const int32_t nf = min(tail - head, kWave);
    int32_t a = 0, b = 0, ng = 0, v = 0;
    double sk = 0.0;
    if (lane < nf) {
      v = L.queue[head + lane];
      a = G.in_off[v];
      b = G.in_off[v + 1];
      if (G.skip) sk = G.skip[v];
      if (sk == 0.0) {
        if (a < b) ng = ((b - 1) >> 2) - (a >> 2) + 1;
        s_ex += (uint32_t)(b - a);
      }
    }
    // run-length vertices: their geometric gaps, drawn across the wavefront
    rl_walks(sk != 0.0, (uint32_t)v, a, b - a, sk, G.seed_lo, G.seed_hi, G.stream, i, L.gbase,
             &s_ex, &s_lv, [&](int32_t e) { stage_push(L, G.in_src, e, &over); });
    const int32_t inc = wave_inclusive_scan(ng);
    const int32_t total = __shfl(inc, kWave - 1, kWave);
    L.pre[lane] = inc;
    L.gbase[lane] = (a >> 2) - (inc - ng);
    L.ea[lane] = a;
    L.eb[lane] = b;
    head += nf;
    wave_sync();
    for (int32_t base = 0; base < total; base += kWave * kUnroll) {
      // one owner for the whole chunk (a large in-edge list) skips the search
      const int o_b = owner_of<kWave>(L.pre, base);
      const bool uni = L.pre[o_b] >= min(total, base + kWave * kUnroll);
      uint4 q[kUnroll];
      uint32_t g[kUnroll];
      int32_t ea[kUnroll], eb[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int32_t gi = base + u * kWave + lane;
        ea[u] = eb[u] = 0;
        g[u] = 0;
        if (gi < total) {
          const int o = uni ? o_b : owner_of<kWave>(L.pre, gi);
          g[u] = (uint32_t)(L.gbase[o] + gi);
          ea[u] = L.ea[o];
          eb[u] = L.eb[o];
          q[u] = reinterpret_cast<const uint4*>(G.thr)[g[u]];
        }
      }
      uint32_t lm = 0;  // live words of this lane's groups, bit u * 4 + w
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (ea[u] < eb[u]) {
          const uint4 r = philox4x32_10(make_uint4(g[u], i, kTagEdge, G.stream), G.seed_lo,
                                        G.seed_hi);
          const int32_t e0 = (int32_t)(g[u] << 2);
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int32_t e = e0 + w;
            const uint32_t qw = pick_word(q[u], w), rw = pick_word(r, w);
            if (e >= ea[u] && e < eb[u] && (qw == 0xFFFFFFFFu || rw < qw)) lm |= 1u << (u * 4 + w);
          }
        }
      }
      {  // stage this iteration's live edges at wave-scanned positions
        const int32_t c = __popc(lm);
        const int32_t incl = wave_inclusive_scan(c);
        const int32_t base = L.nst;
        int32_t k = base + incl - c;
        s_lv += (uint32_t)c;
        while (lm) {
          const int bit = __ffs(lm) - 1;
          lm &= lm - 1;
          uint32_t gb = g[0];
#pragma unroll
          for (int u = 1; u < kUnroll; ++u)
            if ((bit >> 2) == u) gb = g[u];
          const int32_t e = (int32_t)(gb << 2) + (bit & 3);
          if (k < kStage)
            L.stage[k] = e;
          else
            lds_insert(L, G.in_src[e], &over);
          ++k;
        }
        wave_sync();
        if (lane == kWave - 1) L.nst = base + incl;
      }
      stage_flush(L, G.in_src, lane, &over);
      if (__any(over)) break;
    }
    stage_flush(L, G.in_src, lane, &over);  // the walks' edges when no groups ran
    tail = L.tail;
    if (__any(over) || tail > kSmallCap) {
      over = true;
      break;
    }
  }
  if (over) {
    const unsigned long long hex = wave_sum((unsigned long long)ex0);
    const unsigned long long hlv = wave_sum((unsigned long long)lv0);
    const unsigned long long redo = wave_sum((unsigned long long)(s_ex - ex0));
    if (lane == 0 && redo) atomicAdd(&A.ctr[9], redo);
    uint32_t slot = 0;
    if (lane == 0) slot = (uint32_t)atomicAdd(&A.ctr[2], 1ull);
    slot = __shfl(slot, 0, kWave);
    if (slot < kMaxHandoff) {
      Handoff& H = A.handoff[slot];
      for (int j = lane; j < tail0; j += kWave) H.mem[j] = L.queue[j];
      if (lane == 0) {
        H.head = head0;
        H.tail = tail0;
        H.ex = hex;
        H.lv = hlv;
      }
    }
    if (lane == 0) {
      A.big_list[slot] = il;
      A.len[il] = -1;
    }
    wave_sync();
    return;
  }
  // sort queue[0, tail) ascending (bitonic over the next power of two)
  int32_t P = 1;
  while (P < tail) P <<= 1;
  for (int j = tail + lane; j < P; j += kWave) L.queue[j] = 0x7FFFFFFF;
  wave_sync();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < (P >> 1); t += kWave) {
        const int i1 = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int i2 = i1 | j;
        const bool asc = (i1 & k) == 0;
        const int32_t x = L.queue[i1], y = L.queue[i2];
        if ((x > y) == asc) {
          L.queue[i1] = y;
          L.queue[i2] = x;
        }
      }
      wave_sync();
    }
  }
  if (cpos + (unsigned long long)tail > cend) {
    const unsigned long long want = max((unsigned long long)tail, kChunk);
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(&A.ctr[1], want);
    cpos = first_lane_u64(shfl_u64(b, 0));
    cend = cpos + want;
  }
  const unsigned long long pos = cpos;
  cpos += (unsigned long long)tail;
  w_tot += (unsigned long long)tail;
  if (pos + (unsigned long long)tail <= A.arena_cap)
    for (int j = lane; j < tail; j += kWave) A.arena[pos + j] = L.queue[j];
  if (lane == 0) {
    A.start[il] = (int64_t)pos;
    A.len[il] = tail;
  }
  w_ex += s_ex;
  w_lv += s_lv;
  wave_sync();
}

// IC sets: each wavefront claims 64 work items at a time (ctr[0]), runs the
// lane pass over them and then the wavefront path over the items the lane
// pass left, in order.  Once every item is claimed (ctr[16], set by the first
// wavefront to find none), a wavefront hands the items it has not started to
// the large-set launch and stops, so no wavefront works through a long
// private backlog while others idle; that launch takes its sets in list
// order, the long handed-off sets first.
__global__ __launch_bounds__(kSmallBlock) IM_IC_ATTR void k_sample_ic_small(SampleArgs A) {
  __shared__ WaveLds lds_all[kSmallBlock / kWave];
  WaveLds& L = lds_all[threadIdx.x / kWave];
  const int lane = lane_id();
  unsigned long long w_ex = 0, w_lv = 0;  // per-lane sums of finished sets
  unsigned long long w_tot = 0;            // members written by this wave
  unsigned long long cpos = 0, cend = 0;  // reserved arena chunk
  unsigned long long batch = 0, defer = 0;
  for (;;) {
    wave_sync();
    if (defer == 0) {
      unsigned long long b = 0;
      if (lane == 0) b = atomicAdd(&A.ctr[0], (unsigned long long)kWave);
      b = first_lane_u64(shfl_u64(b, 0));
      if (b >= A.count) {
        if (lane == 0) __hip_atomic_store(&A.ctr[16], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      batch = b;
      defer = lane_pass(A, L, b, &cpos, &cend, &w_tot, &w_ex, &w_lv);
      continue;
    }
    unsigned long long ex = 0;
    if (lane == 0) ex = __hip_atomic_load(&A.ctr[16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (first_lane_u64(shfl_u64(ex, 0))) {
      // every item is claimed: the sets not started go to the large-set
      // launch, after the ones handed off so far, with a snapshot of just
      // their root
      uint32_t s0 = 0;
      if (lane == 0) s0 = (uint32_t)atomicAdd(&A.ctr[2], (unsigned long long)__popcll(defer));
      s0 = __shfl(s0, 0, kWave);
      if ((defer >> lane) & 1ull) {
        const uint32_t slot = s0 + (uint32_t)__popcll(defer & ((1ull << lane) - 1ull));
        int tk;
        uint32_t i;
        int64_t il;
        locate_work(A, batch + (unsigned long long)lane, &tk, &i, &il);
        const GView G = view_of(A.tasks[tk]);
        if (slot < kMaxHandoff) {
          Handoff& H = A.handoff[slot];
          H.mem[0] = (int32_t)scale_draw(
              draw1(((uint64_t)G.seed_hi << 32) | G.seed_lo, kTagRoot, G.stream, 0u, i), G.n);
          H.head = 0;
          H.tail = 1;
          H.ex = 0;
          H.lv = 0;
        }
        A.big_list[slot] = (uint32_t)il;
        A.len[il] = -1;
      }
      break;
    }
    const int dl = __ffsll(defer) - 1;
    defer &= defer - 1;
    wave_path(A, L, batch + (unsigned long long)dl, cpos, cend, w_tot, w_ex, w_lv);
  }
  flush_counts(A, w_ex, w_lv, w_tot);
}


// ------------------------------------------------------------------ large sets
struct BigArgs {
  uint32_t nwords;                  // ceil(max n / 32)
  uint32_t qcap;                    // max n over the tasks
  uint32_t* __restrict__ bitmaps;   // per worker, nwords words, all zero between uses
  int32_t* __restrict__ queues;     // per worker, qcap entries
};

template <int kBlock>
__device__ __forceinline__ int64_t block_exclusive_scan64(int64_t x, int64_t* lds,
                                                          int64_t* total) {
  // lds: kBlock / kWave + 1 entries; every thread of the block must call
  const int t = threadIdx.x, l = lane_id(), w = t / kWave;
  int64_t inc = wave_inclusive_scan(x);
  if (l == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    int64_t v = l < kBlock / kWave ? lds[l] : 0;
    int64_t vi = wave_inclusive_scan(v);
    if (l < kBlock / kWave) lds[l] = vi - v;
    if (l == kWave - 1) lds[kBlock / kWave] = vi;
  }
  __syncthreads();
  int64_t r = lds[w] + inc - x;
  *total = lds[kBlock / kWave];
  __syncthreads();
  return r;
}


// A large set is first grown with its visited set in LDS (open addressing,
// kH slots) and its member list in LDS (kCap); a level that would pass kCap
// members is redone with the worker's HBM bitmap and queue.
static_assert(BigNarrow::kCap >= kSmallCap && BigWide::kCap >= kSmallCap,
              "a hand-off snapshot must fit the LDS tier");

// The visited set and member list of the set a workgroup is growing.
// The word of a worker's HBM bitmap that holds u, read at agent scope (past
// the CU's L1, as the bitmap's atomics are performed in L2).  Bits only get
// set while a set grows, so a set bit read here is final.
__device__ __forceinline__ uint32_t bitmap_word(const uint32_t* bm, int32_t u) {
  return __hip_atomic_load(&bm[u >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct BigSet {
  bool lds;             // LDS mode (block-uniform)
  int32_t* mhash;       // LDS: kH slots
  int32_t* mq;          // LDS: kCap members
  uint32_t* bm;         // HBM: n-bit bitmap
  bool bits;            // bitmap in LDS (over mhash and mq) instead of bm (block-uniform)
  int32_t* queue;       // HBM: n members
  int32_t* s_tail;      // members so far
  int32_t* s_over;      // LDS mode only: a member did not fit
};

// Adds u to the set if it is new.  In LDS mode the member count is checked
// before a slot is claimed, so the hash holds at most C::kCap + kBlock - 1
// keys and probing always ends at u or at a free slot.
template <class C>
__device__ __forceinline__ void set_insert(const BigSet& S, int32_t u) {
  if (S.lds) {
    uint32_t h = hash_slot(u, C::kBits);
    for (;;) {
      const int32_t cur = S.mhash[h];
      if (cur == u) return;
      if (cur == kEmpty) {
        if (__atomic_load_n(S.s_tail, __ATOMIC_RELAXED) >= C::kCap) {
          *S.s_over = 1;
          return;
        }
        const int32_t old = atomicCAS(&S.mhash[h], kEmpty, u);
        if (old == kEmpty) {
          const int32_t pos = atomicAdd(S.s_tail, 1);
          if (pos < C::kCap)
            S.mq[pos] = u;
          else
            *S.s_over = 1;
          return;
        }
        if (old == u) return;
      }
      h = (h + 1) & (C::kH - 1);
    }
  } else if (S.bits) {
    const uint32_t bit = 1u << (u & 31);
    const uint32_t old = atomicOr((uint32_t*)&S.mhash[u >> 5], bit);
    if (!(old & bit)) S.queue[atomicAdd(S.s_tail, 1)] = u;
  } else {
    const uint32_t bit = 1u << (u & 31);
    if (bitmap_word(S.bm, u) & bit) return;
    const uint32_t old = atomicOr(&S.bm[u >> 5], bit);
    if (!(old & bit)) S.queue[atomicAdd(S.s_tail, 1)] = u;
  }
}

// As in the small path: live in-edges are staged by index and their sources
// loaded together; an edge that finds the stage full is handled at once.
template <class C>
__device__ __forceinline__ void big_push(int32_t e, int32_t* stage, int32_t* s_nst,
                                         const int32_t* __restrict__ in_src, const BigSet& S) {
  const int32_t k = atomicAdd(s_nst, 1);
  if (k < C::kStage)
    stage[k] = e;
  else
    set_insert<C>(S, in_src[e]);
}

// Every thread of the block must call.  Each thread takes kFlushBatch staged
// edges at a time: their sources are loaded together and, in HBM mode, their
// bitmap atomics issued together before any result is used (a source seen
// twice is appended once: the second atomicOr returns the bit set).
#ifndef IM_FLUSH_BATCH
#define IM_FLUSH_BATCH 8
#endif
constexpr int kFlushBatch = IM_FLUSH_BATCH;
template <class C>
__device__ __forceinline__ void big_flush(const int32_t* stage, int32_t* s_nst,
                                          const int32_t* __restrict__ in_src, const BigSet& S) {
  __syncthreads();
  const int32_t ns = min(*s_nst, C::kStage);
  for (int32_t k0 = threadIdx.x; k0 < ns; k0 += kFlushBatch * C::kBlock) {
    int32_t u[kFlushBatch];
#pragma unroll
    for (int q = 0; q < kFlushBatch; ++q) {
      const int32_t k = k0 + q * C::kBlock;
      u[q] = k < ns ? in_src[stage[k]] : -1;
    }
    if (S.lds || S.bits) {
#pragma unroll
      for (int q = 0; q < kFlushBatch; ++q)
        if (u[q] >= 0) set_insert<C>(S, u[q]);
    } else {
      uint32_t old[kFlushBatch];
      // a coherent load first: a source whose bit is already set (most of
      // the live edges of a large set) costs a read instead of a device atomic
#pragma unroll
      for (int q = 0; q < kFlushBatch; ++q)
        old[q] = u[q] >= 0 ? bitmap_word(S.bm, u[q]) : 0u;
#pragma unroll
      for (int q = 0; q < kFlushBatch; ++q)
        if (u[q] >= 0 && !(old[q] & (1u << (u[q] & 31))))
          old[q] = atomicOr(&S.bm[u[q] >> 5], 1u << (u[q] & 31));
#pragma unroll
      for (int q = 0; q < kFlushBatch; ++q)
        if (u[q] >= 0 && !(old[q] & (1u << (u[q] & 31)))) S.queue[atomicAdd(S.s_tail, 1)] = u[q];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *s_nst = 0;
  __syncthreads();
}

// One workgroup per large set: visited set and members in LDS while they fit
// (sorted in LDS); past that, on graphs of at most C::kBitsN vertices, a
// bitmap in LDS with the members queued in HBM (read in order from the
// bitmap); otherwise the worker's private bitmap and queue in HBM (sorted in
// LDS up to C::kSortCap members, else read in order from the bitmap, a pass
// over all n bits).
template <class C>
__global__ __launch_bounds__(C::kBlock) IM_BIG_ATTR void k_sample_big(SampleArgs A, BigArgs Bg) {
  __shared__ int32_t pre[C::kBlock];
  __shared__ int32_t gbase[C::kBlock];
  __shared__ int32_t ea[C::kBlock];
  __shared__ int32_t eb[C::kBlock];
  __shared__ int64_t scan_lds[C::kBlock / kWave + 1];
  __shared__ int32_t pool[C::kPool];  // LDS-mode hash | members | stage; sort buffer
  int32_t* const mhash = pool;
  int32_t* const mq = pool + C::kH;
  int32_t* const stage = pool + C::kH + C::kCap;
  __shared__ int32_t s_nst;
  __shared__ int32_t s_tail;
  __shared__ int32_t s_over;
  __shared__ uint32_t s_item;
  __shared__ unsigned long long s_pos;
  uint32_t* bm = Bg.bitmaps + (size_t)blockIdx.x * Bg.nwords;
  int32_t* queue = Bg.queues + (size_t)blockIdx.x * (size_t)Bg.qcap;
  const int t = threadIdx.x;
  const uint32_t nbig = (uint32_t)A.ctr[2];
  unsigned long long t_ex = 0, t_lv = 0, t_tot = 0;
  for (;;) {
    if (t == 0) s_item = (uint32_t)atomicAdd(&A.ctr[5], 1ull);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= nbig) break;
    const int64_t il = (int64_t)A.big_list[item];
    const int tk = task_of_pos(A, il);
    const TaskDesc& T = A.tasks[tk];
    const GView G = view_of(T);
    const uint32_t i = T.first + (uint32_t)(il - T.sample_base);
    const uint64_t seed = ((uint64_t)G.seed_hi << 32) | G.seed_lo;
    const int32_t root = (int32_t)scale_draw(draw1(seed, kTagRoot, G.stream, 0u, i), G.n);
    unsigned long long s_ex = 0, s_lv = 0;
    BigSet S{T.model == IM_IC, mhash, mq, bm, false, queue, &s_tail, &s_over};
    if (T.model == IM_IC) {
      int32_t head = 0, tail = 1;
      for (int j = t; j < C::kH; j += C::kBlock) mhash[j] = kEmpty;
      if (t == 0) {
        s_tail = 0;
        s_over = 0;
        s_nst = 0;
      }
      __syncthreads();
      if (item < kMaxHandoff) {  // resume from the small path's snapshot
        const Handoff& H = A.handoff[item];
        head = H.head;
        tail = H.tail;  // <= kSmallCap < C::kCap: the snapshot fits LDS mode
        for (int j = t; j < tail; j += C::kBlock) set_insert<C>(S, H.mem[j]);
        if (t == 0) {
          s_ex = H.ex;
          s_lv = H.lv;
        }
      } else if (t == 0) {
        set_insert<C>(S, root);
      }
      __syncthreads();
      if (S.lds) {  // the snapshot's members were distinct; keep its order
        for (int j = t; j < tail; j += C::kBlock)
          mq[j] = item < kMaxHandoff ? A.handoff[item].mem[j] : root;
      }
      __syncthreads();
      while (head < tail) {
        // level start: what a redo in HBM mode restarts from
        const int32_t head0 = head, tail0 = tail;
        const unsigned long long ex0 = s_ex, lv0 = s_lv;
        const int32_t* Q = S.lds ? mq : queue;
        const int32_t nf = min(tail - head, C::kBlock);
        int32_t a = 0, b = 0, ng = 0, v = 0;
        double sk = 0.0;
        if (t < nf) {
          v = Q[head + t];
          a = G.in_off[v];
          b = G.in_off[v + 1];
          sk = G.skip ? G.skip[v] : 0.0;
          if (sk == 0.0) {
            if (a < b) ng = ((b - 1) >> 2) - (a >> 2) + 1;
            s_ex += (unsigned long long)(b - a);
          }
        }
        {  // run-length vertices: their geometric gaps, drawn across each wavefront
          uint32_t wex = 0, wlv = 0;
          rl_walks(sk != 0.0, (uint32_t)v, a, b - a, sk, G.seed_lo, G.seed_hi, G.stream, i,
                   gbase + (t / kWave) * kWave, &wex, &wlv,
                   [&](int32_t e) { big_push<C>(e, stage, &s_nst, G.in_src, S); });
          s_ex += wex;
          s_lv += wlv;
          if (sk != 0.0) a = b = 0;
        }
        int64_t tot64;
        const int32_t ex = (int32_t)block_exclusive_scan64<C::kBlock>(ng, scan_lds, &tot64);
        const int32_t total = (int32_t)tot64;
        pre[t] = ex + ng;
        gbase[t] = (a >> 2) - ex;
        ea[t] = a;
        eb[t] = b;
        head += nf;
        __syncthreads();
        for (int32_t base = 0; base < total; base += C::kBlock * kUnroll) {
          const int o_b = owner_of<C::kBlock>(pre, base);
          const bool uni = pre[o_b] >= min(total, base + C::kBlock * kUnroll);
          uint4 q[kUnroll];
          uint32_t g[kUnroll];
          int32_t e_a[kUnroll], e_b[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int32_t gi = base + u * C::kBlock + t;
            e_a[u] = e_b[u] = 0;
            g[u] = 0;
            if (gi < total) {
              const int o = uni ? o_b : owner_of<C::kBlock>(pre, gi);
              g[u] = (uint32_t)(gbase[o] + gi);
              e_a[u] = ea[o];
              e_b[u] = eb[o];
              q[u] = reinterpret_cast<const uint4*>(G.thr)[g[u]];
            }
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            if (e_a[u] < e_b[u]) {
              const uint4 r =
                  philox4x32_10(make_uint4(g[u], i, kTagEdge, G.stream), G.seed_lo, G.seed_hi);
              const int32_t e0 = (int32_t)(g[u] << 2);
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                const int32_t e = e0 + w;
                const uint32_t qw = pick_word(q[u], w), rw = pick_word(r, w);
                if (e >= e_a[u] && e < e_b[u] && (qw == 0xFFFFFFFFu || rw < qw)) {
                  ++s_lv;
                  big_push<C>(e, stage, &s_nst, G.in_src, S);
                }
              }
            }
          }
          __syncthreads();
          if (s_nst >= C::kStage / 2) big_flush<C>(stage, &s_nst, G.in_src, S);
        }
        big_flush<C>(stage, &s_nst, G.in_src, S);
        tail = s_tail;
        const bool over = S.lds && s_over;
        __syncthreads();
        if (over) {  // the level passed C::kCap members: redo it in a bitmap mode
          S.bits = G.n <= C::kBitsN;
          for (int j = t; j < tail0; j += C::kBlock) {
            const int32_t u = mq[j];
            queue[j] = u;
            if (!S.bits) atomicOr(&bm[u >> 5], 1u << (u & 31));
          }
          if (S.bits) {  // the bitmap replaces the hash and member list in LDS
            __syncthreads();
            const int32_t nw = (G.n + 31) >> 5;
            for (int j = t; j < nw; j += C::kBlock) mhash[j] = 0;
            __syncthreads();
            for (int j = t; j < tail0; j += C::kBlock) {
              const int32_t u = queue[j];
              atomicOr((uint32_t*)&mhash[u >> 5], 1u << (u & 31));
            }
          }
          S.lds = false;
          head = head0;
          tail = tail0;
          s_ex = ex0;
          s_lv = lv0;
          __syncthreads();
          if (t == 0) {
            s_tail = tail0;
            s_over = 0;
          }
          __syncthreads();
        }
      }
    } else if (t == 0) {  // LT: the chain is sequential; one thread walks it
      int32_t v = root, len = 0;
      bm[v >> 5] |= 1u << (v & 31);
      queue[len++] = v;
      for (;;) {
        const int32_t a = G.in_off[v], b = G.in_off[v + 1];
        if (a == b) break;
        s_ex += ceil_log2_plus1(b - a);
        const uint32_t r = draw1(seed, kTagVert, G.stream, i, (uint32_t)v);
        int32_t u = 0;
        if (lt_pick<false>(G, a, b, r, &u) == b) break;
        ++s_lv;
        const uint32_t bit = 1u << (u & 31);
        if (bm[u >> 5] & bit) break;
        bm[u >> 5] |= bit;
        queue[len++] = u;
        v = u;
      }
      s_tail = len;
    }
    __syncthreads();
    const int32_t tail = s_tail;
    if (t == 0) s_pos = atomicAdd(&A.ctr[1], (unsigned long long)tail);
    __syncthreads();
    const unsigned long long pos = s_pos;
    const bool fits = pos + (unsigned long long)tail <= A.arena_cap;
    if (S.bits) {
      // members in ascending order straight from the LDS bitmap
      const uint32_t nw = ((uint32_t)G.n + 31) >> 5;
      const uint32_t per = (nw + C::kBlock - 1) / C::kBlock;
      const uint32_t w0 = min((uint32_t)t * per, nw);
      const uint32_t w1 = min(w0 + per, nw);
      const uint32_t* lbm = (const uint32_t*)mhash;
      int64_t cnt = 0;
      for (uint32_t w = w0; w < w1; ++w) cnt += __popc(lbm[w]);
      int64_t tot;
      int64_t o = block_exclusive_scan64<C::kBlock>(cnt, scan_lds, &tot);
      if (fits) {
        for (uint32_t w = w0; w < w1; ++w) {
          uint32_t x = lbm[w];
          while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1;
            A.arena[pos + o++] = (int32_t)((w << 5) + b);
          }
        }
      }
    } else if (S.lds || tail <= C::kSortCap) {
      // LDS mode: the members are in mq (tail <= C::kCap); HBM mode: copy them
      // into the (now unused) LDS pool
      int32_t* sorted = S.lds ? mq : pool;
      int32_t P = 1;
      while (P < tail) P <<= 1;
      if (S.lds) {
        for (int j = tail + t; j < P; j += C::kBlock) sorted[j] = 0x7FFFFFFF;
      } else {  // the HBM queue's loads issued 8 at a time
        constexpr int kU = 8;
        for (int j0 = t; j0 < P; j0 += kU * C::kBlock) {
          int32_t x[kU];
#pragma unroll
          for (int q = 0; q < kU; ++q) {
            const int j = j0 + q * C::kBlock;
            x[q] = j < tail ? queue[j] : 0x7FFFFFFF;
          }
#pragma unroll
          for (int q = 0; q < kU; ++q)
            if (j0 + q * C::kBlock < P) sorted[j0 + q * C::kBlock] = x[q];
        }
      }
      __syncthreads();
      for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int u = t; u < (P >> 1); u += C::kBlock) {
            const int i1 = ((u & ~(j - 1)) << 1) | (u & (j - 1));
            const int i2 = i1 | j;
            const bool asc = (i1 & k) == 0;
            const int32_t x = sorted[i1], y = sorted[i2];
            if ((x > y) == asc) {
              sorted[i1] = y;
              sorted[i2] = x;
            }
          }
          __syncthreads();
        }
      }
      if (fits)
        for (int j = t; j < tail; j += C::kBlock) A.arena[pos + j] = sorted[j];
      if (!S.lds)  // clear the set's bits from the LDS copy of its members
        for (int j = t; j < tail; j += C::kBlock) bm[sorted[j] >> 5] = 0u;
    } else {
      // members in ascending order straight from the bitmap
      const uint32_t per = (Bg.nwords + C::kBlock - 1) / C::kBlock;
      const uint32_t w0 = min((uint32_t)t * per, Bg.nwords);
      const uint32_t w1 = min(w0 + per, Bg.nwords);
      int64_t cnt = 0;
      for (uint32_t w = w0; w < w1; ++w) cnt += __popc(bm[w]);
      int64_t tot;
      int64_t o = block_exclusive_scan64<C::kBlock>(cnt, scan_lds, &tot);
      if (fits) {
        for (uint32_t w = w0; w < w1; ++w) {
          uint32_t x = bm[w];
          while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1;
            A.arena[pos + o++] = (int32_t)((w << 5) + b);
          }
        }
      }
    }
    __syncthreads();
    if (!S.lds && !S.bits && tail > C::kSortCap)  // (smaller sets were cleared above)
      for (int j = t; j < tail; j += C::kBlock) bm[queue[j] >> 5] = 0u;
    if (t == 0) {
      A.start[il] = (int64_t)pos;
      A.len[il] = tail;
    }
    t_ex += s_ex;
    t_lv += s_lv;
    if (t == 0) t_tot += (unsigned long long)tail;
    __syncthreads();
  }
  int64_t tot;
  (void)block_exclusive_scan64<C::kBlock>((int64_t)t_ex, scan_lds, &tot);
  if (t == 0 && tot) atomicAdd(&A.ctr[6], (unsigned long long)tot);
  (void)block_exclusive_scan64<C::kBlock>((int64_t)t_lv, scan_lds, &tot);
  if (t == 0 && tot) atomicAdd(&A.ctr[7], (unsigned long long)tot);
  (void)block_exclusive_scan64<C::kBlock>((int64_t)t_tot, scan_lds, &tot);
  if (t == 0 && tot) {
    atomicAdd(&A.ctr[8], (unsigned long long)tot);
    atomicAdd(&A.ctr[10], (unsigned long long)tot);
  }
}

// ------------------------------------------------------------------ LT walks
// A walk's members are kept twice per lane: in order in the lane's list in
// HBM (what is written out), and as a 256-bit Bloom filter in registers.  A
// clear filter bit proves a vertex new, so the common step appends without
// reading anything back; only on a set bit is the list scanned for an exact
// answer.  A short list (kLtOwnScan members) is scanned by its own lane; a
// longer one by the whole wavefront, 256 members per round (one 1 KB
// coalesced load), since the filter fills up on long walks and a lane
// scanning its own list would make such a walk quadratic in its length.
// Nothing has to be cleared between walks.
struct Bloom {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ uint32_t bloom_bit(int32_t u) {
  return ((uint32_t)u * 0x9E3779B1u) >> 24;
}

// Masked updates of all four words, so that the filter stays in registers
// (a selected word becomes an indexed private array in scratch memory).
__device__ __forceinline__ bool bloom_has(const Bloom& b, uint32_t h) {
  const uint64_t m = 1ull << (h & 63u);
  const uint32_t q = h >> 6;
  const uint64_t hit = (b.w0 & (q == 0u ? m : 0ull)) | (b.w1 & (q == 1u ? m : 0ull)) |
                       (b.w2 & (q == 2u ? m : 0ull)) | (b.w3 & (q == 3u ? m : 0ull));
  return hit != 0ull;
}

__device__ __forceinline__ void bloom_add(Bloom& b, uint32_t h) {
  const uint64_t m = 1ull << (h & 63u);
  const uint32_t q = h >> 6;
  b.w0 |= q == 0u ? m : 0ull;
  b.w1 |= q == 1u ? m : 0ull;
  b.w2 |= q == 2u ? m : 0ull;
  b.w3 |= q == 3u ? m : 0ull;
}

// Is u among the first len (<= kLtOwnScan) entries of the lane's list
// (16-byte aligned)?  All of its loads are issued before any compare.
constexpr int32_t kLtOwnScan = 32;

__device__ __forceinline__ bool list_has(const int32_t* Ls, int32_t len, int32_t u) {
  int4 x[kLtOwnScan / 4];
#pragma unroll
  for (int q = 0; q < kLtOwnScan / 4; ++q)
    x[q] = 4 * q < len ? *reinterpret_cast<const int4*>(Ls + 4 * q) : make_int4(-1, -1, -1, -1);
  bool hit = false;
#pragma unroll
  for (int q = 0; q < kLtOwnScan / 4; ++q) {
    const int j = 4 * q;
    hit |= (j < len && x[q].x == u) | (j + 1 < len && x[q].y == u) |
           (j + 2 < len && x[q].z == u) | (j + 3 < len && x[q].w == u);
  }
  return hit;
}

// Second membership filter of a walk, 32 words per lane in LDS, hashed with
// another multiplier than the register filter: it is read only when the
// register filter has the bit, and a clear bit again proves the vertex new.
#ifndef IM_LT_BLOOM2
#define IM_LT_BLOOM2 1
#endif
#ifndef IM_LT_BLOOM2_BITS
#define IM_LT_BLOOM2_BITS 10
#endif
constexpr int kLtBloom2Words = (1 << IM_LT_BLOOM2_BITS) / 32;

__device__ __forceinline__ uint32_t bloom2_bit(int32_t u) {
  return ((uint32_t)u * 0x85EBCA6Bu) >> (32 - IM_LT_BLOOM2_BITS);
}

// One lane per walk.  Lanes take new samples as their walks end (aggregated
// per wave), so a long walk does not hold up the other 63 lanes.  Resident
// wavefronts per SIMD (IM_LT_WAVES): the compiler keeps the registers within
// what that many need.
#ifndef IM_LT_WAVES
#define IM_LT_WAVES 3
#endif
__global__ __launch_bounds__(kLtBlock) __attribute__((amdgpu_waves_per_eu(IM_LT_WAVES)))
void k_sample_lt(SampleArgs A, int32_t* lane_list) {
  const size_t gl = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t* Ls = lane_list + gl * kLtCap;
#if IM_LT_BLOOM2
  __shared__ uint32_t s_f2[kLtBlock * kLtBloom2Words];
  uint32_t* F2 = s_f2 + (size_t)threadIdx.x * kLtBloom2Words;  // this lane's
#endif
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  bool have = false, done = false;
  uint32_t i = 0;
  int64_t il = 0;
  GView G{};
  uint64_t seed = 0;
  int32_t v = 0, len = 0;
  Bloom bl{0ull, 0ull, 0ull, 0ull};
  unsigned long long ex = 0, lv = 0, s_ex = 0, s_lv = 0, w_tot = 0;
  unsigned long long pnext = 0, pend = 0;  // this wave's pool of sample ids
  bool dry = false;                        // no ids left anywhere
  unsigned long long cpos = 0, cend = 0;   // reserved arena chunk
  for (;;) {
    const uint64_t need = __ballot(!have && !done);
    if (need) {
      if (pnext == pend && !dry) {
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(&A.ctr[11], (unsigned long long)A.lt_grab);
        b = shfl_u64(b, 0);
        if (b >= A.count) {
          dry = true;
        } else {
          pnext = b;
          pend = min(b + A.lt_grab, (unsigned long long)A.count);
        }
      }
      const unsigned long long avail = pend - pnext;
      const unsigned long long rank = (unsigned long long)__popcll(need & below);
      if (!have && !done) {
        if (rank < avail) {
          int tk;
          locate_work(A, pnext + rank, &tk, &i, &il);
          G = view_of(A.tasks[tk]);
          seed = ((uint64_t)G.seed_hi << 32) | G.seed_lo;
          v = (int32_t)scale_draw(draw1(seed, kTagRoot, G.stream, 0u, i), G.n);
          bl = Bloom{0ull, 0ull, 0ull, 0ull};
          bloom_add(bl, bloom_bit(v));
#if IM_LT_BLOOM2
#pragma unroll
          for (int q = 0; q < kLtBloom2Words / 4; ++q)
            reinterpret_cast<uint4*>(F2)[q] = make_uint4(0u, 0u, 0u, 0u);
          {
            const uint32_t h2 = bloom2_bit(v);
            F2[h2 >> 5] |= 1u << (h2 & 31u);
          }
#endif
          Ls[0] = v;
          len = 1;
          s_ex = s_lv = 0;
          have = true;
        } else if (dry) {
          done = true;
        }
      }
      pnext += min(avail, (unsigned long long)__popcll(need));
    }
    if (!__any(have)) break;
    bool fin = false, over = false, cand = false, seen = false, wide = false;
    int32_t u = 0;
    uint32_t h = 0;
    if (have) {
      const int32_t a = G.in_off[v], b = G.in_off[v + 1];
      if (a == b) {
        fin = true;
      } else {
        s_ex += ceil_log2_plus1(b - a);
        const uint32_t r = draw1(seed, kTagVert, G.stream, i, (uint32_t)v);
        if (lt_pick(G, a, b, r, &u) == b) {
          fin = true;
        } else {
          ++s_lv;
          h = bloom_bit(u);
          cand = true;
#if IM_LT_BLOOM2
          const uint32_t h2 = bloom2_bit(u);
          if (bloom_has(bl, h) && ((F2[h2 >> 5] >> (h2 & 31u)) & 1u)) {
#else
          if (bloom_has(bl, h)) {
#endif
            if (len <= kLtOwnScan)
              seen = list_has(Ls, len, u);
            else
              wide = true;
          }
        }
      }
    }
    // long lists: the wavefront scans each in turn (a lane's list entries
    // were stored by that lane in earlier rounds of this loop)
    uint64_t pend = __ballot(wide);
    if (pend) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    while (pend) {
      const int j = __ffsll((long long)pend) - 1;
      pend &= pend - 1;
      const int32_t lj = __shfl(len, j, kWave), uj = __shfl(u, j, kWave);
      const int32_t* Lj = lane_list + (gl - (size_t)lane + (size_t)j) * kLtCap;
      bool hit = false;
      // a whole list (kLtCap entries) in one batch of loads: 4 x 16 bytes per lane
      constexpr int kR = kLtCap / (4 * kWave);
      int4 xs[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int32_t p = 4 * lane + r * 4 * kWave;
        xs[r] = p < lj ? *reinterpret_cast<const int4*>(Lj + p) : make_int4(-1, -1, -1, -1);
      }
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int32_t p = 4 * lane + r * 4 * kWave;
        hit |= (p < lj && xs[r].x == uj) | (p + 1 < lj && xs[r].y == uj) |
               (p + 2 < lj && xs[r].z == uj) | (p + 3 < lj && xs[r].w == uj);
      }
      const bool any = __any(hit);
      if (lane == j) seen = any;
    }
    if (cand) {
      if (seen) {
        fin = true;
      } else if (len == kLtCap) {
        fin = true;
        over = true;
      } else {
        bloom_add(bl, h);
#if IM_LT_BLOOM2
        {
          const uint32_t h2 = bloom2_bit(u);
          F2[h2 >> 5] |= 1u << (h2 & 31u);
        }
#endif
        Ls[len++] = u;
        v = u;
      }
    }
    const bool emit = fin && !over;
    const int32_t mylen = emit ? len : 0;
    const int32_t inc = wave_inclusive_scan(mylen);
    const int32_t tot = __shfl(inc, kWave - 1, kWave);
    unsigned long long pos = 0;
    if (tot > 0) {
      if (cpos + (unsigned long long)tot > cend) {
        const unsigned long long want = max((unsigned long long)tot, 4 * kChunk);
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(&A.ctr[1], want);
        cpos = shfl_u64(b, 0);
        cend = cpos + want;
      }
      pos = cpos + (unsigned long long)(inc - mylen);
      cpos += (unsigned long long)tot;
      w_tot += (unsigned long long)tot;
    }
    if (fin) {
      if (over) {
        const uint32_t slot = (uint32_t)atomicAdd(&A.ctr[2], 1ull);
        A.big_list[slot] = il;
        A.len[il] = -1;
      } else {
        if (pos + (unsigned long long)len <= A.arena_cap) {
          for (int32_t j0 = 0; j0 < len; j0 += 32) {  // 32 members per round, loads first
            int4 x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
              x[q] = j0 + 4 * q < len ? *reinterpret_cast<const int4*>(Ls + j0 + 4 * q)
                                      : make_int4(0, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int32_t j = j0 + 4 * q;
              if (j < len) A.arena[pos + j] = x[q].x;
              if (j + 1 < len) A.arena[pos + j + 1] = x[q].y;
              if (j + 2 < len) A.arena[pos + j + 2] = x[q].z;
              if (j + 3 < len) A.arena[pos + j + 3] = x[q].w;
            }
          }
        }
        A.start[il] = (int64_t)pos;
        A.len[il] = len;
        ex += s_ex;
        lv += s_lv;
      }
      have = false;
    }
  }
  ex = wave_sum(ex);
  lv = wave_sum(lv);
  if (lane == 0) {
    if (ex) atomicAdd(&A.ctr[3], ex);
    if (lv) atomicAdd(&A.ctr[4], lv);
    if (w_tot) atomicAdd(&A.ctr[10], w_tot);
  }
}

// ------------------------------------------------------------------ gather
constexpr int kGatherBlock = 256;

constexpr int32_t kGatherLane = 16;  // sets up to this size are copied by one lane

// Copies every set from the arena to its canonical place.  Sets written in
// order (IC): one lane per set, 64 consecutive sets per wavefront, the few
// longer than kGatherLane copied by the whole wavefront.  Sets written
// unsorted (LT walks): one wavefront per set, sorting it on the way.
__global__ __launch_bounds__(kGatherBlock) void k_gather(uint32_t count,
                                                         const int64_t* __restrict__ start,
                                                         const int32_t* __restrict__ len,
                                                         const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ arena,
                                                         int32_t* __restrict__ mem,
                                                         int sort_small) {
  __shared__ int32_t buf_all[kGatherBlock / kWave][kGatherSortCap];
  int32_t* buf = buf_all[threadIdx.x / kWave];
  const int lane = lane_id();
  if (!sort_small) {
    const uint64_t w0 = ((uint64_t)blockIdx.x * kGatherBlock + threadIdx.x) / kWave * kWave;
    const uint64_t step = (uint64_t)gridDim.x * kGatherBlock;
    for (uint64_t base = w0; base < count; base += step) {  // wavefront-uniform
      const uint64_t sid = base + (uint64_t)lane;
      int32_t L = 0;
      int64_t a = 0, d = 0;
      if (sid < count) {
        L = len[sid];
        a = start[sid];
        d = off[sid];
      }
      const bool mine = L <= kGatherLane;
      if (mine)
        for (int32_t j = 0; j < L; ++j) mem[d + j] = arena[a + j];
      unsigned long long todo = __ballot(!mine);
      while (todo) {
        const int src = __ffsll(todo) - 1;
        todo &= todo - 1;
        const int32_t Ls = __shfl(L, src, kWave);
        const int64_t as = shfl_i64(a, src), ds = shfl_i64(d, src);
        for (int32_t j = lane; j < Ls; j += kWave) mem[ds + j] = arena[as + j];
      }
    }
    return;
  }
  const uint32_t wid = (blockIdx.x * kGatherBlock + threadIdx.x) / kWave;
  const uint32_t nw = gridDim.x * (kGatherBlock / kWave);
  for (uint32_t s = wid; s < count; s += nw) {
    const int32_t L = len[s];
    const int32_t* src = arena + start[s];
    int32_t* dst = mem + off[s];
    if (sort_small && L > 1 && L <= kGatherSortCap) {
      int32_t P = 1;
      while (P < L) P <<= 1;
      for (int j = lane; j < P; j += kWave) buf[j] = j < L ? src[j] : 0x7FFFFFFF;
      wave_sync();
      for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int t = lane; t < (P >> 1); t += kWave) {
            const int i1 = ((t & ~(j - 1)) << 1) | (t & (j - 1));
            const int i2 = i1 | j;
            const bool asc = (i1 & k) == 0;
            const int32_t x = buf[i1], y = buf[i2];
            if ((x > y) == asc) {
              buf[i1] = y;
              buf[i2] = x;
            }
          }
          wave_sync();
        }
      }
      for (int j = lane; j < L; j += kWave) dst[j] = buf[j];
      wave_sync();
    } else {
      for (int j = lane; j < L; j += kWave) dst[j] = src[j];
    }
  }
}

// ------------------------------------------------------------------ host
// Arena entries beyond the sets themselves: the unused tails of the chunks
// the wavefronts reserve.  Every reservation holds at least one set and
// exceeds its sets by at most 4 kChunk, which bounds the tails by
// 4 kChunk per set; over many sets they stay below 4 kChunk per resident
// wavefront slot (measured).
static uint64_t arena_slack(int num_cus, uint64_t sets) {
  return std::min<uint64_t>((uint64_t)num_cus * 32 * 4 * kChunk, sets * 4 * kChunk);
}

// Workgroups of the LT launch: the knob's count per CU, or fewer when there
// are fewer walks than lanes to give them out (each wavefront claims
// lt_grab at a time).
static int lt_blocks(int num_cus, int64_t walks) {
  const int64_t per_block = (int64_t)(kLtBlock / kWave) * tune(IM_TUNE_LT_GRAB);
  const int64_t want = (walks + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cus * tune(IM_TUNE_LT_BLOCKS),
                                                     want));
}

static size_t lt_lane_bytes(int blocks) {
  return ws_align((size_t)blocks * kLtBlock * kLtCap * sizeof(int32_t));
}

// One large-set worker: an n-bit bitmap and an n-entry queue.
static size_t big_worker_bytes(int32_t max_n) {
  return (size_t)((max_n + 31) / 32) * 4 + (size_t)max_n * 4;
}

// Phase 1 of sampling every task of a table into one canonical CSR over output
// positions (task t's sets at [sample_base, sample_base + count)).  IC tasks
// share one main launch, LT tasks another; both hand oversized sets to one
// large-path launch.  The sets land in the stream's staging arena; the
// exclusive scan of their sizes is written to off.  R records where they are
// for gather_arena.  sort_all: sort every set on the gather (needed when IC
// and LT tasks share the output); otherwise only LT sets are sorted there.
// expect: a guess of the member total (0: none), used to size the arena.
int sample_to_arena(const TaskDesc* h_tasks, int ntasks, int64_t count_total, int32_t max_n,
                    int64_t* off, int64_t expect, int64_t stop_above, bool sort_all, bool timed,
                    ArenaRun* R, hipStream_t s) {
  *R = ArenaRun{};
  DeviceInfo di;
  IM_TRY(device_info(&di));
  if (count_total == 0) {
    IM_HIP(hipMemsetAsync(off, 0, sizeof(int64_t), s));
    IM_HIP(hipStreamSynchronize(s));
    return IM_OK;
  }
  if (count_total >= ((int64_t)1 << 32)) return IM_EINVAL;
  const uint64_t cnt = (uint64_t)count_total;
  // work segments per model, in task order
  std::vector<int64_t> seg_ic{0}, seg_lt{0};
  std::vector<int32_t> task_ic, task_lt;
  bool any_lt = false;
  for (int t = 0; t < ntasks; ++t) {
    if (h_tasks[t].count == 0) continue;
    if (h_tasks[t].model == IM_IC) {
      task_ic.push_back(t);
      seg_ic.push_back(seg_ic.back() + h_tasks[t].count);
    } else {
      any_lt = true;
      task_lt.push_back(t);
      seg_lt.push_back(seg_lt.back() + h_tasks[t].count);
    }
  }
  // device copies of the task table and the segment lists
  const size_t tab_bytes = (size_t)ntasks * sizeof(TaskDesc);
  const size_t seg_bytes = (seg_ic.size() + seg_lt.size()) * 8 + (task_ic.size() + task_lt.size()) * 4;
  void* tp = nullptr;
  IM_TRY(scratch(s, kSlotSampleTasks, tab_bytes + seg_bytes + 256, &tp));
  char* tc = (char*)tp;
  TaskDesc* d_tasks = (TaskDesc*)tc;
  int64_t* d_seg_ic = (int64_t*)(tc + ((tab_bytes + 63) / 64) * 64);
  int64_t* d_seg_lt = d_seg_ic + seg_ic.size();
  int32_t* d_task_ic = (int32_t*)(d_seg_lt + seg_lt.size());
  int32_t* d_task_lt = d_task_ic + task_ic.size();
  IM_HIP(hipMemcpyAsync(d_tasks, h_tasks, tab_bytes, hipMemcpyHostToDevice, s));
  IM_HIP(hipMemcpyAsync(d_seg_ic, seg_ic.data(), seg_ic.size() * 8, hipMemcpyHostToDevice, s));
  IM_HIP(hipMemcpyAsync(d_seg_lt, seg_lt.data(), seg_lt.size() * 8, hipMemcpyHostToDevice, s));
  if (!task_ic.empty())
    IM_HIP(hipMemcpyAsync(d_task_ic, task_ic.data(), task_ic.size() * 4, hipMemcpyHostToDevice, s));
  if (!task_lt.empty())
    IM_HIP(hipMemcpyAsync(d_task_lt, task_lt.data(), task_lt.size() * 4, hipMemcpyHostToDevice, s));

  // per-position metadata: start (i64), len (i32), big list (u32), counters,
  // hand-off snapshots
  const uint32_t nhand = (uint32_t)std::min<uint64_t>(cnt, kMaxHandoff);
  const size_t meta_bytes = (size_t)cnt * 8 + (size_t)cnt * 4 + (size_t)cnt * 4 + 256 + 256 +
                            (size_t)nhand * sizeof(Handoff) + 64;
  void* mp = nullptr;
  IM_TRY(scratch(s, kSlotSampleMeta, meta_bytes, &mp));
  unsigned long long* ctr = (unsigned long long*)mp;
  int64_t* start = (int64_t*)((char*)mp + 256);
  int32_t* lens = (int32_t*)(start + cnt);
  uint32_t* big_list = (uint32_t*)(lens + cnt);
  Handoff* handoff = (Handoff*)(((uintptr_t)(big_list + cnt) + 63) & ~(uintptr_t)63);

  // room for the sets plus the unfilled tails of the per-wave arena chunks
  // (each wavefront holds at most one partly used chunk); the guess of the
  // member total: `expect` (the caller's capacity, or an estimate), else up
  // to 64 members per set within what the workspace leaves, so that one pass
  // usually suffices (an arena that turns out short means sampling again)
  const uint64_t slack = arena_slack(di.num_cus, cnt);
  // carved after the arena: the LT walks' lists, one large-set worker, the scan
  const size_t later = (any_lt ? lt_lane_bytes(lt_blocks(di.num_cus, seg_lt.back())) : 0) +
                       ws_align(big_worker_bytes(max_n)) +
                       ws_align((size_t)(cnt / 8192 + 2) * 8) + 4096;
  const size_t room = scratch_room();
  const int64_t room_entries =
      room > later ? (int64_t)((room - later) / 4) - (int64_t)slack : (int64_t)0;
  const int64_t guess =
      expect > 0 ? expect + expect / 8
                 : std::max<int64_t>(count_total * 2,
                                     std::min<int64_t>(count_total * 64, room_entries / 2));
  uint64_t arena_cap = (uint64_t)std::max<int64_t>(guess, count_total * 2) + slack;
  unsigned long long hc[16] = {0};
  // device times of the launches, only when statistics are requested
  hipEvent_t ev[4] = {};
  if (timed)
    for (auto& e : ev) IM_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    bool on;
    ~EvGuard() {
      if (on)
        for (int j = 0; j < 4; ++j) (void)hipEventDestroy(e[j]);
    }
  } ev_guard{ev, timed};
  float ms_main = 0.f, ms_large = 0.f;
  void* ap = nullptr;
  for (int attempt = 0; attempt < 3; ++attempt) {
    IM_TRY(scratch(s, kSlotSampleArena, arena_cap * sizeof(int32_t), &ap));
    SampleArgs A{};
    A.tasks = d_tasks;
    A.ntasks = ntasks;
    A.arena = (int32_t*)ap;
    A.arena_cap = arena_cap;
    A.start = start;
    A.len = lens;
    A.big_list = big_list;
    A.handoff = handoff;
    A.ctr = ctr;
    IM_HIP(hipMemsetAsync(ctr, 0, 256, s));
    if (timed) IM_HIP(hipEventRecord(ev[0], s));
    if (!task_ic.empty()) {
      SampleArgs Ai = A;
      Ai.seg_base = d_seg_ic;
      Ai.seg_task = d_task_ic;
      Ai.nseg = (int32_t)task_ic.size();
      Ai.count = (uint64_t)seg_ic.back();
      const int blocks = di.num_cus * (int)tune(IM_TUNE_SAMPLE_BLOCKS);
      k_sample_ic_small<<<dim3(blocks), dim3(kSmallBlock), 0, s>>>(Ai);
      IM_HIP(hipGetLastError());
    }
    if (!task_lt.empty()) {
      SampleArgs Al = A;
      Al.seg_base = d_seg_lt;
      Al.seg_task = d_task_lt;
      Al.nseg = (int32_t)task_lt.size();
      Al.count = (uint64_t)seg_lt.back();
      Al.lt_grab = (uint32_t)tune(IM_TUNE_LT_GRAB);
      const int blocks = lt_blocks(di.num_cus, Al.count);
      const size_t lanes = (size_t)blocks * kLtBlock;
      void* hp = nullptr;
      IM_TRY(scratch(s, kSlotSampleLtLane, lanes * kLtCap * sizeof(int32_t), &hp));
      k_sample_lt<<<dim3(blocks), dim3(kLtBlock), 0, s>>>(Al, (int32_t*)hp);
      IM_HIP(hipGetLastError());
    }
    if (timed) IM_HIP(hipEventRecord(ev[1], s));
    IM_HIP(hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
    IM_HIP(hipStreamSynchronize(s));
    if (timed) IM_HIP(hipEventElapsedTime(&ms_main, ev[0], ev[1]));
    ms_large = 0.f;
    if (hc[2] > 0) {
      const uint32_t nbig = (uint32_t)hc[2];
      const uint32_t nwords = (uint32_t)(((int64_t)max_n + 31) / 32);
      // workers each hold an n-bit bitmap and an n-entry queue
      const size_t per_worker = (size_t)nwords * 4 + (size_t)max_n * 4;
      // up to kPerCu workers per CU, within a budget of IM_BIG_BUDGET_GIB per
      // stream (at 2^20 vertices 16 GiB holds 3.9 K workers, as fast as any
      // larger number; 8 GiB is 40% slower); the bitmaps are zero
      // between uses (each set clears its own bits), so only a new buffer
      // needs clearing
      // one wavefront per set unless most sets were handed off
      const int64_t shape = tune(IM_TUNE_BIG_SHAPE);
      const bool narrow = shape == 1 || (shape == 0 && (uint64_t)nbig * 8 <= (uint64_t)cnt);
      const uint32_t max_workers =
          (uint32_t)di.num_cus * (narrow ? BigNarrow::kPerCu : BigWide::kPerCu);
      const size_t budget = (size_t)IM_BIG_BUDGET_GIB << 30;
      // within the budget and what the workspace leaves beside the offset
      // scan that follows (at least one worker)
      const size_t scan = ws_align((size_t)(cnt / 8192 + 2) * 8) + 256;
      const size_t room = scratch_largest();
      const size_t fit = room > scan ? (room - scan) / per_worker : 0;
      if (fit < 1) {
        scratch_need(per_worker + scan);
        set_error_text("workspace too small for one large-set worker (" +
                       std::to_string(per_worker) + " bytes; im_workspace_need)");
        return IM_ENOMEM;
      }
      const uint32_t best = (uint32_t)std::min<size_t>(
          std::min<size_t>(max_workers, budget / per_worker), (size_t)nbig);
      const uint32_t workers = (uint32_t)std::max<size_t>(1, std::min<size_t>(best, fit));
      if (workers < best) scratch_wish((size_t)best * per_worker + 4096);
      void* bp = nullptr;
      IM_TRY(scratch(s, kSlotSampleBig, (size_t)workers * per_worker, &bp));
      BigArgs Bg;
      Bg.nwords = nwords;
      Bg.qcap = (uint32_t)max_n;
      Bg.bitmaps = (uint32_t*)bp;
      Bg.queues = (int32_t*)((char*)bp + (size_t)workers * nwords * 4);
      // every worker's bitmap starts empty (each set clears its own bits
      // again before the worker takes the next one)
      IM_HIP(hipMemsetAsync(Bg.bitmaps, 0, (size_t)workers * nwords * 4, s));
      if (timed) IM_HIP(hipEventRecord(ev[2], s));
      if (narrow)
        k_sample_big<BigNarrow><<<dim3(workers), dim3(BigNarrow::kBlock), 0, s>>>(A, Bg);
      else
        k_sample_big<BigWide><<<dim3(workers), dim3(BigWide::kBlock), 0, s>>>(A, Bg);
      IM_HIP(hipGetLastError());
      if (timed) IM_HIP(hipEventRecord(ev[3], s));
      IM_HIP(hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
      IM_HIP(hipStreamSynchronize(s));
      if (timed) IM_HIP(hipEventElapsedTime(&ms_large, ev[2], ev[3]));
    }
    R->passes = attempt + 1;
    R->total = (int64_t)hc[10];  // exact even when the arena was short
    if (hc[1] <= arena_cap) break;
    // more members than the caller can take: the call reports the total and
    // returns IM_ERANGE, so the sets need not be kept
    if (stop_above > 0 && (int64_t)hc[10] > stop_above) break;
    if (attempt == 2) {
      set_error_text("im_sample_rrr: arena still short after 3 passes (needed " +
                     std::to_string(hc[1]) + " of " + std::to_string(arena_cap) + " entries)");
      return IM_ENOMEM;
    }
    // the sets are deterministic, the chunk slack is not: leave room for it
    arena_cap = hc[1] + hc[1] / 8 + slack;
  }
  const int64_t tot = (int64_t)hc[10];
  IM_TRY(exclusive_scan_i32_to_i64(lens, (int64_t)cnt, off, s));
  R->cnt = cnt;
  R->arena = (const int32_t*)ap;
  R->start = start;
  R->lens = lens;
  R->sort = sort_all || any_lt;
  R->total = tot;
  R->examined = (int64_t)(hc[3] + hc[6]);
  R->live = (int64_t)(hc[4] + hc[7]);
  R->large_sets = (int64_t)hc[2];
  R->large_total = (int64_t)hc[8];
  R->large_examined = (int64_t)hc[6];
  R->large_live = (int64_t)hc[7];
  R->redo_examined = (int64_t)hc[9];
  R->ms_main = ms_main;
  R->ms_large = ms_large;
  return IM_OK;
}

// Phase 2: copies every set of R from the arena to mem at the offsets written
// by phase 1 (sorting the sets that need it).  The arena must be untouched
// since phase 1 (same stream, no other sampling in between).
int gather_arena(const ArenaRun& R, const int64_t* off, int32_t* mem, double* ms, hipStream_t s) {
  if (ms) *ms = 0.0;
  if (R.cnt == 0) return IM_OK;
  DeviceInfo di;
  IM_TRY(device_info(&di));
  hipEvent_t ev[2] = {};
  const bool timed = ms != nullptr;
  if (timed)
    for (auto& e : ev) IM_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    bool on;
    ~EvGuard() {
      if (on)
        for (int j = 0; j < 2; ++j) (void)hipEventDestroy(e[j]);
    }
  } ev_guard{ev, timed};
  if (timed) IM_HIP(hipEventRecord(ev[0], s));
  const int gblocks = (int)std::min<int64_t>(((int64_t)R.cnt + 3) / 4, (int64_t)di.num_cus * 16);
  k_gather<<<dim3(std::max(gblocks, 1)), dim3(kGatherBlock), 0, s>>>(
      (uint32_t)R.cnt, R.start, R.lens, off, R.arena, mem, R.sort ? 1 : 0);
  IM_HIP(hipGetLastError());
  if (timed) {
    IM_HIP(hipEventRecord(ev[1], s));
    IM_HIP(hipEventSynchronize(ev[1]));
    float t = 0.f;
    IM_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
    *ms = t;
  }
  return IM_OK;
}

static void fill_stats(const ArenaRun& R, double ms_canon, im_sample_stats* stats) {
  if (!stats) return;
  stats->total = R.total;
  stats->examined = R.examined;
  stats->live = R.live;
  stats->large_sets = R.large_sets;
  stats->large_total = R.large_total;
  stats->large_examined = R.large_examined;
  stats->large_live = R.large_live;
  stats->redo_examined = R.redo_examined;
  stats->ms_main = R.ms_main;
  stats->ms_large = R.ms_large;
  stats->ms_canon = ms_canon;
}

int sample_tasks(const TaskDesc* h_tasks, int ntasks, int64_t count_total, int32_t max_n,
                 int64_t* off, int32_t* mem, int64_t capacity, int64_t* total,
                 im_sample_stats* stats, bool sort_all, hipStream_t s) {
  ArenaRun R;
  IM_TRY(sample_to_arena(h_tasks, ntasks, count_total, max_n, off, capacity, capacity, sort_all,
                         stats != nullptr, &R, s));
  *total = R.total;
  if (R.total > capacity) {
    IM_HIP(hipStreamSynchronize(s));
    fill_stats(R, 0.0, stats);
    return IM_ERANGE;
  }
  double ms_canon = 0.0;
  IM_TRY(gather_arena(R, off, mem, stats ? &ms_canon : nullptr, s));
  IM_HIP(hipStreamSynchronize(s));
  fill_stats(R, ms_canon, stats);
  return IM_OK;
}

void release_sampling() {
  for (int slot : {kSlotSampleTasks, kSlotSampleMeta, kSlotSampleArena, kSlotSampleLtLane,
                   kSlotSampleBig})
    scratch_release(slot);
}

// Workspace of one sampling call (one task): the task table, per-set
// metadata, the staging arena for `capacity` members, the LT walks' lists,
// large-set workers (one at least; `full`: as many as the launch can use
// within IM_BIG_BUDGET_GIB, 16 for LT whose walks rarely overflow) and the
// offset scan.
size_t ws_sample(int num_cus, int64_t count, int64_t capacity, int32_t max_n, int32_t model,
                 bool full) {
  if (count <= 0) return 0;
  const uint64_t cnt = (uint64_t)count;
  size_t b = ws_align(sizeof(TaskDesc) + 64 + 256) + 64;  // task table, segments
  const uint32_t nhand = (uint32_t)std::min<uint64_t>(cnt, kMaxHandoff);
  b += ws_align((size_t)cnt * 16 + 512 + (size_t)nhand * sizeof(Handoff) + 64);
  const int64_t guess = capacity > 0 ? capacity + capacity / 8 : 0;
  const uint64_t arena = (uint64_t)std::max<int64_t>(guess, count * 2) + arena_slack(num_cus, cnt);
  b += ws_align((size_t)arena * 4);
  if (model == IM_LT) b += lt_lane_bytes(lt_blocks(num_cus, count));
  const size_t per_worker = big_worker_bytes(max_n);
  size_t workers = 1;
  if (full) {
    const size_t budget = (size_t)IM_BIG_BUDGET_GIB << 30;
    const size_t most = model == IM_LT ? 16 : (size_t)num_cus * BigNarrow::kPerCu;
    workers = std::max<size_t>(1, std::min<size_t>(std::min<size_t>(most, budget / per_worker),
                                                   (size_t)count));
  }
  b += ws_align(workers * per_worker);
  b += ws_align((size_t)(cnt / 8192 + 2) * 8) + 8192;
  return b;
}

int graph_ok(const im_graph* g) {
  if (!g || g->n <= 0 || g->num_edges < 0 || g->num_edges >= (int64_t)0x7FFFFFFF ||
      !g->in_off || (g->num_edges > 0 && (!g->in_src || !g->thr)) ||
      (g->model != IM_IC && g->model != IM_LT) || ((uintptr_t)g->thr & 15u) ||
      ((uintptr_t)g->lt_index & 15u))
    return 0;
  return 1;
}

TaskDesc task_of(const im_graph* g, uint64_t seed, uint32_t stream_tag, int64_t first,
                 int64_t count, int64_t sample_base) {
  TaskDesc T;
  T.in_off = g->in_off;
  T.in_src = g->in_src;
  T.thr = g->thr;
  T.skip = g->skip;
  T.lt_index = g->lt_index;
  T.num_edges = g->num_edges;
  T.n = g->n;
  T.model = g->model;
  T.seed_lo = (uint32_t)seed;
  T.seed_hi = (uint32_t)(seed >> 32);
  T.stream = stream_tag;
  T.first = (uint32_t)first;
  T.sample_base = sample_base;
  T.count = count;
  return T;
}

}  // namespace im

// ------------------------------------------------------------------ entry
extern "C" int im_sample_rrr(const im_graph* g, uint64_t seed, uint32_t stream_tag,
                             int64_t first, int64_t count, int64_t* off, int32_t* mem,
                             int64_t capacity, int64_t* total, im_sample_stats* stats, void* ws,
                             size_t ws_bytes, void* stream) {
  using namespace im;
  if (!off || !total || first < 0 || count < 0 || capacity < 0 ||
      first + count > (int64_t)1 << 32 || (capacity > 0 && !mem) || !graph_ok(g))
    return IM_EINVAL;
  DeviceInfo di;
  IM_TRY(device_info(&di));
  WsScope scope(ws, ws_bytes);
  if (!scope.check(ws_sample(di.num_cus, count, capacity, g->n, g->model, false)))
    return IM_ENOMEM;
  const TaskDesc T = task_of(g, seed, stream_tag, first, count, 0);
  return sample_tasks(&T, 1, count, g->n, off, mem, capacity, total, stats, false,
                      (hipStream_t)stream);
}
