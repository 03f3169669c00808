// common.h -- shared device helpers and host plumbing of the HIP library.
//
// gfx950 (CDNA4): 64-lane wavefronts, 160 KB LDS per CU, 256 CUs.  Nothing
// here uses matrix cores: every operation on the path is integer graph or
// set work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "../../include/im.h"

namespace im {

constexpr int kWave = 64;

// Random-number domains and counter layout (key = seed, counter =
// (id >> 2, sample, tag, stream), word id & 3).
constexpr uint32_t kTagRoot = 0, kTagEdge = 1, kTagVert = 2, kTagPart = 3;
// Levels of the LT search index (16^7 edge ids per top window: every vertex's
// in-edges lie in one aligned group of 16 top windows, as E < 2^31).
constexpr int kLtLevels = 7;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each 32x32 product is
// formed as one 64-bit product (a single v_mad_u64_u32 on gfx950) rather than
// separate high and low multiplies.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t pa = (uint64_t)0xD2511F53u * c.x;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb, (uint32_t)(pa >> 32) ^ c.w ^ k1,
                   (uint32_t)pa);
  }
  return c;
}

__device__ __forceinline__ uint32_t pick_word(uint4 v, uint32_t w) {
  return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
}

__device__ __forceinline__ uint32_t draw1(uint64_t seed, uint32_t tag, uint32_t stream,
                                          uint32_t sample, uint32_t id) {
  uint4 r = philox4x32_10(make_uint4(id >> 2, sample, tag, stream), (uint32_t)seed,
                          (uint32_t)(seed >> 32));
  return pick_word(r, id & 3u);
}

// Natural log for x > 0 (normal) from IEEE-754 basic operations only, so the
// result is the same bits on every implementation of the method: split
// x = m 2^e, fold m into [sqrt(1/2), sqrt(2)), log m = 2 atanh(s) with
// s = (m-1)/(m+1) as the odd series up to s^19.
__host__ __device__ inline double im_log(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
#else
  unsigned long long bits;
  __builtin_memcpy(&bits, &x, sizeof bits);
#endif
  int e = (int)((bits >> 52) & 0x7FF) - 1023;
  const unsigned long long mb = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
#if defined(__HIP_DEVICE_COMPILE__)
  double m = __longlong_as_double((long long)mb);
#else
  double m;
  __builtin_memcpy(&m, &mb, sizeof m);
#endif
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double t = 2.0 / 19.0;
  t = t * z + 2.0 / 17.0;
  t = t * z + 2.0 / 15.0;
  t = t * z + 2.0 / 13.0;
  t = t * z + 2.0 / 11.0;
  t = t * z + 2.0 / 9.0;
  t = t * z + 2.0 / 7.0;
  t = t * z + 2.0 / 5.0;
  t = t * z + 2.0 / 3.0;
  t = t * z + 2.0;
  return (double)e * 0.6931471805599453 + s * t;
}

// Uniform on (0, 1] from 53 bits of draw pair j of (sample i, vertex v):
// counter (v, i, 2^31 | j/2, stream), words 2(j&1) (high 21 bits) and
// 2(j&1)+1.
__device__ __forceinline__ double skip_uniform(uint32_t seed_lo, uint32_t seed_hi,
                                               uint32_t stream, uint32_t i, uint32_t v,
                                               uint32_t j) {
  const uint4 r = philox4x32_10(make_uint4(v, i, 0x80000000u | (j >> 1), stream), seed_lo, seed_hi);
  const uint32_t hi = ((j & 1u) ? r.z : r.x) >> 11, lo = (j & 1u) ? r.w : r.y;
  const double u = (double)(((unsigned long long)hi << 32) | lo) + 1.0;
  return u * 1.1102230246251565e-16;  // 2^-53
}

// The same uniform, for draws j = 0, 1, 2, ... in order: draws 2t and 2t+1
// come from one Philox block, which is computed at even j into *blk.
__device__ __forceinline__ double skip_uniform_seq(uint32_t seed_lo, uint32_t seed_hi,
                                                   uint32_t stream, uint32_t i, uint32_t v,
                                                   uint32_t j, uint4* blk) {
  if (!(j & 1u))
    *blk = philox4x32_10(make_uint4(v, i, 0x80000000u | (j >> 1), stream), seed_lo, seed_hi);
  const uint32_t hi = ((j & 1u) ? blk->z : blk->x) >> 11, lo = (j & 1u) ? blk->w : blk->y;
  const double u = (double)(((unsigned long long)hi << 32) | lo) + 1.0;
  return u * 1.1102230246251565e-16;  // 2^-53
}

// floor(r * n / 2^32): maps a uniform word onto [0, n).
__device__ __forceinline__ uint32_t scale_draw(uint32_t r, uint32_t n) {
  return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders LDS traffic of one wavefront (the wave's lanes run in lockstep; this
// keeps the compiler from moving LDS accesses across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Cross-lane moves by DPP (register to register, no LDS): lane i reads lane
// i - n of its row of 16 (row_shr:n, dpp_ctrl 0x110 + n) or the last lane of
// row 0 / row 1 (row_bcast:15 = 0x142, row_bcast:31 = 0x143, for the rows in
// RowMask); a lane without a source reads 0.  Every lane must be active.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xF, false);
}
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = dpp_u32<Ctrl, RowMask>((uint32_t)v);
  const uint32_t hi = dpp_u32<Ctrl, RowMask>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <int Ctrl, int RowMask, typename T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(T) == 4)
    return (T)dpp_u32<Ctrl, RowMask>((uint32_t)v);
  else
    return (T)dpp_u64<Ctrl, RowMask>((uint64_t)v);
}

// Inclusive prefix sum over the wavefront's 64 lanes: within each row of 16
// by shifts of 1, 2, 4, 8; then rows 1 and 3 add the last lane of rows 0 and
// 2, and rows 2 and 3 add lane 31.  Every lane must be active.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  x += dpp_move<0x111, 0xF>(x);
  x += dpp_move<0x112, 0xF>(x);
  x += dpp_move<0x114, 0xF>(x);
  x += dpp_move<0x118, 0xF>(x);
  x += dpp_move<0x142, 0xA>(x);
  x += dpp_move<0x143, 0xC>(x);
  return x;
}

// Sum over the wavefront, the same in every lane.  Every lane must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  const T incl = wave_inclusive_scan(x);
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  } else {
    const uint64_t u = (uint64_t)incl;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), kWave - 1);
    return (T)(((uint64_t)hi << 32) | lo);
  }
}

// Maximum over the wavefront, the same in every lane (the DPP steps of
// wave_inclusive_scan with max for +; 0, the shifted-in value, is max's
// identity).  Every lane must be active.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
  uint64_t y;
  y = dpp_u64<0x111, 0xF>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x112, 0xF>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x114, 0xF>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x118, 0xF>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x142, 0xA>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x143, 0xC>(x);
  x = y > x ? y : x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, kWave - 1);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), kWave - 1);
  return ((uint64_t)hi << 32) | lo;
}

// Argmax key: larger count first, then lower vertex id.
__device__ __forceinline__ uint64_t argmax_key(uint32_t count, uint32_t v) {
  return ((uint64_t)count << 32) | (uint64_t)(0xFFFFFFFFu - v);
}
__device__ __forceinline__ uint32_t key_vertex(uint64_t key) {
  return 0xFFFFFFFFu - (uint32_t)key;
}
__device__ __forceinline__ uint32_t key_count(uint64_t key) { return (uint32_t)(key >> 32); }

}  // namespace im

// ----------------------------------------------------------------- host side
namespace im {

// Per-thread last error text (im_last_error).
void set_error(hipError_t e, const char* where);
void set_error_text(const std::string& text);

#define IM_HIP(call)                                   \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) {                            \
      ::im::set_error(_e, #call);                      \
      return IM_EDEVICE;                               \
    }                                                  \
  } while (0)

#define IM_TRY(call)                 \
  do {                               \
    int _s = (call);                 \
    if (_s != IM_OK) return _s;      \
  } while (0)

// The caller's workspace for the current entry point (see WsScope).
// scratch: a region of at least `bytes` for `slot`, kept while later requests
// fit it; contents undefined.  IM_ENOMEM when the workspace is exhausted (the
// shortfall is kept for im_workspace_need).  Regions are used on the call's
// stream only.
int scratch(hipStream_t stream, int slot, size_t bytes, void** ptr);
// Same, keeping the first `keep` bytes of the slot's previous region (grown
// in place when it is the topmost, else copied on `stream`).
int scratch_grow(hipStream_t stream, int slot, size_t keep, size_t bytes, void** ptr);
// Returns the slot's region to the workspace (its contents are then dead).
void scratch_release(int slot);
// Bytes of workspace above the highest region carved so far.
size_t scratch_room();
// The largest region one request could get now (a free hole or the room).
size_t scratch_largest();
// Records that the call needs `more` bytes beyond its highest region.
void scratch_need(size_t more);
// Records that `more` bytes beyond the highest region would have let the
// call take a faster launch shape (reported by im_workspace_need).
void scratch_wish(size_t more);
// `bytes` rounded up to the workspace's alignment (256).
size_t ws_align(size_t bytes);

// Entries of the LT search index for E edges (im_lt_index_size).
int64_t lt_index_entries(int64_t E);

// Workspace bytes of the entry points (the op of im_workspace_size);
// sampling, covering subsets and the cover kernels declare theirs beside
// their launches.
size_t ws_forward(int32_t n);
size_t ws_influence(int32_t n, int64_t nsims, int32_t nseeds);
size_t ws_solve(int num_cus, int32_t n, int32_t model, int64_t count, int64_t total, int32_t k,
                int32_t selector, int32_t m, double delta, bool full);
size_t ws_opim(int num_cus, int32_t n, int32_t model, int64_t count, int64_t total, int32_t k,
               int32_t selector, int32_t m, double delta, bool full);
size_t ws_batch(int num_cus, int32_t nt, int64_t S, int64_t V, int64_t total, int32_t max_n,
                int32_t max_k, int32_t model, bool full);

// Installs the caller's workspace (ws, ws_bytes) for an entry point, unless
// an outer entry point of this thread already did (then its workspace
// serves).  check(need): the outermost call's workspace holds `need` bytes
// (else the shortfall is recorded and the call returns IM_ENOMEM before any
// device work).
class WsScope {
 public:
  WsScope(void* ws, size_t bytes);
  ~WsScope();
  WsScope(const WsScope&) = delete;
  WsScope& operator=(const WsScope&) = delete;
  bool nested() const { return nested_; }
  bool check(size_t need) const;

 private:
  bool nested_ = false;
  void* ctx_ = nullptr;
};

// Scratch slots (each caller of a slot owns it for the duration of its call).
enum Slot {
  kSlotSampleArena = 0,
  kSlotSampleMeta,
  kSlotSampleBig,
  kSlotSampleLtLane,
  kSlotScan,
  kSlotIncidence,
  kSlotGreedy,
  kSlotLocal,
  kSlotStream,
  kSlotSolvePool,
  kSlotSolveOff,
  kSlotSolveInc,
  kSlotSolveIncOff,
  kSlotSolveOut,
  kSlotSolveLocal,
  kSlotSampleTasks,
  kSlotBatch,
  kSlotBatchMem,
  kSlotBatchInc,
  kSlotIncPairs,
  kSlotOffline,
  kSlotForward,
  kSlotOpim,
  kSlotOpimIncOff,
  kSlotOpimInc,
  kSlotPoolOff0,
  kSlotPoolMem0,
  kSlotPoolOff1,
  kSlotPoolMem1,
  kSlotCount
};

// Launch-shape knob in effect (im_tune_set; the default when unset).
int64_t tune(im_tune_key key);

struct DeviceInfo {
  int device;
  int num_cus;
};
int device_info(DeviceInfo* out);

// Exclusive scan of n int64/int32 values into int64 outputs (out[n] = total).
int exclusive_scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, hipStream_t s);
int exclusive_scan_u32_to_i64(const uint32_t* in, int64_t n, int64_t* out, hipStream_t s);

}  // namespace im
