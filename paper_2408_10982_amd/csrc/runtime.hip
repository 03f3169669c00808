// runtime.hip -- error text, per-stream scratch, device facts, device-wide scan.
#include <algorithm>
#include <atomic>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <string>

#include "common.h"
#include "cover.h"
#include "incidence.h"
#include "sample.h"

namespace im {

static thread_local std::string g_last_error;

void set_error(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
}

void set_error_text(const std::string& text) { g_last_error = text; }

// ------------------------------------------------------------ workspace
// Every device buffer beyond a call's inputs and outputs is carved from the
// workspace its caller passed (ws, ws_bytes), by a first-fit allocator
// installed for the duration of the outermost entry point on the calling
// thread.  Nested entry points (im_solve calling the selectors, and so on)
// share it.  A slot keeps its region while later requests fit it; a larger
// request, or scratch_release, returns the region to the free list.  Every
// region is used on the call's one stream, so a region freed and carved again
// is reused in stream order.
namespace {
constexpr size_t kAlign = 256;
struct WsCtx {
  char* base = nullptr;
  size_t cap = 0;
  size_t top = 0;                  // end of the highest carved region
  size_t peak = 0;                 // largest `top` of the call
  std::map<size_t, size_t> holes;  // offset -> bytes, free regions below top
  size_t at[kSlotCount] = {};
  size_t bytes[kSlotCount] = {};   // 0: the slot holds no region
};
thread_local WsCtx* t_ws = nullptr;
thread_local size_t t_need = 0;  // the least the last short call needed
thread_local size_t t_want = 0;  // what the last call could have used

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

void give_back(WsCtx* c, size_t at, size_t len) {
  auto it = c->holes.emplace(at, len).first;
  // merge with the following and the preceding hole
  auto nx = std::next(it);
  if (nx != c->holes.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    c->holes.erase(nx);
  }
  if (it != c->holes.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      c->holes.erase(it);
      it = pv;
    }
  }
  if (it->first + it->second == c->top) {  // the top hole lowers the top
    c->top = it->first;
    c->holes.erase(it);
  }
}

int take(WsCtx* c, size_t len, size_t* at) {
  for (auto it = c->holes.begin(); it != c->holes.end(); ++it) {
    if (it->second < len) continue;
    *at = it->first;
    const size_t rest = it->second - len, rat = it->first + len;
    c->holes.erase(it);
    if (rest) c->holes.emplace(rat, rest);
    return IM_OK;
  }
  if (!c->base || c->top + len > c->cap) {
    // what the whole call needs at least: its high-water mark and this
    t_need = std::max(t_need, std::max(c->peak, c->top + len));
    set_error_text("workspace exhausted: " + std::to_string(c->top + len) + " of " +
                   std::to_string(c->cap) + " bytes needed so far (im_workspace_need)");
    return IM_ENOMEM;
  }
  *at = c->top;
  c->top += len;
  c->peak = std::max(c->peak, c->top);
  return IM_OK;
}

WsCtx* current(const char* what) {
  if (!t_ws) set_error_text(std::string("no workspace installed for ") + what);
  return t_ws;
}
}  // namespace

WsScope::WsScope(void* ws, size_t bytes) {
  if (t_ws) {  // a nested entry point: the outer call's workspace
    nested_ = true;
    return;
  }
  WsCtx* c = new (std::nothrow) WsCtx();
  ctx_ = c;
  if (c) {
    // the base is aligned up; what precedes the alignment is unused
    const uintptr_t b0 = (uintptr_t)ws, b1 = (b0 + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
    c->base = ws ? (char*)b1 : nullptr;
    c->cap = ws && bytes > (size_t)(b1 - b0) ? bytes - (size_t)(b1 - b0) : 0;
    t_ws = c;
  }
  t_need = 0;
  t_want = 0;
}

WsScope::~WsScope() {
  if (nested_ || !ctx_) return;
  WsCtx* c = (WsCtx*)ctx_;
  t_want = std::max(std::max(t_want, t_need), c->peak);
  t_ws = nullptr;
  delete c;
}

bool WsScope::check(size_t need) const {
  if (nested_) return true;
  if (!ctx_) {
    set_error_text("workspace bookkeeping could not be allocated on the host");
    return false;
  }
  const WsCtx* c = (const WsCtx*)ctx_;
  if (c->cap >= need) return true;
  t_need = need;
  set_error_text("workspace of " + std::to_string(c->cap) + " bytes; this call needs at least " +
                 std::to_string(need) + " (im_workspace_size)");
  return false;
}

int scratch(hipStream_t, int slot, size_t bytes, void** ptr) {
  WsCtx* c = current("scratch");
  if (!c) return IM_ENOMEM;
  const size_t len = align_up(std::max<size_t>(bytes, 1));
  if (c->bytes[slot] >= len) {
    *ptr = c->base + c->at[slot];
    return IM_OK;
  }
  if (c->bytes[slot]) {  // contents need not survive: give the region back first
    give_back(c, c->at[slot], c->bytes[slot]);
    c->bytes[slot] = 0;
  }
  size_t at = 0;
  IM_TRY(take(c, len, &at));
  c->at[slot] = at;
  c->bytes[slot] = len;
  *ptr = c->base + at;
  return IM_OK;
}

int scratch_grow(hipStream_t s, int slot, size_t keep, size_t bytes, void** ptr) {
  WsCtx* c = current("scratch_grow");
  if (!c) return IM_ENOMEM;
  const size_t len = align_up(std::max<size_t>(bytes, 1));
  if (c->bytes[slot] >= len) {
    *ptr = c->base + c->at[slot];
    return IM_OK;
  }
  const size_t old_at = c->at[slot], old_len = c->bytes[slot];
  if (old_len && old_at + old_len == c->top && old_at + len <= c->cap) {
    // the topmost region grows in place
    c->top = old_at + len;
    c->peak = std::max(c->peak, c->top);
    c->bytes[slot] = len;
    *ptr = c->base + old_at;
    return IM_OK;
  }
  size_t at = 0;
  IM_TRY(take(c, len, &at));
  if (old_len) {
    if (keep)
      IM_HIP(hipMemcpyAsync(c->base + at, c->base + old_at, std::min(keep, old_len),
                            hipMemcpyDeviceToDevice, s));
    give_back(c, old_at, old_len);
  }
  c->at[slot] = at;
  c->bytes[slot] = len;
  *ptr = c->base + at;
  return IM_OK;
}

void scratch_release(int slot) {
  WsCtx* c = t_ws;
  if (!c || !c->bytes[slot]) return;
  give_back(c, c->at[slot], c->bytes[slot]);
  c->bytes[slot] = 0;
}

size_t scratch_room() {
  const WsCtx* c = t_ws;
  if (!c) return 0;
  return c->cap > c->top ? c->cap - c->top : 0;
}

size_t scratch_largest() {
  const WsCtx* c = t_ws;
  if (!c) return 0;
  size_t best = c->cap > c->top ? c->cap - c->top : 0;
  for (const auto& h : c->holes) best = std::max(best, h.second);
  return best;
}

void scratch_need(size_t more) {
  const WsCtx* c = t_ws;
  if (c) t_need = std::max(t_need, std::max(c->peak, c->top + more));
}

void scratch_need_whole(size_t bytes) {
  const WsCtx* c = t_ws;
  if (c && c->cap < bytes) t_need = std::max(t_need, bytes);
}

void scratch_wish(size_t more) {
  const WsCtx* c = t_ws;
  if (c) t_want = std::max(t_want, std::max(c->peak, c->top + more));
}

size_t ws_align(size_t bytes) { return align_up(bytes); }

int device_info(DeviceInfo* out) {
  static std::mutex mu;
  static std::map<int, int> cus;
  int dev = 0;
  IM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = cus.find(dev);
  if (it == cus.end()) {
    int n = 0;
    IM_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    it = cus.emplace(dev, n).first;
  }
  out->device = dev;
  out->num_cus = it->second;
  return IM_OK;
}

// ------------------------------------------------------------ exclusive scan
// Three passes: per-tile sums, a single-block scan of the tile sums, then a
// per-tile scan that adds the tile's base.  Tiles of 1024 threads x 8 items.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t* lds, int64_t* total) {
  // lds: kScanThreads / kWave entries
  const int t = threadIdx.x, l = lane_id(), w = t / kWave;
  int64_t inc = wave_inclusive_scan(x);
  if (l == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    int64_t v = l < kScanThreads / kWave ? lds[l] : 0;
    int64_t vi = wave_inclusive_scan(v);
    if (l < kScanThreads / kWave) lds[l] = vi - v;
    if (l == kWave - 1) lds[kScanThreads / kWave] = vi;
  }
  __syncthreads();
  int64_t r = lds[w] + inc - x;
  *total = lds[kScanThreads / kWave];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(const T* in, int64_t n,
                                                                 int64_t* sums) {
  __shared__ int64_t lds[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
  int64_t tot;
  (void)block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int64_t* sums, int64_t nb) {
  __shared__ int64_t lds[kScanThreads / kWave + 1];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < nb ? sums[i] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(v, lds, &tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const T* in, int64_t n,
                                                             const int64_t* sums, int64_t* out) {
  __shared__ int64_t lds[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // each thread owns kScanItems consecutive entries
  const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = my + j;
    v[j] = i < n ? (int64_t)in[i] : 0;
    s += v[j];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(s, lds, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = my + j;
    if (i < n) out[i] = ex;
    ex += v[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = sums[gridDim.x];
}

template <typename T>
static int exclusive_scan_impl(const T* in, int64_t n, int64_t* out, hipStream_t s) {
  if (n <= 0) {
    IM_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    return IM_OK;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotScan, (size_t)(nb + 1) * sizeof(int64_t), &p));
  int64_t* sums = (int64_t*)p;
  k_scan_tile_sums<T><<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(in, n, sums);
  k_scan_sums<<<1, kScanThreads, 0, s>>>(sums, nb);
  k_scan_apply<T><<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(in, n, sums, out);
  IM_HIP(hipGetLastError());
  return IM_OK;
}

int exclusive_scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, hipStream_t s) {
  return exclusive_scan_impl<int32_t>(in, n, out, s);
}
int exclusive_scan_u32_to_i64(const uint32_t* in, int64_t n, int64_t* out, hipStream_t s) {
  return exclusive_scan_impl<uint32_t>(in, n, out, s);
}

namespace {
constexpr int kTuneKeys = 8;
constexpr int64_t kTuneDefault[kTuneKeys] = {5, 0, 1, 256, 2, 16, 0, 1};
constexpr int64_t kTuneMin[kTuneKeys] = {1, 0, 1, 0, 1, 1, 0, 0};
constexpr int64_t kTuneMax[kTuneKeys] = {64, 2, 16, (int64_t)1 << 40, 32, 4096, 1, 1};
std::atomic<int64_t> g_tune[kTuneKeys] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
}  // namespace

int64_t tune(im_tune_key key) {
  const int64_t v = g_tune[key].load(std::memory_order_relaxed);
  return v < 0 ? kTuneDefault[key] : v;
}

}  // namespace im

extern "C" {

int im_tune_set(int32_t key, int64_t value) {
  if (key < 0 || key >= im::kTuneKeys) return IM_EINVAL;
  if (value != -1 && (value < im::kTuneMin[key] || value > im::kTuneMax[key])) return IM_EINVAL;
  im::g_tune[key].store(value, std::memory_order_relaxed);
  return IM_OK;
}

int im_tune_get(int32_t key, int64_t* value) {
  if (key < 0 || key >= im::kTuneKeys || !value) return IM_EINVAL;
  *value = im::tune((im_tune_key)key);
  return IM_OK;
}

const char* im_version(void) { return "im-mi355x 0.1 (gfx950)"; }

const char* im_last_error(void) { return im::g_last_error.c_str(); }

int im_workspace_size(int32_t op, const im_ws_shape* sh, size_t* bytes) {
  using namespace im;
  if (!sh || !bytes || sh->n < 0 || sh->count < 0 || sh->total < 0 || sh->k < 0 || sh->m < 0 ||
      sh->ntasks < 0 || sh->num_cus < 0)
    return IM_EINVAL;
  int cus = sh->num_cus;
  if (cus == 0 && (op == IM_WS_SAMPLE || op == IM_WS_SOLVE || op == IM_WS_OPIM ||
                   op == IM_WS_BATCH)) {
    DeviceInfo di;
    IM_TRY(device_info(&di));
    cus = di.num_cus;
  }
  const bool full = sh->full != 0;
  const int32_t m = std::max(sh->m, 1), k = std::max(sh->k, 1);
  const bool stream_op = (op == IM_WS_STREAM) ||
                         ((op == IM_WS_SOLVE || op == IM_WS_OPIM) && sh->selector == IM_SEL_GREEDIRIS);
  if (stream_op && !(sh->delta > 0.0 && sh->delta < 0.5)) return IM_EINVAL;
  size_t b = 0;
  switch (op) {
    case IM_WS_PREPARE_GRAPH: b = ws_align(64); break;
    case IM_WS_SAMPLE: b = ws_sample(cus, sh->count, sh->total, sh->n, sh->model, full); break;
    case IM_WS_INCIDENCE: b = ws_incidence(sh->n, sh->total, 0, full); break;
    case IM_WS_GREEDY: b = ws_greedy(sh->n, sh->count, k); break;
    case IM_WS_RANDGREEDI: b = ws_randgreedi(sh->n, sh->count, sh->total, k, m); break;
    case IM_WS_STREAM: b = ws_stream(sh->n, sh->count, k, m, sh->delta); break;
    case IM_WS_OFFLINE: b = ws_offline(sh->n, sh->count, k, m); break;
    case IM_WS_FORWARD: b = ws_forward(sh->n); break;
    case IM_WS_INFLUENCE: b = ws_influence(sh->n, sh->count, sh->k); break;
    case IM_WS_SOLVE:
      b = ws_solve(cus, sh->n, sh->model, sh->count, sh->total, k, sh->selector, m, sh->delta, full);
      break;
    case IM_WS_OPIM:
      b = ws_opim(cus, sh->n, sh->model, sh->count, sh->total, k, sh->selector, m, sh->delta, full);
      break;
    case IM_WS_BATCH:
      b = ws_batch(cus, std::min(std::max(sh->ntasks, 1), kMaxParts), sh->count, sh->n, sh->total,
                   sh->n, k, sh->model, full);
      break;
    default: return IM_EINVAL;
  }
  *bytes = b;
  return IM_OK;
}

int im_workspace_need(size_t* need, size_t* want) {
  if (!need && !want) return IM_EINVAL;
  if (need) *need = im::t_need;
  if (want) *want = im::t_want;
  return IM_OK;
}

int im_release(void) {
  IM_HIP(hipDeviceSynchronize());
  im::release_cover_graphs();
  return IM_OK;
}

}  // extern "C"
