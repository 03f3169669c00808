// runtime.hip -- error text, per-stream scratch, device facts, device-wide scan.
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.h"
#include "cover.h"

namespace im {

static thread_local std::string g_last_error;

void set_error(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
}

void set_error_text(const std::string& text) { g_last_error = text; }

namespace {
struct ScratchBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_mu;
std::map<std::tuple<int, uintptr_t, int>, ScratchBuf> g_scratch;
}  // namespace

int scratch(hipStream_t stream, int slot, size_t bytes, void** ptr) {
  bool fresh = false;
  return scratch_fresh(stream, slot, bytes, ptr, &fresh);
}

int scratch_fresh(hipStream_t stream, int slot, size_t bytes, void** ptr, bool* fresh) {
  *fresh = false;
  int dev = 0;
  IM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  ScratchBuf& b = g_scratch[std::make_tuple(dev, (uintptr_t)stream, slot)];
  if (bytes == 0) bytes = 256;
  if (b.bytes < bytes) {
    if (b.ptr) {
      IM_HIP(hipStreamSynchronize(stream));
      IM_HIP(hipFree(b.ptr));
      b.ptr = nullptr;
      b.bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 4095) & ~(size_t)4095;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      e = hipMalloc(&p, bytes);
      want = bytes;
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error_text("hipMalloc(scratch) of " + std::to_string(bytes) + " bytes: " +
                       hipGetErrorString(e));
        return IM_ENOMEM;
      }
    }
    b.ptr = p;
    b.bytes = want;
    *fresh = true;
  }
  *ptr = b.ptr;
  return IM_OK;
}

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
constexpr int kTuneKeys = 7;
constexpr int64_t kTuneDefault[kTuneKeys] = {5, 0, 1, 256, 7, 16, 0};
constexpr int64_t kTuneMin[kTuneKeys] = {1, 0, 1, 0, 1, 1, 0};
constexpr int64_t kTuneMax[kTuneKeys] = {64, 2, 16, (int64_t)1 << 40, 32, 4096, 1};
std::atomic<int64_t> g_tune[kTuneKeys] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
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

int im_scratch_bytes(void* stream, size_t* bytes) {
  if (!bytes) return IM_EINVAL;
  int dev = 0;
  IM_HIP(hipGetDevice(&dev));
  size_t b = 0;
  std::lock_guard<std::mutex> lk(im::g_mu);
  for (const auto& kv : im::g_scratch)
    if (std::get<0>(kv.first) == dev && std::get<1>(kv.first) == (uintptr_t)stream)
      b += kv.second.bytes;
  *bytes = b;
  return IM_OK;
}

int im_release(void) {
  int dev = 0;
  IM_HIP(hipGetDevice(&dev));
  IM_HIP(hipDeviceSynchronize());
  im::release_cover_graphs();
  std::lock_guard<std::mutex> lk(im::g_mu);
  for (auto it = im::g_scratch.begin(); it != im::g_scratch.end();) {
    if (std::get<0>(it->first) == dev) {
      if (it->second.ptr) IM_HIP(hipFree(it->second.ptr));
      it = im::g_scratch.erase(it);
    } else {
      ++it;
    }
  }
  return IM_OK;
}

}  // extern "C"
