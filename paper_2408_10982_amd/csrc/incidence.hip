// incidence.hip -- covering subsets S(v) = {j : v in R(j)} (im_build_incidence).
//
// Sec. 3.2 / Alg. 3 per-vertex step: the transpose of the sample-major RRR
// collection.  A degree histogram (global atomics), an exclusive scan for the
// vertex-major offsets, then a scatter in which every thread walks a short
// contiguous run of members, knowing the sample that owns each member.
#include <algorithm>

#include "common.h"

namespace im {

constexpr int kIncBlock = 256;
constexpr int kRun = 16;  // members per thread in the scatter

__global__ __launch_bounds__(kIncBlock) void k_degree(const int32_t* __restrict__ mem,
                                                      int64_t total, uint32_t* __restrict__ deg) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&deg[mem[t]], 1u);
}

__global__ __launch_bounds__(kIncBlock) void k_scatter(int64_t count,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ mem,
                                                       int64_t total,
                                                       const int64_t* __restrict__ inc_off,
                                                       uint32_t* __restrict__ fill,
                                                       int32_t* __restrict__ inc_mem) {
  const int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRun;
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
  const int64_t t1 = min(t0 + kRun, total);
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

}  // namespace im

extern "C" int im_build_incidence(int32_t n, int64_t count, const int64_t* off,
                                  const int32_t* mem, int64_t total, int64_t* inc_off,
                                  int32_t* inc_mem, void* stream) {
  using namespace im;
  if (n <= 0 || count < 0 || total < 0 || !off || !inc_off || (total > 0 && (!mem || !inc_mem)) ||
      count >= ((int64_t)1 << 31))
    return IM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  void* p = nullptr;
  IM_TRY(scratch(s, kSlotIncidence, (size_t)n * 8, &p));
  uint32_t* deg = (uint32_t*)p;
  uint32_t* fill = deg + n;
  IM_HIP(hipMemsetAsync(deg, 0, (size_t)n * 8, s));
  DeviceInfo di;
  IM_TRY(device_info(&di));
  if (total > 0) {
    int64_t blocks = std::min<int64_t>((total + kIncBlock - 1) / kIncBlock, (int64_t)di.num_cus * 16);
    k_degree<<<dim3((unsigned)blocks), dim3(kIncBlock), 0, s>>>(mem, total, deg);
    IM_HIP(hipGetLastError());
  }
  IM_TRY(exclusive_scan_u32_to_i64(deg, n, inc_off, s));
  if (total > 0 && count > 0) {
    const int64_t threads = (total + kRun - 1) / kRun;
    const int64_t blocks = (threads + kIncBlock - 1) / kIncBlock;
    k_scatter<<<dim3((unsigned)blocks), dim3(kIncBlock), 0, s>>>(count, off, mem, total, inc_off,
                                                                 fill, inc_mem);
    IM_HIP(hipGetLastError());
  }
  return IM_OK;
}
