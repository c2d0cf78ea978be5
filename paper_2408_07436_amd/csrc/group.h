// Device side of the grouped launches (kernels.h): workgroup b of a grouped
// launch belongs to job j with pre[j] <= b < pre[j + 1]; this finds j by
// binary search (the prefix sums are uniform across the workgroup, so the
// loads are scalar) and the job-local workgroup index.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kifmm {

__device__ inline int group_job(const int64_t* __restrict__ pre, int nj, int64_t& local) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nj;  // pre[lo] <= b < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  local = b - pre[lo];
  return lo;
}

}  // namespace kifmm
