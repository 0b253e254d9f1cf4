// Grouped launches: one launch covers a phase of many independent tasks (factors or
// layers).  Task t owns the flat block range [off[t], off[t+1]) laid out as a gx[t]-wide
// 2-D grid; the wrapper maps blockIdx.x to (task, bx, by) and runs the same body as the
// single-task kernel.  Tables live in device memory (the caller's workspace).
#pragma once
#include <hip/hip_runtime.h>

namespace kfac {

struct GroupMap {
  const int* off;   // ntasks + 1 prefix offsets
  const int* gx;    // ntasks grid widths
  int ntasks;
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  This
// bijection on [0, n) gives every XCD a contiguous range of logical block indices, so
// neighbouring tiles that share an operand panel run under the same L2.
__device__ __forceinline__ int xcd_swizzle(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, slot = b >> 3;
  return x * q + (x < r ? x : r) + slot;
}

__device__ __forceinline__ void group_locate_at(const GroupMap& g, int b, int& t, int& bx, int& by) {
  int lo = 0, hi = g.ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  // every lane computed the same values: make them scalar, so the task record is read
  // with scalar loads and kept in SGPRs
  t = __builtin_amdgcn_readfirstlane(lo);
  const int local = __builtin_amdgcn_readfirstlane(b - g.off[t]);
  const int w = __builtin_amdgcn_readfirstlane(g.gx[t]);
  bx = local % w;
  by = local / w;
}

__device__ __forceinline__ void group_locate(const GroupMap& g, int& t, int& bx, int& by) {
  group_locate_at(g, blockIdx.x, t, bx, by);
}

__device__ __forceinline__ void group_locate_xcd(const GroupMap& g, int& t, int& bx, int& by) {
  group_locate_at(g, xcd_swizzle(blockIdx.x, gridDim.x), t, bx, by);
}

// Work-balanced XCD mapping for launches whose task block counts are multiples of 8:
// every XCD takes one contiguous eighth of every task, so each XCD gets the same share
// of each task's work while neighbouring blocks of a task still share its L2.  Block b
// is the (b / 8)-th workgroup dispatched to XCD b % 8.
__device__ __forceinline__ void group_locate_xcd8(const GroupMap& g, int& t, int& bx, int& by) {
  const int x = blockIdx.x & 7, s = blockIdx.x >> 3;
  int lo = 0, hi = g.ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.off[mid] <= 8 * s) lo = mid; else hi = mid - 1;
  }
  t = __builtin_amdgcn_readfirstlane(lo);
  const int o = __builtin_amdgcn_readfirstlane(g.off[t]);
  const int per = __builtin_amdgcn_readfirstlane((g.off[t + 1] - o) >> 3);
  const int local = x * per + (s - (o >> 3));
  const int w = __builtin_amdgcn_readfirstlane(g.gx[t]);
  bx = local % w;
  by = local / w;
}

#define KFAC_GROUPED_KERNEL(NAME, BODY, PARAMS, NT)                                   \
  __global__ __launch_bounds__(NT) void NAME(const PARAMS* tasks, GroupMap gm) {        \
    int t_, bx_, by_;                                                                   \
    group_locate(gm, t_, bx_, by_);                                                     \
    BODY(tasks[t_], bx_, by_);                                                          \
  }

#define KFAC_GROUPED_KERNEL_XCD(NAME, BODY, PARAMS, NT)                               \
  __global__ __launch_bounds__(NT) void NAME(const PARAMS* tasks, GroupMap gm) {        \
    int t_, bx_, by_;                                                                   \
    group_locate_xcd(gm, t_, bx_, by_);                                                 \
    BODY(tasks[t_], bx_, by_);                                                          \
  }

}  // namespace kfac
