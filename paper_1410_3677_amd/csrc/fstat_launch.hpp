// Host-side check of a kernel launch's configuration against the device's limits and the
// kernel's compiled ones, made before every dispatch so that a configuration the queue
// would reject (a malformed dispatch packet aborts the whole queue) is refused with an
// error naming the kernel and the limit instead.  Plain host C++ (no HIP types), so that
// the rules are testable on a machine without a GPU.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>

namespace fstat {

struct DeviceLaunchLimits {
  int64_t max_threads_per_block = 1024;
  int64_t max_block[3] = {1024, 1024, 1024};
  int64_t max_grid[3] = {2147483647, 65536, 65536};   // workgroups per dimension
  int64_t max_lds_per_block = 65536;                   // bytes of LDS one workgroup may hold
};

struct KernelLaunchLimits {
  int64_t max_threads_per_block = 1024;   // the kernel's compiled maximum workgroup size
  int64_t static_lds = 0;                 // bytes of LDS the kernel declares
};

// A dispatch packet holds the grid as work-items per dimension in 32 bits.
constexpr int64_t MAX_WORK_ITEMS_PER_DIM = 0xFFFFFFFFLL;

// Why a launch of `grid` workgroups of `block` work-items with `dyn_lds` bytes of dynamic
// LDS would be rejected, or "" when it is within every limit.
inline std::string launch_problem(const DeviceLaunchLimits& d, const KernelLaunchLimits& k, const int64_t grid[3],
                                  const int64_t block[3], int64_t dyn_lds) {
  static const char axis[3] = {'x', 'y', 'z'};
  char msg[200];
  for (int i = 0; i < 3; ++i) {
    if (grid[i] < 1) {
      std::snprintf(msg, sizeof msg, "grid %c dimension %lld (must be >= 1)", axis[i], (long long)grid[i]);
      return msg;
    }
    if (block[i] < 1) {
      std::snprintf(msg, sizeof msg, "workgroup %c dimension %lld (must be >= 1)", axis[i], (long long)block[i]);
      return msg;
    }
  }
  for (int i = 0; i < 3; ++i) {
    if (block[i] > d.max_block[i]) {
      std::snprintf(msg, sizeof msg, "workgroup %c dimension %lld above the device's %lld", axis[i],
                    (long long)block[i], (long long)d.max_block[i]);
      return msg;
    }
  }
  const int64_t threads = block[0] * block[1] * block[2];
  if (threads > d.max_threads_per_block) {
    std::snprintf(msg, sizeof msg, "%lld work-items per workgroup above the device's %lld", (long long)threads,
                  (long long)d.max_threads_per_block);
    return msg;
  }
  if (threads > k.max_threads_per_block) {
    std::snprintf(msg, sizeof msg, "%lld work-items per workgroup above the kernel's compiled maximum %lld",
                  (long long)threads, (long long)k.max_threads_per_block);
    return msg;
  }
  for (int i = 0; i < 3; ++i) {
    if (grid[i] > d.max_grid[i]) {
      std::snprintf(msg, sizeof msg, "grid %c dimension %lld above the device's %lld workgroups", axis[i],
                    (long long)grid[i], (long long)d.max_grid[i]);
      return msg;
    }
    if (grid[i] > MAX_WORK_ITEMS_PER_DIM / block[i]) {
      std::snprintf(msg, sizeof msg, "grid %c dimension of %lld x %lld work-items exceeds 2^32 - 1", axis[i],
                    (long long)grid[i], (long long)block[i]);
      return msg;
    }
  }
  if (dyn_lds < 0 || k.static_lds + dyn_lds > d.max_lds_per_block) {
    std::snprintf(msg, sizeof msg, "%lld bytes of LDS (%lld static + %lld dynamic) above the %lld a workgroup may hold",
                  (long long)(k.static_lds + dyn_lds), (long long)k.static_lds, (long long)dyn_lds,
                  (long long)d.max_lds_per_block);
    return msg;
  }
  return std::string();
}

}  // namespace fstat
