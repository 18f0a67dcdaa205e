// fss_plan.hpp -- the host side of a work-list plan, shared by the pooled plan
// (fss_plan_create) and the evaluation that allocates nothing
// (fss_eval_batch_noalloc).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/fusefss.h"
#include "fss_kernels.hpp"

namespace fss {

// A planned work-list in host memory, ready to upload.
struct HostPlan {
  std::vector<DevItem> items;
  std::vector<uint32_t> units;  // kUnitWords u32 per unit
  std::vector<uint32_t> split;  // items whose tiles run in parts (y zeroed before the launch)
  uint64_t max_split_elems = 0;
  int parts = 1;                // parts per tile chosen for call 2
  bool merged_pred = true;      // call 1 runs in call 2's first unit of a tile
  fss_tune tune{};              // resolved launch configuration
  int grid = 0;                 // persistent blocks
  double aes = 0, lookups = 0;  // algorithmic work of one launch
};

// Reads each item's key header to the host (on `*header_stream`, which may
// be the null stream, or on the library's own stream when `header_stream` is
// null), validates the items and plans the units.  Allocates host memory only.
int build_host_plan(const fss_work_item* items, int32_t n_items, const fss_tune* tune,
                    const hipStream_t* header_stream, HostPlan* out);

// log2 of a resolved tune's lane groups (1, 2 or 4 lanes per element).
inline int lanes_log2(int lanes) { return lanes >= 4 ? 2 : lanes == 2 ? 1 : 0; }

// Record the thread-local error message of the C ABI and return `code`.
int set_error(int code, const char* fmt, ...);
int set_hip_error(hipError_t e, const char* what);

// Address of the no-alloc path's status word on the current device, or null
// when that path has not run on it.
int* noalloc_status_word();

}  // namespace fss
