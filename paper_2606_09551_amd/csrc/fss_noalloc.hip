// fss_noalloc.hip -- work-list evaluation for callers that cannot allocate
// device memory (fss_eval_batch_noalloc in include/fusefss.h).
//
// The persistent kernel's work-list (items, units, the work counter, the list
// of items whose tiles run in parts) and a status word live in one file-scope
// device array of fixed size instead of buffers from the library's pool.
// Each device holds its own copy of the array.  Its address on a device is
// looked up once, with that device current, and only that address is handed
// to HIP calls and kernels (in host code the array's name is not a device
// address).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/fusefss.h"
#include "fss_kernels.hpp"
#include "fss_plan.hpp"

namespace fss {
namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;
// Layout: the work counter at 0, the status word at 64, then the items, the
// split-item list and the units.
constexpr size_t kOffCounter = 0, kOffStatus = 64, kOffItems = 256;
constexpr size_t kMaxItems = FSS_NOALLOC_MAX_ITEMS;
constexpr size_t kOffSplit = kOffItems + kMaxItems * sizeof(DevItem);
constexpr size_t kOffUnits = (kOffSplit + kMaxItems * sizeof(uint32_t) + 255) & ~(size_t)255;
constexpr size_t kUnitBytes = kUnitWords * sizeof(uint32_t);
static_assert(kOffUnits + (size_t)FSS_NOALLOC_MAX_UNITS * kUnitBytes <= kScratchBytes,
              "the documented unit limit does not fit the scratch array");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, uint8_t*> g_ptr;  // device -> address of `scratch` on that device

// The array's address on the current device, looked up on the first call there.
int scratch_ptr(uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_hip_error(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(dev);
  if (it == g_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return set_hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(FSS_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    it = g_ptr.emplace(dev, (uint8_t*)p).first;
  }
  *out = it->second;
  return FSS_OK;
}

}  // namespace

int* noalloc_status_word() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(dev);
  return it == g_ptr.end() ? nullptr : (int*)(it->second + kOffStatus);
}

}  // namespace fss

extern "C" int fss_eval_batch_noalloc(int32_t party, const fss_work_item* items, int32_t n_items, void* stream) {
  using namespace fss;
  hipStream_t st = (hipStream_t)stream;
  if (party != FSS_PARTY_ANY && party != 0 && party != 1)
    return set_error(FSS_E_PARTY, "party must be 0, 1 or FSS_PARTY_ANY (got %d)", party);
  if (n_items < 0 || (n_items > 0 && !items)) return set_error(FSS_E_ARG, "bad items");
  if (n_items > FSS_NOALLOC_MAX_ITEMS)
    return set_error(FSS_E_ARG, "%d items exceed the no-alloc limit of %d", n_items, FSS_NOALLOC_MAX_ITEMS);
  for (int i = 0; i < n_items; ++i)
    if (party != FSS_PARTY_ANY && items[i].party != party)
      return set_error(FSS_E_PARTY, "item %d is party %d's, the batch party %d's", i, items[i].party, party);
  uint8_t* base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  if (n_items == 0) return FSS_OK;
  // Key headers are read on the caller's stream once the work already
  // enqueued there (the keygen that wrote them) has finished.
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_hip_error(e, "hipStreamSynchronize(eval_batch_noalloc)");
  HostPlan hp;
  if ((rc = build_host_plan(items, n_items, nullptr, &st, &hp))) return rc;
  const size_t n_units = hp.units.size() / kUnitWords;
  if (n_units > (size_t)FSS_NOALLOC_MAX_UNITS)
    return set_error(FSS_E_ARG, "%zu work-list units exceed the no-alloc limit of %d", n_units,
                     FSS_NOALLOC_MAX_UNITS);
  if (n_units == 0) return FSS_OK;
  DevItem* d_items = (DevItem*)(base + kOffItems);
  uint32_t* d_split = (uint32_t*)(base + kOffSplit);
  uint32_t* d_units = (uint32_t*)(base + kOffUnits);
  uint32_t* d_counter = (uint32_t*)(base + kOffCounter);
  int* d_status = (int*)(base + kOffStatus);
  e = hipMemcpyAsync(d_items, hp.items.data(), sizeof(DevItem) * hp.items.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !hp.split.empty())
    e = hipMemcpyAsync(d_split, hp.split.data(), sizeof(uint32_t) * hp.split.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_units, hp.units.data(), sizeof(uint32_t) * hp.units.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return set_hip_error(e, "upload work-list (no-alloc)");
  // the host copies of the work-list go out of scope when this call returns
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_hip_error(e, "hipStreamSynchronize(upload, no-alloc)");
  // launch_fused resets the work counter and zeroes the split items' y with
  // kernels before the persistent launch
  e = launch_fused(hp.tune.aes_variant, d_items, d_units, (uint32_t)n_units, d_counter, d_status, hp.grid,
                   lanes_log2(hp.tune.lanes), d_split,
                   (uint32_t)hp.split.size(), hp.max_split_elems, st);
  if (e != hipSuccess) return set_hip_error(e, "fused launch (no-alloc)");
  return FSS_OK;
}
