// Stand-ins for the library's kernel launchers, so that its host code
// (fss_api.cpp) links into a CPU-only sanitizer build without device code.
// The host driver never reaches them: every one reports that it cannot run.
#include "fss_kernels.hpp"
#include "fss_plan.hpp"

namespace fss {

hipError_t launch_header_init(uint8_t*, const uint8_t*, int64_t, uint64_t, uint32_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_keygen(int, int, int, const KeyHeader*, const KgArgs&, uint8_t*, uint8_t*, uint64_t*, uint64_t*,
                         int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_mask(const int64_t*, const uint64_t*, int64_t, uint64_t*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_eval_pred(int, int, const uint8_t*, const uint64_t*, int64_t, uint64_t*, int*, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_eval_coeff(int, int, const uint8_t*, const uint64_t*, int64_t, uint64_t*, int*, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_fused(int, const DevItem*, const uint32_t*, uint32_t, uint32_t*, int*, int, int, const uint32_t*,
                        uint32_t, uint64_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_rescale_keygen(int, int, const KeyHeader*, const KgArgs&, const uint64_t*, uint8_t*, uint8_t*,
                                 uint64_t*, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_rescale_eval(int, int, const uint8_t*, const uint64_t*, int64_t, uint64_t*, int*, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_open(const uint64_t*, const uint64_t*, int64_t, uint64_t*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_lit_keygen(int, int, const KeyHeader*, const KgArgs&, uint8_t*, uint8_t*, uint64_t*, uint64_t*,
                             hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_lit_eval(int, const uint8_t*, const uint64_t*, int64_t, uint64_t*, uint64_t*, int*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_correlations(const RoundKeys&, int, int64_t, uint32_t, uint64_t*, uint64_t*, uint64_t*, uint64_t*,
                               uint64_t*, uint64_t*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_phi(int, int, const uint64_t*, const uint64_t*, const uint64_t*, const uint64_t*, const uint64_t*,
                      const uint64_t*, int64_t, uint64_t*, uint64_t*, uint64_t*, hipStream_t) {
  return hipErrorNotSupported;
}
int variant_block(int) { return 768; }
int variant_lds_bytes(int) { return 0; }
int* noalloc_status_word() { return nullptr; }

}  // namespace fss
