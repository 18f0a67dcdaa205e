// fss_kernels.hpp -- launch wrappers between the C ABI (fss_api.cpp) and the
// HIP kernels (fss_kernels.hip).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fss_common.hpp"

namespace fss {

constexpr int kNumAesVariants = 5;  // 0-3: T-table layouts in LDS, 4: bitsliced PRG

struct RoundKeys { uint32_t w[44]; };

// Keygen arguments passed by value: round keys of the dealer-seed AES key
// and the per-atom thresholds in view space (public, spec-derived).
struct KgArgs {
  RoundKeys rk;
  uint64_t bprime[kMaxAtoms];
  int64_t n_elems;
  uint64_t n_tiles;
  int32_t jobs;  // waves per tile: 1 (one wave does all) or 2 (masks + call 1 | call 2)
};

// One work-list entry as the persistent kernel sees it.
struct DevItem {
  const uint8_t* keys;
  const uint64_t* xhat;
  uint64_t* y;
  uint64_t* z;
  int64_t n_elems;
  int32_t party;
  int32_t words;  // ceil(n_elems / 64): stride of the z bit-planes
};

// One unit of the fused kernel's work-list, kUnitWords u32: item, tile,
// lookup-point range (i0 | i1 << 16) and flags.  A tile has a call-1 unit and
// call 2 either whole (y stored) or in parts whose shares of y are added.
constexpr int kUnitWords = 4;
constexpr uint32_t kUnitPred = 1u;        // call 1 (the predicate bits)
constexpr uint32_t kUnitBase = 2u;        // the walk at v, tab_0 rho and r_out terms of call 2
constexpr uint32_t kUnitAccumulate = 4u;  // add the part's y to memory zeroed before the launch
// A call-2 unit over 64 / G elements of a tile (G = lane groups of the launch,
// 2 or 4): lane l takes element slot s0 + l mod (64 / G) and, with the other
// lanes of its group l / (64 / G), an even share of the unit's lookup points
// (group 0 also takes the base); the groups' shares of y are summed across
// lanes.  Flags bits 16..21: s0.
constexpr uint32_t kUnitLanes = 8u;
constexpr int kMaxLaneGroupsLog2 = 2;
// Table layouts with lane-group kernels (the others would only add build time).
constexpr bool lanes_variant(int v) { return v == 1 || v == 2; }

// Launchers of one AES table layout V (0 .. kNumAesVariants-1).
template <int V>
struct VariantOps {
  static int block();
  static int lds_bytes();
  // `cus`: compute units of the device; batches with fewer tiles than a full
  // grid get smaller blocks so their tiles spread over the CUs.
  static hipError_t keygen(const KeyHeader* h, int p, int r, const KgArgs& ga, uint8_t* k0, uint8_t* k1, uint64_t* ri,
                           uint64_t* ro, int cus, hipStream_t st);
  static hipError_t pred(int party, const uint8_t* keys, const uint64_t* xhat, int64_t n, uint64_t* z,
                         int* status, int cus, hipStream_t st);
  static hipError_t coeff(int party, const uint8_t* keys, const uint64_t* xhat, int64_t n, uint64_t* y,
                          int* status, int cus, hipStream_t st);
  // lanes_log2: log2 of the lane groups of the launch's kUnitLanes units (0: none)
  static hipError_t fused(const DevItem* items, const uint32_t* units, uint32_t n_units, uint32_t* counter,
                          int* status, int grid, int lanes_log2, hipStream_t st);
  // the rescaling gate (ARS of a masked value)
  static hipError_t rescale_keygen(const KeyHeader* h, int r, const KgArgs& ga, const uint64_t* r_in, uint8_t* k0,
                                   uint8_t* k1, uint64_t* r_out, int cus, hipStream_t st);
  static hipError_t rescale_eval(int party, const uint8_t* keys, const uint64_t* yhat, int64_t n, uint64_t* z,
                                 int* status, int cus, hipStream_t st);
};
extern template struct VariantOps<0>;
extern template struct VariantOps<1>;
extern template struct VariantOps<2>;
extern template struct VariantOps<3>;
extern template struct VariantOps<4>;

hipError_t launch_header_init(uint8_t* dst, const uint8_t* src, int64_t n_elems, uint64_t n_tiles,
                              uint32_t party, hipStream_t st);
hipError_t launch_keygen(int variant, int p, int r, const KeyHeader* dev_hdr, const KgArgs& ga, uint8_t* key0,
                         uint8_t* key1, uint64_t* r_in, uint64_t* r_out, int cus, hipStream_t st);
hipError_t launch_mask(const int64_t* x, const uint64_t* r_in, int64_t n, uint64_t* xhat,
                       hipStream_t st);
hipError_t launch_eval_pred(int variant, int party, const uint8_t* keys, const uint64_t* xhat,
                            int64_t n, uint64_t* z, int* status, int cus, hipStream_t st);
hipError_t launch_eval_coeff(int variant, int party, const uint8_t* keys, const uint64_t* xhat,
                             int64_t n, uint64_t* y, int* status, int cus, hipStream_t st);
// Resets the work counter and zeroes y of the split items with kernels
// (graph-safe), then launches the persistent kernel with `grid` blocks of the
// variant's block size over `n_units` work-list units.
hipError_t launch_fused(int variant, const DevItem* items, const uint32_t* units, uint32_t n_units,
                        uint32_t* counter, int* status, int grid, int lanes_log2, const uint32_t* split_items,
                        uint32_t n_split, uint64_t max_split_elems, hipStream_t st);
hipError_t launch_rescale_keygen(int variant, int r, const KeyHeader* dev_hdr, const KgArgs& ga, const uint64_t* r_in,
                                 uint8_t* key0, uint8_t* key1, uint64_t* r_out, int cus, hipStream_t st);
hipError_t launch_rescale_eval(int variant, int party, const uint8_t* keys, const uint64_t* yhat, int64_t n,
                               uint64_t* z, int* status, int cus, hipStream_t st);
// yhat = y0 + y1 (the opening of two additive shares, both on this device).
hipError_t launch_open(const uint64_t* y0, const uint64_t* y1, int64_t n, uint64_t* yhat, hipStream_t st);
// The literal interval lookup (table layout 1) and the post-processing
// subprotocols (fss_phi.hip).
hipError_t launch_lit_keygen(int p, int r, const KeyHeader* dev_hdr, const KgArgs& ga, uint8_t* key0, uint8_t* key1,
                             uint64_t* r_in, uint64_t* r_out, hipStream_t st);
hipError_t launch_lit_eval(int party, const uint8_t* keys, const uint64_t* xhat, int64_t n, uint64_t* coef,
                           uint64_t* x_share, int* status, hipStream_t st);
// kind 0: Beaver triples, 1: AND triples, 2: B2A bits (a0 / a1: XOR-share
// words, c0 / c1: additive shares)
hipError_t launch_correlations(const RoundKeys& rk, int kind, int64_t n, uint32_t step, uint64_t* a0, uint64_t* b0,
                               uint64_t* c0, uint64_t* a1, uint64_t* b1, uint64_t* c1, hipStream_t st);
// a party's local step of a subprotocol (see k_phi)
hipError_t launch_phi(int kind, int party, const uint64_t* u, const uint64_t* v, const uint64_t* a,
                      const uint64_t* b, const uint64_t* c, const uint64_t* add, int64_t n, uint64_t* d,
                      uint64_t* e, uint64_t* z, hipStream_t st);
int variant_block(int variant);
int variant_lds_bytes(int variant);

}  // namespace fss
