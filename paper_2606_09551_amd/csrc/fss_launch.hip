// fss_launch.hip -- layout-independent kernels and the dispatch from an AES
// table-layout index to its launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fss_kernels.hpp"

namespace fss {

// Copy the cached per-spec header into a key buffer, stamping size and party;
// the rest of the header region is zeroed so key bytes are fully determined.
__global__ void k_header_init(uint8_t* dst, const uint8_t* src, int64_t n_elems, uint64_t n_tiles,
                              uint32_t party) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (uint32_t i = threadIdx.x; i < kHeaderBytes / 4; i += blockDim.x)
    d[i] = i < sizeof(KeyHeader) / 4 ? s[i] : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    KeyHeader* h = reinterpret_cast<KeyHeader*>(dst);
    h->party = party;
    h->n_elems = (uint64_t)n_elems;
    h->n_tiles = n_tiles;
  }
}

// Masked opening collapsed to one process: xhat = x + r_in mod 2^64.
__global__ void k_mask(const int64_t* x, const uint64_t* r_in, int64_t n, uint64_t* xhat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) xhat[i] = (uint64_t)x[i] + r_in[i];
}

// The opening of two additive shares held on one device: yhat = y0 + y1.
__global__ void k_open(const uint64_t* y0, const uint64_t* y1, int64_t n, uint64_t* yhat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) yhat[i] = y0[i] + y1[i];
}

// Work counters are cleared by a kernel rather than a memset node so a
// captured graph replays correctly.
__global__ void k_reset_counter(uint32_t* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

hipError_t launch_header_init(uint8_t* dst, const uint8_t* src, int64_t n_elems, uint64_t n_tiles,
                              uint32_t party, hipStream_t st) {
  hipLaunchKernelGGL(k_header_init, dim3(1), dim3(256), 0, st, dst, src, n_elems, n_tiles, party);
  return hipGetLastError();
}

hipError_t launch_mask(const int64_t* x, const uint64_t* r_in, int64_t n, uint64_t* xhat, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_mask, dim3(grid), dim3(256), 0, st, x, r_in, n, xhat);
  return hipGetLastError();
}

hipError_t launch_open(const uint64_t* y0, const uint64_t* y1, int64_t n, uint64_t* yhat, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_open, dim3(grid), dim3(256), 0, st, y0, y1, n, yhat);
  return hipGetLastError();
}

hipError_t launch_rescale_keygen(int v, int r, const KeyHeader* h, const KgArgs& ga, const uint64_t* r_in,
                                 uint8_t* k0, uint8_t* k1, uint64_t* ro, int cus, hipStream_t st) {
  switch (v) {
    case 0: return VariantOps<0>::rescale_keygen(h, r, ga, r_in, k0, k1, ro, cus, st);
    case 1: return VariantOps<1>::rescale_keygen(h, r, ga, r_in, k0, k1, ro, cus, st);
    case 2: return VariantOps<2>::rescale_keygen(h, r, ga, r_in, k0, k1, ro, cus, st);
    case 3: return VariantOps<3>::rescale_keygen(h, r, ga, r_in, k0, k1, ro, cus, st);
    case 4: return VariantOps<4>::rescale_keygen(h, r, ga, r_in, k0, k1, ro, cus, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rescale_eval(int v, int party, const uint8_t* keys, const uint64_t* yhat, int64_t n, uint64_t* z,
                               int* status, int cus, hipStream_t st) {
  switch (v) {
    case 0: return VariantOps<0>::rescale_eval(party, keys, yhat, n, z, status, cus, st);
    case 1: return VariantOps<1>::rescale_eval(party, keys, yhat, n, z, status, cus, st);
    case 2: return VariantOps<2>::rescale_eval(party, keys, yhat, n, z, status, cus, st);
    case 3: return VariantOps<3>::rescale_eval(party, keys, yhat, n, z, status, cus, st);
    case 4: return VariantOps<4>::rescale_eval(party, keys, yhat, n, z, status, cus, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_keygen(int v, int p, int r, const KeyHeader* h, const KgArgs& ga, uint8_t* k0, uint8_t* k1,
                         uint64_t* ri, uint64_t* ro, int cus, hipStream_t st) {
  switch (v) {
    case 0: return VariantOps<0>::keygen(h, p, r, ga, k0, k1, ri, ro, cus, st);
    case 1: return VariantOps<1>::keygen(h, p, r, ga, k0, k1, ri, ro, cus, st);
    case 2: return VariantOps<2>::keygen(h, p, r, ga, k0, k1, ri, ro, cus, st);
    case 3: return VariantOps<3>::keygen(h, p, r, ga, k0, k1, ri, ro, cus, st);
    case 4: return VariantOps<4>::keygen(h, p, r, ga, k0, k1, ri, ro, cus, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eval_pred(int v, int party, const uint8_t* keys, const uint64_t* xhat, int64_t n,
                            uint64_t* z, int* status, int cus, hipStream_t st) {
  switch (v) {
    case 0: return VariantOps<0>::pred(party, keys, xhat, n, z, status, cus, st);
    case 1: return VariantOps<1>::pred(party, keys, xhat, n, z, status, cus, st);
    case 2: return VariantOps<2>::pred(party, keys, xhat, n, z, status, cus, st);
    case 3: return VariantOps<3>::pred(party, keys, xhat, n, z, status, cus, st);
    case 4: return VariantOps<4>::pred(party, keys, xhat, n, z, status, cus, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eval_coeff(int v, int party, const uint8_t* keys, const uint64_t* xhat, int64_t n,
                             uint64_t* y, int* status, int cus, hipStream_t st) {
  switch (v) {
    case 0: return VariantOps<0>::coeff(party, keys, xhat, n, y, status, cus, st);
    case 1: return VariantOps<1>::coeff(party, keys, xhat, n, y, status, cus, st);
    case 2: return VariantOps<2>::coeff(party, keys, xhat, n, y, status, cus, st);
    case 3: return VariantOps<3>::coeff(party, keys, xhat, n, y, status, cus, st);
    case 4: return VariantOps<4>::coeff(party, keys, xhat, n, y, status, cus, st);
    default: return hipErrorInvalidValue;
  }
}

// Zeroes y of the items whose tiles run in parts (the parts add into it).
__global__ void k_zero_split(const DevItem* items, const uint32_t* split_items, uint32_t n_split) {
  for (uint32_t s = blockIdx.y; s < n_split; s += gridDim.y) {
    const DevItem* ip = items + split_items[s];
    uint64_t* y = ip->y;
    const int64_t n = ip->n_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
      y[e] = 0;
  }
}

hipError_t launch_fused(int v, const DevItem* items, const uint32_t* tiles, uint32_t n_tiles, uint32_t* counter,
                        int* status, int grid, int lanes_log2, const uint32_t* split_items, uint32_t n_split,
                        uint64_t max_split_elems, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_split > 0 && max_split_elems > 0) {
    const uint64_t bx = std::min<uint64_t>((max_split_elems + 255) / 256, 1024);
    const unsigned by = std::min<uint32_t>(n_split, 1024);
    hipLaunchKernelGGL(k_zero_split, dim3((unsigned)bx, by), dim3(256), 0, st, items, split_items, n_split);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (v) {
    case 0: return VariantOps<0>::fused(items, tiles, n_tiles, counter, status, grid, lanes_log2, st);
    case 1: return VariantOps<1>::fused(items, tiles, n_tiles, counter, status, grid, lanes_log2, st);
    case 2: return VariantOps<2>::fused(items, tiles, n_tiles, counter, status, grid, lanes_log2, st);
    case 3: return VariantOps<3>::fused(items, tiles, n_tiles, counter, status, grid, lanes_log2, st);
    case 4: return VariantOps<4>::fused(items, tiles, n_tiles, counter, status, grid, lanes_log2, st);
    default: return hipErrorInvalidValue;
  }
}

int variant_block(int v) {
  switch (v) {
    case 0: return VariantOps<0>::block();
    case 1: return VariantOps<1>::block();
    case 2: return VariantOps<2>::block();
    case 3: return VariantOps<3>::block();
    default: return VariantOps<4>::block();
  }
}

int variant_lds_bytes(int v) {
  switch (v) {
    case 0: return VariantOps<0>::lds_bytes();
    case 1: return VariantOps<1>::lds_bytes();
    case 2: return VariantOps<2>::lds_bytes();
    case 3: return VariantOps<3>::lds_bytes();
    default: return VariantOps<4>::lds_bytes();
  }
}

}  // namespace fss
