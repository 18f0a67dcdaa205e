// fss_phi.hip -- the literal interval lookup (one vector DCF per inner
// boundary of the translated partition) and the post-processing
// subprotocols over shares: Beaver multiplication, AND on XOR-shared bit
// words, B2A.  The lookup runs AES table layout 1; the dealer's correlated
// randomness runs layout 0 (small tables: a few blocks per element).
#include "fss_kernels_impl.hpp"

namespace fss {

// ---------------------------------------------------------------------------
// Literal lookup partition of v-space (compilation protocol, step (1)) for
// one lane's mask.  Unpadded, position k (0 <= k < cnt) starts at S(k) and
// holds piece ord(k): position 0 starts at v = 0 inside the piece `first`
// that holds the preimage of v = 0; positions 1 .. m-1 start at the other
// pieces' translated starts, in cyclic order; if the first piece's own
// translated start is not 0, it returns at the top as position m (cut).  A
// partition that was not cut is padded to M = min(m + 1, 2^n) positions: the
// last position of length >= 2 gives its top value to a new position with
// the same piece.
// ---------------------------------------------------------------------------
struct LitPart {
  GHdr h;
  int m, M, first, cnt, kp;  // kp: position split by the padding, or -1
  uint64_t rn, nmask, N;

  __device__ uint64_t start(int k) const {  // unpadded start of position k <= cnt
    if (k == 0) return 0;
    if (k >= cnt) return N;
    if (k < m) return (h->aprime[(first + k) % m] + rn) & nmask;
    return (h->aprime[first] + rn) & nmask;  // the cut-off top of the first piece
  }
  __device__ int piece(int k) const { return k < m ? (first + k) % m : first; }
  __device__ uint64_t boundary(int j) const {  // B_j of the padded partition, 1 <= j < M
    if (kp < 0 || j <= kp) return start(j);
    return j == kp + 1 ? start(kp + 1) - 1 : start(j - 1);
  }
  __device__ int order(int j) const {  // ord_j of the padded partition, 0 <= j < M
    if (kp < 0 || j <= kp) return piece(j);
    return j == kp + 1 ? piece(kp) : piece(j - 1);
  }
};

__device__ __forceinline__ LitPart lit_partition(GHdr h, uint64_t r_in) {
  LitPart P;
  P.h = h;
  P.m = (int)h->m;
  P.M = (int)h->lit_M;
  const int n = (int)h->n;
  P.N = 1ull << n;
  P.nmask = P.N - 1;
  P.rn = r_in & P.nmask;
  const uint64_t x0 = (P.N - P.rn) & P.nmask;  // the preimage of v = 0
  P.first = 0;
  for (int i = 1; i < P.m; ++i)
    if (h->aprime[i] <= x0) P.first = i;
  P.cnt = P.m + (((h->aprime[P.first] + P.rn) & P.nmask) != 0 ? 1 : 0);
  P.kp = -1;
  if (P.cnt < P.M)
    for (int k = P.cnt - 1; k >= 0; --k)
      if (P.start(k + 1) - P.start(k) >= 2) {
        P.kp = k;
        break;
      }
  return P;
}

// Dealer keys of the literal lookup, one wave per tile and lane = element.
// Randomness R(e, ., .): 0 -> r_in, r_out; 1 -> party 0's r_out share; 200
// -> party 0's r_in share; 201 / 202 (ctr j) -> roots of DCF j; 203 + k
// (ctr 64 j + level) -> its on-path corrections; 210 / 211 -> party 0's
// shares of the last interval's payload.
template <int V, int P, int R>
__global__ __launch_bounds__((keygen_block<V, P>())) void k_lit_keygen(const KeyHeader* hdr, KgArgs ga, uint8_t* key0,
                                                                  uint8_t* key1, uint64_t* r_in, uint64_t* r_out) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (tile >= ga.n_tiles) return;
  TB tb(lds, lane);
  const GHdr h = ghdr(hdr);
  const int n = (int)h->n, M = (int)h->lit_M;
  const uint64_t tbb = h->tile_bytes, off_lrin = h->off_lrin, off_crout = h->off_crout, off_lbase = h->off_lbase;
  const uint64_t off_root = h->off_croot, dcf_bytes = h->dcf_bytes;
  const uint64_t e = tile * kTile + lane;
  uint8_t* t0 = key0 + kHeaderBytes + tile * tbb;
  uint8_t* t1 = key1 ? key1 + kHeaderBytes + tile * tbb : nullptr;
  uint32_t r[4];
  rand_blk(tb, ga.rk, e, 0, 0, r);
  const uint64_t rin = mk64(r[0], r[1]), rout = mk64(r[2], r[3]);
  if (e < (uint64_t)ga.n_elems) {
    if (r_in) stg64(r_in + e, rin);
    if (r_out) stg64(r_out + e, rout);
  }
  rand_blk(tb, ga.rk, e, 1, 0, r);
  st8(t0 + off_crout + lane * 8, mk64(r[0], r[1]));
  if (t1) st8(t1 + off_crout + lane * 8, rout - mk64(r[0], r[1]));
  rand_blk(tb, ga.rk, e, 200, 0, r);
  st8(t0 + off_lrin + lane * 8, mk64(r[0], r[1]));
  if (t1) st8(t1 + off_lrin + lane * 8, rin - mk64(r[0], r[1]));
  init_record(tb, ga.rk, tile, h->off_seen, h->off_sentinel, tbb, t0, t1, lane);
  const LitPart part = lit_partition(h, rin);
#pragma unroll 1
  for (int j = 1; j < M; ++j) {
    const int lo = part.order(j - 1), hi = part.order(j);
    uint64_t beta[P];
#pragma unroll
    for (int q = 0; q < P; ++q) beta[q] = h->lcoef[lo][q] - h->lcoef[hi][q];
    uint32_t c0[4], c1[4];
    rand_blk(tb, ga.rk, e, 201, (uint32_t)j, c0);
    rand_blk(tb, ga.rk, e, 202, (uint32_t)j, c1);
    const uint64_t off = off_root + (uint64_t)(j - 1) * dcf_bytes;
    gen_vec_at<P, R>(tb, off, off + (uint64_t)kTile * 16, 203u, 64u * (uint32_t)j, n, part.boundary(j), beta, c0,
                     c1, ga.rk, e, t0, t1, lane);
  }
  const int last = part.order(M - 1);
  uint32_t ra[4], rb[4];
  rand_blk(tb, ga.rk, e, 210, 0, ra);
  rand_blk(tb, ga.rk, e, 211, 0, rb);
  const uint64_t sh[4] = {mk64(ra[0], ra[1]), mk64(ra[2], ra[3]), mk64(rb[0], rb[1]), mk64(rb[2], rb[3])};
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const uint64_t o = off_lbase + ((uint64_t)q * kTile + lane) * 8;
    st8(t0 + o, sh[q]);
    if (t1) st8(t1 + o, h->lcoef[last][q] - sh[q]);
  }
}

// Party b's shares of the active piece's coefficients and of x = xhat - r_in:
// the last interval's payload share plus every DCF at v = (xhat + c) mod 2^n.
template <int P, int R, class TB>
__device__ __forceinline__ void lit_walks(const TB& tb, GHdr h, const uint8_t* tp, int lane, int b, uint64_t xh,
                                          uint64_t (&acc)[P]) {
  const int n = (int)h->n, M = (int)h->lit_M;
  const uint64_t nmask = n >= 64 ? ~0ull : ((1ull << n) - 1);
  const uint32_t v = (uint32_t)((xh + h->lookup_c) & nmask);
  const uint64_t off_root = h->off_croot, dcf_bytes = h->dcf_bytes;
#pragma unroll 1
  for (int j = 1; j < M; ++j) {
    const uint8_t* d = tp + off_root + (uint64_t)(j - 1) * dcf_bytes;
    VState<P> st = vroot_at<P>(d, lane, b);
    vec_walk_at<P, R>(tb, n, d + (uint64_t)kTile * 16, lane, b, v, 0, (n + R - 1) / R, st);
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] += st.V[q];
  }
}

template <int V>
__global__ __launch_bounds__(TabOf<V>::kBlock) void k_lit_eval(const uint8_t* keys, const uint64_t* xhat, int64_t n,
                                                                int party, uint64_t* coef, uint64_t* xs,
                                                                int* status) {
  using TB = typename TabOf<V>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const GHdr h = ghdr(keys);
  if (h->magic != kMagic || h->version != kVersion || h->kind != kGateLiteral || (int)h->party != party ||
      (uint64_t)n > h->n_elems) {
    if (threadIdx.x == 0) set_status(status, (int)h->party != party ? kStatusParty : kStatusShape);
    return;
  }
  const int lane = threadIdx.x & 63;
  const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (tile * kTile >= (uint64_t)n) return;
  const uint64_t e = tile * kTile + lane;
  const bool valid = e < (uint64_t)n;
  const uint64_t xh = valid ? ldg64(xhat + e) : 0;
  TB tb(lds, lane);
  const uint8_t* tp = keys + kHeaderBytes + tile * h->tile_bytes;
  const int p = (int)h->p;
  uint64_t acc[kMaxP];
#pragma unroll
  for (int q = 0; q < kMaxP; ++q) acc[q] = q < p ? ld8(tp + h->off_lbase + ((uint64_t)q * kTile + lane) * 8) : 0ull;
  auto run = [&](auto pc, auto rc) {
    constexpr int PP = decltype(pc)::value, RR = decltype(rc)::value;
    uint64_t a[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) a[q] = acc[q];
    lit_walks<PP, RR>(tb, h, tp, lane, party, xh, a);
#pragma unroll
    for (int q = 0; q < PP; ++q) acc[q] = a[q];
  };
  auto by_r = [&](auto pc) {
    switch (h->lookup_r) {
      case 2: run(pc, std::integral_constant<int, 2>{}); break;
      case 3: run(pc, std::integral_constant<int, 3>{}); break;
      default: run(pc, std::integral_constant<int, 4>{}); break;
    }
  };
  switch (p) {
    case 1: by_r(std::integral_constant<int, 1>{}); break;
    case 2: by_r(std::integral_constant<int, 2>{}); break;
    case 3: by_r(std::integral_constant<int, 3>{}); break;
    default: by_r(std::integral_constant<int, 4>{}); break;
  }
  const uint64_t rin = ld8(tp + h->off_lrin + lane * 8);
  acc[0] += ld8(tp + h->off_crout + lane * 8);  // the output mask rides in the constant term
  const bool ok = claim_once(h, tp, lane, xh, valid, status);
  if (valid) {
    for (int q = 0; q < p; ++q) stg64(coef + (uint64_t)q * (uint64_t)n + e, ok ? acc[q] : 0ull);
    stg64(xs + e, ok ? (party == 0 ? xh - rin : 0ull - rin) : 0ull);
  }
}

// ---------------------------------------------------------------------------
// Dealer correlations, element (or bit word) i of `n`, step `step`:
//   Beaver triple: R(i, 220, step) -> a, b; R(i, 221, step) -> party 0's
//   shares of a, b; R(i, 222, step).lo -> party 0's share of c = a b.
//   AND triple of word i: the same with 230, 231, 232 and c = a & b, XOR.
//   B2A: t = R(i, 240, step).lo bit 0; R(i, 241, step): party 0's XOR share
//   of t (lo bit 0) and additive share T_0 (hi); bits packed 64 to a word.
// ---------------------------------------------------------------------------
constexpr int kDealerV = 0;

__global__ __launch_bounds__(TabOf<kDealerV>::kBlock) void k_correlations(RoundKeys rk, int kind, int64_t n,
                                                                           uint32_t step, uint64_t* a0, uint64_t* b0,
                                                                           uint64_t* c0, uint64_t* a1, uint64_t* b1,
                                                                           uint64_t* c1) {
  using TB = typename TabOf<kDealerV>::T;
  __shared__ __align__(16) uint32_t lds[TB::kWords];
  TB::fill(lds, threadIdx.x, blockDim.x);
  __syncthreads();
  TB tb(lds, threadIdx.x & 63);
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every lane of a wave runs the AES (the tables are shared per wave); the
  // B2A bit words need whole waves for their ballot
  const uint32_t base = kind == 0 ? 220u : kind == 1 ? 230u : 240u;
  uint32_t x[4], y[4], z[4];
  rand_blk(tb, rk, i, base, step, x);
  rand_blk(tb, rk, i, base + 1, step, y);
  if (kind == 2) {
    const uint64_t t = x[0] & 1u, s = y[0] & 1u, T0 = mk64(y[2], y[3]);
    const uint64_t w0 = __ballot(s != 0), w1 = __ballot((s ^ t) != 0);
    if (i < (uint64_t)n) {
      c0[i] = T0;
      c1[i] = t - T0;
    }
    if ((threadIdx.x & 63) == 0 && i < (uint64_t)n) {
      a0[i >> 6] = w0;
      a1[i >> 6] = w1;
    }
    return;
  }
  rand_blk(tb, rk, i, base + 2, step, z);
  if (i >= (uint64_t)n) return;
  const uint64_t A = mk64(x[0], x[1]), B = mk64(x[2], x[3]), A0 = mk64(y[0], y[1]), B0 = mk64(y[2], y[3]);
  const uint64_t C0 = mk64(z[0], z[1]);
  if (kind == 0) {
    a0[i] = A0; a1[i] = A - A0;
    b0[i] = B0; b1[i] = B - B0;
    c0[i] = C0; c1[i] = A * B - C0;
  } else {
    a0[i] = A0; a1[i] = A ^ A0;
    b0[i] = B0; b1[i] = B ^ B0;
    c0[i] = C0; c1[i] = (A & B) ^ C0;
  }
}

// One party's local steps, element (or word) i of n.
//   kind 0: d = u - a, e = v - b                    (Beaver, before the opening)
//   kind 1: z = c + d b + e a (+ d e for party 0) (+ add)   (Beaver, after it)
//   kind 2: d = x ^ a, e = y ^ b (e skipped if y is null)   (AND / B2A, before)
//   kind 3: z = c ^ (d & b) ^ (e & a) (^ d & e for party 0) (AND, after)
//   kind 4: z = c ^ d                                (XOR opening)
//   kind 5: z = (party 0: bit) + (1 - 2 bit) T, bit i of the opened words c  (B2A, after)
struct PhiArgs {
  const uint64_t *u, *v, *a, *b, *c, *add;
  uint64_t *d, *e, *z;
  int64_t n;
  int kind, party;
};

__global__ void k_phi(PhiArgs g) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x) {
    switch (g.kind) {
      case 0:
        g.d[i] = g.u[i] - g.a[i];
        g.e[i] = g.v[i] - g.b[i];
        break;
      case 1: {
        const uint64_t D = g.u[i], E = g.v[i];
        uint64_t z = g.c[i] + D * g.b[i] + E * g.a[i];
        if (g.party == 0) z += D * E;
        if (g.add) z += g.add[i];
        g.z[i] = z;
        break;
      }
      case 2:
        g.d[i] = g.u[i] ^ g.a[i];
        if (g.v) g.e[i] = g.v[i] ^ g.b[i];
        break;
      case 3: {
        const uint64_t D = g.u[i], E = g.v[i];
        uint64_t z = g.c[i] ^ (D & g.b[i]) ^ (E & g.a[i]);
        if (g.party == 0) z ^= D & E;
        g.z[i] = z;
        break;
      }
      case 4:
        g.z[i] = g.u[i] ^ g.v[i];
        break;
      default: {
        const uint64_t bit = (g.c[i >> 6] >> (i & 63)) & 1ull;
        g.z[i] = (g.party == 0 ? bit : 0ull) + (1ull - 2ull * bit) * g.a[i];
        break;
      }
    }
  }
}

hipError_t launch_lit_keygen(int p, int r, const KeyHeader* h, const KgArgs& ga, uint8_t* k0, uint8_t* k1,
                             uint64_t* ri, uint64_t* ro, hipStream_t st) {
  constexpr int V = 1;
  auto go = [&](auto kern, int block) {
    const unsigned grid = (unsigned)((ga.n_tiles + block / 64 - 1) / (block / 64));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, h, ga, k0, k1, ri, ro);
    return hipGetLastError();
  };
#define FSS_LIT_CASE(PP, RR) \
  if (p == PP && r == RR) return go(k_lit_keygen<V, PP, RR>, keygen_block<V, PP>());
  FSS_LIT_CASE(1, 2) FSS_LIT_CASE(1, 3) FSS_LIT_CASE(1, 4)
  FSS_LIT_CASE(2, 2) FSS_LIT_CASE(2, 3) FSS_LIT_CASE(2, 4)
  FSS_LIT_CASE(3, 2) FSS_LIT_CASE(3, 3) FSS_LIT_CASE(3, 4)
  FSS_LIT_CASE(4, 2) FSS_LIT_CASE(4, 3) FSS_LIT_CASE(4, 4)
#undef FSS_LIT_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_lit_eval(int party, const uint8_t* keys, const uint64_t* xhat, int64_t n, uint64_t* coef,
                           uint64_t* xs, int* status, hipStream_t st) {
  constexpr int V = 1, B = TabOf<V>::kBlock;
  if (n <= 0) return hipSuccess;
  const uint64_t tiles = ((uint64_t)n + kTile - 1) / kTile;
  const unsigned grid = (unsigned)((tiles + B / 64 - 1) / (B / 64));
  hipLaunchKernelGGL((k_lit_eval<V>), dim3(grid), dim3(B), 0, st, keys, xhat, n, party, coef, xs, status);
  return hipGetLastError();
}

hipError_t launch_correlations(const RoundKeys& rk, int kind, int64_t n, uint32_t step, uint64_t* a0, uint64_t* b0,
                               uint64_t* c0, uint64_t* a1, uint64_t* b1, uint64_t* c1, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  constexpr int B = TabOf<kDealerV>::kBlock;
  const unsigned grid = (unsigned)((n + B - 1) / B);
  hipLaunchKernelGGL(k_correlations, dim3(grid), dim3(B), 0, st, rk, kind, n, step, a0, b0, c0, a1, b1, c1);
  return hipGetLastError();
}

hipError_t launch_phi(int kind, int party, const uint64_t* u, const uint64_t* v, const uint64_t* a,
                      const uint64_t* b, const uint64_t* c, const uint64_t* add, int64_t n, uint64_t* d,
                      uint64_t* e, uint64_t* z, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  PhiArgs g{u, v, a, b, c, add, d, e, z, n, kind, party};
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_phi, dim3(grid), dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace fss
