/*
 * fusefss.h -- C ABI of the MI355X (gfx950) FuseFSS hot-path library.
 *
 * The library implements the two FSS calls the paper's compiler emits for a
 * scalar fixed-point operator (Sec. 4.4 "Compiling One Operator Gate with Two
 * FSS Calls", Theorem "Two-call evaluation"), evaluated on the public masked
 * input xhat = x + r_in (Sec. 3.5 masked-wire invariant):
 *   call 1, packed comparison: XOR shares of all predicate bits
 *           (Definition "Multi-view packed predicate primitive");
 *   call 2, vector interval lookup: additive shares of the active piece's
 *           coefficients (Definition "Interval lookup with vector payload"),
 *           combined locally into shares of P_{i*}(x) + r_out mod 2^64,
 * together with the dealer's key generation (Sec. 5.2 "Preprocessing").
 *
 * Conventions for every function:
 *   - Return value: FSS_OK (0) or a negative FSS_E_* code; fss_last_error()
 *     returns a thread-local message for the last failure.  No C++ exception
 *     crosses the ABI.
 *   - Pointers documented as "device" point to HIP device memory allocated by
 *     the caller; "host" pointers are ordinary host memory.  The caller owns
 *     every buffer.  The library owns only fss_spec / fss_plan / fss_graph
 *     handles, released with the matching *_free call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that take a stream only enqueue work; they return before the GPU
 *     finishes.  Kernel-side validation failures (for example a key buffer of
 *     the wrong party) are recorded in a device status word and reported by
 *     fss_status().
 *   - Ring: all arithmetic outputs live in Z_{2^64}; comparison views use
 *     n_bits in [2, 32]; fixed-point inputs are n_bits-wide signed values with
 *     frac_bits fractional bits, sign-extended to 64 bits.
 */
#ifndef FUSEFSS_H
#define FUSEFSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSS_OK 0
#define FSS_E_INVALID_SPEC (-1) /* partition not increasing, degree > 3, |P| >= 2^62, NaN */
#define FSS_E_UNSUPPORTED (-2)  /* n_bits outside [2,32], frac_bits >= n_bits, too many atoms */
#define FSS_E_NEEDS_PHI (-3)    /* AND/OR predicate: needs the interactive post-processing */
#define FSS_E_SHAPE (-4)        /* key header / buffer does not match the call */
#define FSS_E_PARTY (-5)        /* party not 0 or 1 */
#define FSS_E_HIP (-6)          /* a HIP runtime call failed (message has the hipError_t) */
#define FSS_E_OOM (-7)          /* host allocation failed */
#define FSS_E_ARG (-8)          /* NULL pointer, negative size, bad tuning value */
#define FSS_E_CONSUMED (-9)     /* (device status) a key evaluated again at another masked input */

#define FSS_MAX_INTERVALS 64
#define FSS_MAX_PREDS 16
#define FSS_MAX_ATOMS 16
#define FSS_MAX_DEGREE 3

/* ---- operator specification (Definition "Operator specification") ------ */

/* Half-open real interval [lo, hi); lo = -INFINITY / hi = +INFINITY for tails. */
typedef struct { double lo, hi; } fss_interval;

/* Polynomial piece a_0 + a_1 x + ... + a_d x^d over real x (lowest first), d <= 3. */
typedef struct { int32_t degree; double coef[4]; } fss_piece;

enum {
  FSS_PRED_LT_SIGNED = 0,   /* x <_signed thr (real threshold)                    */
  FSS_PRED_LT_UNSIGNED = 1, /* rep(x) < thr over canonical representatives        */
  FSS_PRED_LOWBITS_LT = 2,  /* (x mod 2^f_bits) < gamma  (primitive D_{gamma,f})   */
  FSS_PRED_MSB_SHIFT = 3    /* MSB(x + c) for a public shift c                     */
};
enum { FSS_COMBINE_XOR = 0, FSS_COMBINE_AND = 1, FSS_COMBINE_OR = 2 };

/* One primitive predicate.  Predicates with the same `out` are combined into
 * output bit `out` with XOR (local); AND / OR need the post-processing
 * circuit and are rejected with FSS_E_NEEDS_PHI (appendix "Typed
 * specification language"). */
typedef struct {
  int32_t kind;     /* FSS_PRED_* */
  int32_t negate;   /* nonzero: XOR the predicate with 1 */
  int32_t out;      /* output bit index, 0 <= out < 64 */
  int32_t combine;  /* FSS_COMBINE_* */
  int32_t f_bits;   /* LOWBITS_LT: low-bit width, 1 <= f_bits <= n_bits */
  int32_t reserved;
  double thr;       /* LT_SIGNED / LT_UNSIGNED: real threshold */
  int64_t gamma;    /* LOWBITS_LT: integer threshold in [0, 2^f_bits] */
  int64_t c;        /* MSB_SHIFT: public shift (taken mod 2^n_bits) */
} fss_pred;

typedef struct fss_spec fss_spec;

/* Validate and store a real-valued operator specification.  Quantisation to
 * (n_bits, frac_bits) happens on first use and is cached per spec (compiled
 * program reuse, ablation "Program Reuse Across Layers").
 *   iv[m], pieces[m]: host arrays; iv must be contiguous from -inf to +inf.
 *   preds[n_preds]: host array (may be NULL when n_preds == 0).
 *   out_frac_bits: fractional bits of the arithmetic output; < 0 selects
 *     2*frac_bits for degree <= 1 and 4*frac_bits otherwise.
 *   *out receives a handle owned by the caller (free with fss_spec_free). */
int fss_compile_spec(const fss_interval* iv, int32_t m, const fss_piece* pieces,
                     const fss_pred* preds, int32_t n_preds, int32_t out_frac_bits,
                     fss_spec** out);
void fss_spec_free(fss_spec* spec);

/* The Definition "Operator specification" in its integer form, as the paper
 * states it over Z_{2^n}: boundaries 0 = alpha_0 < alpha_1 < ... < alpha_m =
 * 2^n_bits over the canonical representatives {0, ..., 2^n_bits - 1}, piece i
 * applying to the inputs whose representative lies in [alpha_i, alpha_{i+1}),
 * and ring coefficients in Z_{2^64} (the polynomial is evaluated at the
 * input's 64-bit value, mod 2^64).  This is the form of the appendix's worked
 * example (ReLU with alpha_1 = 2^(n-1)).
 *   alpha: host, m + 1 u64.  coef: host, m * (degree + 1) u64, row-major,
 *     lowest degree first.  preds: host (NULL when n_preds == 0); comparison
 *     thresholds `thr` must be integers (there are no fractional bits).
 *   The spec is used at (n_bits, frac_bits = 0) only; other sizes return
 *   FSS_E_SHAPE.  Call 2 then reads the unshifted view xhat mod 2^n_bits
 *   (real-valued specs read the offset-binary view of the signed order).
 *   Errors: FSS_E_INVALID_SPEC for boundaries that do not run increasing from
 *   0 to 2^n_bits, a degree outside [0, 3] or a non-integer threshold;
 *   FSS_E_UNSUPPORTED for n_bits outside [2, 32]; FSS_E_NEEDS_PHI for AND/OR.
 *   *out receives a handle owned by the caller (free with fss_spec_free). */
int fss_compile_spec_int(int32_t n_bits, int32_t m, const uint64_t* alpha, int32_t degree,
                         const uint64_t* coef, const fss_pred* preds, int32_t n_preds, fss_spec** out);

/* Input bits per level of call 2's vector DCF (the interval lookup of
 * Definition "Interval lookup with vector payload", realised as one DCF
 * evaluated at m points): 2, 3 or 4, i.e. 4, 8 or 16 children per level and
 * ceil(n_bits / bits) levels.  More bits per level walk fewer levels at each
 * lookup point (fewer AES blocks in evaluation) and generate and store more
 * children per level (more AES in keygen, larger keys).  The paper leaves
 * the DCF open; this is the 2^k-ary form.  Applies to keys generated and
 * sizes queried after the call (each setting is cached separately); keys
 * record it in their header, so evaluation needs no setting.  Returns
 * FSS_E_ARG for other values.  The default is 3 until changed. */
int fss_spec_set_lookup_radix(fss_spec* spec, int32_t bits);
/* The current setting (or a negative FSS_E_* code for a NULL spec). */
int fss_spec_get_lookup_radix(const fss_spec* spec);

/* Public, mask-independent shape of a quantised spec (leakage L_shape of
 * the appendix "A standard real/ideal security statement"). */
typedef struct {
  int32_t n_bits, frac_bits, m, degree, p, out_frac_bits;
  int32_t T;        /* comparison atoms in the packed comparison */
  int32_t ell;      /* predicate output bits */
  int32_t atom_k[FSS_MAX_ATOMS];    /* bit width of each atom's view */
  int64_t atom_c[FSS_MAX_ATOMS];    /* public shift of each atom's view */
  int32_t atom_is_mask[FSS_MAX_ATOMS]; /* 1: the 1[view < r_k] atom of its view */
  int32_t lookup_r;  /* input bits per level of call 2's DCF */
  int32_t top_depth; /* its levels walked once per block of lookup points */
  int32_t top_blocks; /* aligned blocks of lookup points that share them */
} fss_spec_info;

/* Quantise at (n_bits, frac_bits) and report the shape and integer tables.
 *   aprime: host, m+1 u64 (offset-binary boundaries alpha_i + 2^(n-1)), may be NULL.
 *   coef:   host, m*p u64 ring coefficients (row-major, lowest degree first), may be NULL. */
int fss_spec_query(const fss_spec* spec, int32_t n_bits, int32_t frac_bits, fss_spec_info* info,
                   uint64_t* aprime, uint64_t* coef);

/* ---- dealer key generation (Sec. 5.2, Protocol "Compile a scalar gate") -- */

/* Bytes of one party's key buffer for n_elems elements.  Depends only on
 * (spec, n_bits, frac_bits, n_elems), never on masks (Proposition
 * "Mask-independent shape via padding"). */
int fss_key_bytes(const fss_spec* spec, int32_t n_bits, int32_t frac_bits, int64_t n_elems,
                  size_t* per_party);

/* Generate both parties' keys for n_elems fresh gate instances.
 *   seed: host, 16 bytes: the AES-128 key of the dealer's randomness (a
 *     128-bit integer in little-endian byte order), so the masks have the
 *     security parameter of Gen(1^lambda) (Sec. "Threat Model and
 *     Preprocessing").  Read before the call returns.
 *   key0, key1: device, fss_key_bytes each (key1 may be NULL to skip party 1).
 *   r_in, r_out: device, n_elems u64 each (the dealer's masks; may be NULL).
 * Each element e draws all of its randomness from AES keyed by `seed`
 * (counter mode over e), so the output is a pure function of the arguments.
 * Keys are one-time material: evaluate each buffer on one input only. */
int fss_keygen(const fss_spec* spec, int32_t n_bits, int32_t frac_bits, const uint8_t* seed,
               int64_t n_elems, void* key0, void* key1, uint64_t* r_in, uint64_t* r_out,
               void* stream);

/* Work of one fss_keygen call over n_elems elements, as the kernel computes
 * it (host out-params): AES-128 blocks, and T-table lookups (16 per round,
 * less the 24 lookups of rounds 1-2 shared by the blocks that expand one seed
 * under several tweaks).  Per element: both parties' two children of every
 * comparison-DCF level, both parties' 2^r children of every lookup-DCF level,
 * and the counter-mode randomness blocks.  Used for throughput reporting. */
int fss_keygen_work(const fss_spec* spec, int32_t n_bits, int32_t frac_bits, int64_t n_elems,
                    double* aes_blocks, double* table_lookups);

/* Protocol "Shares -> masked opening" collapsed to one process that holds
 * the plaintext: xhat[e] = x[e] + r_in[e] mod 2^64 (all device, n each). */
int fss_mask_input(const int64_t* x, const uint64_t* r_in, int64_t n, uint64_t* xhat,
                   void* stream);

/* ---- rescaling gate: ARS of a masked value ---------------------------------
 * Fixed-point rescaling by arithmetic right shift (Sec. 3.2 encoding; the
 * paper counts truncation and ARS among the specification-compatible gates
 * of Definition "Specification-compatible scalar gate").  The gate composes
 * with an operator gate the way FSS gates compose: the operator's output
 * mask r_out is the rescaling gate's input mask, the parties open
 * yhat = y_0 + y_1 = y + r_out (fss_open), and each evaluates its key on
 * yhat.  For a signed y with |y| < 2^62 (every compiled piece satisfies the
 * bound) the outputs are shares of floor(y / 2^shift_bits) + r_out', with a
 * fresh output mask r_out'.  shift_bits in [1, 32]; lookup_bits (2, 3 or 4)
 * is the input bits per level of the gate's comparison DCF. */

/* Bytes of one party's rescaling-gate key buffer (mask-independent). */
int fss_rescale_key_bytes(int32_t shift_bits, int32_t lookup_bits, int64_t n_elems, size_t* per_party);
/* Dealer keygen of n_elems rescaling gates.
 *   seed: host, 16 bytes (the gate's own dealer seed, as in fss_keygen).
 *   r_in: device, n_elems u64: the input masks (the previous gate's r_out).
 *   key0, key1: device, fss_rescale_key_bytes each (key1 may be NULL).
 *   r_out: device, n_elems u64 output masks (may be NULL).
 * Errors: FSS_E_UNSUPPORTED (shift_bits), FSS_E_ARG. */
int fss_rescale_keygen(int32_t shift_bits, int32_t lookup_bits, const uint8_t* seed, int64_t n_elems,
                       const uint64_t* r_in, void* key0, void* key1, uint64_t* r_out, void* stream);
/* Party `party`'s evaluation at the openings yhat (device, n_elems u64);
 * z: device, n_elems u64 output shares.  Key-buffer mismatches are recorded
 * in the device status word (fss_status). */
int fss_rescale_eval(int32_t party, const void* keys, const uint64_t* yhat, int64_t n_elems, uint64_t* z,
                     void* stream);
/* The opening of additive shares held on one device (both parties simulated
 * in one process; across two devices each party would send its share):
 * yhat[e] = y0[e] + y1[e] mod 2^64, all device, n each. */
int fss_open(const uint64_t* y0, const uint64_t* y1, int64_t n, uint64_t* yhat, void* stream);

/* ---- online evaluation (Sec. 5.3 "Online Evaluation", steps 2-3) ------- */

/* One-time keys (Sec. "Threat Model and Preprocessing": all preprocessing
 * material is one-time; two openings under one mask would reveal x - x').
 * Every evaluator below records, in the key buffer itself, the masked input
 * each element is first evaluated at (8 bytes per element, set by one atomic
 * compare-and-swap against a random per-tile sentinel that keygen writes).
 * Evaluating an element again at the same masked input is a replay and
 * allowed (it reveals nothing new: graphs, retries, the two calls of the
 * plain path); at a different one the element is refused: its output shares
 * are zero and fss_status reports FSS_E_CONSUMED.  Key buffers are therefore
 * written by evaluation; launches that overlap on one key buffer are checked
 * against each other too.  This guards against accidental reuse by the
 * caller, not against a party that copies its key bytes. */

/* Plain evaluator: call 1 then call 2 as two kernel launches.
 *   keys: device key buffer of `party` (self-describing header).
 *   xhat: device, n_elems u64.  y: device, n_elems u64 output shares.
 *   zbits: device, ell * ceil(n_elems/64) u64 output shares; predicate j of
 *          element e is bit (e & 63) of word j*ceil(n_elems/64) + (e >> 6).
 *          May be NULL when ell == 0. */
int fss_eval(int32_t party, const void* keys, const uint64_t* xhat, int64_t n_elems,
             uint64_t* y, uint64_t* zbits, void* stream);
/* The two calls separately (same buffers as fss_eval). */
int fss_eval_pred(int32_t party, const void* keys, const uint64_t* xhat, int64_t n_elems,
                  uint64_t* zbits, void* stream);
int fss_eval_coeff(int32_t party, const void* keys, const uint64_t* xhat, int64_t n_elems,
                   uint64_t* y, void* stream);

/* ---- fused, batched evaluation over a work-list --------------------------- */

typedef struct {
  int32_t party;
  int32_t reserved;
  const void* keys;       /* device key buffer of `party` */
  const uint64_t* xhat;   /* device, n_elems */
  uint64_t* y;            /* device, n_elems */
  uint64_t* zbits;        /* device, ell * ceil(n_elems/64), may be NULL if ell == 0 */
  int64_t n_elems;
} fss_work_item;

/* Launch configuration of the persistent kernel (0 = library default). */
typedef struct {
  int32_t block_threads;  /* set by the library from the table layout */
  int32_t blocks_per_cu;  /* resident blocks per compute unit */
  int32_t aes_variant;    /* AES table layout, 0 .. fss_aes_variants()-1 */
  int32_t order;          /* 0: costliest tiles first, 1: work-list order */
  int32_t parts;          /* units call 2 of a tile is split into: 0 = planner's choice, 1 .. 4 */
  int32_t pred_unit;      /* call 1 of a tile: 0 = planner's choice, 1 = in the unit that runs
                             call 2's first part (one pass over the elements), 2 = its own unit */
  int32_t lanes;          /* lanes per element in call 2, i.e. elements per wave = 64 / lanes:
                             0 or 1 = one lane per element; 2 or 4 = each element's lookup
                             points split over that many lanes, whose shares of y are summed
                             across the wave (then parts <= 1, call 1 in its own unit, and
                             aes_variant 1 or 2) */
} fss_tune;

typedef struct fss_plan fss_plan;

/* Build a work-list plan: reads each item's key header (synchronously, once;
 * the keys must have been generated), uploads the unit list, and records the
 * launch configuration (`tune` may be NULL for defaults).  Items may mix
 * parties, specs and sizes.  A unit is normally one tile's call 1 and call 2
 * in one pass over its elements; when whole tiles would leave waves idle the
 * planner splits call 2 into parts and may run call 1 as a unit of its own
 * (fss_plan_config reports the choice). */
int fss_plan_create(const fss_work_item* items, int32_t n_items, const fss_tune* tune,
                    fss_plan** out);
/* One persistent launch evaluating both calls of every element of every item.
 * Enqueue-only and safe to capture into a HIP graph. */
int fss_plan_launch(fss_plan* plan, void* stream);
/* Releases the plan without waiting: its device buffers return to the
 * library's pool once its last launch (direct or through a graph) has
 * completed.  Free graphs that captured a plan before the plan itself. */
int fss_plan_free(fss_plan* plan);

/* Fused, batched evaluation of a work-list in one call (Sec. 5.3 "Online
 * Evaluation" for many gate instances at once): plan, one persistent launch
 * on `stream`, release.  `party` is 0 or 1, and then every item must be that
 * party's, or FSS_PARTY_ANY to let the items mix parties (both parties
 * simulated on one device).  The planner reads the items' key headers on the
 * host, so the call first waits for the work already enqueued on `stream`
 * (for example the keygen that wrote them); it returns once the launch is
 * enqueued.  Errors: FSS_E_PARTY (an item of the other party, or a bad
 * `party`), FSS_E_SHAPE (not a key buffer, n_elems beyond the keys),
 * FSS_E_ARG (NULL buffers), FSS_E_HIP. */
#define FSS_PARTY_ANY (-1)
int fss_eval_batch(int32_t party, const fss_work_item* items, int32_t n_items, void* stream);
/* AES-128 blocks one launch of `plan` evaluates, as the kernels compute them
 * (per element and party, with B = 1 + ceil(p/2) blocks per level of the
 * lookup DCF and ceil(p/2) at its last level, L = ceil(n/r) levels of 2^r
 * children, D shared top levels and T of the spec's top blocks:
 * sum_t (k_t - min(7, k_t) + 1) + (L - 1 + T D + (m-1)(L-D-1)) B + m ceil(p/2),
 * each comparison atom walking its tree above the 128-bit leaves and one
 * leaf conversion; the m-1 lookup
 * points share their first D levels, walked once for each of the T aligned
 * blocks they fall in; a tile run in parts walks them once per part).  Used
 * for throughput reporting. */
double fss_plan_aes_blocks(const fss_plan* plan);
/* T-table lookups of one launch: 16 per AES round, less the 24 lookups of
 * rounds 1-2 that the blocks expanding one seed under K tweaks share
 * (160 K - 24 (K - 1) per expansion).  The table-lookup rate of the CUs'
 * local memory bounds the evaluation, so this is the roofline's work figure. */
double fss_plan_table_lookups(const fss_plan* plan);
/* Parts per tile the planner chose (1 = every tile runs whole).  When the
 * tiles do not divide evenly over the resident waves, the planner splits each
 * tile's lookup points into up to 4 parts run by different waves; each part
 * adds its share of y (mod 2^64, exact) into y, which the launch zeroes first.
 * Returns 0 for a NULL plan. */
int fss_plan_parts(const fss_plan* plan);
/* fss_eval_batch for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs and errors as fss_eval_batch, but the work-list
 * lives in a fixed device array of 8 MiB that the library holds on each
 * device it runs on until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call (the key headers are read on `stream`).
 * Limits: at most FSS_NOALLOC_MAX_ITEMS items and FSS_NOALLOC_MAX_UNITS
 * work-list units (a unit is a 64-element tile of one item, or one of up to
 * five parts of it); larger work-lists return FSS_E_ARG before anything is
 * enqueued.  Every call on a device uses that device's one array: calls that
 * overlap on one device race (order them, e.g. on one stream).  Kernel-side
 * validation failures are reported by fss_status like the others. */
#define FSS_NOALLOC_MAX_ITEMS 1024
#define FSS_NOALLOC_MAX_UNITS 491520
int fss_eval_batch_noalloc(int32_t party, const fss_work_item* items, int32_t n_items, void* stream);

/* Resolved launch configuration of a plan (host out-params): the tune with
 * `parts`, `pred_unit` and `lanes` set to the planner's choice. */
int fss_plan_config(const fss_plan* plan, fss_tune* tune, int32_t* grid);

/* Capture the launches of n_plans plans, in order, into one HIP graph. */
typedef struct fss_graph fss_graph;
int fss_graph_capture(fss_plan* const* plans, int32_t n_plans, fss_graph** out);
int fss_graph_launch(fss_graph* graph, void* stream);
int fss_graph_free(fss_graph* graph);

/* Time candidate launch configurations on this work-list (the items' outputs
 * are overwritten) and return the fastest in *best; results are cached in
 * `cache_path` (may be NULL) keyed by the work-list's shape and the device. */
int fss_autotune(const fss_work_item* items, int32_t n_items, const char* cache_path,
                 fss_tune* best);
int fss_aes_variants(void);

/* The key-layout knob: pick the input bits per level of call 2's DCF (2, 3
 * or 4, fss_spec_set_lookup_radix) for `spec` at (n_bits, frac_bits) over
 * n_elems elements by timing one step per candidate -- both parties' keygen
 * and one fused launch of both parties' evaluation, at masked inputs spread
 * uniformly over the ring -- on scratch buffers this call allocates and
 * frees; the fastest of four timed steps counts.  A larger radix (larger keys) must be faster by
 * 2 % to be chosen.  Sets the spec's radix to the winner and returns it in
 * *best_bits; results are cached in `cache_path` (may be NULL) keyed by the
 * spec, sizes and device.  Keys generated afterwards use the chosen radix. */
int fss_autotune_radix(fss_spec* spec, int32_t n_bits, int32_t frac_bits, int64_t n_elems, const char* cache_path,
                       int32_t* best_bits);

/* ---- the literal interval lookup (Definition "Interval lookup with vector
 * payload"; Appendix "Full Compilation Protocol", Protocol "Compile a scalar
 * gate instance to two backend primitive instances", steps (1) and (5)) ----
 *
 * The lookup as the compilation protocol builds it, for comparison with the
 * single-key lookup of fss_keygen / fss_eval: per element, the partition of
 * the lookup view v = (xhat + c) mod 2^n translated by the mask, padded to
 * M = min(m + 1, 2^n) intervals, one vector DCF (2^r children per level, the
 * spec's lookup radix) per inner boundary B_j with payload v_{j-1} - v_j,
 * and shares of v_{M-1}; v_j is the ring coefficient vector (x-space, p
 * words) of the piece that interval j maps to.  Evaluation returns additive
 * shares of the active piece's coefficients (the constant term's share
 * includes the party's share of r_out) and of x = xhat - r_in; the
 * polynomial is then evaluated on shares by Horner's rule with one Beaver
 * multiplication per degree (fss_triples, fss_beaver_mask, fss_open,
 * fss_beaver_mul).  Keys are one-time like the operator gate's.  Built for
 * AES table layout 1. */

/* Bytes of one party's literal key buffer for n_elems elements. */
int fss_lit_key_bytes(const fss_spec* spec, int32_t n_bits, int32_t frac_bits, int64_t n_elems, size_t* bytes);
/* Dealer: both parties' literal keys (key1 may be NULL), with r_in and r_out
 * (device, n_elems u64 each, may be NULL) drawn exactly as fss_keygen draws
 * them from the same seed. */
int fss_lit_keygen(const fss_spec* spec, int32_t n_bits, int32_t frac_bits, const uint8_t* seed, int64_t n_elems,
                   void* key0, void* key1, uint64_t* r_in, uint64_t* r_out, void* stream);
/* Party `party`'s shares: coef (device, p * n_elems u64; coefficient k of
 * element e at k * n_elems + e) and x_share (device, n_elems u64). */
int fss_lit_eval(int32_t party, const void* keys, const uint64_t* xhat, int64_t n_elems, uint64_t* coef,
                 uint64_t* x_share, void* stream);

/* ---- post-processing subprotocols (Sec. "Standard Preprocessing
 * Subprotocols": Beaver multiplication over Z_2^64, AND on XOR shares; Sec.
 * "Mixed-Domain Conversions": B2A) -------------------------------------------
 *
 * All buffers are device arrays.  The dealer's correlations are drawn from
 * its 16-byte seed, per element (or 64-bit word) index i and `step` in
 * [0, 65535], so that several gates can use one seed.  A party's local steps
 * run before and after the opening; fss_open (additive) and fss_xopen (XOR)
 * are the openings, both parties' shares being on this device. */

/* Beaver triples for n products: a, b uniform, c = a b, additively shared. */
int fss_triples(const uint8_t* seed, int64_t n, int32_t step, uint64_t* a0, uint64_t* b0, uint64_t* c0,
                uint64_t* a1, uint64_t* b1, uint64_t* c1, void* stream);
/* A party's masked shares d = u - a and e = v - b (to be opened). */
int fss_beaver_mask(const uint64_t* u, const uint64_t* v, const uint64_t* a, const uint64_t* b, int64_t n,
                    uint64_t* d, uint64_t* e, void* stream);
/* A party's share of u v from the openings d, e: c + d b + e a (+ d e for
 * party 0), plus `add` (a share to add, may be NULL). */
int fss_beaver_mul(int32_t party, const uint64_t* d, const uint64_t* e, const uint64_t* a, const uint64_t* b,
                   const uint64_t* c, const uint64_t* add, int64_t n, uint64_t* z, void* stream);
/* AND triples for `words` 64-bit words of independent bits, XOR-shared. */
int fss_and_triples(const uint8_t* seed, int64_t words, int32_t step, uint64_t* a0, uint64_t* b0, uint64_t* c0,
                    uint64_t* a1, uint64_t* b1, uint64_t* c1, void* stream);
/* d = x ^ a and, if y is not NULL, e = y ^ b (a party's masked bit words). */
int fss_xor_mask(const uint64_t* x, const uint64_t* a, const uint64_t* y, const uint64_t* b, int64_t words,
                 uint64_t* d, uint64_t* e, void* stream);
/* The XOR opening: out = s0 ^ s1. */
int fss_xopen(const uint64_t* s0, const uint64_t* s1, int64_t words, uint64_t* out, void* stream);
/* A party's XOR share of x & y from the openings d, e: c ^ (d & b) ^ (e & a)
 * (^ d & e for party 0). */
int fss_and(int32_t party, const uint64_t* d, const uint64_t* e, const uint64_t* a, const uint64_t* b,
            const uint64_t* c, int64_t words, uint64_t* z, void* stream);
/* B2A correlation for n bits: a uniform bit t per element, XOR-shared in
 * bit words t0 / t1 (ceil(n / 64) words, bit i of word i / 64) and
 * additively shared in T0 / T1 (n words). */
int fss_b2a_rand(const uint8_t* seed, int64_t n, int32_t step, uint64_t* t0, uint64_t* t1, uint64_t* T0,
                 uint64_t* T1, void* stream);
/* A party's additive share of bit z from the opened c = z ^ t (bit words):
 * z = c + (1 - 2c) t. */
int fss_b2a(int32_t party, const uint64_t* c, const uint64_t* T, int64_t n, uint64_t* out, void* stream);

/* ---- status ------------------------------------------------------------ */

/* Synchronise `stream`, then read and clear the device status word.
 * *device_code receives 0 or the FSS_E_* code a kernel recorded. */
int fss_status(void* stream, int32_t* device_code);
const char* fss_last_error(void);
/* Library version string. */
const char* fss_version(void);

#ifdef __cplusplus
}
#endif
#endif
