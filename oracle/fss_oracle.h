/*
 * fss_oracle.h -- plain CPU oracle for the FuseFSS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; only
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant generator with the GPU path.
 *
 * What it computes (paper sections in brackets):
 *   - AES-128 from FIPS-197, byte oriented, S-box derived from GF(2^8)
 *     inversion + the affine map.
 *   - A fixed-key AES PRG (tweaked Matyas-Meyer-Oseas) and a counter-based
 *     randomness source keyed by the dealer seed.
 *   - The distributed comparison function of Boyle et al. (EUROCRYPT 2021),
 *     cited by the paper for its backend [Backend Interface appendix], with
 *     payload group Z_2 (predicates) or Z_{2^64}^p (coefficient lookup).
 *   - Operator-specification quantisation [Definition "Operator
 *     specification", Sec. 3.2 fixed-point encoding].
 *   - Dealer key generation and per-party evaluation of the packed
 *     comparison [Lemma "Masked rewrite for unsigned comparison", signed /
 *     MSB appendix, low-bit appendix] and of the vector interval lookup
 *     [Definition "Interval lookup with vector payload"], followed by the
 *     local combination at the public masked input.
 *   - Protocol "Compile a scalar gate instance" (translated lookup table),
 *     used only to cross-check the lookup.
 *   - A plaintext evaluator of the quantised specification.
 */
#ifndef FSS_ORACLE_H
#define FSS_ORACLE_H
#include <stdint.h>

#define ORC_MAXN 32   /* comparison bit width n */
#define ORC_MAXP 4    /* payload length p = d + 1 */
#define ORC_MAXM 64   /* intervals m */
#define ORC_MAXPRED 16 /* primitive predicates */
#define ORC_MAXT 16    /* comparison atoms */
#define ORC_MAXL 64    /* predicate output bits (one 64-bit word) */

typedef struct { uint64_t lo, hi; } orc_blk;

typedef struct { uint8_t rk[176]; } orc_aes_sched;

/* ---- AES / PRG / randomness --------------------------------------------- */
void orc_aes128_expand(const uint8_t key[16], orc_aes_sched* ks);
void orc_aes128_encrypt(const orc_aes_sched* ks, const uint8_t in[16], uint8_t out[16]);
void orc_aes128_encrypt_key(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]);
void orc_sbox(uint8_t out[256]);
/* H(s, j) = AES_K(s ^ J_j) ^ s ^ J_j with the fixed PRG key. */
orc_blk orc_prg(orc_blk s, int j);
/* K_seed: the AES-128 key schedule of the dealer's 16-byte seed. */
void orc_seed_sched(const uint8_t seed[16], orc_aes_sched* ks);
/* R(e, purpose, ctr) = AES_{K_seed}(e || purpose || ctr || 0). */
orc_blk orc_rand(const orc_aes_sched* kseed, uint64_t e, int purpose, int ctr);

/* ---- DCF ------------------------------------------------------------------ */
/* group: p == 0 means Z_2 (one bit, XOR); p in 1..4 means Z_{2^64}^p. */
typedef struct {
  int32_t n, p;
  orc_blk root;                     /* this party's root seed (bits 0..1 zero) */
  orc_blk scw[ORC_MAXN];            /* seed corrections (bits 0..1 zero) */
  uint8_t tl[ORC_MAXN], tr[ORC_MAXN];
  uint64_t vcw[ORC_MAXN][ORC_MAXP]; /* value corrections (Z_2: vcw[i][0] in {0,1}) */
  uint64_t fin[ORC_MAXP];           /* final correction */
} orc_dcf_key;

void orc_dcf_gen(int n, int p, uint64_t alpha, const uint64_t* beta,
                 orc_blk root0, orc_blk root1, orc_dcf_key* k0, orc_dcf_key* k1);
void orc_dcf_eval(int b, const orc_dcf_key* k, uint64_t x, uint64_t* out);

/* ---- Z_2 DCF with early termination -------------------------------------- */
/* f(x) = 1[x < alpha] over n bits, the construction above (p = 0, beta = 1)
 * on the high n - nu bits, nu = min(7, n), with each leaf seed s converted
 * into the 128-bit vector H(s, 2): the output at x is the XOR of the path's
 * values and bit (x mod 2^nu) of the leaf vector (plus the leaf correction
 * when the control bit is set).  At alpha's leaf the correction makes the two
 * parties' vectors XOR to (1[j < alpha mod 2^nu])_j; at every other leaf the
 * parties' seeds agree and their vectors cancel.  Evaluation walks n - nu
 * levels and one conversion block. */
typedef struct {
  int32_t n, nu;
  orc_blk root;                     /* this party's root seed (bits 0..1 zero) */
  orc_blk scw[ORC_MAXN];            /* levels 0 .. n - nu - 1 */
  uint8_t tl[ORC_MAXN], tr[ORC_MAXN], vcw[ORC_MAXN];
  orc_blk leaf;                     /* the leaf correction (bit j: low input bits j) */
} orc_dcfz_key;

int orc_dcfz_nu(int n);
void orc_dcfz_gen(int n, uint64_t alpha, orc_blk root0, orc_blk root1, orc_dcfz_key* k0, orc_dcfz_key* k1);
int orc_dcfz_eval(int b, const orc_dcfz_key* k, uint64_t x);

/* ---- DCF with 2^r children per level --------------------------------------- */
/* The same construction with r input bits (one base-2^r digit) per level, r in
 * {2, 3, 4}: each level has 2^r children, and the key carries a seed,
 * control-bit and value correction for each child.  For a child off alpha's
 * path they are the corrections above (with beta entering when that child's
 * digit is below alpha's); for the child on the path they are fresh dealer
 * randomness (`keep_rand`, 1 + ceil(p/2) blocks per level, the last level's
 * unused), so the key does not show which child alpha takes.  At the last
 * level alpha's child gets the equalising value correction as well (without
 * beta): it cancels the sum along alpha's path, so there is no leaf
 * conversion and no final correction; the last level's seed and control-bit
 * corrections are never used and are zero.  The input is walked as
 * r * ceil(n / r) bits with leading zeros.  Child c of seed s is H(s, c)
 * (seed and control bit); its value is words c p .. c p + p - 1 of the
 * stream H(s, 2^r), H(s, 2^r + 1), ... (two 64-bit words per block). */
#define ORC_MAXLR ((ORC_MAXN + 1) / 2) /* levels at r = 2 */
#define ORC_MAXC 16                    /* children at r = 4 */
typedef struct {
  int32_t n, p, r;                      /* levels = ceil(n / r) */
  orc_blk root;
  orc_blk scw[ORC_MAXLR][ORC_MAXC];            /* seed corrections (bits 0..1 zero) */
  uint8_t tcw[ORC_MAXLR][ORC_MAXC];            /* control-bit corrections */
  uint64_t vcw[ORC_MAXLR][ORC_MAXC][ORC_MAXP]; /* value corrections */
} orc_dcfr_key;

void orc_dcfr_gen(int n, int r, int p, uint64_t alpha, const uint64_t* beta, orc_blk root0, orc_blk root1,
                  const orc_blk* keep_rand, orc_dcfr_key* k0, orc_dcfr_key* k1);
void orc_dcfr_eval(int b, const orc_dcfr_key* k, uint64_t x, uint64_t* out);

/* ---- operator specification ------------------------------------------------ */
typedef struct { double lo, hi; } orc_interval;
typedef struct { int32_t degree; double coef[4]; } orc_piece;
enum { ORC_LT_SIGNED = 0, ORC_LT_UNSIGNED = 1, ORC_LOWBITS_LT = 2, ORC_MSB_SHIFT = 3 };
typedef struct {
  int32_t kind, negate, out, f_bits;
  double thr;      /* real threshold for LT_SIGNED / LT_UNSIGNED */
  int64_t gamma;   /* integer threshold for LOWBITS_LT */
  int64_t c;       /* public shift for MSB_SHIFT */
} orc_pred;

typedef struct {
  int32_t n, f, m, d, p, F_out, ell;
  int64_t alpha[ORC_MAXM + 1];          /* signed integer boundaries, alpha[0]=-s, alpha[m]=s */
  uint64_t aprime[ORC_MAXM + 1];        /* offset-binary boundaries alpha + s */
  uint64_t coef[ORC_MAXM][ORC_MAXP];    /* ring coefficients, lowest degree first */
  /* user predicates, quantised, evaluated directly by the plaintext path */
  int32_t n_user;
  int32_t u_kind[ORC_MAXPRED], u_out[ORC_MAXPRED], u_neg[ORC_MAXPRED], u_f[ORC_MAXPRED];
  int64_t u_beta[ORC_MAXPRED];          /* signed beta / unsigned beta / gamma */
  uint64_t u_c[ORC_MAXPRED];
  /* compiled (masked) predicate form */
  int32_t n_prim;                       /* non-constant primitive predicates */
  int32_t prim_k[ORC_MAXPRED], prim_view[ORC_MAXPRED], prim_out[ORC_MAXPRED];
  uint64_t prim_bprime[ORC_MAXPRED];    /* threshold in view space */
  int32_t n_views;
  int32_t view_k[ORC_MAXPRED];
  uint64_t view_c[ORC_MAXPRED];
  int32_t T;                            /* atoms: n_prim thresholds, then the mask atoms of the
                                           views other than lookup_view */
  uint8_t negate[ORC_MAXL];             /* public constant flip per output bit */
  int32_t lookup_r;                     /* input bits per level of call 2's DCF (2, 3 or 4) */
  int32_t is_int;                       /* 1: integer spec over canonical representatives */
  uint64_t lookup_c;                    /* public shift of the lookup's view: 2^(n-1) or 0 */
  /* The view whose mask query 1[view < r_k] is the lookup's own comparison
   * 1[v < r_n] (k = n, c = lookup_c), or -1: that query has no atom of its
   * own; its bit is the lookup DCF's first output at v reduced mod 2. */
  int32_t lookup_view;
} orc_spec;

/* Returns 0 on success, negative on an invalid or unsupported spec.  Sets
 * lookup_r = 3; a caller may change it before keygen. */
int orc_spec_compile(const orc_interval* iv, int32_t m, const orc_piece* pc,
                     const orc_pred* pr, int32_t n_pred, int32_t n_bits,
                     int32_t frac_bits, int32_t out_frac_bits, orc_spec* S);

/* Integer form of the Definition: boundaries alpha[0..m] with 0 = alpha_0 <
 * ... < alpha_m = 2^n over canonical representatives, ring coefficients
 * coef[i * (degree + 1) + l] (lowest degree first), predicate thresholds
 * given as integers.  Returns 0 or a negative code like orc_spec_compile. */
int orc_spec_compile_int(int32_t n_bits, int32_t m, const uint64_t* alpha, int32_t degree,
                         const uint64_t* coef, const orc_pred* pr, int32_t n_pred, orc_spec* S);

/* ---- per-element keys ------------------------------------------------------- */
typedef struct {
  orc_dcfz_key atom[ORC_MAXT];
  uint64_t wshare;                      /* bit j: this party's share of the carry of output j */
  orc_dcfr_key coeff;                   /* call 2's vector DCF, 2^r children per level */
  uint64_t rho[ORC_MAXP];               /* additive share of rho = ((-r_in)^k)_k */
  uint64_t rout;                        /* additive share of r_out */
} orc_elem_key;

void orc_keygen_elem(const orc_spec* S, const orc_aes_sched* kseed, uint64_t e,
                     orc_elem_key* k0, orc_elem_key* k1, uint64_t* r_in, uint64_t* r_out);
void orc_eval_elem(int b, const orc_spec* S, const orc_elem_key* K, uint64_t xhat,
                   uint64_t* y, uint64_t* zbits);
/* Plaintext fixed-point evaluation of the quantised spec at signed x. */
void orc_plain_eval(const orc_spec* S, int64_t x, uint64_t* y, uint64_t* zbits);

/* Batched drivers over a list of element indices (threads: 0 = all cores). */
int orc_keygen_batch(const orc_spec* S, const uint8_t seed[16], const int64_t* elems, int64_t count,
                     orc_elem_key* k0, orc_elem_key* k1, uint64_t* r_in, uint64_t* r_out,
                     int threads);
int orc_eval_batch(int b, const orc_spec* S, const orc_elem_key* K, const uint64_t* xhat,
                   int64_t count, uint64_t* y, uint64_t* zbits, int threads);
/* keygen + both parties' evaluation without storing keys (CPU baseline and
 * full-size parity checks); r_in / r_out may be NULL. */
int orc_full_batch(const orc_spec* S, const uint8_t seed[16], const int64_t* elems, int64_t count,
                   const int64_t* x, uint64_t* y0, uint64_t* y1, uint64_t* z0, uint64_t* z1,
                   uint64_t* r_in, uint64_t* r_out, int threads);
int orc_hw_threads(void);
/* AES-128 blocks the batched drivers have encrypted so far (all threads). */
uint64_t orc_aes_blocks(void);
int orc_sizeof_elem_key(void);
int orc_sizeof_dcf_key(void);
int orc_sizeof_dcfz_key(void);
int orc_sizeof_dcfr_key(void);
int orc_sizeof_spec(void);

/* ---- rescaling gate: ARS of a masked 64-bit value ------------------------- */
/* Input: the opening yhat = y + r_in of a signed y, |y| < 2^62, masked by the
 * previous gate's output mask r_in.  Output: additive shares of
 * floor(y / 2^s) + r_out, 1 <= s <= 32.  Key: a DCF with payload -1 over the
 * s low bits (2^r children per level, r in {2, 3, 4}) at alpha = r_in mod 2^s,
 * and additive shares of k0 = r_out - (r_in >> s) and k1 = 2^(64-s) MSB(r_in).
 * Randomness R(e, .): purpose 0 -> r_out (lo), 1 -> party-0 shares of k0 (lo)
 * and k1 (hi), 64 / 65 -> DCF roots, 69 + k -> on-path corrections. */
typedef struct {
  orc_dcfr_key dcf;
  uint64_t k0, k1;
} orc_trunc_key;

uint64_t orc_ars(int64_t y, int s);
void orc_trunc_keygen_elem(int s, int r, const orc_aes_sched* kseed, uint64_t e, uint64_t r_in,
                           orc_trunc_key* k0, orc_trunc_key* k1, uint64_t* r_out);
uint64_t orc_trunc_eval_elem(int b, int s, const orc_trunc_key* K, uint64_t yhat);
/* Keygen at the given r_in and both parties' evaluation at yhat, per element. */
int orc_trunc_batch(int s, int r, const uint8_t seed[16], const int64_t* elems, int64_t count,
                    const uint64_t* r_in, const uint64_t* yhat, uint64_t* z0, uint64_t* z1, uint64_t* r_out,
                    int threads);

/* ---- Protocol "Compile a scalar gate instance", lookup part ---------------- */
/* alpha: boundaries 0=a_0<...<a_m=N of the partition being translated; r: mask.
 * Writes B[0..M] and ord[0..M-1] (B needs room for m + 2 entries); returns M. */
int orc_protocol3(int n, const uint64_t* alpha, int m, uint64_t r, uint64_t* B, int32_t* ord);

/* ---- literal interval lookup (Definition "Interval lookup with vector payload",
 * built as the compilation protocol's steps (1) and (5) state it) ------------- */
/* For the lookup view v = (xhat + lookup_c) mod 2^n and the element's mask,
 * the partition (B, ord) of v-space from orc_protocol3 and payload v_j = the
 * ring coefficients of piece ord_j (x-space, lowest degree first):
 * LUT(v) = v_{M-1} + sum_{j=1}^{M-1} (v_{j-1} - v_j) 1[v < B_j], one vector
 * DCF (2^r children per level) per inner boundary.  Randomness R(e, ., .) of
 * the dealer seed: 0 -> r_in, r_out; 1 -> party 0's r_out share; 200 ->
 * party 0's r_in share; 201 / 202 (ctr j) -> roots of DCF j; 203 + k
 * (ctr 64 j + level) -> its on-path corrections; 210, 211 -> party 0's
 * share of v_{M-1}. */
typedef struct {
  int32_t M;                  /* intervals after padding; M - 1 DCFs */
  orc_dcfr_key dcf[ORC_MAXM]; /* DCF of boundary B_j at index j - 1 */
  uint64_t base[ORC_MAXP];    /* additive share of v_{M-1} */
  uint64_t rin, rout;         /* additive shares of r_in and r_out */
} orc_lit_key;

int orc_lit_keygen_elem(const orc_spec* S, const orc_aes_sched* kseed, uint64_t e, orc_lit_key* k0,
                        orc_lit_key* k1, uint64_t* r_in, uint64_t* r_out);
/* Party b's additive shares of the active piece's coefficients (p words; the
 * constant term's share includes the party's r_out share) and of
 * x = xhat - r_in. */
void orc_lit_eval_elem(int b, const orc_spec* S, const orc_lit_key* K, uint64_t xhat, uint64_t* coef,
                       uint64_t* x_share);

/* ---- post-processing subprotocols (Sec. "Standard Preprocessing Subprotocols",
 * Sec. "Mixed-Domain Conversions") ------------------------------------------ */
/* Beaver triple for multiplication `step` of element e: a, b uniform, c = a b
 * mod 2^64, additively shared.  R(e, 220, step) -> (a, b); R(e, 221, step)
 * -> party 0's shares of (a, b); R(e, 222, step).lo -> party 0's share of c. */
void orc_triple(const orc_aes_sched* kseed, uint64_t e, int step, uint64_t a[2], uint64_t b[2], uint64_t c[2]);
/* Party `party`'s share of u v from the opened d = u - a and e = v - b. */
uint64_t orc_beaver_mul(int party, uint64_t d, uint64_t e, uint64_t a, uint64_t b, uint64_t c);
/* AND triple for word w (64 independent bits): a, b uniform, c = a & b,
 * XOR-shared.  R(w, 230, step) -> (a, b); R(w, 231, step) -> party 0's
 * shares of (a, b); R(w, 232, step).lo -> party 0's share of c. */
void orc_and_triple(const orc_aes_sched* kseed, uint64_t w, int step, uint64_t a[2], uint64_t b[2], uint64_t c[2]);
/* Party `party`'s XOR share of x & y from the opened d = x ^ a, e = y ^ b. */
uint64_t orc_and(int party, uint64_t d, uint64_t e, uint64_t a, uint64_t b, uint64_t c);
/* B2A randomness for element e: a uniform bit t, XOR-shared (t_0 from
 * R(e, 241, step).lo bit 0) and additively shared (T_0 = R(e, 241, step).hi),
 * t = R(e, 240, step).lo bit 0. */
void orc_b2a_rand(const orc_aes_sched* kseed, uint64_t e, int step, uint64_t tbit[2], uint64_t T[2]);
/* Party `party`'s additive share of bit z from the opened c = z ^ t:
 * z = c + (1 - 2c) t. */
uint64_t orc_b2a(int party, uint64_t c, uint64_t T);

/* The paper's lookup-plus-post-processing pipeline for `count` elements:
 * literal lookup keys, both parties' coefficient shares at xhat = x + r_in,
 * then Horner's rule on the shares with one Beaver multiplication per degree
 * (triple `step` t of element e for the t-th multiplication, openings between
 * the parties); the r_out shares ride in the constant term, so
 * y0 + y1 = P(x) + r_out.  coef0 / coef1: count * p words (element-major),
 * may be NULL. */
int orc_lit_batch(const orc_spec* S, const uint8_t seed[16], const int64_t* elems, int64_t count,
                  const int64_t* x, uint64_t* coef0, uint64_t* coef1, uint64_t* y0, uint64_t* y1,
                  uint64_t* r_in, uint64_t* r_out, int threads);

#endif
