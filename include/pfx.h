/*
 * pfx — RNS-CKKS homomorphic evaluation on AMD Instinct MI355X (gfx950).
 *
 * C-ABI of libpfx.so.  Plain pointers and sizes only.  The calls follow the
 * roles of the paper's private database exploration (arXiv 2412.13269, Sec. 3
 * and Sec. 5.5, Alg. 2): the scientist creates keys, encrypts and decrypts;
 * the database owner evaluates on ciphertexts.  The scheme is RNS-CKKS with
 * hybrid key switching (Sec. 2.3-2.5, App. A).
 *
 * Conventions
 * -----------
 * Status: every call returns PFX_OK (0) or a negative PFX_E* code; on error the
 *   outputs are untouched and pfx_last_error() (thread-local) describes it.
 * Ownership: objects come back through out-parameters; the caller frees them
 *   with the matching pfx_*_destroy.  Host arrays are borrowed for the call.
 * Device work: evaluation calls are enqueued on `stream` (a hipStream_t, NULL
 *   for the default stream) and return before the device finishes.  An object
 *   must outlive the stream work that reads it.  Outputs may alias inputs.
 *   Calls that share a context and run on different streams each use that
 *   stream's own scratch space; they are safe as long as they do not write
 *   the same objects.
 * Interchange words: uint64 residues in [0, q_i), COEFFICIENT domain, natural
 *   coefficient order, limb-major: word (k, i, c) of a ciphertext sits at
 *   ((k * n_limbs) + i) * N + c for polynomial k, limb i (prime q_i),
 *   coefficient c.  On the device the library keeps its own representation
 *   (NTT domain, residues held as exact FP64 integers); exported words are
 *   canonical and bit-comparable.
 * Randomness: the library draws nothing.  The secret key, the uniform
 *   polynomials `a` and the errors `e` of encryption and key generation
 *   (Sec. 2.3, Sec. 2.4.1) are inputs supplied by the caller.
 * Moduli: every prime is below 2^50 and 1 mod 2^mod_log2 (see pfx_params).
 */
#ifndef PFX_H
#define PFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pfx_status;
#define PFX_OK 0
#define PFX_EINVAL (-1)  /* bad argument, size or pointer */
#define PFX_EPARAM (-2)  /* parameter set not supported */
#define PFX_ELEVEL (-3)  /* too few limbs for the operation */
#define PFX_ESCALE (-4)  /* operand scales differ by more than 2^-10 relative */
#define PFX_ENOKEY (-5)  /* no key for the needed Galois element */
#define PFX_ENOMEM (-6)  /* device allocation failed or budget exceeded */
#define PFX_EBUSY (-7)   /* server did not admit the request (retry later) */
#define PFX_EDEVICE (-8) /* HIP runtime error or no usable gfx950 device */

#define PFX_MAX_PRIMES 64
#define PFX_MAX_LOGN 16
#define PFX_MIN_LOGN 4

/*
 * Parameter set (Sec. 6.1, Tab. 1 gives the paper's sets by bit sizes only).
 * Ciphertext primes q_0..q_{n_q-1}, special primes p_0..p_{n_p-1} (the
 * modulus P of hybrid key switching, Sec. 2.4.1).  Prime rule: every prime is
 * 1 mod 2^mod_log2 (0 means log_n + 1); a prime of 50 bits is the next unused
 * prime below 2^50, a smaller one the next unused prime nearest 2^bits
 * (offsets 0, +1, -1, +2, ... multiples of 2^mod_log2); q's are chosen first,
 * in order, then p's.  Bit sizes must lie in [20, 50]; at most 7 special primes
 * (device contexts).  alpha (<= 8) = primes per
 * key-switching digit; digit j holds primes [alpha*j, alpha*j + alpha).
 */
typedef struct pfx_params {
    uint32_t log_n;
    uint32_t n_q;
    uint32_t q_bits[PFX_MAX_PRIMES];
    uint32_t n_p;
    uint32_t p_bits[PFX_MAX_PRIMES];
    uint32_t alpha;
    uint32_t mod_log2;
} pfx_params;

typedef struct pfx_info {
    uint32_t log_n;
    uint32_t n_limbs;
    uint32_t degree; /* 0 plaintext, 1 ciphertext, 2 after a product */
    double scale;
} pfx_info;

typedef struct pfx_ctx pfx_ctx;
typedef struct pfx_sk pfx_sk;
typedef struct pfx_swk pfx_swk;
typedef struct pfx_ct pfx_ct; /* ciphertexts and plaintexts (degree 0) */
typedef struct pfx_ct pfx_pt;

const char *pfx_status_str(pfx_status s);
const char *pfx_last_error(void);

/* Host only, no device needed: the primes q, p and the roots psi (2N-th,
 * one per prime, q's then p's) that pfx_ctx_create would choose.  Arrays of
 * n_q, n_p and n_q + n_p entries. */
pfx_status pfx_params_primes(const pfx_params *prm, uint64_t *q, uint64_t *p, uint64_t *psi);

/* Host only: the words of pfx_encode (n_limbs * N canonical residues,
 * coefficient domain) without a device. */
pfx_status pfx_encode_words(const pfx_params *prm, const double *re, const double *im, size_t n_slots,
                            uint32_t n_limbs, double scale, uint64_t *words);
/* Host only: pfx_decode of canonical coefficient-domain words. */
pfx_status pfx_decode_words(const pfx_params *prm, const uint64_t *words, uint32_t n_limbs,
                            double scale, double *re, double *im, size_t n_slots);

/* ------------------------------------------------------------------ context */
pfx_status pfx_ctx_create(const pfx_params *prm, int hip_device, pfx_ctx **out);
void pfx_ctx_destroy(pfx_ctx *ctx);

/*
 * Device memory of a context.  Every device allocation the library makes for
 * the context after pfx_ctx_create's own tables (twiddles and conversion
 * constants) goes through one path: ciphertexts and plaintexts, keys, the
 * per-stream scratch and its batch and repacking regions, the temporaries of
 * key generation and export, pfx_dev_alloc, and a request server's arena.
 *   alloc(bytes, stream, user) returns device memory of the context's device
 *   (NULL when it cannot), free(p, stream, user) gives it back; stream is the
 *   stream the memory is first used on or NULL.  Both NULL: hipMalloc/hipFree.
 *   hbm_budget: bytes the context may hold at once, counted from creation
 *   (tables included, pfx_ctx_mem); 0 = no cap.  An allocation that would
 *   exceed it, or that the allocator refuses, fails the call with PFX_ENOMEM
 *   and leaves its outputs untouched.
 * Memory is freed by the allocator that made it, so the allocator may be
 * changed at any time; a budget below what the context already holds only
 * refuses further allocations.  Not thread-safe against calls running on the
 * context.  user is passed through unchanged.
 */
typedef void *(*pfx_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*pfx_free_fn)(void *p, void *stream, void *user);
pfx_status pfx_ctx_set_allocator(pfx_ctx *ctx, pfx_alloc_fn alloc, pfx_free_fn free_fn, void *user,
                                 size_t hbm_budget);
/* Bytes of device memory the context holds now and at most so far. */
pfx_status pfx_ctx_mem(const pfx_ctx *ctx, size_t *in_use, size_t *peak);

/*
 * Launch geometry of the NTT passes per ring degree (process-wide; every
 * context of that degree uses it, graphs captured earlier keep theirs):
 *   row_wg256 / col_wg256: a row / column pass takes 256-thread workgroups
 *     when that gives at least this many of them, 128 otherwise;
 *   widen_wg: launches over few limbs (standalone passes, the special-prime
 *     INTT of key switching) narrow their tiles until they have this many
 *     workgroups, down to min_col columns (min_col_special for the
 *     special-prime INTT; powers of two);
 *   rs_widen_wg: the same for the INTT of a rescale's dropped limb;
 *   ks_fuse: key switches (other than hoisted automorphisms and repacking
 *     rounds) run the ModUp row pass, the key inner product and the first
 *     pass of the special-prime INTT as one launch of ks_fuse threads per
 *     workgroup (128 or 256); 0 keeps them separate launches;
 *   ks_batch: batched key switches (pfx_rotate_batch, pfx_apply_galois_batch,
 *     pfx_mul_relin_batch, pfx_relinearize_batch) split a run of entries of
 *     one level into batches of at most ks_batch (1..8) entries, as equal in
 *     size as possible;
 *   ks_modup_batch: inside a batched key switch the ModUp conversion, its row
 *     pass and the inner product run for this many entries at a time (0: the
 *     whole batch), so that the ModUp limbs stay in the last-level cache from
 *     one launch to the next.
 * Defaults {2048, 0, 1024, 16, 8, 256, 0, 8, 0}.  The geometry never changes
 * a result, only its speed.  pfx_tuning_load reads lines "log_n row_wg256
 * col_wg256 widen_wg min_col min_col_special rs_widen_wg [ks_fuse [ks_batch
 * [ks_modup_batch]]]"
 * ('#' starts a comment line; fields left out keep their defaults);
 * the first pfx_ctx_create loads tuning.txt next to libpfx.so if there is one
 * (the package's autotuner writes it).
 */
typedef struct pfx_pass_tuning {
    uint32_t log_n;
    uint32_t row_wg256, col_wg256, widen_wg, min_col, min_col_special, rs_widen_wg;
    uint32_t ks_fuse, ks_batch, ks_modup_batch;
} pfx_pass_tuning;
pfx_status pfx_tuning_set(const pfx_pass_tuning *t);
pfx_status pfx_tuning_get(uint32_t log_n, pfx_pass_tuning *t);
pfx_status pfx_tuning_reset(void);
pfx_status pfx_tuning_load(const char *path);
pfx_status pfx_ctx_moduli(const pfx_ctx *ctx, uint64_t *q, uint64_t *p, uint64_t *psi);
/* Blocks until all work the library enqueued on `stream` has finished. */
pfx_status pfx_sync(pfx_ctx *ctx, void *stream);

/* ---------------------------------------------------------- scientist side */
/* Secret key from its N coefficients in {-1, 0, 1} (Sec. 2.3). */
pfx_status pfx_sk_create(pfx_ctx *ctx, const int8_t *s, pfx_sk **out);
void pfx_sk_destroy(pfx_sk *sk);

/*
 * Switching key (Sec. 2.4.1 SwitchKeyGen): for each digit j < beta,
 *   swk_j = (-a_j s + e_j + P w_j s_from, a_j)  over all n_q + n_p primes,
 * w_j the CRT idempotent of digit j over the full Q.  galois = 0 builds the
 * relinearisation key (s_from = s^2, App. A.2); an odd galois element g < 2N
 * builds the key for phi_g (s_from = phi_g(s)), used by rotation (g = 5^k mod
 * 2N rotates slots left by k, App. A.1) and conjugation (g = 2N - 1).
 *   a: beta * (n_q + n_p) * N words, [j][prime][coefficient], each < its prime.
 *   e: beta * N integers, [j][coefficient].
 */
pfx_status pfx_swk_create(pfx_ctx *ctx, const pfx_sk *sk, uint32_t galois, const uint64_t *a,
                          const int64_t *e, pfx_swk **out);
/* The same with an arbitrary s_from (N integer coefficients, host): the key
 * of ring switching (Sec. 3.3), from the secret of a smaller ring embedded in
 * this one (s_small(X^(N/n)), coefficient j N/n = s_small[j]) to sk.  Such a
 * key is neither a relinearisation nor a Galois key (PFX_ENOKEY there); a, e as
 * for pfx_swk_create. */
pfx_status pfx_swk_create_from(pfx_ctx *ctx, const pfx_sk *sk, const int8_t *s_from, const uint64_t *a,
                               const int64_t *e, pfx_swk **out);
/* Words [j][t][prime][coefficient], t = 0 for the b part, 1 for a. */
pfx_status pfx_swk_export(pfx_ctx *ctx, const pfx_swk *k, uint64_t *words, size_t cap_words);
/* A switching key from the words pfx_swk_export writes (canonical residues,
 * coefficient domain, beta * 2 * (n_q + n_p) * N of them, each below its
 * prime: PFX_EINVAL otherwise), for Galois element `galois` (0: a
 * relinearisation key).  Word for word the exported key. */
pfx_status pfx_swk_import(pfx_ctx *ctx, uint32_t galois, const uint64_t *words, size_t n_words, pfx_swk **out);
uint32_t pfx_swk_galois(const pfx_swk *k);
void pfx_swk_destroy(pfx_swk *k);
/* The secret's N coefficients in {-1, 0, 1} (the scientist's copy, host). */
pfx_status pfx_sk_export(const pfx_sk *sk, int8_t *s, size_t n);

/*
 * Seeded key generation and encryption (Sec. 2.3, Sec. 2.4.1), drawing their
 * randomness on the host from SHAKE-256 (FIPS 202) streams keyed by
 *   seed (32 bytes) || tag || index || limb   (little-endian uint32 each):
 *   uniform below m: 8-byte little-endian words masked to bitlen(m - 1) bits,
 *     rejected while >= m;
 *   uniform ternary: bytes b, v = b & 3 rejected while 3; 0, 1, 2 -> 0, +1, -1;
 *   h-sparse ternary: positions 0..N-1, for i < h swap entry i with entry
 *     i + u (u uniform below N - i); then one byte per chosen position in
 *     order, bit 0 its sign (0: +1, 1: -1);
 *   discrete Gaussian, sigma 3.2, |e| <= 19: the cumulative table T[k] =
 *     floor(2^63 P(|X| <= k)), k < 19 (weights exp(-k^2 / 2 sigma^2), doubled
 *     for k > 0, summed in order in FP64), T[19] = 2^63; u = word >> 1, |e| the
 *     least k with u < T[k]; a non-zero |e| takes bit 0 of one more byte as
 *     its sign.
 * Tags: 1 the secret (index 0); 2 a switching key's a (index 256 g + j for
 * Galois element g, 0 for relinearisation, digit j; limb the prime index over
 * Q then P); 3 its error (index as for a, limb 0); 4 an encryption's a (index
 * 0, limb the prime index); 5 its error (index 0, limb 0).  Equal seeds give
 * equal keys and ciphertexts, word for word, on any device.
 */
/* Secret with h non-zero coefficients (h < 0: uniform ternary, Sec. 2.3). */
pfx_status pfx_keygen_secret(pfx_ctx *ctx, const uint8_t *seed, int32_t h, pfx_sk **out);
/* Relinearisation key (s^2 -> s) from seed. */
pfx_status pfx_keygen_relin(pfx_ctx *ctx, const pfx_sk *sk, const uint8_t *seed, pfx_swk **out);
/* Galois keys for slot rotations by steps[0..n) (left, Galois element 5^step
 * mod 2N) and, when conj is non-zero, conjugation (2N - 1) last: n + (conj !=
 * 0) keys into out[].  All or nothing: on an error none is kept. */
pfx_status pfx_keygen_galois(pfx_ctx *ctx, const pfx_sk *sk, const int32_t *steps, size_t n, int conj,
                             const uint8_t *seed, pfx_swk **out);
/* pfx_encrypt with a and e drawn from seed (tags 4 and 5). */
pfx_status pfx_encrypt_seeded(pfx_ctx *ctx, const pfx_sk *sk, const pfx_pt *pt, const uint8_t *seed, pfx_ct *out,
                              void *stream);
/* Host only (no device): the draws above, for checking them against another
 * implementation.  pfx_shake256: outlen bytes of SHAKE-256(msg). */
pfx_status pfx_shake256(const uint8_t *msg, size_t n, uint8_t *out, size_t outlen);
pfx_status pfx_sample_uniform(const uint8_t *seed, uint32_t tag, uint32_t index, uint32_t limb, uint64_t q,
                              size_t n, uint64_t *out);
/* The secret's coefficients (tag 1): h-sparse, or uniform ternary for h < 0. */
pfx_status pfx_sample_secret(const uint8_t *seed, size_t n, int32_t h, int8_t *out);
pfx_status pfx_sample_gaussian(const uint8_t *seed, uint32_t tag, uint32_t index, size_t n, int64_t *out);

/* Slot encoding (App. A.1): n_slots (power of two, <= N/2) complex values
 * (im may be NULL) -> round(scale * tau^-1(z)) at n_limbs limbs.  Rounding
 * is half away from zero. */
pfx_status pfx_encode(pfx_ctx *ctx, const double *re, const double *im, size_t n_slots,
                      uint32_t n_limbs, double scale, pfx_pt **out);
/* Inverse of pfx_encode on the centred CRT lift of the plaintext. */
pfx_status pfx_decode(pfx_ctx *ctx, const pfx_pt *pt, double *re, double *im, size_t n_slots);
pfx_status pfx_pt_import(pfx_ctx *ctx, const uint64_t *words, uint32_t n_limbs, double scale,
                         pfx_pt **out);

/* (c0, c1) = (-a s + e + m, a) at the plaintext's level (Sec. 2.3).
 * a: n_limbs * N words; e: N integers.  `out` needs capacity >= n_limbs. */
pfx_status pfx_encrypt(pfx_ctx *ctx, const pfx_sk *sk, const pfx_pt *pt, const uint64_t *a,
                       const int64_t *e, pfx_ct *out, void *stream);
/* m + e = c0 + c1 s (+ c2 s^2) into a new plaintext. */
pfx_status pfx_decrypt(pfx_ctx *ctx, const pfx_sk *sk, const pfx_ct *ct, pfx_pt **out,
                       void *stream);

/* ----------------------------------------------------------- ciphertexts */
/* Device ciphertext with room for cap_limbs limbs and cap_degree + 1
 * polynomials (cap_degree 0 = plaintext).  Starts at degree 0, 0 limbs. */
pfx_status pfx_ct_create(pfx_ctx *ctx, uint32_t cap_limbs, uint32_t cap_degree, pfx_ct **out);
void pfx_ct_destroy(pfx_ct *ct);
pfx_status pfx_ct_info(const pfx_ct *ct, pfx_info *info);
pfx_status pfx_ct_set_scale(pfx_ct *ct, double scale);
/* Import canonical words (layout above) of a degree-`degree` ciphertext. */
pfx_status pfx_ct_import(pfx_ctx *ctx, const uint64_t *words, uint32_t n_limbs, uint32_t degree,
                         double scale, pfx_ct *out, void *stream);
/* Export to canonical words; cap_words >= (degree + 1) * n_limbs * N.
 * Synchronises `stream`. */
pfx_status pfx_ct_export(pfx_ctx *ctx, const pfx_ct *ct, uint64_t *words, size_t cap_words,
                         pfx_info *info, void *stream);
pfx_status pfx_ct_copy(pfx_ctx *ctx, const pfx_ct *src, pfx_ct *dst, void *stream);

/* ------------------------------------------------------ database owner side */
/* Binary operands at different levels: the higher one's extra limbs are
 * dropped (exact).  Additions need scales within 2^-10 relative (PFX_ESCALE
 * otherwise); the result carries the first operand's scale. */
pfx_status pfx_add(pfx_ctx *ctx, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream);
pfx_status pfx_sub(pfx_ctx *ctx, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream);
pfx_status pfx_neg(pfx_ctx *ctx, const pfx_ct *a, pfx_ct *out, void *stream);
pfx_status pfx_add_plain(pfx_ctx *ctx, const pfx_ct *a, const pfx_pt *m, pfx_ct *out, void *stream);
/* Slot-wise product with a plaintext (App. A.1); scale multiplies. */
pfx_status pfx_mul_plain(pfx_ctx *ctx, const pfx_ct *a, const pfx_pt *m, pfx_ct *out, void *stream);
/* Product with an integer; the scale is unchanged. */
pfx_status pfx_mul_int(pfx_ctx *ctx, const pfx_ct *a, int64_t k, pfx_ct *out, void *stream);
/* Tensor product (a0 b0, a0 b1 + a1 b0, a1 b1): degree-2 result. */
pfx_status pfx_mul(pfx_ctx *ctx, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream);
/* Accumulating products, one launch each: acc += a * b (tensor product; acc of
 * degree 2) and acc += a * m (plaintext product; acc of a's degree).  The
 * scale of acc is kept (it must be within 2^-10 of the product's, PFX_ESCALE
 * otherwise); the level becomes the smallest of the operands'; acc must not
 * alias an operand.  Word for word the product followed by pfx_add. */
pfx_status pfx_mul_acc(pfx_ctx *ctx, const pfx_ct *a, const pfx_ct *b, pfx_ct *acc, void *stream);
pfx_status pfx_mul_plain_acc(pfx_ctx *ctx, const pfx_ct *a, const pfx_pt *m, pfx_ct *acc, void *stream);
/* acc += a * k for an integer k (acc of a's degree, scales within 2^-10). */
pfx_status pfx_mul_int_acc(pfx_ctx *ctx, const pfx_ct *a, int64_t k, pfx_ct *acc, void *stream);
/* Relinearisation (App. A.2): (d0, d1) + SwitchKey(d2, swk_{s^2 -> s}). */
pfx_status pfx_relinearize(pfx_ctx *ctx, const pfx_ct *a, const pfx_swk *rlk, pfx_ct *out,
                           void *stream);
/* Relinearisation of n degree-2 ciphertexts: out[i] = relin(a[i]), word for
 * word n calls of pfx_relinearize; those of one level share batched key-switch
 * launches (up to 8).  out[i] may be a[i]; it must not alias another entry's
 * input or output (PFX_EINVAL).  Scratch as pfx_mul_relin_batch. */
pfx_status pfx_relinearize_batch(pfx_ctx *ctx, const pfx_ct *const *a, size_t n, const pfx_swk *rlk,
                                 pfx_ct *const *out, void *stream);
/* HMult + relinearisation in one call. */
pfx_status pfx_mul_relin(pfx_ctx *ctx, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk,
                         pfx_ct *out, void *stream);
/* pfx_mul_relin for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, checks and words as pfx_mul_relin; it calls no hipMalloc,
 * hipFree or allocating library routine.  Its key-switch scratch is a fixed
 * device array of the library (pfx_noalloc_scratch_bytes(), 64 MiB, held on
 * each GPU the library runs on until the process ends; its address is taken
 * once per device by pfx_ctx_create), not the stream's workspace.  A product
 * whose scratch would exceed it (N (l + beta (l + K) + 2 (l + K) + 2 l)
 * doubles at l limbs, plus 3 l N when out aliases an operand; e.g. N = 2^16
 * at 24 + 4 primes) returns PFX_ENOMEM with nothing launched.  Every call on
 * one GPU uses the same array and it keeps the last call's contents: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  PFX_EINVAL while the library's profiler is on (it
 * creates events). */
pfx_status pfx_mul_relin_noalloc(pfx_ctx *ctx, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk,
                                 pfx_ct *out, void *stream);
/* Bytes of the no-allocation scratch array (per GPU). */
size_t pfx_noalloc_scratch_bytes(void);
/* HMult + relinearisation of n pairs under one context and key: out[i] =
 * relin(a[i] * b[i]), word for word what n calls of pfx_mul_relin give.  Pairs
 * of the same level (min of the operands' levels) share the launches of one
 * batched key switch, up to 8 pairs per launch: the key residues are read once
 * for all of them.  Outputs must be distinct and alias no operand of any pair
 * (PFX_EINVAL); the call validates every pair before it launches anything.
 * Scratch for the batch is kept with the stream and grows on first use. */
pfx_status pfx_mul_relin_batch(pfx_ctx *ctx, const pfx_ct *const *a, const pfx_ct *const *b, size_t n,
                               const pfx_swk *rlk, pfx_ct *const *out, void *stream);
/* Rescale (Sec. 2.5): round(c / q_last) with round-half-up of the [0, Q)
 * lift; one limb fewer; scale / q_last.  PFX_ELEVEL below 2 limbs. */
pfx_status pfx_rescale(pfx_ctx *ctx, const pfx_ct *a, pfx_ct *out, void *stream);
/* Rescale of n ciphertexts: out[i] = rescale(a[i]), word for word what n calls
 * of pfx_rescale give.  Ciphertexts of the same level and degree share the
 * four launches of one batched rescale (up to 8 per launch).  out[i] may be
 * a[i] (in place); it must not alias another entry's input or output
 * (PFX_EINVAL).  Every entry is validated before anything is launched.
 * Scratch: the stream's batch region (as pfx_mul_relin_batch). */
pfx_status pfx_rescale_batch(pfx_ctx *ctx, const pfx_ct *const *a, size_t n, pfx_ct *const *out, void *stream);
/* Keep the first n_limbs limbs (exact modulus switch to Q_{n_limbs}). */
pfx_status pfx_drop_level(pfx_ctx *ctx, const pfx_ct *a, uint32_t n_limbs, pfx_ct *out,
                          void *stream);
/* SwitchKey(d, swk) of the first polynomial of d (Sec. 2.4.1): out = (k0, k1)
 * with k0 + k1 s ~ d s_from. */
pfx_status pfx_key_switch(pfx_ctx *ctx, const pfx_ct *d, const pfx_swk *k, pfx_ct *out,
                          void *stream);
/* Automorphism phi_g with key switching back to s (Sec. 2.4.2, App. A.2):
 * g is the key's Galois element. */
pfx_status pfx_apply_galois(pfx_ctx *ctx, const pfx_ct *a, const pfx_swk *gk, pfx_ct *out,
                            void *stream);
/* n automorphisms by the Galois element of gk: out[i] = phi_g(a[i]), word for
 * word n calls of pfx_apply_galois; entries of one level share batched
 * key-switch launches (up to 8; the key residues read once for them).
 * Outputs must be distinct and alias no input of any entry (PFX_EINVAL). */
pfx_status pfx_apply_galois_batch(pfx_ctx *ctx, const pfx_ct *const *a, size_t n, const pfx_swk *gk,
                                  pfx_ct *const *out, void *stream);
/*
 * Rotations of n ciphertexts, entry i by its own step steps[i] (slots left by
 * steps[i], as pfx_rotate), each with its own Galois key found among gks
 * (PFX_ENOKEY if one is missing).  Entries of one level run as batched key
 * switches of up to 8 entries: every launch of the key switch covers the whole
 * batch, so the small launches of a single key switch fill the GPU; the inner
 * product reads each entry's own key.  A step of 0 (mod n_slots) copies.
 * Outputs must be distinct and must not alias any input (PFX_EINVAL).  Word
 * for word the results of pfx_rotate.  Scratch as pfx_mul_relin_batch.
 */
pfx_status pfx_rotate_batch(pfx_ctx *ctx, const pfx_ct *const *a, const int32_t *steps, size_t n,
                            const pfx_swk *const *gks, size_t n_gks, pfx_ct *const *out, void *stream);
/* Hoisted automorphisms (the baby steps of the BSGS linear transforms, App.
 * A.4): out[i] = phi_(g_i)(a) for the Galois elements of gks[0..n), the
 * decomposition (ModUp) of c1 computed once and each key switch fed with its
 * permutation; decrypts to the same messages as pfx_apply_galois (not the same
 * words: the permuted decomposition lifts negated residues differently).
 * Outputs must be distinct and not a (PFX_EINVAL); non-Galois keys
 * PFX_ENOKEY. */
pfx_status pfx_apply_galois_hoisted(pfx_ctx *ctx, const pfx_ct *a, const pfx_swk *const *gks, size_t n,
                                    pfx_ct *const *out, void *stream);
/* Plaintext-matrix product on the slots by the diagonal method with the
 * baby-step giant-step split (CoeffsToSlots / SlotsToCoeffs, App. A.4):
 *   out = sum_k diags[k] (.) rot(a, steps[k])     (steps taken mod N/2)
 * computed as sum_j rot(sum_{k: s_k = n1 j + i} rot(diags[k], -n1 j) (.) rot(a, i), n1 j):
 * the distinct baby steps i != 0 as hoisted automorphisms, the diagonals
 * rotated as plaintexts (no key), one rotation per distinct giant step j != 0.
 * diags: n plaintexts with at least a's limbs, one scale (PFX_ESCALE);
 * keys: Galois keys of every baby and giant step (PFX_ENOKEY).  out has a's
 * level and the scale a.scale * diags' scale (no rescale); out != a. */
pfx_status pfx_linear_transform(pfx_ctx *ctx, const pfx_ct *a, const pfx_pt *const *diags, const int32_t *steps,
                                size_t n, uint32_t n1, const pfx_swk *const *keys, size_t n_keys, pfx_ct *out,
                                void *stream);
/* a * X^k in R_Q = Z_Q[X]/(X^N + 1) (k taken mod 2N; X^N = -1): the lookup of
 * plaintext point k in an encrypted table (Sec. 3.4) and the X^t of ring
 * repacking (Alg. 1).  Scale and level are kept; out may be a. */
pfx_status pfx_mul_monomial(pfx_ctx *ctx, const pfx_ct *a, int64_t k, pfx_ct *out, void *stream);
/* a * N^-1 mod Q (every residue times N^-1 mod q_i), the pre-multiplication
 * of ring repacking (Alg. 1); the scale is kept.  out may be a. */
pfx_status pfx_mul_inv_n(pfx_ctx *ctx, const pfx_ct *a, pfx_ct *out, void *stream);
/* Ring repacking (Sec. 3.2, Alg. 1) of in[0..n), degree-1 ciphertexts of one
 * level and scale, in groups of N: out[g] (g < ceil(n / N)) encrypts
 * sum_j m_(gN+j)[0] X^j, the constant coefficients of the group's inputs
 * (Lemma 1).  Inputs are multiplied by N^-1, the last group is padded with
 * zero ciphertexts, then round i < log N with t = N / 2^(i+1) and g = 2N - 1
 * (i = 0) or 5^(2^(i-1)) mod 2N updates c_j <- c_j + X^t c_(j+t) +
 * phi_g(c_j - X^t c_(j+t)) for j < t, every pair of every group of a round in
 * batched key-switch launches.  The log N Galois keys must be among gks
 * (PFX_ENOKEY).  Outputs keep the inputs' level and scale and alias no input
 * (PFX_EINVAL).  The stream's repacking arrays (1.5 ceil(n/N) N ciphertexts)
 * are allocated on first use, not under graph capture. */
pfx_status pfx_repack(pfx_ctx *ctx, const pfx_ct *const *in, size_t n, const pfx_swk *const *gks, size_t n_gks,
                      pfx_ct *const *out, void *stream);
/* Private lookup-table evaluation with score aggregation, then ring repacking
 * (Sec. 3.4, Sec. 4.2 "Encrypted Scoring Functions", Alg. 1): record r < n is
 * the ciphertext sum_l tables[l] X^(exps[r m + l]) (tables[l] encrypts u_f of
 * function l, Sec. 3.4, and its constant coefficient is then sum_l f_l(k_rl)),
 * and out[g] encrypts the records g N .. g N + N - 1 in its coefficients, as
 * pfx_repack of those records would (word for word).  exps: device memory,
 * n * m int64 exponents, row-major by record, taken mod 2N; the records are
 * formed directly in the repacking arrays.  tables: m degree-1 ciphertexts of
 * one level and scale; out as for pfx_repack. */
pfx_status pfx_pfe_repack(pfx_ctx *ctx, const pfx_ct *const *tables, size_t m, const int64_t *exps, size_t n,
                          const pfx_swk *const *gks, size_t n_gks, pfx_ct *const *out, void *stream);
/* ModRaise, the first step of bootstrapping (App. A.3): a ciphertext of one
 * limb (q_0) read modulo the first n_limbs primes: every coefficient's q_0
 * residue lifted to [-(q_0-1)/2, (q_0-1)/2] and reduced modulo each prime, so
 * out decrypts to m + q_0 I(X) with I small.  Scale and degree are kept; out
 * may be a when its capacity holds n_limbs. */
pfx_status pfx_mod_raise(pfx_ctx *ctx, const pfx_ct *a, uint32_t n_limbs, pfx_ct *out, void *stream);
/* The trace-like map after ModRaise (App. A.3): out = prod_{t < log_r}
 * (1 + phi_{N/2^t + 1}) a, which keeps the coefficients of degree a multiple of
 * r = 2^log_r (times r) and cancels the others; log_r automorphisms, whose keys
 * (Galois elements N/2^t + 1) must be among keys (PFX_ENOKEY).  out may be a. */
pfx_status pfx_subring_trace(pfx_ctx *ctx, const pfx_ct *a, uint32_t log_r, const pfx_swk *const *keys,
                             size_t n_keys, pfx_ct *out, void *stream);
/* Ring merging and ring switching (Sec. 3.3, Sec. 4.3): n <= N/n_small
 * degree-1 ciphertexts of one limb in the small ring (context `small`, degree
 * n_small) -> one of one limb in the large ring (context `big`, degree N)
 * whose plaintext has coefficient j of input i at X^(j N/n_small + i), i.e.
 * sum_i X^i m_i(X^(N/n_small)) (missing inputs are zero).  The inputs are
 * embedded (X -> X^(N/n_small), an encryption under the embedded small
 * secret), shifted by X^i and summed, then key-switched to the large secret
 * with `swk`, made by pfx_swk_create_from in `big` from the embedded small
 * secret (PFX_ENOKEY otherwise).  Both contexts must share their first prime
 * (PFX_EPARAM) and n_small < N.  The scale is the inputs' (PFX_ESCALE if they
 * differ); out is a ciphertext of `big`. */
pfx_status pfx_ring_merge(pfx_ctx *big, pfx_ctx *small, const pfx_ct *const *in, size_t n, const pfx_swk *swk,
                          pfx_ct *out, void *stream);
/* Rotate slots left by `step` (App. A.1); the key for 5^step mod 2N must be
 * among keys[0..n_keys) (PFX_ENOKEY otherwise). */
pfx_status pfx_rotate(pfx_ctx *ctx, const pfx_ct *a, int32_t step, const pfx_swk *const *keys,
                      size_t n_keys, pfx_ct *out, void *stream);
pfx_status pfx_conjugate(pfx_ctx *ctx, const pfx_ct *a, const pfx_swk *const *keys, size_t n_keys,
                         pfx_ct *out, void *stream);
/* InnerSum (Alg. 2, last step): x <- x + rot(x, 2^k) for k < log_steps. */
pfx_status pfx_rotate_sum(pfx_ctx *ctx, const pfx_ct *a, uint32_t log_steps,
                          const pfx_swk *const *keys, size_t n_keys, pfx_ct *out, void *stream);

/* x + value in every slot: the constant polynomial round(value * scale_x)
 * (App. A.1: a constant has only coefficient 0) added to c0. */
pfx_status pfx_add_const(pfx_ctx *ctx, const pfx_ct *a, double value, pfx_ct *out, void *stream);
/* x times the constant round(value * cscale) (every slot times value); the
 * scale multiplies by cscale.  cscale <= 0 takes the last prime of x, so that
 * a following rescale returns x's scale. */
pfx_status pfx_mul_const(pfx_ctx *ctx, const pfx_ct *a, double value, double cscale, pfx_ct *out,
                         void *stream);

/* Standalone negacyclic NTT on device words (canonical residues), in place:
 * d_words holds `batch` blocks of n_limbs limbs of N words; limb i of every
 * block uses prime first_prime + i (prime index: q's then p's).  Output order
 * is NTT(a)[j] = sum_k a_k psi^(k (2 bitrev(j) + 1)); inverse = 1 undoes it. */
pfx_status pfx_ntt(pfx_ctx *ctx, uint64_t *d_words, uint32_t first_prime, uint32_t n_limbs,
                   size_t batch, int inverse, void *stream);

/* ------------------------------------------------------------ circuits */
/*
 * Op-list executor: a query circuit (e.g. Alg. 2's threshold and count) as a
 * list of register operations run natively, optionally captured once into a
 * HIP graph and replayed.  Registers are caller-created ciphertexts (capacity
 * n_q limbs, degree 2); registers [0, n_inputs) are read-only inputs.
 * Plaintexts are the database operands.  `gks` holds the Galois keys that
 * ROTATE / ROTATE_SUM need; `rlk` the relinearisation key.
 *   op            effect                                         operands
 *   COPY          dst = a
 *   ADD, SUB      dst = a +- b (scale of a)                      b register
 *   MUL_PLAIN     dst = a * pts[b]                               b plaintext
 *   ADD_PLAIN     dst = a + pts[b]                               b plaintext
 *   MUL_INT       dst = a * k                                    k
 *   MUL_RELIN     dst = relin(a * b)                             b register
 *   MUL           dst = a * b, degree 2 (pfx_mul; dst needs     b register
 *                 capacity for degree 2)
 *   RELIN         dst = relin(a), a of degree 2
 *   MUL_ACC       dst = dst + a * b (dst of degree 2)            b register
 *   MUL_PLAIN_ACC dst = dst + a * pts[b]                         b plaintext
 *   MUL_INT_ACC   dst = dst + a * k                              k
 *   DROP          dst = the first k limbs of a (pfx_drop_level)  k
 *   MONO          dst = a * X^k (pfx_mul_monomial)               k
 *   INV_N         dst = a * N^-1 mod Q (pfx_mul_inv_n)
 *   GALOIS        dst = phi_k(a) (pfx_apply_galois; the key of    k
 *                 Galois element k among gks)
 *   RESCALE       dst = rescale(a)
 *   ADD_CONST     dst = a + value (pfx_add_const)                value
 *   MUL_CONST     dst = a * value at the last prime's scale      value
 *   MUL_CONST_TO  dst = a * value, the constant taken at the       value,
 *                 scale c = scale_b * q_last / scale_a (q_last    b register
 *                 a's last prime), so that after one RESCALE dst
 *                 has register b's scale: terms of a sum meet at
 *                 one scale exactly (App. A.3, EvalMod); only b's
 *                 scale is read
 *   MUL_CONST_LIKE dst = a * value, the constant taken at the      value,
 *                 scale scale_b / scale_a, so that dst has register b register
 *                 b's scale exactly: a term joins a sum formed
 *                 before its one RESCALE (App. A.3, EvalMod);
 *                 only b's scale is read
 *   SCALE_MUL     dst = a with scale * value (value / factor)    value
 *   ROTATE        dst = rotate(a, k)                             k
 *   ROTATE_SUM    dst = InnerSum(a) over 2^k slots               k
 * `mode` is a combination of
 *   PFX_RUN_GRAPH (non-NULL stream required): the first call for a given op
 *     list, register set, plaintexts and keys is captured into a HIP graph and
 *     launched; later calls replay it.  Register metadata (limbs, scale) after
 *     a replay equals that of the captured run.  Graphs are cached process-wide
 *     (at most 64, least recently used dropped) under the identities of the
 *     objects (never their addresses), the registers' capacities, the inputs'
 *     shapes, the plaintexts' levels and scales, the stream and the mode;
 *     destroying any object a graph uses drops that graph, and a graph
 *     captured before any library scratch region was freed or moved (stream
 *     or context destroyed, a batch or repacking region grown) is captured
 *     again instead of replayed.  Every object must be library-created
 *     (PFX_EINVAL otherwise).
 *   PFX_RUN_LANES: LANE markers in the list are honoured.  The first marker
 *     LANE k (0 <= k < 8) of a fork records an event on `stream` that all of
 *     the library's lane streams wait for, and the ops after LANE k run on
 *     lane k; LANE -1 (or the end of the list) joins every lane back into
 *     `stream`.  Ops on different lanes of one fork run concurrently (e.g. the
 *     record blocks of a query), so none of them may depend on another's
 *     registers (read-after-write, write-after-read, write-after-write):
 *     the list is checked before anything is launched (PFX_EINVAL).  With
 *     PFX_RUN_GRAPH the forks are captured into one multi-stream graph.
 *     Without PFX_RUN_LANES the markers are ignored and the list runs in
 *     program order on `stream`.
 * Results are identical in every mode.
 *   LANE          switch lane (see PFX_RUN_LANES)                k
 */
#define PFX_RUN_EAGER 0
#define PFX_RUN_GRAPH 1
#define PFX_RUN_LANES 2
#define PFX_OP_COPY 0
#define PFX_OP_ADD 1
#define PFX_OP_SUB 2
#define PFX_OP_MUL_PLAIN 3
#define PFX_OP_ADD_PLAIN 4
#define PFX_OP_MUL_INT 5
#define PFX_OP_MUL_RELIN 6
#define PFX_OP_RESCALE 7
#define PFX_OP_ADD_CONST 8
#define PFX_OP_MUL_CONST 9
#define PFX_OP_SCALE_MUL 10
#define PFX_OP_ROTATE 11
#define PFX_OP_ROTATE_SUM 12
#define PFX_OP_LANE 13
#define PFX_OP_MUL 14
#define PFX_OP_RELIN 15
#define PFX_OP_MUL_ACC 16
#define PFX_OP_MUL_PLAIN_ACC 17
#define PFX_OP_MUL_INT_ACC 18
#define PFX_OP_DROP 19
#define PFX_OP_MONO 20
#define PFX_OP_INV_N 21
#define PFX_OP_GALOIS 22
#define PFX_OP_MUL_CONST_TO 23
#define PFX_OP_MUL_CONST_LIKE 24

typedef struct pfx_op {
    int32_t code;
    int32_t dst;
    int32_t a;
    int32_t b;
    int64_t k;
    double value;
} pfx_op;

pfx_status pfx_run_circuit(pfx_ctx *ctx, const pfx_op *ops, size_t n_ops, pfx_ct *const *regs,
                           size_t n_regs, size_t n_inputs, const pfx_pt *const *pts, size_t n_pts,
                           const pfx_swk *rlk, const pfx_swk *const *gks, size_t n_gks, int mode,
                           void *stream);

/*
 * Batched HMult + relinearisation + rescale over ciphertexts of uneven ring
 * degree and level: out[i] = rescale(relin(a[i] * b[i])) under ctxs[i]
 * (one context per ring degree; rlk[i] its relinearisation key).
 *   mode 0: one ciphertext after the other on `stream` (the per-ciphertext path)
 *   mode 1: spread over the library's lane streams, forked from and joined back
 *           to `stream` with events, so that the launches of different
 *           ciphertexts overlap on the device (lanes balanced by estimated work)
 *   mode 2: mode 1 captured once into a HIP graph (non-NULL stream) and replayed
 *   mode 3: mode 1 with entries of the same context and level grouped (up to 8)
 *           into batched key switches and rescales (pfx_mul_relin_batch,
 *           pfx_rescale_batch); an entry whose output aliases its own operand
 *           runs alone
 *   mode 4: mode 3 captured once into a HIP graph and replayed
 *   mode 5: one persistent cooperative launch for the whole batch: the
 *           thirteen steps of the key switch and rescale run in order, each
 *           step's tiles of every entry (any ring degree and level) dealt to
 *           one grid of resident workgroups, a grid barrier between steps.
 *           Needs 2^12 <= N <= 2^16, digits of at most 4 primes and at most 4
 *           special primes (PFX_EINVAL).  An entry whose output aliases an
 *           operand of any entry runs first, on the per-ciphertext path.
 *           Scratch for every entry is kept with the stream (grown on
 *           demand, counted against the first entry's context).  Returns
 *           after the batch has finished; PFX_EDEVICE if a grid barrier
 *           timed out (not expected: every workgroup is resident).
 *   mode 6: mode 5's tiles in step-major order without the persistent grid:
 *           one launch per step over the tiles of every entry (13 launches
 *           for the whole batch, each with the registers and occupancy of its
 *           own step); at most 1024 entries besides those that run alone.
 * Results are identical in every mode.  Outputs must not alias inputs of other
 * batch entries.
 */
pfx_status pfx_batch_mul_relin_rescale(pfx_ctx *const *ctxs, const pfx_ct *const *a,
                                       const pfx_ct *const *b, const pfx_swk *const *rlk,
                                       pfx_ct *const *out, size_t n, int mode, void *stream);

/*
 * The process-wide cache of captured graphs (PFX_RUN_GRAPH, batched modes 2
 * and 4): entries held now, and captures made since the library was loaded
 * (a replay does not count).  Either pointer may be NULL.  Never fails.
 */
pfx_status pfx_graph_cache_stats(size_t *entries, uint64_t *captures);

/* ------------------------------------------------------------ served form */
/*
 * A query server over one context: the database owner's side of the private
 * query (Sec. 5 and Alg. 2 of the paper) run as a service.  Requests are op
 * lists (the pfx_op codes above) that arrive at any time; the server admits
 * them first-come first-served whenever one of its `slots` streams is free and
 * the request's footprint fits in what is left of the HBM budget, and runs
 * every admitted request on its own stream, so that requests overlap on the
 * device (continuous batching at request granularity: a finishing request
 * frees its slot and memory, which admits the next one at once).
 *
 * Batching inside a request.  With max_batch > 1 a request's runs of
 * independent HMult + relin ops or rescales (as pfx_run_circuit batches them,
 * e.g. the record blocks of an interleaved query plan) share batched launches
 * of up to max_batch (at most 8) entries; 1 runs every op alone.
 *
 * Memory.  At creation the server takes `hbm_budget` bytes: each slot's
 * key-switching scratch (fixed; with max_batch > 1 it includes the batch
 * region for max_batch entries), and the rest as one arena from which each
 * admitted request's work registers are carved.  A request's footprint is
 * its work registers at the largest level among its inputs: (degree + 1) *
 * max(inputs' n_limbs) * N * 8 bytes each, degree from reg_degree (1 when
 * NULL).  The evaluation keys
 * (rlk, gks: resident, shared by every request), the input ciphertexts and the
 * plaintexts are the caller's and are not counted.
 *
 * Ownership.  rlk and gks must outlive the server.  A request's inputs, pts
 * and out are borrowed until pfx_server_poll reports the ticket finished; the
 * server copies the request's op list and pointer arrays at submit.  Inputs
 * are registers 0..n_inputs-1 and are only read; out receives a copy of
 * register out_reg (its capacity must hold that register's limbs).
 *
 * Results are identical to pfx_run_circuit of the same op list on the same
 * inputs, whatever else runs beside them.  A server launches from a thread of
 * its own; calls on the same context from other threads may run meanwhile.
 */
typedef struct pfx_server pfx_server;

typedef struct pfx_request {
    const pfx_op *ops;
    size_t n_ops;
    size_t n_regs;                 /* registers of the op list */
    size_t n_inputs;               /* registers 0..n_inputs-1 are inputs[...] */
    const pfx_ct *const *inputs;
    const pfx_pt *const *pts;      /* plaintext operands, by op field b */
    size_t n_pts;
    int32_t out_reg;               /* in [n_inputs, n_regs) */
    pfx_ct *out;
    const uint8_t *reg_degree;     /* per register: capacity degree (1 or 2) of a work
                                      register; NULL: every work register degree 1 */
} pfx_request;

typedef struct pfx_request_info {
    pfx_status status;             /* of the evaluation (PFX_OK, or the failing op's error) */
    int32_t slot;                  /* stream slot it ran on */
    size_t footprint;              /* arena bytes it held while running */
    double queued_s;               /* submit -> admission, seconds */
    double latency_s;              /* submit -> the end of its last launch, seconds */
    char error[160];               /* message of a failed evaluation */
} pfx_request_info;

typedef struct pfx_server_stats {
    uint64_t submitted, completed, queued, running;
    size_t budget, scratch_bytes, arena_bytes, bytes_in_use, peak_bytes;
    uint32_t slots, peak_running;
} pfx_server_stats;

/* PFX_ENOMEM if the budget does not cover the slots' scratch; slots in [1, 16],
 * max_batch in [1, 8] (PFX_EINVAL otherwise). */
pfx_status pfx_server_create(pfx_ctx *ctx, size_t hbm_budget, uint32_t slots, uint32_t max_batch,
                             const pfx_swk *rlk, const pfx_swk *const *gks, size_t n_gks, pfx_server **out);
/* Queues a request and returns its ticket.  PFX_EINVAL for a malformed request
 * (registers out of range, an input of another context), PFX_ENOMEM if its
 * footprint exceeds the whole arena (it could never be admitted). */
pfx_status pfx_server_submit(pfx_server *s, const pfx_request *rq, uint64_t *ticket);
/* PFX_OK once the ticket has finished (info filled, the ticket released),
 * PFX_EBUSY while it is queued or running and wait == 0 (wait != 0 blocks until
 * it finishes), PFX_EINVAL for an unknown or already released ticket. */
pfx_status pfx_server_poll(pfx_server *s, uint64_t ticket, int wait, pfx_request_info *info);
pfx_status pfx_server_stats_get(pfx_server *s, pfx_server_stats *st);
/* Waits for the running requests, drops the queued ones, frees the arena and
 * the slots. */
void pfx_server_destroy(pfx_server *s);

/* ------------------------------------------------------------ plumbing */
/* Device memory and streams for callers that hold raw words (pfx_ntt).  The
 * library links the system HIP runtime; a process should not load a second
 * HIP runtime beside it (PyTorch wheels bundle their own), so these cover what
 * such a caller would otherwise take from a framework. */
pfx_status pfx_dev_alloc(pfx_ctx *ctx, size_t bytes, void **out);
pfx_status pfx_dev_free(pfx_ctx *ctx, void *p);
pfx_status pfx_memcpy_htod(pfx_ctx *ctx, void *dst, const void *src, size_t bytes, void *stream);
pfx_status pfx_memcpy_dtoh(pfx_ctx *ctx, void *dst, const void *src, size_t bytes, void *stream);
/* Streams at the default priority. */
pfx_status pfx_stream_create(pfx_ctx *ctx, void **out);
pfx_status pfx_stream_destroy(pfx_ctx *ctx, void *stream);
/* Timing events on a stream, for callers that time calls on the device: record
 * one before and one after a call on the stream it runs on; pfx_event_elapsed
 * waits for `end` and gives the device time between the two (ms). */
pfx_status pfx_event_create(pfx_ctx *ctx, void **out);
pfx_status pfx_event_record(pfx_ctx *ctx, void *event, void *stream);
pfx_status pfx_event_elapsed(pfx_ctx *ctx, void *start, void *end, float *ms);
pfx_status pfx_event_destroy(pfx_ctx *ctx, void *event);
/* Work enqueued on `stream` after this call waits until `event` (recorded on
 * another stream) has completed: independent calls on two streams joined. */
pfx_status pfx_stream_wait_event(pfx_ctx *ctx, void *stream, void *event);

/* ------------------------------------------------------------ profiling */
/* When on, the library brackets each kernel launch with HIP events on the
 * stream it launches on and accumulates per-kernel device time. */
pfx_status pfx_profile_enable(pfx_ctx *ctx, int on);
/* Completed launches, their summed device time (ms) and summed algorithmic
 * HBM bytes (each launch's minimal reads + writes of its operands, no
 * re-reads, no twiddle or constant tables) for a kernel name (see
 * pfx_profile_names); synchronises pending events. */
pfx_status pfx_profile_get(pfx_ctx *ctx, const char *kernel, uint64_t *launches, double *total_ms,
                           double *bytes);
/* Newline-separated kernel names seen so far. */
pfx_status pfx_profile_names(pfx_ctx *ctx, char *buf, size_t cap);
pfx_status pfx_profile_reset(pfx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PFX_H */
