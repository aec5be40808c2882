// Internal structures of libpfx: context, objects, device tables, launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "graph_cache.h"
#include "pfx.h"

namespace pfx {

constexpr int kMaxAlpha = 8;
constexpr int kMaxSpecial = 8;    // special primes p_k
constexpr int kMaxMapLimbs = 256;   // limbs per NTT launch (kernel-argument map)

// Per-prime device record.  Prime ids: q_0..q_{L-1} are 0..L-1, p_k is L+k.
struct PrimeDev {
    double q, qinv;              // q and fl(1/q)
    double ninv, ninv_q;         // N^-1 mod q and fl(N^-1 / q)
    double ninv_w1, ninv_w1_q;   // N^-1 * psi^-(N/2), the last inverse stage folded with N^-1
    const double2 *tw;           // tw[k]  = {psi^bitrev(k),  fl(./q)}, k < N
    const double2 *itw;          // itw[k] = {psi^-bitrev(k), fl(./q)}, k < N
    // On-the-fly twiddles of the last R2 stages of the row pass (T = log N - R2):
    // stage T + k, twiddle for j = (P << R2) | u is rc[2^k - 1 + x] * B_k with
    // x = u >> (R2 - k), B_{R2-1} = rtw[P] = psi^(2 bitrev_T(P)), B_{k-1} = B_k^2.
    const double *rtw;           // 2^T entries
    const double *irtw;          // same with psi^-1
    double rc[16];
    double irc[16];
};

// Limbs of one batched NTT launch: limb b sits at base + off[b] * N and uses prime pid[b].
struct LimbMap {
    int n;
    int32_t off[kMaxMapLimbs];
    int16_t pid[kMaxMapLimbs];
};

// Constants of the fast basis conversion of one key-switching digit variant
// (digit j with sz active primes): y_i = [d_i * inv_i]_{q_i};
// out_m = sum_i y_i * hat[i][m] mod m, for every prime id m.
struct ModUpConst {
    double2 inv[kMaxAlpha];                   // {(Q'/q_i)^-1 mod q_i, ./q_i}
    double2 hat[kMaxAlpha][PFX_MAX_PRIMES];   // {(Q'/q_i) mod m, ./m}
};

// ModDown constants (independent of the level).
struct ModDownConst {
    double2 phat_inv[PFX_MAX_PRIMES];                   // (P/p_k)^-1 mod p_k
    double2 phat[PFX_MAX_PRIMES][PFX_MAX_PRIMES];       // [k][i]: (P/p_k) mod q_i
    double2 pinv[PFX_MAX_PRIMES];                       // P^-1 mod q_i
    double half[2 * PFX_MAX_PRIMES];                    // floor(P/2) mod prime id m
    double2 pmod[PFX_MAX_PRIMES];                       // P mod q_i (key generation gadget)
};

// Rescale constants for dropping prime l: entry [l][i], i < l.
struct RescaleConst {
    double2 inv;     // q_l^-1 mod q_i
    double half;     // floor(q_l / 2) mod q_i
    double pad;
};

struct Workspace {
    hipStream_t stream = nullptr;
    double *buf = nullptr;
    size_t doubles = 0;
    double *bbuf = nullptr;   // batched key-switch scratch (bcap entries), on demand
    int bcap = 0;
    double *rbuf = nullptr;   // ring-repacking arrays (rcap doubles), on demand
    size_t rcap = 0;
    double *pbuf = nullptr;   // persistent batched form: every entry's scratch (pcap doubles), on demand
    size_t pcap = 0;
};

// The device memory of a context: its allocator (the caller's, or hipMalloc
// when alloc is null), the bytes it holds and their cap (0: none).
struct MemAccount {
    std::mutex mu;
    pfx_alloc_fn alloc = nullptr;
    pfx_free_fn free = nullptr;
    void *user = nullptr;
    size_t budget = 0, in_use = 0, peak = 0;
};

// Launch geometry of the transform passes per ring degree (process-wide; set
// by pfx_tuning_set / pfx_tuning_load, chosen by the package's autotuner):
//   row_wg256 / col_wg256: a row / column pass over `limbs` limbs takes 256
//     threads when that gives at least this many workgroups, 128 otherwise;
//   widen_wg: small launches (standalone passes, the special-prime INTT)
//     narrow their tiles until they have this many workgroups, down to
//     min_col columns (min_col_special for the special-prime INTT);
//   rs_widen_wg: the same for the INTT of the rescale's last limbs.
// Defaults: rows 128 threads below 2048 workgroups (eight per CU), columns
// always 256 (16-column tiles read whole 128-byte rows), widen to 1024
// workgroups (16 / 8 columns), the rescale's INTT to 256.
struct PassTuning {
    int row_wg256 = 2048, col_wg256 = 0, widen_wg = 1024, min_col = 16, min_col_special = 8, rs_widen_wg = 256;
    int ks_fuse = 0;     // threads of the fused ModUp row pass + inner product (0: separate launches)
    int ks_batch = 8;    // entries per batched key switch (at most kMaxBatch)
    int ks_modup_batch = 0;   // entries per ModUp + inner-product launch inside a batch (0: all)
};
const PassTuning &pass_tuning(int logn);   // api.cpp

struct ProfEntry {
    hipEvent_t start, stop;
    std::string name;
    double bytes;   // algorithmic HBM bytes of the launch
};

struct ProfTotal {
    uint64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
};

}  // namespace pfx

struct pfx_ctx {
    int device = 0;
    int logn = 0;
    int N = 0;
    int L = 0, K = 0, alpha = 0, beta = 0, mod_log2 = 0;
    std::vector<uint64_t> primes;   // L q's then K p's
    std::vector<uint64_t> psi;

    pfx::PrimeDev *d_primes = nullptr;
    double2 *d_tw = nullptr;
    double *d_rtw = nullptr;
    pfx::ModUpConst *d_modup = nullptr;     // [beta][alpha] variants (j, sz-1)
    pfx::ModDownConst *d_moddown = nullptr;
    pfx::RescaleConst *d_rescale = nullptr; // [L][L]
    std::vector<pfx::PrimeDev> h_primes;

    uint64_t uid = 0;                 // identity for the graph cache (never reused)

    // Device memory of the context (dmalloc / dfree), shared with the
    // allocations it made so that they can be freed after the context.
    std::shared_ptr<pfx::MemAccount> mem = std::make_shared<pfx::MemAccount>();
    std::mutex mu;
    std::map<hipStream_t, pfx::Workspace *> ws;

    std::vector<hipStream_t> lanes;       // batch lanes (default priority)
    std::vector<hipEvent_t> lane_events;
    std::atomic<bool> capturing{false};

    std::atomic<bool> prof_on{false};
    std::vector<pfx::ProfEntry> prof_pending;
    std::map<std::string, pfx::ProfTotal> prof_done;
    std::vector<hipEvent_t> prof_pool;
};

struct pfx_sk {
    pfx_ctx *ctx;
    uint64_t uid = 0;
    double *d_s;          // (L + K) limbs, NTT domain
    std::vector<int8_t> h_s;
};

struct pfx_swk {
    pfx_ctx *ctx;
    uint64_t uid = 0;
    uint32_t galois;
    double *d_k;               // [beta][2][L + K][N], NTT domain
    bool from_secret = false;  // pfx_swk_create_from: neither a relinearisation nor a Galois key
};

struct pfx_ct {
    pfx_ctx *ctx;
    uint64_t uid = 0;     // identity for the graph cache (0: library-internal temporary)
    uint32_t cap_limbs, cap_degree;
    uint32_t n_limbs = 0, degree = 0;
    double scale = 1.0;
    double *d = nullptr;  // poly k, limb i at d + (k * cap_limbs + i) * N
    bool owns = true;     // false for views into memory the library manages elsewhere (server arena)
    double *poly(uint32_t k) const { return d + (size_t)k * cap_limbs * (size_t)ctx->N; }
};

namespace pfx {

// ---------------------------------------------------------------- host helpers
// Drops every captured graph that depends on the object (api.cpp).
void graph_forget(uint64_t uid);
// Device allocation of `bytes` for context c (api.cpp): through the caller's
// allocator when set, within the context's budget; PFX_ENOMEM (*p untouched)
// when the budget or the allocator refuses.  dfree releases memory dmalloc
// made through the allocator that made it, and returns the bytes to its
// context's account (also after the context is gone); null and pointers
// dmalloc did not make are ignored.
pfx_status dmalloc(pfx_ctx *c, void **p, size_t bytes);
template <class T>
pfx_status dmalloc(pfx_ctx *c, T **p, size_t bytes) {
    void *v = nullptr;
    pfx_status r = dmalloc(c, &v, bytes);
    if (!r) *p = static_cast<T *>(v);
    return r;
}
void dfree(void *p);
// Device address of the no-allocation scratch array on `device`, taken once
// with that device current (noalloc.hip; pfx_ctx_create calls it).
pfx_status noalloc_init(int device);
// Seeded sampling (sampler.cpp): SHAKE-256 streams keyed by seed, tag, index
// and limb, and the draws of the secret, of uniform residues and of the
// discrete Gaussian errors (sigma 3.2, |e| <= 19) read from them.
constexpr uint32_t kTagSecret = 1, kTagKeyA = 2, kTagKeyE = 3, kTagEncA = 4, kTagEncE = 5;
void shake256(const uint8_t *msg, size_t n, uint8_t *out, size_t outlen);
void sample_uniform(const uint8_t seed[32], uint32_t tag, uint32_t index, uint32_t limb, uint64_t q, size_t n,
                    uint64_t *out);
void sample_secret(const uint8_t seed[32], size_t n, int32_t h, int8_t *out);
void sample_gaussian(const uint8_t seed[32], uint32_t tag, uint32_t index, size_t n, int64_t *out);
void set_error(const std::string &msg);
pfx_status fail(pfx_status s, const std::string &msg);

bool build_primes(const pfx_params *prm, std::vector<uint64_t> &q, std::vector<uint64_t> &p,
                  std::vector<uint64_t> &psi, std::string &err);
uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t m);
uint64_t powmod_u64(uint64_t a, uint64_t e, uint64_t m);
uint64_t invmod_u64(uint64_t a, uint64_t m);

// Host encoder (slot FFT) in encoder.cpp.
bool encode_coeffs(int logn, const double *re, const double *im, size_t n, double scale,
                   const std::vector<uint64_t> &mods, std::vector<uint64_t> &words, std::string &err);
void decode_words(int logn, const uint64_t *words, int n_limbs, const std::vector<uint64_t> &mods,
                  double scale, size_t n, double *re, double *im);

// Op-list interpreter behind pfx_run_circuit (api.cpp): registers 0..n_inputs-1
// are read-only, every op is launched on `stream`.  With max_batch > 1, runs of
// up to max_batch independent HMult + relin ops share one batched key switch
// (its scratch grows with the stream's workspace); 1 runs every op alone.
pfx_status run_ops(pfx_ctx *c, const pfx_op *ops, size_t n_ops, pfx_ct *const *regs, size_t n_regs,
                   size_t n_inputs, const pfx_pt *const *pts, size_t n_pts, const pfx_swk *rlk,
                   const pfx_swk *const *gks, size_t n_gks, void *stream, int max_batch);
// Bytes of the per-stream scratch, and its allocation for one stream; the same
// for the stream's batch region of nb entries (batched key switch / rescale).
size_t ws_bytes(const pfx_ctx *c);
pfx_status ws_reserve(pfx_ctx *c, hipStream_t st);
size_t batch_ws_bytes(const pfx_ctx *c, int nb);
pfx_status batch_ws_reserve(pfx_ctx *c, hipStream_t st, int nb);

// ---------------------------------------------------------------- launchers
struct Launch {
    pfx_ctx *ctx;
    hipStream_t st;
};

void prof_begin(const Launch &L, const char *name, hipEvent_t *ev);
void prof_end(const Launch &L, const char *name, hipEvent_t ev, double bytes);

// Batched NTT over the limbs of `map`; src == nullptr means in place.
void launch_ntt(const Launch &L, double *base, const double *src, const LimbMap &map, bool inverse);
// One pass (column: the first log N / 2 stages; row: the rest) of the same transform;
// nb copies of the map at base + b * bstride (doubles).
void launch_ntt_pass(const Launch &L, double *base, const double *src, const LimbMap &map, bool row, bool inverse,
                     int nb = 1, size_t bstride = 0);
// NTT / INTT of `limbs` limbs of canonical uint64 words in place (kernels.hip);
// limb l uses prime first + l % nl.
void launch_ntt_words(const Launch &L, uint64_t *words, size_t limbs, int first, int nl, bool inverse);
void launch_u64_to_f64(const Launch &L, double *out, const uint64_t *in, size_t n);
void launch_f64_to_u64(const Launch &L, uint64_t *out, const double *in, size_t n);
void launch_int_to_rns(const Launch &L, double *out, const int64_t *in, int n_limbs, int pid0,
                       int pid_gap_at, int pid_gap);
void launch_s8_to_rns(const Launch &L, double *out, const int8_t *in, int n_limbs);

// EW_MAC: out = out + a * b (out read and written by the same thread).  The
// last three are the per-limb constant forms of collected launches.
enum EwOp { EW_ADD = 0, EW_SUB = 1, EW_MUL = 2, EW_NEG = 3, EW_COPY = 4, EW_MAC = 5, EW_MULC = 6, EW_MULC_ACC = 7,
            EW_ADDC = 8, EW_MONO = 9 };
// out = a * X^k (k in [0, 2N)) in the NTT domain, npoly polynomials of nl limbs
// (kernels.hip): slot j is multiplied by psi^(k (2 bitrev(j) + 1)).
void launch_monomial(const Launch &L, double *out, const double *a, size_t so, size_t sa, int npoly, int nl,
                     uint32_t k);
// Collection of independent elementwise / constant / tensor launches on one
// stream by the calling thread (kernels.hip): between begin and end the
// launchers record instead of launching; end issues one launch per kernel
// variant over up to kMaxBatch records.
void ew_collect_begin(const Launch &L);
void ew_collect_end(const Launch &L);
// out[k][i] = a[k][i] op b[k][i] over npoly polynomials of nl limbs (prime ids 0..nl-1).
void launch_ew(const Launch &L, EwOp op, double *out, const double *a, const double *b, size_t so,
               size_t sa, size_t sb, int npoly, int nl);
// out[k][i] = a[k][i] * cst_i (+ 0) with per-limb constant words.
// acc: out += a * cst (per limb constant) instead of out = a * cst.
void launch_mulconst(const Launch &L, double *out, const double *a, size_t so, size_t sa, int npoly,
                     int nl, const uint64_t *cst, bool acc = false);
void launch_addconst(const Launch &L, double *out, const double *a, int nl, const uint64_t *cst);
// acc: add the product to what d0, d1, d2 hold.
void launch_tensor(const Launch &L, double *d0, double *d1, double *d2, const double *a0,
                   const double *a1, const double *b0, const double *b1, int nl, bool acc = false);
void launch_automorph(const Launch &L, double *out, const double *in, size_t so, size_t si, int npoly,
                      int nl, uint32_t g);
// The operand of a key switch and what it adds (keyswitch.hip):
//   KS_PLAIN:   switch d, add base0 / base1 (either may be null)
//   KS_GALOIS:  switch phi_galois(d), add phi_galois(base0) (base1 null)
//   KS_PRODUCT: switch a1 b1, add a0 b0 and a0 b1 + a1 b0 (HMult + relin)
//   KS_REPACK:  one update of ring repacking (Alg. 1) per entry, entries
//               described by a RepackDesc instead of operand pointers
enum KsMode { KS_PLAIN = 0, KS_GALOIS = 1, KS_PRODUCT = 2, KS_REPACK = 3 };
struct KsOperand {
    int mode = KS_PLAIN;
    const double *d = nullptr;
    const double *base0 = nullptr, *base1 = nullptr;
    uint32_t galois = 0;
    const double *a0 = nullptr, *a1 = nullptr, *b0 = nullptr, *b1 = nullptr;
};
// A batch of key switches at one level with one key and one mode: entry b
// switches op[b] into (out0[b], out1[b]); its scratch regions sit at entry 0's
// (dcoef, ext, acc, tmp) plus b times the strides, in doubles.  Every kernel of
// the key switch covers the whole batch in one launch, and the inner product
// reads each key residue once for all entries.
constexpr int kMaxBatch = 8;
// Ring repacking round of Alg. 1, t = 2^tlog pairs per group: the ciphertexts
// of a round sit in arrays of groups (group stride in_gs / out_gs, ciphertext
// stride cs, polynomial stride ps, doubles); batch entry b is pair
// e = e0 + b, group e >> tlog, j = e mod t, and computes, with
// lo = c_j and hi = c_(j+t) of the input array,
//   out_j = lo + X^t hi + phi_g(lo - X^t hi)        (phi_g with key switching)
// into slot j of its group in the output array (which must not be the input).
struct RepackDesc {
    const double *in = nullptr;
    double *out = nullptr;
    size_t in_gs = 0, out_gs = 0, cs = 0, ps = 0;
    int tlog = 0, e0 = 0;
    uint32_t galois = 0;
};
struct KsBatch {
    int nb = 1, mode = KS_PLAIN;      // KS_REPACK: nb is not bounded by kMaxBatch
    bool hoisted = false;             // KS_GALOIS inner product: ext is the unpermuted (hoisted) ModUp
    RepackDesc rp;
    KsOperand op[kMaxBatch];
    const double *keys[kMaxBatch] = {};   // per-entry key data (all null: the launch's one key)
    double *out0[kMaxBatch] = {}, *out1[kMaxBatch] = {};
    double *dcoef = nullptr, *ext = nullptr, *acc = nullptr, *tmp = nullptr;
    size_t sdc = 0, sext = 0, sacc = 0, stmp = 0;
};
void launch_ks_inner(const Launch &L, const KsBatch &kb, const double *key, int lv);
// Scratch of one key switch (KsBatch entry 0) plus room for a tensor product.
struct KsScratch {
    double *dcoef = nullptr, *ext = nullptr, *acc = nullptr, *tmp = nullptr, *t3 = nullptr;
    size_t t3_stride = 0;
};
// HMult + relinearisation (api.cpp): the argument checks of pfx_mul_relin, and
// its launches with the scratch regions given instead of the stream's.
pfx_status mul_relin_check(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk, pfx_ct *out);
void mul_relin_run(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk, pfx_ct *out, hipStream_t st,
                   const KsScratch &s);
void launch_ks_inner_repack(const Launch &L, const KsBatch &kb, const double *key, int lv);
// The whole repacking key switch of an entry in one workgroup (N = 2^12, one
// ciphertext limb, one special prime, digits of one prime: repack_fused_ok);
// scr: kb.nb * N doubles of scratch.  Same words as ks_run in KS_REPACK mode.
bool repack_fused_ok(const pfx_ctx *c, int lv);
void launch_repack_fused(const Launch &L, const KsBatch &kb, const double *key, double *scr);
// Output slot r < n_slots (2 polynomials of lv limbs, slots cs apart,
// polynomial stride ps) = sum_l tables[l] X^(exps[r m + l]) for r < n, zero for
// r >= n; m tables of 2 polynomials at `tables` (table stride st, polynomial
// stride tps); exps in device memory (int64, taken mod 2N); ninv: times N^-1.
void launch_mono_sum(const Launch &L, double *out, size_t cs, size_t ps, const double *tables, size_t st,
                     size_t tps, int m, const int64_t *exps, int n, int n_slots, int lv, bool ninv);
// The same for 2^9 <= N <= 2^12 and at most 16 tables (mono_sum_lds_ok),
// tables in registers and twiddles in LDS.
// Ring merging: out (2 polynomials of the large ring, coefficient domain, one
// limb, N apart) from the coefficient-domain inputs at `stage` (input i,
// polynomial u at (2i + u) n), coefficient j of input i at j r + i, r = 2^log_r;
// zero where i >= n_in.
void launch_merge_gather(const Launch &L, double *out, const double *stage, int n_in, int log_r, int logn_small);
// ModRaise: coefficient-domain q_0 residues (npoly polynomials si apart) lifted
// to the centred range and reduced modulo the first nl primes (out, so apart).
void launch_mod_raise(const Launch &L, double *out, size_t so, const double *in, size_t si, int npoly, int nl);
bool mono_sum_lds_ok(const pfx_ctx *c, int m);
void launch_mono_sum_lds(const Launch &L, double *out, size_t cs, size_t ps, const double *tables, size_t st,
                         size_t tps, int m, const int64_t *exps, int n, int n_slots, int lv, bool ninv);
// Rescale of nb ciphertexts of np polynomials at lv limbs (rescale.hip): entry
// b reads ents[b].in and writes ents[b].out (which may equal in), polynomials
// si / so doubles apart; scratch `last` (nb np limbs) and `tmp` (nb np (lv - 1)
// limbs).
struct RsEntry {
    const double *in = nullptr;
    double *out = nullptr;
    size_t si = 0, so = 0;
};
void launch_rescale(const Launch &L, const RsEntry *ents, int nb, int np, int lv, double *last, double *tmp);
// Batched HMult + relin + rescale in one persistent cooperative launch, or
// step-major (one launch per step over every entry), (persist.hip) for the
// entries idx of the batch arrays; every entry's scratch
// sits in `region` (persist_entry_doubles per entry, plus the descriptors and barrier words:
// persist_tail_bytes).  Returns after the launch has finished.
bool persist_shape_ok(const pfx_ctx *c);
size_t persist_entry_doubles(const pfx_ctx *c, int lv);
size_t persist_tail_bytes(size_t n);
pfx_status launch_batch_persistent(pfx_ctx *const *ctxs, const pfx_ct *const *a, const pfx_ct *const *b,
                                   const pfx_swk *const *rlk, pfx_ct *const *out, const std::vector<size_t> &idx,
                                   double *region, size_t region_doubles, hipStream_t st, bool step_major);
// Fused key-switching steps (keyswitch.hip).
void launch_intt_scale(const Launch &L, const KsBatch &kb, int lv);
void launch_modup_col(const Launch &L, const KsBatch &kb, int lv);
void launch_intt_special(const Launch &L, const KsBatch &kb, int lv, bool col_only = false);
// The ModUp row pass fused with the inner product (and the first pass of the
// special limbs' INTT) where the tuning enables it and the batch is not
// hoisted or a repacking round (keyswitch.hip).
bool row_inner_ok(const pfx_ctx *c, const KsBatch &kb);
void launch_row_inner(const Launch &L, const KsBatch &kb, const double *key, int lv);
void launch_moddown_col(const Launch &L, const KsBatch &kb, int lv);
void launch_row_moddown(const Launch &L, const KsBatch &kb, int lv);
void launch_keygen_b(const Launch &L, double *b, const double *a, const double *e, const double *s,
                     const double *sfrom, int digit);
void launch_encrypt(const Launch &L, double *c0, const double *a, const double *e, const double *s,
                    const double *m, int lv);
void launch_decrypt(const Launch &L, double *m, const double *c0, const double *c1, const double *c2,
                    const double *s, int lv);

}  // namespace pfx
