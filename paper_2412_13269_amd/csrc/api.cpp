// C-ABI of libpfx: argument checks, host-side constants, and the sequence of
// device launches behind each call.  The kernels are in kernels.hip.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.h"
#include "linear.h"

using namespace pfx;

namespace pfx {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
pfx_status fail(pfx_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

// A captured graph and the event recorded after its last replay (waited for
// before the graph is destroyed).
struct GraphExec {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    int device = 0;
};

constexpr size_t kGraphCacheEntries = 64;

// Process-wide, deliberately never destroyed: a static destructor would run
// after the HIP runtime has been torn down at exit.
GraphCache<GraphExec> &graphs() {
    static GraphCache<GraphExec> *g = new GraphCache<GraphExec>(kGraphCacheEntries, [](GraphExec &x) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(x.device);
        if (x.done) (void)hipEventSynchronize(x.done);
        if (x.exec) (void)hipGraphExecDestroy(x.exec);
        if (x.done) (void)hipEventDestroy(x.done);
        (void)hipSetDevice(prev);
    });
    return *g;
}

// ---- pass geometry per ring degree (PassTuning), process-wide
namespace {
std::mutex g_tune_mu;
PassTuning g_tune[32];

// Loads the tuning file next to libpfx.so (written by the package's
// autotuner); a missing file leaves the defaults.
void tune_autoload() {
    Dl_info info;
    if (!dladdr(reinterpret_cast<void *>(&tune_autoload), &info) || !info.dli_fname) return;
    std::string path(info.dli_fname);
    const size_t slash = path.rfind('/');
    path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tuning.txt";
    (void)pfx_tuning_load(path.c_str());
}
}  // namespace

const PassTuning &pass_tuning(int logn) {
    if (logn < 0 || logn >= 32) logn = 0;
    return g_tune[logn];
}

void graph_forget(uint64_t uid) {
    if (uid) graphs().drop_uid(uid);
}

namespace {

struct MemRecord {
    std::shared_ptr<MemAccount> acct;
    size_t bytes;
    pfx_free_fn free;   // the caller's free function, or null for hipFree
    void *user;
};
std::mutex g_mem_mu;
std::map<void *, MemRecord> &mem_records() {
    static std::map<void *, MemRecord> *m = new std::map<void *, MemRecord>;   // never destroyed (see graphs())
    return *m;
}

}  // namespace

pfx_status dmalloc(pfx_ctx *c, void **p, size_t bytes) {
    if (!bytes) bytes = 1;
    MemAccount &a = *c->mem;
    std::lock_guard<std::mutex> g(a.mu);
    if (a.budget && a.in_use + bytes > a.budget)
        return fail(PFX_ENOMEM, "HBM budget of the context exceeded: " + std::to_string(a.in_use) + " + " +
                                    std::to_string(bytes) + " > " + std::to_string(a.budget) + " bytes");
    void *q = nullptr;
    if (a.alloc) {
        q = a.alloc(bytes, nullptr, a.user);
        if (!q) return fail(PFX_ENOMEM, "the context's allocator refused " + std::to_string(bytes) + " bytes");
    } else if (hipMalloc(&q, bytes) != hipSuccess || !q) {
        (void)hipGetLastError();
        return fail(PFX_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    {
        std::lock_guard<std::mutex> gm(g_mem_mu);
        mem_records()[q] = MemRecord{c->mem, bytes, a.alloc ? a.free : nullptr, a.user};
    }
    a.in_use += bytes;
    a.peak = std::max(a.peak, a.in_use);
    *p = q;
    return PFX_OK;
}

void dfree(void *p) {
    if (!p) return;
    MemRecord rec;
    {
        std::lock_guard<std::mutex> gm(g_mem_mu);
        auto it = mem_records().find(p);
        if (it == mem_records().end()) return;
        rec = it->second;
        mem_records().erase(it);
    }
    if (rec.free) rec.free(p, nullptr, rec.user);
    else (void)hipFree(p);
    std::lock_guard<std::mutex> g(rec.acct->mu);
    rec.acct->in_use -= rec.bytes;
}

}  // namespace pfx

#define HIPCHECK(x)                                                                          \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) return fail(PFX_EDEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

#define PFX_DMALLOC(ctx, pp, bytes)                               \
    do {                                                          \
        pfx_status r_ = dmalloc((ctx), (pp), (bytes));            \
        if (r_) return r_;                                        \
    } while (0)

// Device memory of a context held for one call: freed when the holder goes out
// of scope unless released, so an early error return leaks nothing.
template <class T>
struct DevTmp {
    T *p = nullptr;
    DevTmp() = default;
    DevTmp(const DevTmp &) = delete;
    DevTmp &operator=(const DevTmp &) = delete;
    ~DevTmp() { pfx::dfree(p); }
    T *release() {
        T *q = p;
        p = nullptr;
        return q;
    }
};

#define REQUIRE(cond, code, msg) \
    do {                         \
        if (!(cond)) return fail(code, msg); \
    } while (0)

namespace {

unsigned bitrev(unsigned x, int bits) {
    unsigned r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

double2 shoup_pair(uint64_t w, uint64_t q) { return make_double2((double)w, (double)w / (double)q); }

hipStream_t S(void *stream) { return (hipStream_t)stream; }

// Scratch of one stream, sized for the top level.
struct WsLayout {
    size_t dcoef, ext, acc, mdtmp, t3, rs_last, rs_tmp, xport, rot, total;
};

WsLayout ws_layout(const pfx_ctx *c) {
    const size_t N = c->N, L = c->L, K = c->K, E = L + K;
    WsLayout w;
    size_t o = 0;
    w.dcoef = o; o += L * N;
    w.ext = o; o += (size_t)c->beta * E * N;
    w.acc = o; o += 2 * E * N;
    w.mdtmp = o; o += 2 * L * N;
    w.t3 = o; o += 3 * L * N;
    w.rs_last = o; o += 3 * N;
    w.rs_tmp = o; o += 3 * L * N;
    w.xport = o; o += std::max<size_t>(3 * L, (size_t)E) * N;   // u64 staging (same word size)
    w.rot = o; o += 2 * L * N;                                   // rotate-sum temporary ciphertext
    w.total = o;
    return w;
}

struct Ws {
    double *base;
    WsLayout lay;
    double *at(size_t off) const { return base + off; }
};

// Key-switch scratch of nb batch entries on one stream (dcoef, ext, acc, tmp per
// entry, sized for the top level), grown on demand and kept with the stream's
// workspace.
size_t batch_entry_doubles(const pfx_ctx *c) {
    const size_t N = c->N, L = c->L, K = c->K, E = L + K;
    return L * N + (size_t)c->beta * E * N + 2 * E * N + 2 * L * N;
}

pfx_status get_batch_ws(pfx_ctx *c, hipStream_t st, int nb, KsBatch &kb) {
    const size_t N = c->N, L = c->L, K = c->K, E = L + K;
    const size_t sdc = L * N, sext = (size_t)c->beta * E * N, sacc = 2 * E * N, stmp = 2 * L * N;
    const size_t per = batch_entry_doubles(c);
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->ws.find(st);
    if (it == c->ws.end()) return fail(PFX_EINVAL, "stream has no workspace");
    Workspace *w = it->second;
    if (w->bcap < nb) {
        if (c->capturing) return fail(PFX_EINVAL, "batch workspace must be reserved before graph capture");
        (void)hipStreamSynchronize(st);   // the old region may still be in use on this stream
        bump_scratch_epoch();             // graphs captured against the old region are stale
        dfree(w->bbuf);
        w->bbuf = nullptr;
        w->bcap = 0;
        pfx_status r = dmalloc(c, &w->bbuf, (size_t)nb * per * sizeof(double));
        if (r) return r;
        w->bcap = nb;
    }
    double *base = w->bbuf;
    kb.dcoef = base;
    kb.ext = base + (size_t)nb * sdc;
    kb.acc = kb.ext + (size_t)nb * sext;
    kb.tmp = kb.acc + (size_t)nb * sacc;
    kb.sdc = sdc;
    kb.sext = sext;
    kb.sacc = sacc;
    kb.stmp = stmp;
    return PFX_OK;
}

pfx_status get_ws(pfx_ctx *c, hipStream_t st, Ws &out) {
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->ws.find(st);
    if (it == c->ws.end()) {
        Workspace *w = new Workspace;
        w->stream = st;
        WsLayout lay = ws_layout(c);
        w->doubles = lay.total;
        pfx_status r = dmalloc(c, &w->buf, lay.total * sizeof(double));
        if (r) {
            delete w;
            return r;
        }
        it = c->ws.emplace(st, w).first;
    }
    out.base = it->second->buf;
    out.lay = ws_layout(c);
    return PFX_OK;
}

LimbMap contiguous_map(int n, int pid0, int off0 = 0) {
    LimbMap m;
    m.n = n;
    for (int i = 0; i < n; ++i) {
        m.off[i] = off0 + i;
        m.pid[i] = (int16_t)(pid0 + i);
    }
    return m;
}

// limbs [0, lv) of npoly polynomials spaced `stride_limbs` apart
LimbMap poly_map(int npoly, int lv, int stride_limbs) {
    LimbMap m;
    m.n = npoly * lv;
    for (int k = 0; k < npoly; ++k)
        for (int i = 0; i < lv; ++i) {
            m.off[k * lv + i] = k * stride_limbs + i;
            m.pid[k * lv + i] = (int16_t)i;
        }
    return m;
}

bool scale_close(double a, double b) { return std::fabs(a / b - 1.0) <= std::ldexp(1.0, -10); }

pfx_status check_ct(const pfx_ctx *c, const pfx_ct *x, const char *what) {
    if (!x) return fail(PFX_EINVAL, std::string(what) + " is null");
    if (x->ctx != c) return fail(PFX_EINVAL, std::string(what) + " belongs to another context");
    if (x->n_limbs == 0) return fail(PFX_EINVAL, std::string(what) + " is empty");
    return PFX_OK;
}

pfx_status check_out(const pfx_ct *o, uint32_t lv, uint32_t deg) {
    if (!o) return fail(PFX_EINVAL, "output is null");
    if (o->cap_limbs < lv || o->cap_degree < deg) return fail(PFX_EINVAL, "output capacity too small");
    return PFX_OK;
}

// Key switching (Sec. 2.4.1) of a batch: for every entry b, out_u = ModDown(
// sum_j ModUp_j(d) * swk_{j,u}) + base_u, with d and the bases as the
// operand describes them (KsOperand: plain, read through an automorphism, or
// formed from a ciphertext product).  Six kernels and one row-pass launch,
// each covering the whole batch (keyswitch.hip).  The last kernel reads the
// bases while other workgroups write the outputs, so no output may alias a
// permuted base (KS_GALOIS) or a product operand (KS_PRODUCT) of any entry;
// callers copy or fall back first.
// Steps 1-3a (ModUp into the NTT domain of every target limb) of a batch.
void ks_modup_ext(const Launch &L, const KsBatch &kb, int lv);

void ks_modup(const Launch &L, const KsBatch &kb, int lv) {
    launch_intt_scale(L, kb, lv);
    ks_modup_ext(L, kb, lv);
}

// Steps 2-3a: the conversion into the column pass and the row pass of the
// ModUp limbs.
void ks_modup_ext(const Launch &L, const KsBatch &kb, int lv) {
    pfx_ctx *c = L.ctx;
    const int E = lv + c->K;
    launch_modup_col(L, kb, lv);
    const int beta = (lv + c->alpha - 1) / c->alpha;
    LimbMap m;
    m.n = 0;
    for (int j = 0; j < beta; ++j) {
        const int sz = std::min(c->alpha, lv - j * c->alpha);
        for (int t = 0; t < E - sz; ++t) {
            m.off[m.n] = j * E + t;
            m.pid[m.n] = (int16_t)(t < j * c->alpha ? t : (t < lv - sz ? t + sz : c->L + (t - (lv - sz))));
            if (++m.n == kMaxMapLimbs) {
                launch_ntt_pass(L, kb.ext, nullptr, m, true, false, kb.nb, kb.sext);
                m.n = 0;
            }
        }
    }
    launch_ntt_pass(L, kb.ext, nullptr, m, true, false, kb.nb, kb.sext);
}

// Steps 4-6 (ModDown and the combination with the bases) of a batch.
void ks_moddown(const Launch &L, const KsBatch &kb, int lv) {
    launch_intt_special(L, kb, lv);
    launch_moddown_col(L, kb, lv);
    launch_row_moddown(L, kb, lv);
}

// End of the key-switch batch that starts at order[s0]: entries of one
// level; a run of equal levels is split into batches of at most the tuned
// bound (ks_batch, at most kMaxBatch) of sizes as equal as possible.
template <class Lv>
size_t ks_batch_end(const pfx_ctx *c, const int *order, size_t n, const Lv &lvs, size_t s0) {
    size_t e = s0;
    while (e < n && lvs[order[e]] == lvs[order[s0]]) ++e;
    const size_t run = e - s0;
    const size_t bound = (size_t)std::max(1, std::min(kMaxBatch, pass_tuning(c->logn).ks_batch));
    const size_t nbat = (run + bound - 1) / bound;
    return s0 + (run + nbat - 1) / nbat;
}

// Entries [b0, b0 + n) of a batch (not a repacking round) as a batch of their
// own: the same kernels over the entries' scratch regions.
KsBatch ks_slice(const KsBatch &kb, int b0, int n) {
    KsBatch s = kb;
    s.nb = n;
    for (int e = 0; e < kMaxBatch; ++e) {
        const bool on = e < n;
        s.op[e] = on ? kb.op[b0 + e] : KsOperand{};
        s.keys[e] = on ? kb.keys[b0 + e] : nullptr;
        s.out0[e] = on ? kb.out0[b0 + e] : nullptr;
        s.out1[e] = on ? kb.out1[b0 + e] : nullptr;
    }
    s.dcoef = kb.dcoef + (size_t)b0 * kb.sdc;
    s.ext = kb.ext + (size_t)b0 * kb.sext;
    s.acc = kb.acc + (size_t)b0 * kb.sacc;
    s.tmp = kb.tmp + (size_t)b0 * kb.stmp;
    return s;
}

void ks_run(const Launch &L, const KsBatch &kb, int lv, const pfx_swk *key) {
    const int sub = pass_tuning(L.ctx->logn).ks_modup_batch;
    if (kb.mode != KS_REPACK && !kb.hoisted && sub > 0 && sub < kb.nb && !row_inner_ok(L.ctx, kb)) {
        // the ModUp limbs of a few entries at a time, written by the
        // conversion, read and rewritten by the row pass and read by the inner
        // product while they still sit in the last-level cache; the small
        // launches before and after cover the whole batch
        launch_intt_scale(L, kb, lv);
        for (int b0 = 0; b0 < kb.nb; b0 += sub) {
            const KsBatch s = ks_slice(kb, b0, std::min(sub, kb.nb - b0));
            ks_modup_ext(L, s, lv);
            launch_ks_inner(L, s, key->d_k, lv);
        }
        ks_moddown(L, kb, lv);
        return;
    }
    if (row_inner_ok(L.ctx, kb)) {
        // the ModUp row pass, the inner product and the special limbs' first
        // INTT pass in one launch
        launch_intt_scale(L, kb, lv);
        launch_modup_col(L, kb, lv);
        launch_row_inner(L, kb, key->d_k, lv);
        launch_intt_special(L, kb, lv, true);
        launch_moddown_col(L, kb, lv);
        launch_row_moddown(L, kb, lv);
        return;
    }
    ks_modup(L, kb, lv);
    if (kb.mode == KS_REPACK) launch_ks_inner_repack(L, kb, key->d_k, lv);
    else launch_ks_inner(L, kb, key->d_k, lv);
    ks_moddown(L, kb, lv);
}

// One key switch in the stream's scratch.
void ks_core(pfx_ctx *c, const Launch &L, const Ws &w, const KsOperand &op, int lv, const pfx_swk *key,
             double *out0, double *out1) {
    (void)c;
    KsBatch kb;
    kb.nb = 1;
    kb.mode = op.mode;
    kb.op[0] = op;
    kb.out0[0] = out0;
    kb.out1[0] = out1;
    kb.dcoef = w.at(w.lay.dcoef);
    kb.ext = w.at(w.lay.ext);
    kb.acc = w.at(w.lay.acc);
    kb.tmp = w.at(w.lay.mdtmp);
    ks_run(L, kb, lv, key);
}

KsOperand ks_plain(const double *d, const double *base0, const double *base1) {
    KsOperand op;
    op.mode = KS_PLAIN;
    op.d = d;
    op.base0 = base0;
    op.base1 = base1;
    return op;
}

pfx_swk *find_key(pfx_ctx *c, uint32_t g, const pfx_swk *const *keys, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (keys[i] && keys[i]->ctx == c && keys[i]->galois == g) return const_cast<pfx_swk *>(keys[i]);
    return nullptr;
}

pfx_status galois_apply(pfx_ctx *c, const pfx_ct *a, const pfx_swk *gk, pfx_ct *out, hipStream_t st) {
    Ws w;
    pfx_status r = get_ws(c, st, w);
    if (r) return r;
    const int lv = a->n_limbs;
    Launch L{c, st};
    KsOperand op;
    op.mode = KS_GALOIS;
    op.d = a->poly(1);
    op.base0 = a->poly(0);
    op.galois = gk->galois;
    if (out->d == a->d) {
        // in place: c0 is read through the permutation while out0 is written,
        // so it is read from a copy (c1 is only written by the last launch)
        double *t0 = w.at(w.lay.t3);
        launch_ew(L, EW_COPY, t0, a->poly(0), nullptr, (size_t)c->L * c->N, (size_t)a->cap_limbs * c->N, 0, 1, lv);
        op.base0 = t0;
    }
    ks_core(c, L, w, op, lv, gk, out->poly(0), out->poly(1));
    out->n_limbs = lv;
    out->degree = 1;
    out->scale = a->scale;
    return PFX_OK;
}

uint32_t rot_element(const pfx_ctx *c, int64_t step) {
    const int64_t half = c->N / 2;
    int64_t s = ((step % half) + half) % half;
    return (uint32_t)powmod_u64(5, (uint64_t)s, 2ull * c->N);
}

}  // namespace

namespace pfx {

size_t ws_bytes(const pfx_ctx *c) { return ws_layout(c).total * sizeof(double); }

size_t batch_ws_bytes(const pfx_ctx *c, int nb) { return (size_t)nb * batch_entry_doubles(c) * sizeof(double); }

pfx_status batch_ws_reserve(pfx_ctx *c, hipStream_t st, int nb) {
    KsBatch kb;
    return get_batch_ws(c, st, nb, kb);
}

pfx_status ws_reserve(pfx_ctx *c, hipStream_t st) {
    Ws w;
    return get_ws(c, st, w);
}

// One op of an op list on `stream`.
static pfx_status run_op(pfx_ctx *c, size_t i, const pfx_op &o, pfx_ct *const *regs, size_t n_regs, size_t n_inputs,
                         const pfx_pt *const *pts, size_t n_pts, const pfx_swk *rlk, const pfx_swk *const *gks,
                         size_t n_gks, void *stream) {
    if (o.code == PFX_OP_LANE) return PFX_OK;
    auto R = [&](int32_t k) -> pfx_ct * { return (k >= 0 && (size_t)k < n_regs) ? regs[k] : nullptr; };
    pfx_ct *d = R(o.dst), *A = R(o.a);
    const std::string at = "op " + std::to_string(i) + ": ";
    if (!d || !A) return fail(PFX_EINVAL, at + "register index out of range");
    if ((size_t)o.dst < n_inputs) return fail(PFX_EINVAL, at + "writes an input register");
    const pfx_pt *pt = (o.b >= 0 && (size_t)o.b < n_pts) ? pts[o.b] : nullptr;
    pfx_status r;
    switch (o.code) {
        case PFX_OP_COPY: r = pfx_ct_copy(c, A, d, stream); break;
        case PFX_OP_ADD: r = pfx_add(c, A, R(o.b), d, stream); break;
        case PFX_OP_SUB: r = pfx_sub(c, A, R(o.b), d, stream); break;
        case PFX_OP_MUL_PLAIN: r = pfx_mul_plain(c, A, pt, d, stream); break;
        case PFX_OP_ADD_PLAIN: r = pfx_add_plain(c, A, pt, d, stream); break;
        case PFX_OP_MUL_INT: r = pfx_mul_int(c, A, o.k, d, stream); break;
        case PFX_OP_MUL_RELIN: r = pfx_mul_relin(c, A, R(o.b), rlk, d, stream); break;
        case PFX_OP_MUL: r = pfx_mul(c, A, R(o.b), d, stream); break;
        case PFX_OP_MUL_ACC: r = pfx_mul_acc(c, A, R(o.b), d, stream); break;
        case PFX_OP_MUL_PLAIN_ACC: r = pfx_mul_plain_acc(c, A, pt, d, stream); break;
        case PFX_OP_MUL_INT_ACC: r = pfx_mul_int_acc(c, A, o.k, d, stream); break;
        case PFX_OP_MONO: r = pfx_mul_monomial(c, A, o.k, d, stream); break;
        case PFX_OP_INV_N: r = pfx_mul_inv_n(c, A, d, stream); break;
        case PFX_OP_GALOIS: {
            pfx_swk *gk = (o.k > 0 && o.k < 2 * (int64_t)c->N) ? find_key(c, (uint32_t)o.k, gks, n_gks) : nullptr;
            if (!gk) return fail(PFX_ENOKEY, at + "no Galois key for element " + std::to_string(o.k));
            r = pfx_apply_galois(c, A, gk, d, stream);
            break;
        }
        case PFX_OP_DROP:
            if (o.k < 1 || o.k > (int64_t)A->n_limbs) return fail(PFX_ELEVEL, at + "cannot drop to that many limbs");
            r = pfx_drop_level(c, A, (uint32_t)o.k, d, stream);
            break;
        case PFX_OP_RELIN: r = pfx_relinearize(c, A, rlk, d, stream); break;
        case PFX_OP_RESCALE: r = pfx_rescale(c, A, d, stream); break;
        case PFX_OP_ADD_CONST: r = pfx_add_const(c, A, o.value, d, stream); break;
        case PFX_OP_MUL_CONST: r = pfx_mul_const(c, A, o.value, 0.0, d, stream); break;
        case PFX_OP_MUL_CONST_TO: {
            const pfx_ct *B = R(o.b);
            if (!B) return fail(PFX_EINVAL, at + "register index out of range");
            if (A->n_limbs < 2) return fail(PFX_ELEVEL, at + "no prime left to rescale by");
            const double cs = B->scale * (double)c->primes[A->n_limbs - 1] / A->scale;
            r = pfx_mul_const(c, A, o.value, cs, d, stream);
            break;
        }
        case PFX_OP_MUL_CONST_LIKE: {
            const pfx_ct *B = R(o.b);
            if (!B) return fail(PFX_EINVAL, at + "register index out of range");
            r = pfx_mul_const(c, A, o.value, B->scale / A->scale, d, stream);
            break;
        }
        case PFX_OP_SCALE_MUL: {
            const double sc = A->scale * o.value;
            r = pfx_ct_copy(c, A, d, stream);
            if (!r) d->scale = sc;
            break;
        }
        case PFX_OP_ROTATE: r = pfx_rotate(c, A, (int32_t)o.k, gks, n_gks, d, stream); break;
        case PFX_OP_ROTATE_SUM: r = pfx_rotate_sum(c, A, (uint32_t)o.k, gks, n_gks, d, stream); break;
        default: return fail(PFX_EINVAL, at + "unknown op code");
    }
    if (r) return fail(r, at + g_err);
    return PFX_OK;
}

// Length of the run of ops starting at ops[i] that one batched launch sequence
// may take: consecutive HMult + relin ops (or consecutive relinearisations,
// rescales, or automorphisms by one Galois element), at most max_batch,
// outputs distinct and none of them an operand of another op of the run, so
// the ops are independent.  An HMult + relin or automorphism output must not
// alias its own operands either (the batched key switch reads them while it
// writes); a relinearisation or a rescale may work in place.  1 if ops[i]
// alone; 0 for any other op.
size_t mr_run(const pfx_op *ops, size_t n_ops, size_t i, int max_batch) {
    const int32_t code = ops[i].code;
    if (code != PFX_OP_MUL_RELIN && code != PFX_OP_RESCALE && code != PFX_OP_RELIN && code != PFX_OP_GALOIS) return 0;
    const bool rb = code == PFX_OP_MUL_RELIN;                      // b is a register
    const bool no_self = rb || code == PFX_OP_GALOIS;              // no in-place output
    auto reads = [&](const pfx_op &o, int32_t r) { return o.a == r || (rb && o.b == r); };
    const pfx_op &f = ops[i];
    if (no_self && reads(f, f.dst)) return 1;
    size_t j = i + 1;
    for (; j < n_ops && j - i < (size_t)max_batch && ops[j].code == code; ++j) {
        const pfx_op &o = ops[j];
        bool ok = !(no_self && reads(o, o.dst)) && (code != PFX_OP_GALOIS || o.k == f.k);
        for (size_t k = i; k < j && ok; ++k) {
            const pfx_op &p = ops[k];
            ok = o.dst != p.dst && !reads(p, o.dst) && !reads(o, p.dst);
        }
        if (!ok) break;
    }
    return j - i;
}

// Elementwise ops (one or two elementwise, constant or tensor launches each,
// no scratch): runs of independent ones are issued as collected launches.
bool ew_code(int32_t code) {
    switch (code) {
        case PFX_OP_COPY: case PFX_OP_ADD: case PFX_OP_SUB: case PFX_OP_MUL_PLAIN: case PFX_OP_ADD_PLAIN:
        case PFX_OP_MUL_INT: case PFX_OP_MUL: case PFX_OP_MUL_ACC: case PFX_OP_MUL_PLAIN_ACC:
        case PFX_OP_MUL_INT_ACC: case PFX_OP_ADD_CONST: case PFX_OP_MUL_CONST: case PFX_OP_SCALE_MUL:
        case PFX_OP_DROP: case PFX_OP_MONO: case PFX_OP_INV_N: case PFX_OP_MUL_CONST_TO:
        case PFX_OP_MUL_CONST_LIKE:
            return true;
        default:
            return false;
    }
}

bool accumulates(int32_t code) {
    return code == PFX_OP_MUL_ACC || code == PFX_OP_MUL_PLAIN_ACC || code == PFX_OP_MUL_INT_ACC;
}

bool reads_b_reg(int32_t code) {
    return code == PFX_OP_ADD || code == PFX_OP_SUB || code == PFX_OP_MUL_RELIN || code == PFX_OP_MUL ||
           code == PFX_OP_MUL_ACC || code == PFX_OP_MUL_CONST_TO ||
           code == PFX_OP_MUL_CONST_LIKE;
}

// Registers an op reads (a, a register b, and an accumulator), as indices.
int op_reads(const pfx_op &o, int32_t out[3]) {
    int n = 0;
    out[n++] = o.a;
    if (reads_b_reg(o.code)) out[n++] = o.b;
    if (accumulates(o.code)) out[n++] = o.dst;
    return n;
}

// Run of consecutive ops with the same elementwise code from ops[i], at most
// max_batch, none writing what another of the run reads or writes.
size_t ew_run(const pfx_op *ops, size_t n_ops, size_t i, int max_batch) {
    if (!ew_code(ops[i].code)) return 0;
    size_t j = i + 1;
    for (; j < n_ops && j - i < (size_t)max_batch && ops[j].code == ops[i].code; ++j) {
        bool ok = true;
        int32_t rj[3];
        const int nj = op_reads(ops[j], rj);
        for (size_t k = i; k < j && ok; ++k) {
            int32_t rk[3];
            const int nk = op_reads(ops[k], rk);
            ok = ops[j].dst != ops[k].dst;
            for (int x = 0; x < nk && ok; ++x) ok = rk[x] != ops[j].dst;
            for (int x = 0; x < nj && ok; ++x) ok = rj[x] != ops[k].dst;
        }
        if (!ok) break;
    }
    return j - i;
}

// The same independence on the ciphertexts the registers name (two registers
// may hold one ciphertext).
bool ew_run_distinct(const pfx_op *ops, size_t i, size_t run, pfx_ct *const *regs, size_t n_regs) {
    auto R = [&](int32_t x) -> const pfx_ct * { return (x >= 0 && (size_t)x < n_regs) ? regs[x] : nullptr; };
    for (size_t k = 0; k < run; ++k) {
        const pfx_ct *dk = R(ops[i + k].dst);
        if (!dk) return false;
        for (size_t m = 0; m < run; ++m) {
            if (m == k) continue;
            const pfx_ct *dm = R(ops[i + m].dst);
            if (!dm || dm->d == dk->d) return false;
            int32_t rm[3];
            const int nm = op_reads(ops[i + m], rm);
            for (int x = 0; x < nm; ++x) {
                const pfx_ct *r = R(rm[x]);
                if (!r || r->d == dk->d) return false;
            }
        }
    }
    return true;
}

// Largest batch that run_span will hand to one batched call.
size_t max_mr_run(const pfx_op *ops, size_t n_ops, int max_batch) {
    size_t m = 0;
    for (size_t i = 0; i < n_ops;) {
        const size_t r = mr_run(ops, n_ops, i, max_batch);
        m = std::max(m, r);
        i += r ? r : 1;
    }
    return m;
}

// ops[lo, hi) on one stream; runs of independent HMult + relin ops,
// relinearisations or rescales (mr_run) go to pfx_mul_relin_batch /
// pfx_relinearize_batch / pfx_rescale_batch when max_batch > 1.
pfx_status run_span(pfx_ctx *c, const pfx_op *ops, size_t lo, size_t hi, pfx_ct *const *regs, size_t n_regs,
                    size_t n_inputs, const pfx_pt *const *pts, size_t n_pts, const pfx_swk *rlk,
                    const pfx_swk *const *gks, size_t n_gks, void *stream, int max_batch) {
    for (size_t i = lo; i < hi;) {
        const size_t ew = max_batch > 1 ? ew_run(ops, hi, i, kMaxBatch) : 0;
        if (ew > 1 && ew_run_distinct(ops, i, ew, regs, n_regs)) {
            const Launch L{c, S(stream)};
            ew_collect_begin(L);
            pfx_status r = PFX_OK;
            for (size_t k = 0; k < ew && !r; ++k)
                r = run_op(c, i + k, ops[i + k], regs, n_regs, n_inputs, pts, n_pts, rlk, gks, n_gks, stream);
            ew_collect_end(L);      // what was recorded is issued, also after a failed op
            if (r) return r;
            i += ew;
            continue;
        }
        const size_t run = max_batch > 1 ? mr_run(ops, hi, i, max_batch) : 0;
        if (run > 1) {
            const bool mr = ops[i].code == PFX_OP_MUL_RELIN;
            const bool gal = ops[i].code == PFX_OP_GALOIS;
            const pfx_ct *a[kMaxBatch], *b[kMaxBatch];
            pfx_ct *out[kMaxBatch];
            bool distinct = true;       // distinct registers may still name one ciphertext
            for (size_t k = 0; k < run; ++k) {
                const pfx_op &o = ops[i + k];
                auto R = [&](int32_t x) -> pfx_ct * { return (x >= 0 && (size_t)x < n_regs) ? regs[x] : nullptr; };
                a[k] = R(o.a);
                b[k] = mr ? R(o.b) : a[k];
                out[k] = R(o.dst);
                if (!a[k] || !b[k] || !out[k] || (size_t)o.dst < n_inputs) {
                    distinct = false;   // run_op reports the error
                    break;
                }
            }
            for (size_t k = 0; k < run && distinct; ++k)
                for (size_t m = 0; m < run && distinct; ++m) {
                    if (k != m) distinct = out[k]->d != a[m]->d && out[k]->d != b[m]->d && out[k]->d != out[m]->d;
                    else if (mr || gal) distinct = out[k]->d != a[k]->d && out[k]->d != b[k]->d;
                }
            pfx_swk *gk = nullptr;
            if (gal) {
                const int64_t g = ops[i].k;
                gk = (g > 0 && g < 2 * (int64_t)c->N) ? find_key(c, (uint32_t)g, gks, n_gks) : nullptr;
                distinct = distinct && gk;     // a missing key: run_op reports it
            }
            if (distinct) {
                pfx_status r = mr ? pfx_mul_relin_batch(c, a, b, run, rlk, out, stream)
                               : gal ? pfx_apply_galois_batch(c, a, run, gk, out, stream)
                               : ops[i].code == PFX_OP_RELIN ? pfx_relinearize_batch(c, a, run, rlk, out, stream)
                                                             : pfx_rescale_batch(c, a, run, out, stream);
                if (r) return fail(r, "ops " + std::to_string(i) + ".." + std::to_string(i + run - 1) + ": " + g_err);
                i += run;
                continue;
            }
        }
        pfx_status r = run_op(c, i, ops[i], regs, n_regs, n_inputs, pts, n_pts, rlk, gks, n_gks, stream);
        if (r) return r;
        ++i;
    }
    return PFX_OK;
}

pfx_status run_ops(pfx_ctx *c, const pfx_op *ops, size_t n_ops, pfx_ct *const *regs, size_t n_regs,
                   size_t n_inputs, const pfx_pt *const *pts, size_t n_pts, const pfx_swk *rlk,
                   const pfx_swk *const *gks, size_t n_gks, void *stream, int max_batch) {
    return run_span(c, ops, 0, n_ops, regs, n_regs, n_inputs, pts, n_pts, rlk, gks, n_gks, stream, max_batch);
}

}  // namespace pfx

// ======================================================================= API
extern "C" {

const char *pfx_status_str(pfx_status s) {
    switch (s) {
        case PFX_OK: return "ok";
        case PFX_EINVAL: return "invalid argument";
        case PFX_EPARAM: return "unsupported parameters";
        case PFX_ELEVEL: return "not enough limbs";
        case PFX_ESCALE: return "scale mismatch";
        case PFX_ENOKEY: return "missing key";
        case PFX_ENOMEM: return "out of memory";
        case PFX_EBUSY: return "busy";
        case PFX_EDEVICE: return "device error";
        default: return "unknown status";
    }
}

const char *pfx_last_error(void) { return g_err.c_str(); }

pfx_status pfx_params_primes(const pfx_params *prm, uint64_t *q, uint64_t *p, uint64_t *psi) {
    std::vector<uint64_t> vq, vp, vpsi;
    std::string err;
    if (!build_primes(prm, vq, vp, vpsi, err)) return fail(PFX_EPARAM, err);
    if (q) std::copy(vq.begin(), vq.end(), q);
    if (p) std::copy(vp.begin(), vp.end(), p);
    if (psi) std::copy(vpsi.begin(), vpsi.end(), psi);
    return PFX_OK;
}

pfx_status pfx_encode_words(const pfx_params *prm, const double *re, const double *im, size_t n, uint32_t n_limbs,
                            double scale, uint64_t *words) {
    REQUIRE(re && words, PFX_EINVAL, "null argument");
    std::vector<uint64_t> q, p, psi, out;
    std::string err;
    if (!build_primes(prm, q, p, psi, err)) return fail(PFX_EPARAM, err);
    REQUIRE(n_limbs >= 1 && n_limbs <= q.size(), PFX_EINVAL, "n_limbs out of range");
    REQUIRE(scale > 0 && std::isfinite(scale), PFX_EINVAL, "bad scale");
    std::vector<uint64_t> mods(q.begin(), q.begin() + n_limbs);
    if (!encode_coeffs(prm->log_n, re, im, n, scale, mods, out, err)) return fail(PFX_EINVAL, err);
    std::copy(out.begin(), out.end(), words);
    return PFX_OK;
}

pfx_status pfx_decode_words(const pfx_params *prm, const uint64_t *words, uint32_t n_limbs, double scale, double *re,
                            double *im, size_t n) {
    REQUIRE(re && words, PFX_EINVAL, "null argument");
    std::vector<uint64_t> q, p, psi;
    std::string err;
    if (!build_primes(prm, q, p, psi, err)) return fail(PFX_EPARAM, err);
    REQUIRE(n_limbs >= 1 && n_limbs <= q.size(), PFX_EINVAL, "n_limbs out of range");
    const size_t N = (size_t)1 << prm->log_n;
    REQUIRE(n >= 1 && !(n & (n - 1)) && n <= N / 2, PFX_EINVAL, "n_slots must be a power of two <= N/2");
    for (size_t i = 0; i < (size_t)n_limbs * N; ++i) REQUIRE(words[i] < q[i / N], PFX_EINVAL, "word not below its prime");
    std::vector<uint64_t> mods(q.begin(), q.begin() + n_limbs);
    decode_words(prm->log_n, words, n_limbs, mods, scale, n, re, im);
    return PFX_OK;
}

pfx_status pfx_ctx_create(const pfx_params *prm, int device, pfx_ctx **out) {
    REQUIRE(out, PFX_EINVAL, "out is null");
    std::vector<uint64_t> q, p, psi;
    std::string err;
    if (!build_primes(prm, q, p, psi, err)) return fail(PFX_EPARAM, err);
    REQUIRE(prm->n_p <= 7, PFX_EPARAM, "at most 7 special primes");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
        return fail(PFX_EDEVICE, "no such HIP device");
    HIPCHECK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHECK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PFX_EDEVICE, std::string("libpfx is built for gfx950, device is ") + prop.gcnArchName);

    static std::once_flag tune_once;
    std::call_once(tune_once, tune_autoload);   // the autotuner's table, if one sits next to the library
    pfx_status nr = noalloc_init(device);   // once per device, this device current
    if (nr) return nr;
    std::unique_ptr<pfx_ctx> c(new pfx_ctx);
    c->uid = next_uid();
    c->device = device;
    c->logn = prm->log_n;
    c->N = 1 << prm->log_n;
    c->L = prm->n_q;
    c->K = prm->n_p;
    c->alpha = prm->alpha;
    c->beta = (c->L + c->alpha - 1) / c->alpha;
    c->mod_log2 = prm->mod_log2 ? prm->mod_log2 : prm->log_n + 1;
    c->primes = q;
    c->primes.insert(c->primes.end(), p.begin(), p.end());
    c->psi = psi;
    const int NP = c->L + c->K;
    const size_t N = c->N;

    // twiddles: tw[k] = psi^bitrev(k), itw[k] = psi^-bitrev(k), with their fl(w/q)
    std::vector<double2> tw((size_t)2 * NP * N);
    std::vector<uint64_t> pw(N), ipw(N);
    for (int m = 0; m < NP; ++m) {
        const uint64_t qq = c->primes[m];
        const uint64_t ps = psi[m], ips = invmod_u64(ps, qq);
        pw[0] = ipw[0] = 1;
        for (size_t i = 1; i < N; ++i) {
            pw[i] = mulmod_u64(pw[i - 1], ps, qq);
            ipw[i] = mulmod_u64(ipw[i - 1], ips, qq);
        }
        for (size_t k = 0; k < N; ++k) {
            const unsigned b = bitrev((unsigned)k, c->logn);
            tw[(2 * (size_t)m) * N + k] = shoup_pair(pw[b], qq);
            tw[(2 * (size_t)m + 1) * N + k] = shoup_pair(ipw[b], qq);
        }
    }
    {
        pfx_status r = dmalloc(c.get(), &c->d_tw, tw.size() * sizeof(double2));
        if (r) return r;
    }
    HIPCHECK(hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
    // row-pass generated twiddles (see PrimeDev)
    const int Srow = c->logn - c->logn / 2, R2 = Srow - (Srow + 1) / 2, T = c->logn - R2;
    const size_t nT = (size_t)1 << T;
    std::vector<double> rtw((size_t)2 * NP * nT);
    for (int m = 0; m < NP; ++m) {
        const uint64_t qq = c->primes[m];
        const uint64_t ps = psi[m], ips = invmod_u64(ps, qq);
        for (size_t P = 0; P < nT; ++P) {
            const uint64_t e = 2ull * bitrev((unsigned)P, T);
            rtw[(2 * (size_t)m) * nT + P] = (double)powmod_u64(ps, e, qq);
            rtw[(2 * (size_t)m + 1) * nT + P] = (double)powmod_u64(ips, e, qq);
        }
    }
    {
        pfx_status r = dmalloc(c.get(), &c->d_rtw, rtw.size() * sizeof(double));
        if (r) return r;
    }
    HIPCHECK(hipMemcpy(c->d_rtw, rtw.data(), rtw.size() * sizeof(double), hipMemcpyHostToDevice));
    c->h_primes.resize(NP);
    for (int m = 0; m < NP; ++m) {
        const uint64_t qq = c->primes[m];
        PrimeDev &d = c->h_primes[m];
        d.q = (double)qq;
        d.qinv = 1.0 / (double)qq;
        const uint64_t ninv = invmod_u64(N % qq, qq);
        d.ninv = (double)ninv;
        d.ninv_q = (double)ninv / (double)qq;
        const uint64_t w1 = mulmod_u64(ninv, powmod_u64(invmod_u64(psi[m], qq), N / 2, qq), qq);
        d.ninv_w1 = (double)w1;
        d.ninv_w1_q = (double)w1 / (double)qq;
        d.tw = c->d_tw + (2 * (size_t)m) * N;
        d.itw = c->d_tw + (2 * (size_t)m + 1) * N;
        d.rtw = c->d_rtw + (2 * (size_t)m) * nT;
        d.irtw = c->d_rtw + (2 * (size_t)m + 1) * nT;
        std::memset(d.rc, 0, sizeof d.rc);
        std::memset(d.irc, 0, sizeof d.irc);
        const uint64_t ips = invmod_u64(psi[m], qq);
        for (int k = 0; k < R2; ++k)
            for (int x = 0; x < (1 << k); ++x) {
                const uint64_t e = (1ull << (c->logn - 1 - T - k)) + (uint64_t)bitrev((unsigned)x, k) * (1ull << (c->logn - k));
                d.rc[(1 << k) - 1 + x] = (double)powmod_u64(psi[m], e, qq);
                d.irc[(1 << k) - 1 + x] = (double)powmod_u64(ips, e, qq);
            }
    }
    {
        pfx_status r = dmalloc(c.get(), &c->d_primes, NP * sizeof(PrimeDev));
        if (r) return r;
    }
    HIPCHECK(hipMemcpy(c->d_primes, c->h_primes.data(), NP * sizeof(PrimeDev), hipMemcpyHostToDevice));

    // ModUp: for digit j with sz active primes D = {alpha j, ..., alpha j + sz - 1}
    std::vector<ModUpConst> mu((size_t)c->beta * c->alpha);
    std::memset(mu.data(), 0, mu.size() * sizeof(ModUpConst));
    for (int j = 0; j < c->beta; ++j)
        for (int sz = 1; sz <= c->alpha; ++sz) {
            const int j0 = j * c->alpha;
            if (j0 + sz > c->L) continue;
            ModUpConst &x = mu[(size_t)j * c->alpha + (sz - 1)];
            for (int i = 0; i < sz; ++i) {
                const uint64_t qi = c->primes[j0 + i];
                uint64_t prod = 1;   // (Q'/q_i) mod q_i
                for (int i2 = 0; i2 < sz; ++i2)
                    if (i2 != i) prod = mulmod_u64(prod, c->primes[j0 + i2] % qi, qi);
                x.inv[i] = shoup_pair(invmod_u64(prod, qi), qi);
                for (int m = 0; m < NP; ++m) {
                    const uint64_t qm = c->primes[m];
                    uint64_t h = 1;
                    for (int i2 = 0; i2 < sz; ++i2)
                        if (i2 != i) h = mulmod_u64(h, c->primes[j0 + i2] % qm, qm);
                    x.hat[i][m] = shoup_pair(h, qm);
                }
            }
        }
    {
        pfx_status r = dmalloc(c.get(), &c->d_modup, mu.size() * sizeof(ModUpConst));
        if (r) return r;
    }
    HIPCHECK(hipMemcpy(c->d_modup, mu.data(), mu.size() * sizeof(ModUpConst), hipMemcpyHostToDevice));

    // ModDown and key-generation constants
    std::unique_ptr<ModDownConst> md(new ModDownConst);
    std::memset(md.get(), 0, sizeof(ModDownConst));
    for (int k = 0; k < c->K; ++k) {
        const uint64_t pk = c->primes[c->L + k];
        uint64_t prod = 1;
        for (int k2 = 0; k2 < c->K; ++k2)
            if (k2 != k) prod = mulmod_u64(prod, c->primes[c->L + k2] % pk, pk);
        md->phat_inv[k] = shoup_pair(invmod_u64(prod, pk), pk);
        for (int i = 0; i < c->L; ++i) {
            const uint64_t qi = c->primes[i];
            uint64_t h = 1;
            for (int k2 = 0; k2 < c->K; ++k2)
                if (k2 != k) h = mulmod_u64(h, c->primes[c->L + k2] % qi, qi);
            md->phat[k][i] = shoup_pair(h, qi);
        }
    }
    for (int m = 0; m < NP; ++m) {
        const uint64_t qm = c->primes[m];
        uint64_t pmod = 1;
        for (int k = 0; k < c->K; ++k) pmod = mulmod_u64(pmod, c->primes[c->L + k] % qm, qm);
        // floor(P/2) = (P - 1)/2 for odd P
        const uint64_t half = mulmod_u64((pmod + qm - 1) % qm, invmod_u64(2, qm), qm);
        md->half[m] = (double)half;
        if (m < c->L) {
            md->pinv[m] = shoup_pair(invmod_u64(pmod, qm), qm);
            md->pmod[m] = shoup_pair(pmod, qm);
        }
    }
    {
        pfx_status r = dmalloc(c.get(), &c->d_moddown, sizeof(ModDownConst));
        if (r) return r;
    }
    HIPCHECK(hipMemcpy(c->d_moddown, md.get(), sizeof(ModDownConst), hipMemcpyHostToDevice));

    // Rescale: dropping prime l, for i < l
    std::vector<RescaleConst> rc((size_t)PFX_MAX_PRIMES * PFX_MAX_PRIMES);
    std::memset(rc.data(), 0, rc.size() * sizeof(RescaleConst));
    for (int l = 1; l < c->L; ++l)
        for (int i = 0; i < l; ++i) {
            const uint64_t qi = c->primes[i], ql = c->primes[l];
            RescaleConst &r = rc[(size_t)l * PFX_MAX_PRIMES + i];
            r.inv = shoup_pair(invmod_u64(ql % qi, qi), qi);
            r.half = (double)((ql / 2) % qi);
        }
    {
        pfx_status r = dmalloc(c.get(), &c->d_rescale, rc.size() * sizeof(RescaleConst));
        if (r) return r;
    }
    HIPCHECK(hipMemcpy(c->d_rescale, rc.data(), rc.size() * sizeof(RescaleConst), hipMemcpyHostToDevice));
    *out = c.release();
    return PFX_OK;
}

void pfx_ctx_destroy(pfx_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    graph_forget(c->uid);      // every graph that launches on this context's tables or lanes
    bump_scratch_epoch();      // and any that wrote this context's scratch
    for (auto &kv : c->ws) {
        dfree(kv.second->buf);
        dfree(kv.second->bbuf);
        dfree(kv.second->rbuf);
        dfree(kv.second->pbuf);
        delete kv.second;
    }
    for (auto &e : c->prof_pending) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    for (auto e : c->prof_pool) (void)(void)hipEventDestroy(e);
    for (auto st : c->lanes) (void)(void)hipStreamDestroy(st);
    for (auto e : c->lane_events) (void)(void)hipEventDestroy(e);
    dfree(c->d_tw);
    dfree(c->d_rtw);
    dfree(c->d_primes);
    dfree(c->d_modup);
    dfree(c->d_moddown);
    dfree(c->d_rescale);
    delete c;   // objects not yet destroyed keep their memory until they are
}

pfx_status pfx_tuning_set(const pfx_pass_tuning *t) {
    REQUIRE(t, PFX_EINVAL, "null argument");
    REQUIRE(t->log_n >= 2 && t->log_n <= 16, PFX_EINVAL, "log_n out of range");
    REQUIRE(t->widen_wg >= 1 && t->rs_widen_wg >= 1, PFX_EINVAL, "widen thresholds must be positive");
    REQUIRE(t->min_col >= 1 && t->min_col_special >= 1 && !(t->min_col & (t->min_col - 1)) &&
                !(t->min_col_special & (t->min_col_special - 1)),
            PFX_EINVAL, "column widths must be powers of two");
    REQUIRE(t->ks_fuse == 0 || t->ks_fuse == 128 || t->ks_fuse == 256, PFX_EINVAL, "ks_fuse must be 0, 128 or 256");
    REQUIRE(t->ks_batch >= 1 && t->ks_batch <= (uint32_t)kMaxBatch, PFX_EINVAL, "ks_batch must be in [1, 8]");
    REQUIRE(t->ks_modup_batch <= (uint32_t)kMaxBatch, PFX_EINVAL, "ks_modup_batch must be in [0, 8]");
    std::lock_guard<std::mutex> g(g_tune_mu);
    PassTuning &x = g_tune[t->log_n];
    x.row_wg256 = (int)std::min<uint32_t>(t->row_wg256, 1u << 30);
    x.col_wg256 = (int)std::min<uint32_t>(t->col_wg256, 1u << 30);
    x.widen_wg = (int)std::min<uint32_t>(t->widen_wg, 1u << 30);
    x.min_col = (int)t->min_col;
    x.min_col_special = (int)t->min_col_special;
    x.rs_widen_wg = (int)std::min<uint32_t>(t->rs_widen_wg, 1u << 30);
    x.ks_fuse = (int)t->ks_fuse;
    x.ks_batch = (int)t->ks_batch;
    x.ks_modup_batch = (int)t->ks_modup_batch;
    return PFX_OK;
}

pfx_status pfx_tuning_get(uint32_t log_n, pfx_pass_tuning *t) {
    REQUIRE(t && log_n < 32, PFX_EINVAL, "bad argument");
    std::lock_guard<std::mutex> g(g_tune_mu);
    const PassTuning &x = g_tune[log_n];
    *t = pfx_pass_tuning{log_n, (uint32_t)x.row_wg256, (uint32_t)x.col_wg256, (uint32_t)x.widen_wg,
                         (uint32_t)x.min_col, (uint32_t)x.min_col_special, (uint32_t)x.rs_widen_wg,
                         (uint32_t)x.ks_fuse, (uint32_t)x.ks_batch, (uint32_t)x.ks_modup_batch};
    return PFX_OK;
}

pfx_status pfx_tuning_reset(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (PassTuning &x : g_tune) x = PassTuning{};
    return PFX_OK;
}

pfx_status pfx_tuning_load(const char *path) {
    REQUIRE(path, PFX_EINVAL, "null path");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(PFX_EINVAL, std::string("cannot open ") + path);
    char line[512];
    int n = 0;
    pfx_status r = PFX_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        pfx_pass_tuning t;
        t.ks_fuse = (uint32_t)PassTuning{}.ks_fuse;      // fields left out keep their defaults
        t.ks_batch = (uint32_t)PassTuning{}.ks_batch;
        t.ks_modup_batch = (uint32_t)PassTuning{}.ks_modup_batch;
        const int got = std::sscanf(line, "%u %u %u %u %u %u %u %u %u %u", &t.log_n, &t.row_wg256, &t.col_wg256,
                                    &t.widen_wg, &t.min_col, &t.min_col_special, &t.rs_widen_wg, &t.ks_fuse,
                                    &t.ks_batch, &t.ks_modup_batch);
        if (got < 7) {
            r = fail(PFX_EINVAL, std::string("malformed tuning line in ") + path);
            break;
        }
        r = pfx_tuning_set(&t);
        if (r) break;
        ++n;
    }
    std::fclose(f);
    return r;
}

pfx_status pfx_ctx_set_allocator(pfx_ctx *c, pfx_alloc_fn alloc, pfx_free_fn free_fn, void *user,
                                 size_t hbm_budget) {
    REQUIRE(c, PFX_EINVAL, "null context");
    REQUIRE((alloc == nullptr) == (free_fn == nullptr), PFX_EINVAL, "give both alloc and free, or neither");
    std::lock_guard<std::mutex> g(c->mem->mu);
    c->mem->alloc = alloc;
    c->mem->free = free_fn;
    c->mem->user = user;
    c->mem->budget = hbm_budget;
    return PFX_OK;
}

pfx_status pfx_ctx_mem(const pfx_ctx *c, size_t *in_use, size_t *peak) {
    REQUIRE(c, PFX_EINVAL, "null context");
    std::lock_guard<std::mutex> g(c->mem->mu);
    if (in_use) *in_use = c->mem->in_use;
    if (peak) *peak = c->mem->peak;
    return PFX_OK;
}

pfx_status pfx_ctx_moduli(const pfx_ctx *c, uint64_t *q, uint64_t *p, uint64_t *psi) {
    REQUIRE(c, PFX_EINVAL, "null context");
    if (q) std::copy(c->primes.begin(), c->primes.begin() + c->L, q);
    if (p) std::copy(c->primes.begin() + c->L, c->primes.end(), p);
    if (psi) std::copy(c->psi.begin(), c->psi.end(), psi);
    return PFX_OK;
}

pfx_status pfx_sync(pfx_ctx *c, void *stream) {
    REQUIRE(c, PFX_EINVAL, "null context");
    HIPCHECK(hipStreamSynchronize(S(stream)));
    return PFX_OK;
}

// ------------------------------------------------------------------ keys
pfx_status pfx_sk_create(pfx_ctx *c, const int8_t *s, pfx_sk **out) {
    REQUIRE(c && s && out, PFX_EINVAL, "null argument");
    for (int i = 0; i < c->N; ++i) REQUIRE(s[i] >= -1 && s[i] <= 1, PFX_EINVAL, "secret coefficients must be -1, 0 or 1");
    HIPCHECK(hipSetDevice(c->device));
    const int NP = c->L + c->K;
    std::unique_ptr<pfx_sk> k(new pfx_sk);
    k->ctx = c;
    k->uid = next_uid();
    k->h_s.assign(s, s + c->N);
    DevTmp<double> ds;
    DevTmp<int8_t> tmp;
    PFX_DMALLOC(c, &ds.p, (size_t)NP * c->N * sizeof(double));
    PFX_DMALLOC(c, &tmp.p, c->N);
    HIPCHECK(hipMemcpy(tmp.p, s, c->N, hipMemcpyHostToDevice));
    Launch L{c, nullptr};
    launch_s8_to_rns(L, ds.p, tmp.p, NP);
    launch_ntt(L, ds.p, nullptr, contiguous_map(NP, 0), false);
    HIPCHECK(hipStreamSynchronize(nullptr));
    k->d_s = ds.release();
    *out = k.release();
    return PFX_OK;
}

void pfx_sk_destroy(pfx_sk *k) {
    if (!k) return;
    dfree(k->d_s);
    delete k;
}

}  // extern "C"

namespace {

// Inputs of a switching key (Sec. 2.4.1): a words below their primes, errors
// small.
pfx_status check_swk_inputs(const pfx_ctx *c, const uint64_t *a, const int64_t *e) {
    const int NP = c->L + c->K;
    const size_t N = c->N;
    for (int j = 0; j < c->beta; ++j)
        for (int m = 0; m < NP; ++m)
            for (size_t i = 0; i < N; ++i)
                REQUIRE(a[((size_t)j * NP + m) * N + i] < c->primes[m], PFX_EINVAL, "a word not below its prime");
    for (size_t i = 0; i < (size_t)c->beta * N; ++i)
        REQUIRE(e[i] > -(1ll << 40) && e[i] < (1ll << 40), PFX_EINVAL, "error coefficient too large");
    return PFX_OK;
}

// swk_j = (-a_j s + e_j + P w_j s_from, a_j) for every digit j, s_from given
// in the NTT domain over all L + K primes (device).
pfx_status swk_fill(pfx_ctx *c, const pfx_sk *sk, const double *sfrom, const uint64_t *a, const int64_t *e,
                    pfx_swk *k) {
    const int NP = c->L + c->K;
    const size_t N = c->N, limb = N;
    DevTmp<double> dk, etmp_;
    DevTmp<uint64_t> stage_;
    DevTmp<int64_t> edev_;
    PFX_DMALLOC(c, &dk.p, (size_t)c->beta * 2 * NP * limb * sizeof(double));
    PFX_DMALLOC(c, &etmp_.p, (size_t)NP * limb * sizeof(double));
    PFX_DMALLOC(c, &stage_.p, (size_t)NP * limb * sizeof(uint64_t));
    PFX_DMALLOC(c, &edev_.p, N * sizeof(int64_t));
    double *etmp = etmp_.p;
    uint64_t *stage = stage_.p;
    int64_t *edev = edev_.p;
    Launch L{c, nullptr};
    for (int j = 0; j < c->beta; ++j) {
        double *b = dk.p + (size_t)(2 * j) * NP * limb;
        double *aa = dk.p + (size_t)(2 * j + 1) * NP * limb;
        HIPCHECK(hipMemcpy(stage, a + (size_t)j * NP * N, (size_t)NP * N * sizeof(uint64_t), hipMemcpyHostToDevice));
        launch_u64_to_f64(L, aa, stage, (size_t)NP * N);
        launch_ntt(L, aa, nullptr, contiguous_map(NP, 0), false);
        HIPCHECK(hipMemcpy(edev, e + (size_t)j * N, N * sizeof(int64_t), hipMemcpyHostToDevice));
        launch_int_to_rns(L, etmp, edev, NP, 0, 0, 0);
        launch_ntt(L, etmp, nullptr, contiguous_map(NP, 0), false);
        launch_keygen_b(L, b, aa, etmp, sk->d_s, sfrom, j);
        HIPCHECK(hipStreamSynchronize(nullptr));
    }
    k->d_k = dk.release();
    return PFX_OK;
}

}  // namespace

extern "C" {

pfx_status pfx_swk_create(pfx_ctx *c, const pfx_sk *sk, uint32_t galois, const uint64_t *a, const int64_t *e,
                          pfx_swk **out) {
    REQUIRE(c && sk && a && e && out, PFX_EINVAL, "null argument");
    REQUIRE(sk->ctx == c, PFX_EINVAL, "secret key of another context");
    REQUIRE(galois == 0 || ((galois & 1) && galois < 2u * c->N), PFX_EINVAL, "galois must be 0 or odd < 2N");
    pfx_status r = check_swk_inputs(c, a, e);
    if (r) return r;
    HIPCHECK(hipSetDevice(c->device));
    const int NP = c->L + c->K;
    std::unique_ptr<pfx_swk> k(new pfx_swk);
    k->ctx = c;
    k->uid = next_uid();
    k->galois = galois;
    DevTmp<double> sfrom;
    PFX_DMALLOC(c, &sfrom.p, (size_t)NP * c->N * sizeof(double));
    Launch L{c, nullptr};
    if (galois == 0) launch_ew(L, EW_MUL, sfrom.p, sk->d_s, sk->d_s, 0, 0, 0, 1, NP);
    else launch_automorph(L, sfrom.p, sk->d_s, 0, 0, 1, NP, galois);
    r = swk_fill(c, sk, sfrom.p, a, e, k.get());
    if (r) return r;
    *out = k.release();
    return PFX_OK;
}

pfx_status pfx_swk_create_from(pfx_ctx *c, const pfx_sk *sk, const int8_t *s_from, const uint64_t *a,
                               const int64_t *e, pfx_swk **out) {
    REQUIRE(c && sk && s_from && a && e && out, PFX_EINVAL, "null argument");
    REQUIRE(sk->ctx == c, PFX_EINVAL, "secret key of another context");
    pfx_status r = check_swk_inputs(c, a, e);
    if (r) return r;
    HIPCHECK(hipSetDevice(c->device));
    const int NP = c->L + c->K;
    std::unique_ptr<pfx_swk> k(new pfx_swk);
    k->ctx = c;
    k->uid = next_uid();
    k->galois = 0;
    k->from_secret = true;
    DevTmp<double> sfrom;
    DevTmp<int8_t> tmp;
    PFX_DMALLOC(c, &sfrom.p, (size_t)NP * c->N * sizeof(double));
    PFX_DMALLOC(c, &tmp.p, c->N);
    HIPCHECK(hipMemcpy(tmp.p, s_from, c->N, hipMemcpyHostToDevice));
    Launch L{c, nullptr};
    launch_s8_to_rns(L, sfrom.p, tmp.p, NP);
    launch_ntt(L, sfrom.p, nullptr, contiguous_map(NP, 0), false);
    r = swk_fill(c, sk, sfrom.p, a, e, k.get());
    if (r) return r;
    *out = k.release();
    return PFX_OK;
}

pfx_status pfx_swk_export(pfx_ctx *c, const pfx_swk *k, uint64_t *words, size_t cap) {
    REQUIRE(c && k && words, PFX_EINVAL, "null argument");
    const int NP = c->L + c->K;
    const size_t per = (size_t)NP * c->N;
    REQUIRE(cap >= (size_t)c->beta * 2 * per, PFX_EINVAL, "cap_words too small");
    HIPCHECK(hipSetDevice(c->device));
    DevTmp<double> tmp;
    DevTmp<uint64_t> u;
    PFX_DMALLOC(c, &tmp.p, per * sizeof(double));
    PFX_DMALLOC(c, &u.p, per * sizeof(uint64_t));
    Launch L{c, nullptr};
    for (int p = 0; p < 2 * c->beta; ++p) {
        launch_ntt(L, tmp.p, k->d_k + (size_t)p * per, contiguous_map(NP, 0), true);
        launch_f64_to_u64(L, u.p, tmp.p, per);
        HIPCHECK(hipMemcpy(words + (size_t)p * per, u.p, per * sizeof(uint64_t), hipMemcpyDeviceToHost));
    }
    return PFX_OK;
}

pfx_status pfx_swk_import(pfx_ctx *c, uint32_t galois, const uint64_t *words, size_t n_words, pfx_swk **out) {
    REQUIRE(c && words && out, PFX_EINVAL, "null argument");
    REQUIRE(galois == 0 || ((galois & 1) && galois < 2u * c->N), PFX_EINVAL, "galois must be 0 or odd < 2N");
    const int NP = c->L + c->K;
    const size_t N = c->N, per = (size_t)NP * N;
    REQUIRE(n_words == (size_t)c->beta * 2 * per, PFX_EINVAL, "n_words must be beta * 2 * (n_q + n_p) * N");
    for (size_t p = 0; p < (size_t)2 * c->beta; ++p)
        for (int m = 0; m < NP; ++m)
            for (size_t i = 0; i < N; ++i)
                REQUIRE(words[p * per + (size_t)m * N + i] < c->primes[m], PFX_EINVAL, "word not below its prime");
    HIPCHECK(hipSetDevice(c->device));
    std::unique_ptr<pfx_swk> k(new pfx_swk);
    k->ctx = c;
    k->uid = next_uid();
    k->galois = galois;
    DevTmp<double> dk;
    DevTmp<uint64_t> stage;
    PFX_DMALLOC(c, &dk.p, (size_t)c->beta * 2 * per * sizeof(double));
    PFX_DMALLOC(c, &stage.p, per * sizeof(uint64_t));
    Launch L{c, nullptr};
    for (size_t p = 0; p < (size_t)2 * c->beta; ++p) {
        HIPCHECK(hipMemcpy(stage.p, words + p * per, per * sizeof(uint64_t), hipMemcpyHostToDevice));
        launch_u64_to_f64(L, dk.p + p * per, stage.p, per);
        launch_ntt(L, dk.p + p * per, nullptr, contiguous_map(NP, 0), false);
        HIPCHECK(hipStreamSynchronize(nullptr));
    }
    k->d_k = dk.release();
    *out = k.release();
    return PFX_OK;
}

pfx_status pfx_sk_export(const pfx_sk *sk, int8_t *s, size_t n) {
    REQUIRE(sk && s, PFX_EINVAL, "null argument");
    REQUIRE(n == sk->h_s.size(), PFX_EINVAL, "n must be N");
    std::copy(sk->h_s.begin(), sk->h_s.end(), s);
    return PFX_OK;
}

uint32_t pfx_swk_galois(const pfx_swk *k) { return k ? k->galois : 0; }

void pfx_swk_destroy(pfx_swk *k) {
    if (!k) return;
    graph_forget(k->uid);
    dfree(k->d_k);
    delete k;
}

// ------------------------------------------------------------------ ciphertext objects
pfx_status pfx_ct_create(pfx_ctx *c, uint32_t cap_limbs, uint32_t cap_degree, pfx_ct **out) {
    REQUIRE(c && out, PFX_EINVAL, "null argument");
    REQUIRE(cap_limbs >= 1 && cap_limbs <= (uint32_t)c->L, PFX_EINVAL, "cap_limbs must be in [1, n_q]");
    REQUIRE(cap_degree <= 2, PFX_EINVAL, "cap_degree must be 0, 1 or 2");
    HIPCHECK(hipSetDevice(c->device));
    std::unique_ptr<pfx_ct> x(new pfx_ct);
    x->ctx = c;
    x->uid = next_uid();
    x->cap_limbs = cap_limbs;
    x->cap_degree = cap_degree;
    PFX_DMALLOC(c, &x->d, (size_t)(cap_degree + 1) * cap_limbs * c->N * sizeof(double));
    *out = x.release();
    return PFX_OK;
}

void pfx_ct_destroy(pfx_ct *x) {
    if (!x) return;
    graph_forget(x->uid);
    if (x->owns) dfree(x->d);
    delete x;
}

pfx_status pfx_ct_info(const pfx_ct *x, pfx_info *info) {
    REQUIRE(x && info, PFX_EINVAL, "null argument");
    info->log_n = x->ctx->logn;
    info->n_limbs = x->n_limbs;
    info->degree = x->degree;
    info->scale = x->scale;
    return PFX_OK;
}

pfx_status pfx_ct_set_scale(pfx_ct *x, double scale) {
    REQUIRE(x && scale > 0 && std::isfinite(scale), PFX_EINVAL, "bad scale");
    x->scale = scale;
    return PFX_OK;
}

pfx_status pfx_ct_import(pfx_ctx *c, const uint64_t *words, uint32_t n_limbs, uint32_t degree, double scale,
                         pfx_ct *out, void *stream) {
    REQUIRE(c && words && out, PFX_EINVAL, "null argument");
    REQUIRE(n_limbs >= 1 && n_limbs <= (uint32_t)c->L, PFX_EINVAL, "n_limbs out of range");
    REQUIRE(degree <= 2, PFX_EINVAL, "degree out of range");
    pfx_status r = check_out(out, n_limbs, degree);
    if (r) return r;
    const size_t N = c->N;
    for (uint32_t k = 0; k <= degree; ++k)
        for (uint32_t i = 0; i < n_limbs; ++i)
            for (size_t t = 0; t < N; ++t)
                REQUIRE(words[((size_t)k * n_limbs + i) * N + t] < c->primes[i], PFX_EINVAL, "word not below its prime");
    HIPCHECK(hipSetDevice(c->device));
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    uint64_t *stage = (uint64_t *)w.at(w.lay.xport);
    for (uint32_t k = 0; k <= degree; ++k) {
        HIPCHECK(hipMemcpyAsync(stage, words + (size_t)k * n_limbs * N, (size_t)n_limbs * N * sizeof(uint64_t),
                                hipMemcpyHostToDevice, S(stream)));
        launch_u64_to_f64(L, out->poly(k), stage, (size_t)n_limbs * N);
    }
    launch_ntt(L, out->d, nullptr, poly_map(degree + 1, n_limbs, out->cap_limbs), false);
    HIPCHECK(hipStreamSynchronize(S(stream)));
    out->n_limbs = n_limbs;
    out->degree = degree;
    out->scale = scale;
    return PFX_OK;
}

pfx_status pfx_ct_export(pfx_ctx *c, const pfx_ct *x, uint64_t *words, size_t cap, pfx_info *info, void *stream) {
    REQUIRE(c && words, PFX_EINVAL, "null argument");
    pfx_status r = check_ct(c, x, "ciphertext");
    if (r) return r;
    const size_t N = c->N, per = (size_t)x->n_limbs * N;
    REQUIRE(cap >= (size_t)(x->degree + 1) * per, PFX_EINVAL, "cap_words too small");
    HIPCHECK(hipSetDevice(c->device));
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    double *tmp = w.at(w.lay.rs_tmp);
    uint64_t *stage = (uint64_t *)w.at(w.lay.xport);
    for (uint32_t k = 0; k <= x->degree; ++k) {
        launch_ntt(L, tmp, x->poly(k), contiguous_map(x->n_limbs, 0), true);
        launch_f64_to_u64(L, stage, tmp, per);
        HIPCHECK(hipMemcpyAsync(words + k * per, stage, per * sizeof(uint64_t), hipMemcpyDeviceToHost, S(stream)));
        HIPCHECK(hipStreamSynchronize(S(stream)));
    }
    if (info) pfx_ct_info(x, info);
    return PFX_OK;
}

pfx_status pfx_ct_copy(pfx_ctx *c, const pfx_ct *src, pfx_ct *dst, void *stream) {
    pfx_status r = check_ct(c, src, "source");
    if (r) return r;
    r = check_out(dst, src->n_limbs, src->degree);
    if (r) return r;
    if (src != dst) {
        Launch L{c, S(stream)};
        const size_t N = c->N;
        launch_ew(L, EW_COPY, dst->d, src->d, nullptr, dst->cap_limbs * N, src->cap_limbs * N, 0, src->degree + 1,
                  src->n_limbs);
    }
    dst->n_limbs = src->n_limbs;
    dst->degree = src->degree;
    dst->scale = src->scale;
    return PFX_OK;
}

// ------------------------------------------------------------------ encoding and encryption
pfx_status pfx_pt_import(pfx_ctx *c, const uint64_t *words, uint32_t n_limbs, double scale, pfx_pt **out) {
    REQUIRE(c && out, PFX_EINVAL, "null argument");
    REQUIRE(n_limbs >= 1 && n_limbs <= (uint32_t)c->L, PFX_EINVAL, "n_limbs out of range");
    pfx_ct *x = nullptr;
    pfx_status r = pfx_ct_create(c, n_limbs, 0, &x);
    if (r) return r;
    r = pfx_ct_import(c, words, n_limbs, 0, scale, x, nullptr);
    if (r) { pfx_ct_destroy(x); return r; }
    *out = x;
    return PFX_OK;
}

pfx_status pfx_encode(pfx_ctx *c, const double *re, const double *im, size_t n, uint32_t n_limbs, double scale,
                      pfx_pt **out) {
    REQUIRE(c && re && out, PFX_EINVAL, "null argument");
    REQUIRE(n_limbs >= 1 && n_limbs <= (uint32_t)c->L, PFX_EINVAL, "n_limbs out of range");
    REQUIRE(scale > 0 && std::isfinite(scale), PFX_EINVAL, "bad scale");
    std::vector<uint64_t> mods(c->primes.begin(), c->primes.begin() + n_limbs), words;
    std::string err;
    if (!encode_coeffs(c->logn, re, im, n, scale, mods, words, err)) return fail(PFX_EINVAL, err);
    return pfx_pt_import(c, words.data(), n_limbs, scale, out);
}

pfx_status pfx_decode(pfx_ctx *c, const pfx_pt *pt, double *re, double *im, size_t n) {
    REQUIRE(c && re, PFX_EINVAL, "null argument");
    pfx_status r = check_ct(c, pt, "plaintext");
    if (r) return r;
    REQUIRE(pt->degree == 0, PFX_EINVAL, "decode needs a plaintext (degree 0)");
    REQUIRE(n >= 1 && !(n & (n - 1)) && n <= (size_t)c->N / 2, PFX_EINVAL, "n_slots must be a power of two <= N/2");
    std::vector<uint64_t> words((size_t)pt->n_limbs * c->N);
    r = pfx_ct_export(c, pt, words.data(), words.size(), nullptr, nullptr);
    if (r) return r;
    std::vector<uint64_t> mods(c->primes.begin(), c->primes.begin() + pt->n_limbs);
    decode_words(c->logn, words.data(), pt->n_limbs, mods, pt->scale, n, re, im);
    return PFX_OK;
}

pfx_status pfx_encrypt(pfx_ctx *c, const pfx_sk *sk, const pfx_pt *pt, const uint64_t *a, const int64_t *e,
                       pfx_ct *out, void *stream) {
    REQUIRE(c && sk && a && e, PFX_EINVAL, "null argument");
    pfx_status r = check_ct(c, pt, "plaintext");
    if (r) return r;
    const uint32_t lv = pt->n_limbs;
    r = check_out(out, lv, 1);
    if (r) return r;
    const size_t N = c->N;
    for (uint32_t i = 0; i < lv; ++i)
        for (size_t t = 0; t < N; ++t) REQUIRE(a[(size_t)i * N + t] < c->primes[i], PFX_EINVAL, "a word not below its prime");
    for (size_t t = 0; t < N; ++t) REQUIRE(e[t] > -(1ll << 40) && e[t] < (1ll << 40), PFX_EINVAL, "error too large");
    HIPCHECK(hipSetDevice(c->device));
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    uint64_t *stage = (uint64_t *)w.at(w.lay.xport);
    double *etmp = w.at(w.lay.rs_tmp);
    HIPCHECK(hipMemcpyAsync(stage, a, (size_t)lv * N * sizeof(uint64_t), hipMemcpyHostToDevice, S(stream)));
    launch_u64_to_f64(L, out->poly(1), stage, (size_t)lv * N);
    launch_ntt(L, out->poly(1), nullptr, contiguous_map(lv, 0), false);
    int64_t *edev = (int64_t *)w.at(w.lay.t3);
    HIPCHECK(hipMemcpyAsync(edev, e, N * sizeof(int64_t), hipMemcpyHostToDevice, S(stream)));
    launch_int_to_rns(L, etmp, edev, lv, 0, 0, 0);
    launch_ntt(L, etmp, nullptr, contiguous_map(lv, 0), false);
    launch_encrypt(L, out->poly(0), out->poly(1), etmp, sk->d_s, pt->poly(0), lv);
    HIPCHECK(hipStreamSynchronize(S(stream)));
    out->n_limbs = lv;
    out->degree = 1;
    out->scale = pt->scale;
    return PFX_OK;
}

pfx_status pfx_decrypt(pfx_ctx *c, const pfx_sk *sk, const pfx_ct *x, pfx_pt **out, void *stream) {
    REQUIRE(c && sk && out, PFX_EINVAL, "null argument");
    pfx_status r = check_ct(c, x, "ciphertext");
    if (r) return r;
    REQUIRE(x->degree >= 1, PFX_EINVAL, "decrypt needs a ciphertext");
    pfx_ct *m = nullptr;
    r = pfx_ct_create(c, x->n_limbs, 0, &m);
    if (r) return r;
    Launch L{c, S(stream)};
    launch_decrypt(L, m->d, x->poly(0), x->poly(1), x->degree == 2 ? x->poly(2) : nullptr, sk->d_s, x->n_limbs);
    if (hipStreamSynchronize(S(stream)) != hipSuccess) { pfx_ct_destroy(m); return fail(PFX_EDEVICE, "decrypt failed"); }
    m->n_limbs = x->n_limbs;
    m->degree = 0;
    m->scale = x->scale;
    *out = m;
    return PFX_OK;
}

// ------------------------------------------------------------------ evaluation
static pfx_status addsub(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream, bool sub) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, b, "b");
    if (r) return r;
    if (!scale_close(a->scale, b->scale)) return fail(PFX_ESCALE, "operand scales differ");
    const uint32_t lv = std::min(a->n_limbs, b->n_limbs);
    const uint32_t deg = std::max(a->degree, b->degree), dmin = std::min(a->degree, b->degree);
    r = check_out(out, lv, deg);
    if (r) return r;
    Launch L{c, S(stream)};
    const size_t N = c->N;
    launch_ew(L, sub ? EW_SUB : EW_ADD, out->d, a->d, b->d, out->cap_limbs * N, a->cap_limbs * N, b->cap_limbs * N,
              dmin + 1, lv);
    for (uint32_t k = dmin + 1; k <= deg; ++k) {
        const pfx_ct *big = a->degree > b->degree ? a : b;
        const bool negate = sub && big == b;
        launch_ew(L, negate ? EW_NEG : EW_COPY, out->poly(k), big->poly(k), nullptr, 0, 0, 0, 1, lv);
    }
    out->n_limbs = lv;
    out->degree = deg;
    out->scale = a->scale;
    return PFX_OK;
}

pfx_status pfx_add(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream) {
    return addsub(c, a, b, out, stream, false);
}
pfx_status pfx_sub(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream) {
    return addsub(c, a, b, out, stream, true);
}

pfx_status pfx_neg(pfx_ctx *c, const pfx_ct *a, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_out(out, a->n_limbs, a->degree);
    if (r) return r;
    Launch L{c, S(stream)};
    const size_t N = c->N;
    launch_ew(L, EW_NEG, out->d, a->d, nullptr, out->cap_limbs * N, a->cap_limbs * N, 0, a->degree + 1, a->n_limbs);
    out->n_limbs = a->n_limbs;
    out->degree = a->degree;
    out->scale = a->scale;
    return PFX_OK;
}

pfx_status pfx_add_plain(pfx_ctx *c, const pfx_ct *a, const pfx_pt *m, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, m, "plaintext");
    if (r) return r;
    if (!scale_close(a->scale, m->scale)) return fail(PFX_ESCALE, "operand scales differ");
    const uint32_t lv = std::min(a->n_limbs, m->n_limbs);
    r = check_out(out, lv, a->degree);
    if (r) return r;
    Launch L{c, S(stream)};
    launch_ew(L, EW_ADD, out->d, a->d, m->d, 0, 0, 0, 1, lv);
    if (a->degree >= 1 && out != a)
        launch_ew(L, EW_COPY, out->poly(1), a->poly(1), nullptr, out->cap_limbs * c->N, a->cap_limbs * c->N, 0,
                  a->degree, lv);
    out->n_limbs = lv;
    out->degree = a->degree;
    out->scale = a->scale;
    return PFX_OK;
}

pfx_status pfx_mul_plain(pfx_ctx *c, const pfx_ct *a, const pfx_pt *m, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, m, "plaintext");
    if (r) return r;
    const uint32_t lv = std::min(a->n_limbs, m->n_limbs);
    r = check_out(out, lv, a->degree);
    if (r) return r;
    Launch L{c, S(stream)};
    const size_t N = c->N;
    launch_ew(L, EW_MUL, out->d, a->d, m->d, out->cap_limbs * N, a->cap_limbs * N, 0, a->degree + 1, lv);
    out->n_limbs = lv;
    out->degree = a->degree;
    out->scale = a->scale * m->scale;
    return PFX_OK;
}

// [k]_{q_i} for the first n primes.
static std::vector<uint64_t> int_residues(const pfx_ctx *c, int64_t k, uint32_t n) {
    std::vector<uint64_t> cst(n);
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t q = c->primes[i];
        const uint64_t mag = (uint64_t)(k < 0 ? -(k + 1) + 1ull : (uint64_t)k) % q;
        cst[i] = k < 0 ? (q - mag) % q : mag;
    }
    return cst;
}

pfx_status pfx_mul_int_acc(pfx_ctx *c, const pfx_ct *a, int64_t k, pfx_ct *acc, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, acc, "acc");
    if (r) return r;
    REQUIRE(acc->degree == a->degree, PFX_EINVAL, "accumulator and operand degrees differ");
    REQUIRE(acc->d != a->d, PFX_EINVAL, "accumulator aliases the operand");
    if (!scale_close(acc->scale, a->scale)) return fail(PFX_ESCALE, "operand scales differ");
    const uint32_t lv = std::min(a->n_limbs, acc->n_limbs);
    const std::vector<uint64_t> cst = int_residues(c, k, lv);
    Launch L{c, S(stream)};
    const size_t N = c->N;
    launch_mulconst(L, acc->d, a->d, acc->cap_limbs * N, a->cap_limbs * N, a->degree + 1, lv, cst.data(), true);
    acc->n_limbs = lv;
    return PFX_OK;
}

pfx_status pfx_mul_int(pfx_ctx *c, const pfx_ct *a, int64_t k, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_out(out, a->n_limbs, a->degree);
    if (r) return r;
    const std::vector<uint64_t> cst = int_residues(c, k, a->n_limbs);
    Launch L{c, S(stream)};
    const size_t N = c->N;
    launch_mulconst(L, out->d, a->d, out->cap_limbs * N, a->cap_limbs * N, a->degree + 1, a->n_limbs, cst.data());
    out->n_limbs = a->n_limbs;
    out->degree = a->degree;
    out->scale = a->scale;
    return PFX_OK;
}

pfx_status pfx_mul(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, b, "b");
    if (r) return r;
    REQUIRE(a->degree == 1 && b->degree == 1, PFX_EINVAL, "tensor product needs two degree-1 ciphertexts");
    const uint32_t lv = std::min(a->n_limbs, b->n_limbs);
    r = check_out(out, lv, 2);
    if (r) return r;
    Launch L{c, S(stream)};
    const double sc = a->scale * b->scale;
    launch_tensor(L, out->poly(0), out->poly(1), out->poly(2), a->poly(0), a->poly(1), b->poly(0), b->poly(1), lv);
    out->n_limbs = lv;
    out->degree = 2;
    out->scale = sc;
    return PFX_OK;
}

pfx_status pfx_mul_acc(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, pfx_ct *acc, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, b, "b");
    if (r) return r;
    r = check_ct(c, acc, "acc");
    if (r) return r;
    REQUIRE(a->degree == 1 && b->degree == 1, PFX_EINVAL, "tensor product needs two degree-1 ciphertexts");
    REQUIRE(acc->degree == 2, PFX_EINVAL, "accumulator must be of degree 2");
    REQUIRE(acc->d != a->d && acc->d != b->d, PFX_EINVAL, "accumulator aliases an operand");
    if (!scale_close(acc->scale, a->scale * b->scale)) return fail(PFX_ESCALE, "operand scales differ");
    const uint32_t lv = std::min({a->n_limbs, b->n_limbs, acc->n_limbs});
    Launch L{c, S(stream)};
    launch_tensor(L, acc->poly(0), acc->poly(1), acc->poly(2), a->poly(0), a->poly(1), b->poly(0), b->poly(1), lv,
                  true);
    acc->n_limbs = lv;
    return PFX_OK;
}

pfx_status pfx_mul_plain_acc(pfx_ctx *c, const pfx_ct *a, const pfx_pt *m, pfx_ct *acc, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, m, "plaintext");
    if (r) return r;
    r = check_ct(c, acc, "acc");
    if (r) return r;
    REQUIRE(acc->degree == a->degree, PFX_EINVAL, "accumulator and operand degrees differ");
    REQUIRE(acc->d != a->d, PFX_EINVAL, "accumulator aliases the operand");
    if (!scale_close(acc->scale, a->scale * m->scale)) return fail(PFX_ESCALE, "operand scales differ");
    const uint32_t lv = std::min({a->n_limbs, m->n_limbs, acc->n_limbs});
    Launch L{c, S(stream)};
    const size_t N = c->N;
    launch_ew(L, EW_MAC, acc->d, a->d, m->d, acc->cap_limbs * N, a->cap_limbs * N, 0, a->degree + 1, lv);
    acc->n_limbs = lv;
    return PFX_OK;
}

pfx_status pfx_relinearize(pfx_ctx *c, const pfx_ct *a, const pfx_swk *rlk, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(rlk && rlk->ctx == c, PFX_EINVAL, "bad relinearisation key");
    REQUIRE(rlk->galois == 0 && !rlk->from_secret, PFX_ENOKEY, "key is not a relinearisation key");
    REQUIRE(a->degree == 2, PFX_EINVAL, "relinearize needs a degree-2 ciphertext");
    r = check_out(out, a->n_limbs, 1);
    if (r) return r;
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    const double sc = a->scale;
    const uint32_t lv = a->n_limbs;
    ks_core(c, L, w, ks_plain(a->poly(2), a->poly(0), a->poly(1)), lv, rlk, out->poly(0), out->poly(1));
    out->n_limbs = lv;
    out->degree = 1;
    out->scale = sc;
    return PFX_OK;
}

}  // extern "C"

namespace pfx {

pfx_status mul_relin_check(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk, pfx_ct *out) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_ct(c, b, "b");
    if (r) return r;
    REQUIRE(rlk && rlk->ctx == c, PFX_EINVAL, "bad relinearisation key");
    REQUIRE(rlk->galois == 0 && !rlk->from_secret, PFX_ENOKEY, "key is not a relinearisation key");
    REQUIRE(a->degree == 1 && b->degree == 1, PFX_EINVAL, "mul_relin needs two degree-1 ciphertexts");
    return check_out(out, std::min(a->n_limbs, b->n_limbs), 1);
}

// HMult + relin of checked operands with the key-switch scratch given (regions
// sized for the operands' level; t3 with three polynomials t3_stride apart is
// only used when the output aliases an operand).
void mul_relin_run(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk, pfx_ct *out, hipStream_t st,
                   const KsScratch &s) {
    const uint32_t lv = std::min(a->n_limbs, b->n_limbs);
    Launch L{c, st};
    const double sc = a->scale * b->scale;
    KsOperand op;
    if (out->d != a->d && out->d != b->d) {
        // the tensor product is formed inside the key switch, never stored
        op.mode = KS_PRODUCT;
        op.a0 = a->poly(0);
        op.a1 = a->poly(1);
        op.b0 = b->poly(0);
        op.b1 = b->poly(1);
    } else {
        // the output overwrites an operand that other workgroups of the last
        // launch still read: take the tensor product into scratch first
        double *t0 = s.t3, *t1 = t0 + s.t3_stride, *t2 = t1 + s.t3_stride;
        launch_tensor(L, t0, t1, t2, a->poly(0), a->poly(1), b->poly(0), b->poly(1), lv);
        op = ks_plain(t2, t0, t1);
    }
    KsBatch kb;
    kb.nb = 1;
    kb.mode = op.mode;
    kb.op[0] = op;
    kb.out0[0] = out->poly(0);
    kb.out1[0] = out->poly(1);
    kb.dcoef = s.dcoef;
    kb.ext = s.ext;
    kb.acc = s.acc;
    kb.tmp = s.tmp;
    ks_run(L, kb, lv, rlk);
    out->n_limbs = lv;
    out->degree = 1;
    out->scale = sc;
}

}  // namespace pfx

extern "C" {

pfx_status pfx_mul_relin(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk, pfx_ct *out,
                         void *stream) {
    pfx_status r = mul_relin_check(c, a, b, rlk, out);
    if (r) return r;
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    KsScratch s;
    s.dcoef = w.at(w.lay.dcoef);
    s.ext = w.at(w.lay.ext);
    s.acc = w.at(w.lay.acc);
    s.tmp = w.at(w.lay.mdtmp);
    s.t3 = w.at(w.lay.t3);
    s.t3_stride = (size_t)c->L * c->N;
    mul_relin_run(c, a, b, rlk, out, S(stream), s);
    return PFX_OK;
}

// Batched HMult + relinearisation: entries of one level share every launch
// of the key switch (the key residues are read once per launch for all of
// them), at most kMaxBatch entries per launch.
static pfx_status mul_relin_group(pfx_ctx *c, const Launch &L, const pfx_ct *const *a, const pfx_ct *const *b,
                           pfx_ct *const *out, const int *idx, int nb, int lv, const pfx_swk *rlk) {
    KsBatch kb;
    pfx_status r = get_batch_ws(c, L.st, nb, kb);
    if (r) return r;
    kb.nb = nb;
    kb.mode = KS_PRODUCT;
    for (int e = 0; e < nb; ++e) {
        const int i = idx[e];
        KsOperand &op = kb.op[e];
        op.mode = KS_PRODUCT;
        op.a0 = a[i]->poly(0);
        op.a1 = a[i]->poly(1);
        op.b0 = b[i]->poly(0);
        op.b1 = b[i]->poly(1);
        kb.out0[e] = out[i]->poly(0);
        kb.out1[e] = out[i]->poly(1);
    }
    ks_run(L, kb, lv, rlk);
    return PFX_OK;
}

pfx_status pfx_mul_relin_batch(pfx_ctx *c, const pfx_ct *const *a, const pfx_ct *const *b, size_t n,
                               const pfx_swk *rlk, pfx_ct *const *out, void *stream) {
    REQUIRE(c && (n == 0 || (a && b && out)), PFX_EINVAL, "null argument");
    REQUIRE(rlk && rlk->ctx == c, PFX_EINVAL, "bad relinearisation key");
    REQUIRE(rlk->galois == 0 && !rlk->from_secret, PFX_ENOKEY, "key is not a relinearisation key");
    std::vector<uint32_t> lvs(n);
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(c, a[i], "a");
        if (r) return r;
        r = check_ct(c, b[i], "b");
        if (r) return r;
        REQUIRE(a[i]->degree == 1 && b[i]->degree == 1, PFX_EINVAL, "mul_relin needs two degree-1 ciphertexts");
        lvs[i] = std::min(a[i]->n_limbs, b[i]->n_limbs);
        r = check_out(out[i], lvs[i], 1);
        if (r) return r;
    }
    for (size_t i = 0; i < n; ++i)           // the last launch reads operands while writing outputs
        for (size_t j = 0; j < n; ++j) {
            REQUIRE(out[i]->d != a[j]->d && out[i]->d != b[j]->d, PFX_EINVAL,
                    "batched mul_relin output aliases an operand");
            REQUIRE(i == j || out[i]->d != out[j]->d, PFX_EINVAL, "batched mul_relin outputs alias");
        }
    if (n == 0) return PFX_OK;
    Ws w;
    pfx_status r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    std::vector<int> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return lvs[x] > lvs[y]; });
    for (size_t s0 = 0; s0 < n;) {
        const size_t s1 = ks_batch_end(c, order.data(), n, lvs, s0);
        r = mul_relin_group(c, L, a, b, out, &order[s0], (int)(s1 - s0), (int)lvs[order[s0]], rlk);
        if (r) return r;
        s0 = s1;
    }
    for (size_t i = 0; i < n; ++i) {
        const double sc = a[i]->scale * b[i]->scale;
        out[i]->n_limbs = lvs[i];
        out[i]->degree = 1;
        out[i]->scale = sc;
    }
    return PFX_OK;
}

pfx_status pfx_relinearize_batch(pfx_ctx *c, const pfx_ct *const *a, size_t n, const pfx_swk *rlk,
                                 pfx_ct *const *out, void *stream) {
    REQUIRE(c && (n == 0 || (a && out)), PFX_EINVAL, "null argument");
    REQUIRE(rlk && rlk->ctx == c, PFX_EINVAL, "bad relinearisation key");
    REQUIRE(rlk->galois == 0 && !rlk->from_secret, PFX_ENOKEY, "key is not a relinearisation key");
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(c, a[i], "a");
        if (r) return r;
        REQUIRE(a[i]->degree == 2, PFX_EINVAL, "relinearize needs a degree-2 ciphertext");
        r = check_out(out[i], a[i]->n_limbs, 1);
        if (r) return r;
    }
    for (size_t i = 0; i < n; ++i)        // in place allowed; never into another entry
        for (size_t j = 0; j < n; ++j)
            if (i != j) {
                REQUIRE(out[i]->d != a[j]->d, PFX_EINVAL, "batched relinearize output aliases another input");
                REQUIRE(out[i]->d != out[j]->d, PFX_EINVAL, "batched relinearize outputs alias");
            }
    if (n == 0) return PFX_OK;
    Ws w;
    pfx_status r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    std::vector<int> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return a[x]->n_limbs > a[y]->n_limbs; });
    std::vector<double> sc(n);
    std::vector<uint32_t> lvs(n);
    for (size_t i = 0; i < n; ++i) {
        sc[i] = a[i]->scale;
        lvs[i] = a[i]->n_limbs;
    }
    for (size_t s0 = 0; s0 < n;) {
        const size_t s1 = ks_batch_end(c, order.data(), n, lvs, s0);
        KsBatch kb;
        r = get_batch_ws(c, L.st, (int)(s1 - s0), kb);
        if (r) return r;
        kb.nb = (int)(s1 - s0);
        kb.mode = KS_PLAIN;
        for (int e = 0; e < kb.nb; ++e) {
            const int i = order[s0 + e];
            kb.op[e] = ks_plain(a[i]->poly(2), a[i]->poly(0), a[i]->poly(1));
            kb.out0[e] = out[i]->poly(0);
            kb.out1[e] = out[i]->poly(1);
        }
        ks_run(L, kb, (int)lvs[order[s0]], rlk);
        s0 = s1;
    }
    for (size_t i = 0; i < n; ++i) {
        out[i]->n_limbs = lvs[i];
        out[i]->degree = 1;
        out[i]->scale = sc[i];
    }
    return PFX_OK;
}

pfx_status pfx_rescale(pfx_ctx *c, const pfx_ct *a, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    const uint32_t lv = a->n_limbs;
    REQUIRE(lv >= 2, PFX_ELEVEL, "rescale needs at least 2 limbs");
    r = check_out(out, lv - 1, a->degree);
    if (r) return r;
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    const size_t N = c->N;
    const int np = a->degree + 1;
    double *last = w.at(w.lay.rs_last), *tmp = w.at(w.lay.rs_tmp);
    const double sc = a->scale / (double)c->primes[lv - 1];
    const uint32_t deg = a->degree;
    RsEntry e;
    e.in = a->d;
    e.out = out->d;
    e.si = a->cap_limbs * N;
    e.so = out->cap_limbs * N;
    launch_rescale(L, &e, 1, np, lv, last, tmp);
    out->n_limbs = lv - 1;
    out->degree = deg;
    out->scale = sc;
    return PFX_OK;
}

pfx_status pfx_rescale_batch(pfx_ctx *c, const pfx_ct *const *a, size_t n, pfx_ct *const *out, void *stream) {
    REQUIRE(c && (n == 0 || (a && out)), PFX_EINVAL, "null argument");
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(c, a[i], "a");
        if (r) return r;
        REQUIRE(a[i]->n_limbs >= 2, PFX_ELEVEL, "rescale needs at least 2 limbs");
        r = check_out(out[i], a[i]->n_limbs - 1, a[i]->degree);
        if (r) return r;
    }
    for (size_t i = 0; i < n; ++i)        // an entry may rescale in place, never into another's input
        for (size_t j = 0; j < n; ++j)
            if (i != j) {
                REQUIRE(out[i]->d != a[j]->d, PFX_EINVAL, "batched rescale output aliases another input");
                REQUIRE(out[i]->d != out[j]->d, PFX_EINVAL, "batched rescale outputs alias");
            }
    if (n == 0) return PFX_OK;
    Ws w;
    pfx_status r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    const size_t N = c->N;
    std::vector<int> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = (int)i;
    auto shape = [&](int i) { return a[i]->n_limbs * 4 + a[i]->degree; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return shape(x) > shape(y); });
    std::vector<double> sc(n);
    std::vector<uint32_t> deg(n), lvs(n);
    for (size_t i = 0; i < n; ++i) {
        lvs[i] = a[i]->n_limbs;
        deg[i] = a[i]->degree;
        sc[i] = a[i]->scale / (double)c->primes[lvs[i] - 1];
    }
    for (size_t s0 = 0; s0 < n;) {
        size_t s1 = s0;
        while (s1 < n && s1 - s0 < (size_t)kMaxBatch && shape(order[s1]) == shape(order[s0])) ++s1;
        const int nb = (int)(s1 - s0), lv = (int)lvs[order[s0]], np = (int)deg[order[s0]] + 1;
        // scratch: the batch key-switch region, used flat (np lv limbs per entry fit
        // in its dcoef + tmp share of 3 L limbs)
        KsBatch kb;
        r = get_batch_ws(c, S(stream), nb, kb);
        if (r) return r;
        double *last = kb.dcoef, *tmp = last + (size_t)nb * np * N;
        RsEntry ents[kMaxBatch];
        for (int e = 0; e < nb; ++e) {
            const int i = order[s0 + e];
            ents[e].in = a[i]->d;
            ents[e].out = out[i]->d;
            ents[e].si = a[i]->cap_limbs * N;
            ents[e].so = out[i]->cap_limbs * N;
        }
        launch_rescale(L, ents, nb, np, lv, last, tmp);
        s0 = s1;
    }
    for (size_t i = 0; i < n; ++i) {
        out[i]->n_limbs = lvs[i] - 1;
        out[i]->degree = deg[i];
        out[i]->scale = sc[i];
    }
    return PFX_OK;
}

pfx_status pfx_drop_level(pfx_ctx *c, const pfx_ct *a, uint32_t n_limbs, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(n_limbs >= 1 && n_limbs <= a->n_limbs, PFX_ELEVEL, "cannot drop to that many limbs");
    r = check_out(out, n_limbs, a->degree);
    if (r) return r;
    if (out != a) {
        Launch L{c, S(stream)};
        const size_t N = c->N;
        launch_ew(L, EW_COPY, out->d, a->d, nullptr, out->cap_limbs * N, a->cap_limbs * N, 0, a->degree + 1, n_limbs);
    }
    out->n_limbs = n_limbs;
    out->degree = a->degree;
    out->scale = a->scale;
    return PFX_OK;
}

pfx_status pfx_key_switch(pfx_ctx *c, const pfx_ct *d, const pfx_swk *k, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, d, "d");
    if (r) return r;
    REQUIRE(k && k->ctx == c, PFX_EINVAL, "bad key");
    r = check_out(out, d->n_limbs, 1);
    if (r) return r;
    REQUIRE(out != d, PFX_EINVAL, "key_switch output must not alias its input");
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    ks_core(c, L, w, ks_plain(d->poly(0), nullptr, nullptr), d->n_limbs, k, out->poly(0), out->poly(1));
    out->n_limbs = d->n_limbs;
    out->degree = 1;
    out->scale = d->scale;
    return PFX_OK;
}

pfx_status pfx_apply_galois(pfx_ctx *c, const pfx_ct *a, const pfx_swk *gk, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(gk && gk->ctx == c && gk->galois != 0 && !gk->from_secret, PFX_ENOKEY, "not a Galois key");
    REQUIRE(a->degree == 1, PFX_EINVAL, "automorphism needs a degree-1 ciphertext");
    r = check_out(out, a->n_limbs, 1);
    if (r) return r;
    return galois_apply(c, a, gk, out, S(stream));
}

pfx_status pfx_apply_galois_batch(pfx_ctx *c, const pfx_ct *const *a, size_t n, const pfx_swk *gk,
                                  pfx_ct *const *out, void *stream) {
    REQUIRE(c && (n == 0 || (a && out)), PFX_EINVAL, "null argument");
    REQUIRE(gk && gk->ctx == c && gk->galois != 0 && !gk->from_secret, PFX_ENOKEY, "not a Galois key");
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(c, a[i], "a");
        if (r) return r;
        REQUIRE(a[i]->degree == 1, PFX_EINVAL, "automorphism needs a degree-1 ciphertext");
        r = check_out(out[i], a[i]->n_limbs, 1);
        if (r) return r;
    }
    {                                        // the last launch reads the inputs while writing outputs
        std::unordered_set<const double *> ins, outs;
        for (size_t i = 0; i < n; ++i) ins.insert(a[i]->d);
        for (size_t i = 0; i < n; ++i) {
            REQUIRE(!ins.count(out[i]->d), PFX_EINVAL, "batched automorphism output aliases an input");
            REQUIRE(outs.insert(out[i]->d).second, PFX_EINVAL, "batched automorphism outputs alias");
        }
    }
    if (n == 0) return PFX_OK;
    Ws w;
    pfx_status r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    std::vector<int> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return a[x]->n_limbs > a[y]->n_limbs; });
    std::vector<uint32_t> lvs(n);
    std::vector<double> sc(n);
    for (size_t i = 0; i < n; ++i) {
        lvs[i] = a[i]->n_limbs;
        sc[i] = a[i]->scale;
    }
    for (size_t s0 = 0; s0 < n;) {
        const size_t s1 = ks_batch_end(c, order.data(), n, lvs, s0);
        KsBatch kb;
        r = get_batch_ws(c, L.st, (int)(s1 - s0), kb);
        if (r) return r;
        kb.nb = (int)(s1 - s0);
        kb.mode = KS_GALOIS;
        for (int e = 0; e < kb.nb; ++e) {
            const pfx_ct *x = a[order[s0 + e]];
            KsOperand &op = kb.op[e];
            op.mode = KS_GALOIS;
            op.d = x->poly(1);
            op.base0 = x->poly(0);
            op.galois = gk->galois;
            kb.out0[e] = out[order[s0 + e]]->poly(0);
            kb.out1[e] = out[order[s0 + e]]->poly(1);
        }
        ks_run(L, kb, (int)lvs[order[s0]], gk);
        s0 = s1;
    }
    for (size_t i = 0; i < n; ++i) {
        out[i]->n_limbs = lvs[i];
        out[i]->degree = 1;
        out[i]->scale = sc[i];
    }
    return PFX_OK;
}

pfx_status pfx_rotate_batch(pfx_ctx *c, const pfx_ct *const *a, const int32_t *steps, size_t n,
                            const pfx_swk *const *gks, size_t n_gks, pfx_ct *const *out, void *stream) {
    REQUIRE(c && (n == 0 || (a && steps && out)), PFX_EINVAL, "null argument");
    std::vector<const pfx_swk *> key(n, nullptr);
    std::vector<uint32_t> gel(n, 1);
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(c, a[i], "a");
        if (r) return r;
        REQUIRE(a[i]->degree == 1, PFX_EINVAL, "rotate needs a degree-1 ciphertext");
        r = check_out(out[i], a[i]->n_limbs, 1);
        if (r) return r;
        gel[i] = rot_element(c, steps[i]);
        if (gel[i] != 1) {
            key[i] = find_key(c, gel[i], gks, n_gks);
            if (!key[i]) return fail(PFX_ENOKEY, "no Galois key for rotation step " + std::to_string(steps[i]));
        }
    }
    {                                        // the last launch reads the inputs while writing outputs
        std::unordered_set<const double *> ins, outs;
        for (size_t i = 0; i < n; ++i) ins.insert(a[i]->d);
        for (size_t i = 0; i < n; ++i) {
            REQUIRE(!ins.count(out[i]->d), PFX_EINVAL, "batched rotation output aliases an input");
            REQUIRE(outs.insert(out[i]->d).second, PFX_EINVAL, "batched rotation outputs alias");
        }
    }
    if (n == 0) return PFX_OK;
    Launch L{c, S(stream)};
    std::vector<int> order;
    for (size_t i = 0; i < n; ++i) {
        if (gel[i] == 1) {
            pfx_status r = pfx_ct_copy(c, a[i], out[i], stream);
            if (r) return r;
        } else {
            order.push_back((int)i);
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return a[x]->n_limbs > a[y]->n_limbs; });
    std::vector<uint32_t> lvs(n);
    std::vector<double> sc(n);
    for (size_t i = 0; i < n; ++i) {
        lvs[i] = a[i]->n_limbs;
        sc[i] = a[i]->scale;
    }
    for (size_t s0 = 0; s0 < order.size();) {
        const size_t s1 = ks_batch_end(c, order.data(), order.size(), lvs, s0);
        KsBatch kb;
        pfx_status r = get_batch_ws(c, L.st, (int)(s1 - s0), kb);
        if (r) return r;
        kb.nb = (int)(s1 - s0);
        kb.mode = KS_GALOIS;
        for (int e = 0; e < kb.nb; ++e) {
            const int i = order[s0 + e];
            KsOperand &op = kb.op[e];
            op.mode = KS_GALOIS;
            op.d = a[i]->poly(1);
            op.base0 = a[i]->poly(0);
            op.galois = gel[i];
            kb.keys[e] = key[i]->d_k;
            kb.out0[e] = out[i]->poly(0);
            kb.out1[e] = out[i]->poly(1);
        }
        ks_run(L, kb, (int)lvs[order[s0]], key[order[s0]]);
        s0 = s1;
    }
    for (int i : order) {
        out[i]->n_limbs = lvs[i];
        out[i]->degree = 1;
        out[i]->scale = sc[i];
    }
    return PFX_OK;
}

pfx_status pfx_apply_galois_hoisted(pfx_ctx *c, const pfx_ct *a, const pfx_swk *const *gks, size_t n,
                                    pfx_ct *const *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->degree == 1, PFX_EINVAL, "automorphism needs a degree-1 ciphertext");
    REQUIRE(n == 0 || (gks && out), PFX_EINVAL, "null argument");
    {
        std::unordered_set<const double *> outs;
        for (size_t i = 0; i < n; ++i) {
            REQUIRE(gks[i] && gks[i]->ctx == c && gks[i]->galois != 0 && !gks[i]->from_secret, PFX_ENOKEY,
                    "not a Galois key");
            r = check_out(out[i], a->n_limbs, 1);
            if (r) return r;
            REQUIRE(out[i]->d != a->d, PFX_EINVAL, "hoisted automorphism output aliases the input");
            REQUIRE(outs.insert(out[i]->d).second, PFX_EINVAL, "hoisted automorphism outputs alias");
        }
    }
    if (n == 0) return PFX_OK;
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    Launch L{c, S(stream)};
    const int lv = (int)a->n_limbs;
    const double sc = a->scale;
    KsBatch kb;
    r = get_batch_ws(c, L.st, (int)std::min<size_t>(n, kMaxBatch), kb);
    if (r) return r;
    // the decomposition of c1, once, into entry 0's ModUp scratch
    KsBatch up = kb;
    up.nb = 1;
    up.mode = KS_PLAIN;
    up.op[0] = ks_plain(a->poly(1), nullptr, nullptr);
    ks_modup(L, up, lv);
    for (size_t s0 = 0; s0 < n; s0 += kMaxBatch) {
        const int nb = (int)std::min<size_t>(kMaxBatch, n - s0);
        KsBatch g = kb;
        g.nb = nb;
        g.mode = KS_GALOIS;
        for (int e = 0; e < nb; ++e) {
            KsOperand &op = g.op[e];
            op = KsOperand{};
            op.mode = KS_GALOIS;
            op.d = a->poly(1);
            op.base0 = a->poly(0);
            op.galois = gks[s0 + e]->galois;
            g.out0[e] = out[s0 + e]->poly(0);
            g.out1[e] = out[s0 + e]->poly(1);
        }
        for (int e = 0; e < nb; ++e) {               // one key per entry: one inner product each
            KsBatch one = g;
            one.nb = 1;
            one.op[0] = g.op[e];
            one.hoisted = true;
            one.acc = g.acc + (size_t)e * g.sacc;
            launch_ks_inner(L, one, gks[s0 + e]->d_k, lv);
        }
        ks_moddown(L, g, lv);
    }
    for (size_t i = 0; i < n; ++i) {
        out[i]->n_limbs = (uint32_t)lv;
        out[i]->degree = 1;
        out[i]->scale = sc;
    }
    return PFX_OK;
}

pfx_status pfx_mul_monomial(pfx_ctx *c, const pfx_ct *a, int64_t k, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_out(out, a->n_limbs, a->degree);
    if (r) return r;
    const int64_t twoN = 2 * (int64_t)c->N;
    const uint32_t e = (uint32_t)(((k % twoN) + twoN) % twoN);
    Launch L{c, S(stream)};
    const size_t N = c->N;
    const uint32_t lv = a->n_limbs, deg = a->degree;
    const double sc = a->scale;
    launch_monomial(L, out->d, a->d, out->cap_limbs * N, a->cap_limbs * N, (int)deg + 1, (int)lv, e);
    out->n_limbs = lv;
    out->degree = deg;
    out->scale = sc;
    return PFX_OK;
}

pfx_status pfx_mul_inv_n(pfx_ctx *c, const pfx_ct *a, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_out(out, a->n_limbs, a->degree);
    if (r) return r;
    std::vector<uint64_t> cst(a->n_limbs);
    for (uint32_t i = 0; i < a->n_limbs; ++i) cst[i] = invmod_u64((uint64_t)c->N % c->primes[i], c->primes[i]);
    Launch L{c, S(stream)};
    const size_t N = c->N;
    const uint32_t lv = a->n_limbs, deg = a->degree;
    const double sc = a->scale;
    launch_mulconst(L, out->d, a->d, out->cap_limbs * N, a->cap_limbs * N, (int)deg + 1, (int)lv, cst.data());
    out->n_limbs = lv;
    out->degree = deg;
    out->scale = sc;
    return PFX_OK;
}

// ------------------------------------------------------------ ring repacking
}  // extern "C"

namespace {

// Ring-repacking arrays of one stream (doubles), grown on demand.
pfx_status get_repack_ws(pfx_ctx *c, hipStream_t st, size_t doubles, double **out) {
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->ws.find(st);
    if (it == c->ws.end()) return fail(PFX_EINVAL, "stream has no workspace");
    Workspace *w = it->second;
    if (w->rcap < doubles) {
        if (c->capturing) return fail(PFX_EINVAL, "repacking workspace must be reserved before graph capture");
        (void)hipStreamSynchronize(st);
        bump_scratch_epoch();
        dfree(w->rbuf);
        w->rbuf = nullptr;
        w->rcap = 0;
        PFX_DMALLOC(c, &w->rbuf, doubles * sizeof(double));
        w->rcap = doubles;
    }
    *out = w->rbuf;
    return PFX_OK;
}

uint32_t repack_galois(const pfx_ctx *c, int i) {
    const uint64_t two_n = 2 * (uint64_t)c->N;
    if (i == 0) return (uint32_t)(two_n - 1);
    uint64_t g = 5;                                  // 5^(2^(i-1)) mod 2N
    for (int k = 1; k < i; ++k) g = g * g % two_n;
    return (uint32_t)g;
}

// Key-switch entries per repacking launch: the per-entry scratch of a batch
// stays within 512 MiB.
int repack_chunk(const pfx_ctx *c) {
    const size_t per = batch_entry_doubles(c) * sizeof(double);
    return (int)std::max<size_t>(1, std::min<size_t>(4096, ((size_t)512 << 20) / per));
}

// Entries per launch of the fused repacking key switch and its scratch (one
// limb per entry: 256 MiB at N = 2^12).
constexpr int kFusedChunk = 8192;
size_t repack_scratch_doubles(const pfx_ctx *c, int lv) {
    return repack_fused_ok(c, lv) ? (size_t)kFusedChunk * c->N : 0;
}

// Alg. 1 over G groups of N ciphertexts (2 polynomials of lv limbs each, cs =
// 2 lv N doubles apart) already multiplied by N^-1 in A (group stride N cs);
// B holds N/2 ciphertexts per group.  Round i reads one array and writes the
// other; the result of group g is slot 0 of group g of *res (group stride
// *res_gs).  scr: repack_scratch_doubles(c, lv) doubles.
pfx_status repack_rounds(pfx_ctx *c, const Launch &L, double *A, double *B, double *scr, int G, int lv,
                         const pfx_swk *const *gks, size_t n_gks, const double **res, size_t *res_gs) {
    const size_t N = c->N, cs = 2 * (size_t)lv * N;
    const double *in = A;
    double *out = B;
    size_t in_gs = N * cs, out_gs = (N / 2) * cs;
    const bool fused = repack_fused_ok(c, lv);
    const int chunk = fused ? kFusedChunk : repack_chunk(c);
    for (int i = 0; i < c->logn; ++i) {
        const int tlog = c->logn - 1 - i;
        const uint32_t g = repack_galois(c, i);
        const pfx_swk *gk = find_key(c, g, gks, n_gks);
        REQUIRE(gk, PFX_ENOKEY, "no key for a Galois element of ring repacking");
        const int total = G << tlog;
        for (int e0 = 0; e0 < total; e0 += chunk) {
            KsBatch kb;
            const int nb = std::min(chunk, total - e0);
            if (!fused) {
                pfx_status r = get_batch_ws(c, L.st, nb, kb);
                if (r) return r;
            }
            kb.nb = nb;
            kb.mode = KS_REPACK;
            kb.rp.in = in;
            kb.rp.out = out;
            kb.rp.in_gs = in_gs;
            kb.rp.out_gs = out_gs;
            kb.rp.cs = cs;
            kb.rp.ps = (size_t)lv * N;
            kb.rp.tlog = tlog;
            kb.rp.e0 = e0;
            kb.rp.galois = g;
            if (fused) launch_repack_fused(L, kb, gk->d_k, scr);
            else ks_run(L, kb, lv, gk);
        }
        double *next_out = (in == A) ? A : B;        // the array just read is free
        size_t next_gs = in_gs;
        in = out;
        in_gs = out_gs;
        out = next_out;
        out_gs = next_gs;
    }
    *res = in;
    *res_gs = in_gs;
    return PFX_OK;
}

// Slot 0 of each group into the output ciphertexts.
pfx_status repack_store(pfx_ctx *c, hipStream_t st, const double *res, size_t res_gs, int G, int lv, double scale,
                        pfx_ct *const *out) {
    const size_t N = c->N, ps = (size_t)lv * N;
    for (int g = 0; g < G; ++g) {
        const double *src = res + (size_t)g * res_gs;
        for (int u = 0; u < 2; ++u)
            HIPCHECK(hipMemcpyAsync(out[g]->poly((uint32_t)u), src + (size_t)u * ps, ps * sizeof(double),
                                    hipMemcpyDeviceToDevice, st));
        out[g]->n_limbs = (uint32_t)lv;
        out[g]->degree = 1;
        out[g]->scale = scale;
    }
    return PFX_OK;
}

pfx_status check_repack_out(const pfx_ctx *c, pfx_ct *const *out, int G, uint32_t lv) {
    for (int g = 0; g < G; ++g) {
        REQUIRE(out[g] && out[g]->ctx == c, PFX_EINVAL, "repacking output from another context");
        pfx_status r = check_out(out[g], lv, 1);
        if (r) return r;
    }
    return PFX_OK;
}

}  // namespace

extern "C" {

pfx_status pfx_repack(pfx_ctx *c, const pfx_ct *const *in, size_t n, const pfx_swk *const *gks, size_t n_gks,
                      pfx_ct *const *out, void *stream) {
    REQUIRE(c && in && out && n >= 1, PFX_EINVAL, "null argument or no input");
    REQUIRE(n <= (size_t)1 << 24, PFX_EINVAL, "more than 2^24 inputs");
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(c, in[i], "in");
        if (r) return r;
        REQUIRE(in[i]->degree == 1, PFX_EINVAL, "repacking needs degree-1 ciphertexts");
        REQUIRE(in[i]->n_limbs == in[0]->n_limbs, PFX_ELEVEL, "repacking inputs at different levels");
        REQUIRE(in[i]->scale == in[0]->scale, PFX_ESCALE, "repacking inputs at different scales");
    }
    const size_t N = c->N;
    const int G = (int)((n + N - 1) / N);
    const int lv = (int)in[0]->n_limbs;
    pfx_status r = check_repack_out(c, out, G, (uint32_t)lv);
    if (r) return r;
    {
        std::unordered_set<const double *> ins;
        for (size_t i = 0; i < n; ++i) ins.insert(in[i]->d);
        for (int g = 0; g < G; ++g)
            REQUIRE(!ins.count(out[g]->d), PFX_EINVAL, "repacking output aliases an input");
    }
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    const size_t cs = 2 * (size_t)lv * N;
    double *A = nullptr;
    r = get_repack_ws(c, S(stream), (size_t)G * N * cs * 3 / 2 + repack_scratch_doubles(c, lv), &A);
    if (r) return r;
    double *B = A + (size_t)G * N * cs, *scr = B + (size_t)G * (N / 2) * cs;
    Launch L{c, S(stream)};
    // N^-1 c_i into the slots (Alg. 1 pre-multiplication), zeros after the last input
    std::vector<uint64_t> ninv(lv);
    for (int i = 0; i < lv; ++i) ninv[i] = invmod_u64((uint64_t)N % c->primes[i], c->primes[i]);
    ew_collect_begin(L);
    for (size_t i = 0; i < n; ++i)
        launch_mulconst(L, A + i * cs, in[i]->d, (size_t)lv * N, (size_t)in[i]->cap_limbs * N, 2, lv, ninv.data());
    ew_collect_end(L);
    launch_mono_sum(L, A + n * cs, cs, (size_t)lv * N, nullptr, 0, 0, 0, nullptr, 0, (int)((size_t)G * N - n), lv,
                    false);
    const double *res;
    size_t res_gs;
    r = repack_rounds(c, L, A, B, scr, G, lv, gks, n_gks, &res, &res_gs);
    if (r) return r;
    return repack_store(c, L.st, res, res_gs, G, lv, in[0]->scale, out);
}

pfx_status pfx_pfe_repack(pfx_ctx *c, const pfx_ct *const *tables, size_t m, const int64_t *exps, size_t n,
                          const pfx_swk *const *gks, size_t n_gks, pfx_ct *const *out, void *stream) {
    REQUIRE(c && tables && exps && out && m >= 1 && n >= 1, PFX_EINVAL, "null argument, no table or no record");
    REQUIRE(m <= 4096 && n <= (size_t)1 << 24, PFX_EINVAL, "more than 4096 tables or 2^24 records");
    for (size_t l = 0; l < m; ++l) {
        pfx_status r = check_ct(c, tables[l], "tables");
        if (r) return r;
        REQUIRE(tables[l]->degree == 1, PFX_EINVAL, "lookup tables must be degree-1 ciphertexts");
        REQUIRE(tables[l]->n_limbs == tables[0]->n_limbs, PFX_ELEVEL, "lookup tables at different levels");
        REQUIRE(tables[l]->scale == tables[0]->scale, PFX_ESCALE, "lookup tables at different scales");
    }
    const size_t N = c->N;
    const int G = (int)((n + N - 1) / N);
    const int lv = (int)tables[0]->n_limbs;
    pfx_status r = check_repack_out(c, out, G, (uint32_t)lv);
    if (r) return r;
    for (int g = 0; g < G; ++g)
        for (size_t l = 0; l < m; ++l)
            REQUIRE(out[g]->d != tables[l]->d, PFX_EINVAL, "repacking output aliases a table");
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    const size_t cs = 2 * (size_t)lv * N;
    const size_t tbl = (size_t)m * cs;
    double *T = nullptr;
    r = get_repack_ws(c, S(stream), tbl + (size_t)G * N * cs * 3 / 2 + repack_scratch_doubles(c, lv), &T);
    if (r) return r;
    double *A = T + tbl, *B = A + (size_t)G * N * cs, *scr = B + (size_t)G * (N / 2) * cs;
    Launch L{c, S(stream)};
    // the tables side by side (contiguous polynomials), then every record's sum
    for (size_t l = 0; l < m; ++l)
        for (int u = 0; u < 2; ++u)
            HIPCHECK(hipMemcpyAsync(T + l * cs + (size_t)u * lv * N, tables[l]->poly((uint32_t)u),
                                    (size_t)lv * N * sizeof(double), hipMemcpyDeviceToDevice, L.st));
    if (mono_sum_lds_ok(c, (int)m))
        launch_mono_sum_lds(L, A, cs, (size_t)lv * N, T, cs, (size_t)lv * N, (int)m, exps, (int)n,
                            (int)((size_t)G * N), lv, true);
    else
        launch_mono_sum(L, A, cs, (size_t)lv * N, T, cs, (size_t)lv * N, (int)m, exps, (int)n, (int)((size_t)G * N),
                        lv, true);
    const double *res;
    size_t res_gs;
    r = repack_rounds(c, L, A, B, scr, G, lv, gks, n_gks, &res, &res_gs);
    if (r) return r;
    return repack_store(c, L.st, res, res_gs, G, lv, tables[0]->scale, out);
}

pfx_status pfx_linear_transform(pfx_ctx *c, const pfx_ct *a, const pfx_pt *const *diags, const int32_t *steps,
                                size_t n, uint32_t n1, const pfx_swk *const *keys, size_t n_keys, pfx_ct *out,
                                void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->degree == 1, PFX_EINVAL, "linear transform needs a degree-1 ciphertext");
    REQUIRE(n >= 1 && diags && steps && n1 >= 1, PFX_EINVAL, "no diagonal, null argument or n1 = 0");
    const uint32_t lv = a->n_limbs;
    const int64_t half = c->N / 2;
    REQUIRE(n1 <= (uint64_t)half, PFX_EINVAL, "n1 beyond the slot count");
    for (size_t k = 0; k < n; ++k) {
        r = check_ct(c, diags[k], "diagonal");
        if (r) return r;
        REQUIRE(diags[k]->degree == 0 && diags[k]->n_limbs >= lv, PFX_ELEVEL,
                "diagonals must be plaintexts with at least the ciphertext's limbs");
        REQUIRE(diags[k]->scale == diags[0]->scale, PFX_ESCALE, "diagonals at different scales");
    }
    r = check_out(out, lv, 1);
    if (r) return r;
    REQUIRE(out->d != a->d, PFX_EINVAL, "linear transform output aliases the input");
    // steps = n1 j + i; the distinct baby steps i != 0 (hoisted), the distinct giant steps j
    std::vector<int64_t> st(n);
    std::vector<int64_t> babies, giants;
    for (size_t k = 0; k < n; ++k) {
        st[k] = (((int64_t)steps[k] % half) + half) % half;
        babies.push_back(st[k] % n1);
        giants.push_back(st[k] / n1);
    }
    std::sort(babies.begin(), babies.end());
    babies.erase(std::unique(babies.begin(), babies.end()), babies.end());
    if (!babies.empty() && babies[0] == 0) babies.erase(babies.begin());
    std::sort(giants.begin(), giants.end());
    giants.erase(std::unique(giants.begin(), giants.end()), giants.end());
    std::vector<const pfx_swk *> bkeys;
    for (int64_t i : babies) {
        const pfx_swk *k = find_key(c, rot_element(c, i), keys, n_keys);
        if (!k) return fail(PFX_ENOKEY, "no Galois key for baby step " + std::to_string(i));
        bkeys.push_back(k);
    }
    for (int64_t j : giants)
        if (j && !find_key(c, rot_element(c, n1 * j), keys, n_keys))
            return fail(PFX_ENOKEY, "no Galois key for giant step " + std::to_string(n1 * j));
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    const size_t N = c->N, cs = 2 * (size_t)lv * N;
    double *buf = nullptr;                     // baby rotations, the group sum, its rotation
    r = get_repack_ws(c, S(stream), (babies.size() + 2) * cs, &buf);
    if (r) return r;
    auto view = [&](double *d, uint32_t deg, double scale) {
        pfx_ct v;
        v.ctx = c;
        v.cap_limbs = v.n_limbs = lv;
        v.cap_degree = v.degree = deg;
        v.scale = scale;
        v.d = d;
        v.owns = false;
        return v;
    };
    std::vector<pfx_ct> bv;
    for (size_t b = 0; b < babies.size(); ++b) bv.push_back(view(buf + b * cs, 1, a->scale));
    pfx_ct acc = view(buf + babies.size() * cs, 1, 0.0), rot = view(buf + (babies.size() + 1) * cs, 1, 0.0);
    if (!babies.empty()) {
        std::vector<pfx_ct *> bo;
        for (pfx_ct &v : bv) bo.push_back(&v);
        r = pfx_apply_galois_hoisted(c, a, bkeys.data(), bkeys.size(), bo.data(), stream);
        if (r) return r;
    }
    auto baby = [&](int64_t i) -> const pfx_ct * {
        if (i == 0) return a;
        return &bv[std::lower_bound(babies.begin(), babies.end(), i) - babies.begin()];
    };
    Launch L{c, S(stream)};
    bool first = true;
    std::vector<size_t> terms;
    for (int64_t j : giants) {
        // sum_k rot(d_k, -n1 j) (.) rot(z, i_k) over the group, up to kMacTerms
        // terms a launch, the plaintext automorphism applied as the terms are read
        const uint32_t g_back = rot_element(c, half - (int64_t)n1 * j);
        terms.clear();
        for (size_t k = 0; k < n; ++k)
            if (st[k] / n1 == j) terms.push_back(k);
        for (size_t t0 = 0; t0 < terms.size(); t0 += kMacTerms) {
            MacTerms m{};
            const int nt = (int)std::min<size_t>(kMacTerms, terms.size() - t0);
            for (int u = 0; u < nt; ++u) {
                const size_t k = terms[t0 + u];
                const pfx_ct *b = baby(st[k] % n1);
                m.pt[u] = diags[k]->d;
                m.ct[u] = b->d;
                m.cs[u] = (size_t)b->cap_limbs * N;
            }
            launch_diag_mac(L, acc.d, (size_t)acc.cap_limbs * N, m, nt, (int)lv, g_back, t0 > 0);
        }
        acc.scale = a->scale * diags[0]->scale;
        const pfx_ct *part = &acc;
        if (j) {
            r = pfx_rotate(c, &acc, (int32_t)(n1 * j), keys, n_keys, &rot, stream);
            if (r) return r;
            part = &rot;
        }
        r = first ? pfx_ct_copy(c, part, out, stream) : pfx_add(c, out, part, out, stream);
        if (r) return r;
        first = false;
    }
    return PFX_OK;
}

pfx_status pfx_mod_raise(pfx_ctx *c, const pfx_ct *a, uint32_t n_limbs, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->n_limbs == 1, PFX_ELEVEL, "ModRaise starts from one limb (q_0)");
    REQUIRE(n_limbs >= 1 && n_limbs <= (uint32_t)c->L, PFX_ELEVEL, "target level out of range");
    r = check_out(out, n_limbs, a->degree);
    if (r) return r;
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    const size_t N = c->N;
    const int np = (int)a->degree + 1;
    double *stage = nullptr;
    r = get_repack_ws(c, S(stream), (size_t)np * N, &stage);
    if (r) return r;
    for (int u = 0; u < np; ++u)
        HIPCHECK(hipMemcpyAsync(stage + (size_t)u * N, a->poly((uint32_t)u), N * sizeof(double),
                                hipMemcpyDeviceToDevice, S(stream)));
    Launch L{c, S(stream)};
    LimbMap one = contiguous_map(1, 0);
    launch_ntt_pass(L, stage, nullptr, one, true, true, np, N);        // to the coefficient domain over q_0
    launch_ntt_pass(L, stage, nullptr, one, false, true, np, N);
    const double sc = a->scale;
    launch_mod_raise(L, out->d, (size_t)out->cap_limbs * N, stage, N, np, (int)n_limbs);
    const LimbMap m = contiguous_map((int)n_limbs, 0);
    launch_ntt_pass(L, out->d, nullptr, m, false, false, np, (size_t)out->cap_limbs * N);
    launch_ntt_pass(L, out->d, nullptr, m, true, false, np, (size_t)out->cap_limbs * N);
    out->n_limbs = n_limbs;
    out->degree = (uint32_t)np - 1;
    out->scale = sc;
    return PFX_OK;
}

pfx_status pfx_subring_trace(pfx_ctx *c, const pfx_ct *a, uint32_t log_r, const pfx_swk *const *keys, size_t n_keys,
                             pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->degree == 1, PFX_EINVAL, "the trace needs a degree-1 ciphertext");
    REQUIRE(log_r < (uint32_t)c->logn, PFX_EINVAL, "log_r must be below log N");
    r = check_out(out, a->n_limbs, 1);
    if (r) return r;
    std::vector<const pfx_swk *> ks;
    for (uint32_t t = 0; t < log_r; ++t) {
        const pfx_swk *k = find_key(c, (uint32_t)(c->N >> t) + 1u, keys, n_keys);
        if (!k) return fail(PFX_ENOKEY, "no Galois key for N/2^" + std::to_string(t) + " + 1");
        ks.push_back(k);
    }
    const uint32_t lv = a->n_limbs;
    const size_t N = c->N;
    double *tmpd = nullptr;
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    r = get_repack_ws(c, S(stream), 2 * (size_t)lv * N, &tmpd);
    if (r) return r;
    pfx_ct tmp;
    tmp.ctx = c;
    tmp.cap_limbs = lv;
    tmp.cap_degree = 1;
    tmp.d = tmpd;
    tmp.owns = false;
    if (out != a) {
        r = pfx_ct_copy(c, a, out, stream);
        if (r) return r;
    }
    for (const pfx_swk *k : ks) {           // out <- out + phi_{N/2^t + 1}(out)
        r = galois_apply(c, out, k, &tmp, S(stream));
        if (r) return r;
        r = pfx_add(c, out, &tmp, out, stream);
        if (r) return r;
    }
    return PFX_OK;
}

pfx_status pfx_ring_merge(pfx_ctx *big, pfx_ctx *small, const pfx_ct *const *in, size_t n, const pfx_swk *swk,
                          pfx_ct *out, void *stream) {
    REQUIRE(big && small && in && swk && out && n >= 1, PFX_EINVAL, "null argument or no input");
    REQUIRE(small->logn < big->logn, PFX_EINVAL, "the small ring must have the smaller degree");
    const int log_r = big->logn - small->logn;
    REQUIRE(n <= ((size_t)1 << log_r), PFX_EINVAL, "more inputs than the ring ratio N / n");
    REQUIRE(small->primes[0] == big->primes[0], PFX_EPARAM, "the rings do not share their first prime");
    REQUIRE(swk->ctx == big && swk->from_secret, PFX_ENOKEY, "not a key from the embedded secret (pfx_swk_create_from)");
    for (size_t i = 0; i < n; ++i) {
        pfx_status r = check_ct(small, in[i], "in");
        if (r) return r;
        REQUIRE(in[i]->degree == 1 && in[i]->n_limbs == 1, PFX_ELEVEL, "merging needs degree-1 ciphertexts of one limb");
        REQUIRE(in[i]->scale == in[0]->scale, PFX_ESCALE, "merging inputs at different scales");
    }
    pfx_status r = check_out(out, 1, 1);
    if (r) return r;
    REQUIRE(out->ctx == big, PFX_EINVAL, "output of another context");
    Ws w;
    r = get_ws(big, S(stream), w);
    if (r) return r;
    const size_t Ns = small->N, Nb = big->N;
    double *stage = nullptr;                       // 2n small polynomials, then 2 large ones
    r = get_repack_ws(big, S(stream), 2 * ((size_t)n * Ns + Nb), &stage);
    if (r) return r;
    double *merged = stage + 2 * (size_t)n * Ns;
    for (size_t i = 0; i < n; ++i)
        for (uint32_t u = 0; u < 2; ++u)
            HIPCHECK(hipMemcpyAsync(stage + (2 * i + u) * Ns, in[i]->poly(u), Ns * sizeof(double),
                                    hipMemcpyDeviceToDevice, S(stream)));
    LimbMap one;
    one.n = 1;
    one.off[0] = 0;
    one.pid[0] = 0;
    // the inputs to the coefficient domain (small ring), placed in the large
    // ring, back to the NTT domain (large ring; the shared prime)
    Launch Ls{small, S(stream)}, Lb{big, S(stream)};
    launch_ntt_pass(Ls, stage, nullptr, one, true, true, (int)(2 * n), Ns);
    launch_ntt_pass(Ls, stage, nullptr, one, false, true, (int)(2 * n), Ns);
    launch_merge_gather(Lb, merged, stage, (int)n, log_r, small->logn);
    launch_ntt_pass(Lb, merged, nullptr, one, false, false, 2, Nb);
    launch_ntt_pass(Lb, merged, nullptr, one, true, false, 2, Nb);
    // ring switching: (b, 0) + SwitchKey(a) from the embedded secret to the large one
    ks_core(big, Lb, w, ks_plain(merged + Nb, merged, nullptr), 1, swk, out->poly(0), out->poly(1));
    out->n_limbs = 1;
    out->degree = 1;
    out->scale = in[0]->scale;
    return PFX_OK;
}

pfx_status pfx_rotate(pfx_ctx *c, const pfx_ct *a, int32_t step, const pfx_swk *const *keys, size_t n, pfx_ct *out,
                      void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->degree == 1, PFX_EINVAL, "rotate needs a degree-1 ciphertext");
    r = check_out(out, a->n_limbs, 1);
    if (r) return r;
    const uint32_t g = rot_element(c, step);
    if (g == 1) return pfx_ct_copy(c, a, out, stream);
    pfx_swk *k = find_key(c, g, keys, n);
    if (!k) return fail(PFX_ENOKEY, "no Galois key for rotation step " + std::to_string(step));
    return galois_apply(c, a, k, out, S(stream));
}

pfx_status pfx_conjugate(pfx_ctx *c, const pfx_ct *a, const pfx_swk *const *keys, size_t n, pfx_ct *out,
                         void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->degree == 1, PFX_EINVAL, "conjugate needs a degree-1 ciphertext");
    r = check_out(out, a->n_limbs, 1);
    if (r) return r;
    pfx_swk *k = find_key(c, 2u * c->N - 1, keys, n);
    if (!k) return fail(PFX_ENOKEY, "no conjugation key");
    return galois_apply(c, a, k, out, S(stream));
}

pfx_status pfx_rotate_sum(pfx_ctx *c, const pfx_ct *a, uint32_t log_steps, const pfx_swk *const *keys, size_t n,
                          pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    REQUIRE(a->degree == 1, PFX_EINVAL, "rotate_sum needs a degree-1 ciphertext");
    REQUIRE(log_steps < (uint32_t)c->logn, PFX_EINVAL, "log_steps must be < log_n");
    r = check_out(out, a->n_limbs, 1);
    if (r) return r;
    std::vector<pfx_swk *> ks(log_steps);
    for (uint32_t k = 0; k < log_steps; ++k) {
        ks[k] = find_key(c, rot_element(c, 1ll << k), keys, n);
        if (!ks[k]) return fail(PFX_ENOKEY, "no Galois key for rotation step " + std::to_string(1 << k));
    }
    Ws w;
    r = get_ws(c, S(stream), w);
    if (r) return r;
    pfx_ct tmp;                       // a view of the workspace, no allocation
    tmp.ctx = c;
    tmp.cap_limbs = c->L;
    tmp.cap_degree = 1;
    tmp.d = w.at(w.lay.rot);
    r = pfx_ct_copy(c, a, out, stream);
    for (uint32_t k = 0; k < log_steps && !r; ++k) {
        r = galois_apply(c, out, ks[k], &tmp, S(stream));
        if (!r) r = pfx_add(c, out, &tmp, out, stream);
    }
    return r;
}

pfx_status pfx_add_const(pfx_ctx *c, const pfx_ct *a, double value, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    r = check_out(out, a->n_limbs, a->degree);
    if (r) return r;
    const double v = value * a->scale;
    REQUIRE(std::isfinite(v) && std::fabs(v) < 9.0e18, PFX_EINVAL, "constant times scale out of range");
    const int64_t k = (int64_t)(v < 0 ? -std::floor(-v + 0.5) : std::floor(v + 0.5));   // half away from zero
    std::vector<uint64_t> cst(a->n_limbs);
    for (uint32_t i = 0; i < a->n_limbs; ++i) {
        const uint64_t q = c->primes[i];
        const uint64_t mag = (uint64_t)(k < 0 ? -k : k) % q;
        cst[i] = k < 0 ? (q - mag) % q : mag;
    }
    Launch L{c, S(stream)};
    launch_addconst(L, out->poly(0), a->poly(0), a->n_limbs, cst.data());
    if (out != a && a->degree >= 1)
        launch_ew(L, EW_COPY, out->poly(1), a->poly(1), nullptr, out->cap_limbs * (size_t)c->N,
                  a->cap_limbs * (size_t)c->N, 0, a->degree, a->n_limbs);
    out->n_limbs = a->n_limbs;
    out->degree = a->degree;
    out->scale = a->scale;
    return PFX_OK;
}

pfx_status pfx_mul_const(pfx_ctx *c, const pfx_ct *a, double value, double cscale, pfx_ct *out, void *stream) {
    pfx_status r = check_ct(c, a, "a");
    if (r) return r;
    if (cscale <= 0) cscale = (double)c->primes[a->n_limbs - 1];
    const double v = value * cscale;
    REQUIRE(std::isfinite(v) && std::fabs(v) < 9.0e18, PFX_EINVAL, "constant times scale out of range");
    const int64_t k = (int64_t)(v < 0 ? -std::floor(-v + 0.5) : std::floor(v + 0.5));
    const double sc = a->scale * cscale;
    r = pfx_mul_int(c, a, k, out, stream);
    if (r) return r;
    out->scale = sc;
    return PFX_OK;
}

pfx_status pfx_ntt(pfx_ctx *c, uint64_t *d_words, uint32_t first_prime, uint32_t n_limbs, size_t batch, int inverse,
                   void *stream) {
    REQUIRE(c && d_words, PFX_EINVAL, "null argument");
    REQUIRE(n_limbs >= 1 && first_prime + n_limbs <= (uint32_t)(c->L + c->K), PFX_EINVAL, "prime range out of bounds");
    REQUIRE(batch >= 1, PFX_EINVAL, "empty batch");
    Launch L{c, S(stream)};
    // two launches in place: words are converted as the first pass loads them
    // and written back canonical by the last pass; launches of at most 2^20
    // limbs keep the block count within int
    const size_t total_limbs = batch * n_limbs;
    const size_t chunk = (size_t)n_limbs << (20 - std::min(20, (int)std::ceil(std::log2((double)n_limbs))));
    for (size_t l0 = 0; l0 < total_limbs; l0 += chunk) {
        const size_t nl = std::min(chunk, total_limbs - l0);
        launch_ntt_words(L, d_words + l0 * c->N, nl, (int)first_prime, (int)n_limbs, inverse != 0);
    }
    return PFX_OK;
}

static constexpr int kLanes = 8;

static pfx_status ensure_lanes(pfx_ctx *c) {
    if ((int)c->lanes.size() == kLanes) return PFX_OK;
    HIPCHECK(hipSetDevice(c->device));
    for (int i = (int)c->lanes.size(); i < kLanes; ++i) {
        hipStream_t st;
        HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->lanes.push_back(st);
    }
    for (int i = 0; i < kLanes + 1; ++i) {
        hipEvent_t e;
        HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->lane_events.push_back(e);
    }
    return PFX_OK;
}

// Lane structure of an op list (PFX_OP_LANE markers): the caller declares which
// ops may run concurrently.  Before any op is launched, every dependency
// (read-after-write, write-after-read, write-after-write on registers) of an op
// inside a fork is checked to lie on its own lane or before the fork, so that
// the fork/join events alone order the list.
static bool reads_b_register(int32_t code) {
    return code == PFX_OP_ADD || code == PFX_OP_SUB || code == PFX_OP_MUL_RELIN || code == PFX_OP_MUL ||
           code == PFX_OP_MUL_ACC || code == PFX_OP_MUL_CONST_TO ||
           code == PFX_OP_MUL_CONST_LIKE;
}

static pfx_status check_lanes(const pfx_op *ops, size_t n_ops, size_t n_regs) {
    struct Tag {
        int epoch = -1, lane = -1;   // fork epoch and lane of an access; lane -1 = caller stream
    };
    std::vector<Tag> writer(n_regs);
    std::vector<std::vector<Tag>> readers(n_regs);
    int epoch = 0, lane = -1;
    auto ok = [&](const Tag &t) { return t.epoch < epoch || t.lane == -1 || t.lane == lane; };
    for (size_t i = 0; i < n_ops; ++i) {
        const pfx_op &o = ops[i];
        if (o.code == PFX_OP_LANE) {
            if (o.k < -1 || o.k >= kLanes) return fail(PFX_EINVAL, "op " + std::to_string(i) + ": lane out of range");
            if (o.k == -1) {
                if (lane != -1) ++epoch;
                lane = -1;
            } else {
                lane = (int)o.k;
            }
            continue;
        }
        auto in_range = [&](int32_t k) { return k >= 0 && (size_t)k < n_regs; };
        if (!in_range(o.dst) || !in_range(o.a)) continue;   // run_op reports it
        const bool rb = reads_b_register(o.code) && in_range(o.b);
        bool good = ok(writer[o.a]) && (!rb || ok(writer[o.b])) && ok(writer[o.dst]);
        for (const Tag &t : readers[o.dst]) good = good && ok(t);
        if (!good)
            return fail(PFX_EINVAL, "op " + std::to_string(i) + " depends on an op of another lane of the same fork");
        const Tag me{epoch, lane};
        readers[o.a].push_back(me);
        if (rb) readers[o.b].push_back(me);
        writer[o.dst] = me;
        readers[o.dst].clear();
    }
    return PFX_OK;
}

// The op list with its lane markers honoured: the first marker of a fork
// records an event on `stream` that every lane waits for; LANE -1 (and the end
// of the list) joins every lane back into `stream`.
static pfx_status run_ops_lanes(pfx_ctx *c, const pfx_op *ops, size_t n_ops, pfx_ct *const *regs, size_t n_regs,
                                size_t n_inputs, const pfx_pt *const *pts, size_t n_pts, const pfx_swk *rlk,
                                const pfx_swk *const *gks, size_t n_gks, void *stream) {
    pfx_status r = check_lanes(ops, n_ops, n_regs);
    if (!r) r = ensure_lanes(c);
    for (int l = 0; l < kLanes && !r; ++l) {      // scratch of every lane before anything is enqueued or captured
        Ws w;
        r = get_ws(c, c->lanes[l], w);
    }
    if (r) return r;
    bool forked = false;
    void *cur = stream;
    auto join = [&]() -> pfx_status {
        for (int l = 0; l < kLanes; ++l) {
            HIPCHECK(hipEventRecord(c->lane_events[l], c->lanes[l]));
            HIPCHECK(hipStreamWaitEvent(S(stream), c->lane_events[l], 0));
        }
        forked = false;
        cur = stream;
        return PFX_OK;
    };
    pfx_status res = PFX_OK;
    for (size_t i = 0; i < n_ops && !res; ++i) {
        const pfx_op &o = ops[i];
        if (o.code != PFX_OP_LANE) {
            size_t j = i + 1;
            while (j < n_ops && ops[j].code != PFX_OP_LANE) ++j;
            res = run_span(c, ops, i, j, regs, n_regs, n_inputs, pts, n_pts, rlk, gks, n_gks, cur, kMaxBatch);
            i = j - 1;
            continue;
        }
        if (o.k == -1) {
            if (forked) res = join();
            continue;
        }
        if (!forked) {
            HIPCHECK(hipEventRecord(c->lane_events[kLanes], S(stream)));
            for (int l = 0; l < kLanes; ++l) HIPCHECK(hipStreamWaitEvent(c->lanes[l], c->lane_events[kLanes], 0));
            forked = true;
        }
        cur = c->lanes[o.k];
    }
    if (forked) {            // also after a failed op
        pfx_status rj = join();
        if (!res) res = rj;
    }
    return res;
}

pfx_status pfx_run_circuit(pfx_ctx *c, const pfx_op *ops, size_t n_ops, pfx_ct *const *regs, size_t n_regs,
                           size_t n_inputs, const pfx_pt *const *pts, size_t n_pts, const pfx_swk *rlk,
                           const pfx_swk *const *gks, size_t n_gks, int mode, void *stream) {
    REQUIRE(c && ops && regs, PFX_EINVAL, "null argument");
    REQUIRE(n_inputs <= n_regs, PFX_EINVAL, "n_inputs > n_regs");
    REQUIRE((mode & ~(PFX_RUN_GRAPH | PFX_RUN_LANES)) == 0, PFX_EINVAL, "unknown mode bits");
    for (size_t i = 0; i < n_regs; ++i) REQUIRE(regs[i] && regs[i]->ctx == c, PFX_EINVAL, "bad register");
    const bool lanes = (mode & PFX_RUN_LANES) != 0;
    auto exec = [&]() {
        return lanes ? run_ops_lanes(c, ops, n_ops, regs, n_regs, n_inputs, pts, n_pts, rlk, gks, n_gks, stream)
                     : run_ops(c, ops, n_ops, regs, n_regs, n_inputs, pts, n_pts, rlk, gks, n_gks, stream,
                               kMaxBatch);
    };
    if (!(mode & PFX_RUN_GRAPH)) return exec();
    REQUIRE(stream != nullptr, PFX_EINVAL, "graph capture needs a non-default stream");
    // The graph is valid for this op list, these objects (by identity: never
    // an address that a freed object may have left behind), their capacities,
    // these input shapes and plaintext levels, this stream and the scratch
    // epoch it was captured in.
    std::string key((const char *)ops, n_ops * sizeof(pfx_op));
    std::vector<uint64_t> uids{c->uid};
    auto put = [&](const void *p, size_t n) { key.append((const char *)p, n); };
    for (size_t i = 0; i < n_regs; ++i) {
        put(&regs[i]->uid, sizeof(uint64_t));
        put(&regs[i]->cap_limbs, sizeof(uint32_t));
        put(&regs[i]->cap_degree, sizeof(uint32_t));
        uids.push_back(regs[i]->uid);
    }
    for (size_t i = 0; i < n_inputs; ++i) {
        put(&regs[i]->n_limbs, sizeof(uint32_t));
        put(&regs[i]->degree, sizeof(uint32_t));
        put(&regs[i]->scale, sizeof(double));
    }
    for (size_t i = 0; i < n_pts; ++i) {
        REQUIRE(pts[i], PFX_EINVAL, "null plaintext");
        put(&pts[i]->uid, sizeof(uint64_t));
        put(&pts[i]->n_limbs, sizeof(uint32_t));
        put(&pts[i]->scale, sizeof(double));
        uids.push_back(pts[i]->uid);
    }
    for (size_t i = 0; i < n_gks; ++i) {
        REQUIRE(gks[i], PFX_EINVAL, "null Galois key");
        put(&gks[i]->uid, sizeof(uint64_t));
        uids.push_back(gks[i]->uid);
    }
    if (rlk) {
        put(&rlk->uid, sizeof(uint64_t));
        uids.push_back(rlk->uid);
    }
    for (uint64_t u : uids)
        REQUIRE(u != 0, PFX_EINVAL, "graph mode needs library-created objects");
    put(&stream, sizeof(void *));
    put(&mode, sizeof(int));
    pfx_status lr = PFX_OK;
    auto replay = [&](GraphExec &x, const GraphCache<GraphExec>::Meta &meta) {
        for (size_t i = n_inputs; i < n_regs; ++i) {   // register metadata as the capture left it
            regs[i]->n_limbs = meta[i].first & 0xffff;
            regs[i]->degree = meta[i].first >> 16;
            regs[i]->scale = meta[i].second;
        }
        if (hipGraphLaunch(x.exec, S(stream)) != hipSuccess || hipEventRecord(x.done, S(stream)) != hipSuccess)
            lr = fail(PFX_EDEVICE, "graph launch failed");
    };
    if (graphs().launch(key, scratch_epoch().load(), replay)) return lr;

    Ws w;
    pfx_status r = get_ws(c, S(stream), w);   // allocate scratch before capturing
    if (r) return r;
    const int nb = (int)max_mr_run(ops, n_ops, kMaxBatch);
    KsBatch kb;
    if (nb > 1 && !lanes) r = get_batch_ws(c, S(stream), nb, kb);
    if (r) return r;
    if (lanes) {
        r = ensure_lanes(c);
        for (int l = 0; l < kLanes && !r; ++l) {
            r = get_ws(c, c->lanes[l], w);
            if (!r && nb > 1) r = get_batch_ws(c, c->lanes[l], nb, kb);
        }
        if (r) return r;
    }
    // every scratch region this capture writes is in place: the graph belongs
    // to the current epoch
    const uint64_t epoch = scratch_epoch().load();
    const bool prof = c->prof_on;
    c->prof_on = false;
    c->capturing = true;
    HIPCHECK(hipStreamBeginCapture(S(stream), hipStreamCaptureModeThreadLocal));
    r = exec();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(S(stream), &g);
    c->capturing = false;
    c->prof_on = prof;
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(PFX_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    GraphExec x;
    x.device = c->device;
    e = hipGraphInstantiate(&x.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PFX_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (hipEventCreateWithFlags(&x.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(x.exec);
        return fail(PFX_EDEVICE, "graph event creation failed");
    }
    GraphCache<GraphExec>::Meta meta;
    for (size_t i = 0; i < n_regs; ++i) meta.push_back({regs[i]->n_limbs | (regs[i]->degree << 16), regs[i]->scale});
    graphs().insert_and_launch(key, epoch, x, uids, meta, replay);
    return lr;
}

// ------------------------------------------------------------------ batched form
// Entries grouped for batched key switches: same context and level, at most
// kMaxBatch per group, no output aliasing an operand of its own entry (those
// run alone, as pfx_mul_relin handles them); one entry per group otherwise.
static std::vector<std::vector<size_t>> batch_groups(pfx_ctx *const *ctxs, const pfx_ct *const *a,
                                                     const pfx_ct *const *b, pfx_ct *const *out, size_t n,
                                                     bool group) {
    std::vector<std::vector<size_t>> gs;
    std::map<std::pair<const pfx_ctx *, uint32_t>, size_t> open;   // (context, level) -> group being filled
    for (size_t i = 0; i < n; ++i) {
        const bool self_alias = out[i]->d == a[i]->d || out[i]->d == b[i]->d;
        if (!group || self_alias) {
            gs.push_back({i});
            continue;
        }
        const auto key = std::make_pair((const pfx_ctx *)ctxs[i], std::min(a[i]->n_limbs, b[i]->n_limbs));
        auto it = open.find(key);
        if (it == open.end() || gs[it->second].size() == (size_t)kMaxBatch) {
            open[key] = gs.size();
            gs.push_back({i});
        } else {
            gs[it->second].push_back(i);
        }
    }
    return gs;
}

static pfx_status batch_group_run(pfx_ctx *const *ctxs, const pfx_ct *const *a, const pfx_ct *const *b,
                                  const pfx_swk *const *rlk, pfx_ct *const *out, const std::vector<size_t> &g,
                                  void *st) {
    if (g.size() == 1) {
        const size_t i = g[0];
        pfx_status r = pfx_mul_relin(ctxs[i], a[i], b[i], rlk[i], out[i], st);
        if (!r) r = pfx_rescale(ctxs[i], out[i], out[i], st);
        return r;
    }
    const pfx_ct *ga[kMaxBatch], *gb[kMaxBatch];
    pfx_ct *go[kMaxBatch];
    for (size_t k = 0; k < g.size(); ++k) {
        ga[k] = a[g[k]];
        gb[k] = b[g[k]];
        go[k] = out[g[k]];
    }
    pfx_ctx *c = ctxs[g[0]];
    pfx_status r = pfx_mul_relin_batch(c, ga, gb, g.size(), rlk[g[0]], go, st);
    if (!r) r = pfx_rescale_batch(c, go, g.size(), go, st);
    return r;
}

static pfx_status batch_ops(pfx_ctx *const *ctxs, const pfx_ct *const *a, const pfx_ct *const *b,
                            const pfx_swk *const *rlk, pfx_ct *const *out, size_t n, bool lanes, bool group,
                            void *stream) {
    pfx_ctx *c0 = ctxs[0];
    const auto gs = batch_groups(ctxs, a, b, out, n, group);
    if (!lanes) {
        for (const auto &g : gs) {
            pfx_status r = batch_group_run(ctxs, a, b, rlk, out, g, stream);
            if (r) return r;
        }
        return PFX_OK;
    }
    // greedy assignment by estimated work (limbs x ring degree), largest first
    std::vector<size_t> order(gs.size());
    for (size_t i = 0; i < gs.size(); ++i) order[i] = i;
    auto work = [&](size_t k) {
        const size_t i = gs[k][0];
        return (double)std::min(a[i]->n_limbs, b[i]->n_limbs) * ctxs[i]->N * gs[k].size();
    };
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return work(x) > work(y); });
    std::vector<double> load(kLanes, 0.0);
    std::vector<int> lane_of(gs.size());
    for (size_t k : order) {
        int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_of[k] = best;
        load[best] += work(k);
    }
    HIPCHECK(hipEventRecord(c0->lane_events[kLanes], S(stream)));
    for (int l = 0; l < kLanes; ++l) HIPCHECK(hipStreamWaitEvent(c0->lanes[l], c0->lane_events[kLanes], 0));
    pfx_status res = PFX_OK;
    for (size_t k : order) {
        res = batch_group_run(ctxs, a, b, rlk, out, gs[k], c0->lanes[lane_of[k]]);
        if (res) break;
    }
    for (int l = 0; l < kLanes; ++l) {        // joined also after a failure
        HIPCHECK(hipEventRecord(c0->lane_events[l], c0->lanes[l]));
        HIPCHECK(hipStreamWaitEvent(S(stream), c0->lane_events[l], 0));
    }
    return res;
}

}  // extern "C"

namespace {

// Modes 5 and 6: entries whose output aliases an operand of any entry run first
// on the per-ciphertext path (the batch launches read every operand while they
// write every output); the rest in one persistent launch (5) or one launch per
// step (6), with the scratch of all of them in the stream's persistent region
// (grown on demand).
pfx_status batch_persistent(pfx_ctx *const *ctxs, const pfx_ct *const *a, const pfx_ct *const *b,
                            const pfx_swk *const *rlk, pfx_ct *const *out, size_t n, void *stream, bool step_major) {
    std::unordered_set<const double *> operands;
    for (size_t i = 0; i < n; ++i) {
        REQUIRE(persist_shape_ok(ctxs[i]), PFX_EINVAL,
                "persistent mode needs 2^12 <= N <= 2^16, digits of at most 4 primes and at most 4 special primes");
        REQUIRE(rlk[i]->galois == 0 && !rlk[i]->from_secret, PFX_ENOKEY, "key is not a relinearisation key");
        REQUIRE(a[i]->degree == 1 && b[i]->degree == 1, PFX_EINVAL, "batch entries must be degree-1 ciphertexts");
        REQUIRE(out[i]->cap_limbs >= std::min(a[i]->n_limbs, b[i]->n_limbs) && out[i]->cap_degree >= 1, PFX_EINVAL,
                "output capacity too small");
        operands.insert(a[i]->d);
        operands.insert(b[i]->d);
    }
    std::vector<size_t> alone, rest;
    std::unordered_set<const double *> outs;
    for (size_t i = 0; i < n; ++i) {
        REQUIRE(outs.insert(out[i]->d).second, PFX_EINVAL, "two entries write one output");
        (operands.count(out[i]->d) ? alone : rest).push_back(i);
    }
    for (size_t i : alone) {
        pfx_status r = pfx_mul_relin(ctxs[i], a[i], b[i], rlk[i], out[i], stream);
        if (!r) r = pfx_rescale(ctxs[i], out[i], out[i], stream);
        if (r) return r;
    }
    if (rest.empty()) return PFX_OK;
    size_t need = 0;
    for (size_t i : rest) need += persist_entry_doubles(ctxs[i], (int)std::min(a[i]->n_limbs, b[i]->n_limbs));
    need += (persist_tail_bytes(rest.size()) + sizeof(double) - 1) / sizeof(double);
    pfx_ctx *c0 = ctxs[rest[0]];
    Ws w;
    pfx_status r = get_ws(c0, S(stream), w);
    if (r) return r;
    double *region = nullptr;
    size_t cap = 0;
    {
        std::lock_guard<std::mutex> g(c0->mu);
        Workspace *ws = c0->ws[S(stream)];
        if (ws->pcap < need) {
            REQUIRE(!c0->capturing, PFX_EINVAL, "the persistent region must be reserved before graph capture");
            (void)hipStreamSynchronize(S(stream));
            bump_scratch_epoch();
            dfree(ws->pbuf);
            ws->pbuf = nullptr;
            ws->pcap = 0;
            PFX_DMALLOC(c0, &ws->pbuf, need * sizeof(double));
            ws->pcap = need;
        }
        region = ws->pbuf;
        cap = ws->pcap;
    }
    return launch_batch_persistent(ctxs, a, b, rlk, out, rest, region, cap, S(stream), step_major);
}

}  // namespace

extern "C" {

pfx_status pfx_batch_mul_relin_rescale(pfx_ctx *const *ctxs, const pfx_ct *const *a, const pfx_ct *const *b,
                                       const pfx_swk *const *rlk, pfx_ct *const *out, size_t n, int mode,
                                       void *stream) {
    REQUIRE(ctxs && a && b && rlk && out, PFX_EINVAL, "null argument");
    REQUIRE(mode >= 0 && mode <= 6, PFX_EINVAL, "mode must be 0 to 6");
    if (n == 0) return PFX_OK;
    for (size_t i = 0; i < n; ++i) {
        pfx_ctx *c = ctxs[i];
        REQUIRE(c && a[i] && b[i] && rlk[i] && out[i], PFX_EINVAL, "null batch entry");
        REQUIRE(a[i]->ctx == c && b[i]->ctx == c && rlk[i]->ctx == c && out[i]->ctx == c, PFX_EINVAL,
                "batch entry mixes contexts");
        REQUIRE(c->device == ctxs[0]->device, PFX_EINVAL, "batch spans devices");
        REQUIRE(std::min(a[i]->n_limbs, b[i]->n_limbs) >= 2, PFX_ELEVEL, "batch entry below 2 limbs");
    }
    const bool group = mode >= 3;
    if (mode == 0) return batch_ops(ctxs, a, b, rlk, out, n, false, false, stream);
    if (mode >= 5) return batch_persistent(ctxs, a, b, rlk, out, n, stream, mode == 6);
    pfx_ctx *c0 = ctxs[0];
    pfx_status r = ensure_lanes(c0);
    if (r) return r;
    size_t gmax = 1;
    if (group)
        for (const auto &g : batch_groups(ctxs, a, b, out, n, true)) gmax = std::max(gmax, g.size());
    for (size_t i = 0; i < n; ++i)        // scratch for every (context, lane) before any capture
        for (int l = 0; l < kLanes; ++l) {
            Ws w;
            r = get_ws(ctxs[i], c0->lanes[l], w);
            KsBatch kb;
            if (!r && gmax > 1) r = get_batch_ws(ctxs[i], c0->lanes[l], (int)gmax, kb);
            if (r) return r;
        }
    if (mode == 1 || mode == 3) return batch_ops(ctxs, a, b, rlk, out, n, true, group, stream);
    REQUIRE(stream != nullptr, PFX_EINVAL, "graph capture needs a non-default stream");
    // keyed on object identities and shapes, as pfx_run_circuit's graphs
    std::string key = "batch";
    std::vector<uint64_t> uids;
    auto put = [&](const void *p, size_t k) { key.append((const char *)p, k); };
    for (size_t i = 0; i < n; ++i) {
        for (uint64_t u : {ctxs[i]->uid, a[i]->uid, b[i]->uid, out[i]->uid, rlk[i]->uid}) {
            REQUIRE(u != 0, PFX_EINVAL, "graph mode needs library-created objects");
            put(&u, sizeof(uint64_t));
            uids.push_back(u);
        }
        put(&out[i]->cap_limbs, sizeof(uint32_t));
        put(&out[i]->cap_degree, sizeof(uint32_t));
        put(&a[i]->n_limbs, sizeof(uint32_t));
        put(&b[i]->n_limbs, sizeof(uint32_t));
        put(&a[i]->scale, sizeof(double));
        put(&b[i]->scale, sizeof(double));
    }
    put(&stream, sizeof(void *));
    put(&mode, sizeof(int));
    pfx_status lr = PFX_OK;
    auto replay = [&](GraphExec &x, const GraphCache<GraphExec>::Meta &meta) {
        for (size_t i = 0; i < n; ++i) {
            out[i]->n_limbs = meta[i].first & 0xffff;
            out[i]->degree = meta[i].first >> 16;
            out[i]->scale = meta[i].second;
        }
        if (hipGraphLaunch(x.exec, S(stream)) != hipSuccess || hipEventRecord(x.done, S(stream)) != hipSuccess)
            lr = fail(PFX_EDEVICE, "graph launch failed");
    };
    if (graphs().launch(key, scratch_epoch().load(), replay)) return lr;
    const uint64_t epoch = scratch_epoch().load();   // scratch of every (context, lane) reserved above
    for (size_t i = 0; i < n; ++i) ctxs[i]->capturing = true;
    HIPCHECK(hipStreamBeginCapture(S(stream), hipStreamCaptureModeThreadLocal));
    r = batch_ops(ctxs, a, b, rlk, out, n, true, group, stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(S(stream), &g);
    for (size_t i = 0; i < n; ++i) ctxs[i]->capturing = false;
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(PFX_EDEVICE, std::string("batch capture: ") + hipGetErrorString(e));
    GraphExec x;
    x.device = c0->device;
    e = hipGraphInstantiate(&x.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PFX_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (hipEventCreateWithFlags(&x.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(x.exec);
        return fail(PFX_EDEVICE, "graph event creation failed");
    }
    GraphCache<GraphExec>::Meta meta;
    for (size_t i = 0; i < n; ++i) meta.push_back({out[i]->n_limbs | (out[i]->degree << 16), out[i]->scale});
    graphs().insert_and_launch(key, epoch, x, uids, meta, replay);
    return lr;
}

pfx_status pfx_graph_cache_stats(size_t *entries, uint64_t *captures) {
    if (entries) *entries = graphs().size();
    if (captures) *captures = graphs().captures();
    return PFX_OK;
}

// ------------------------------------------------------------------ plumbing
pfx_status pfx_dev_alloc(pfx_ctx *c, size_t bytes, void **out) {
    REQUIRE(c && out, PFX_EINVAL, "null argument");
    HIPCHECK(hipSetDevice(c->device));
    PFX_DMALLOC(c, out, bytes);
    return PFX_OK;
}

pfx_status pfx_dev_free(pfx_ctx *c, void *p) {
    REQUIRE(c, PFX_EINVAL, "null context");
    dfree(p);
    return PFX_OK;
}

pfx_status pfx_memcpy_htod(pfx_ctx *c, void *dst, const void *src, size_t bytes, void *stream) {
    REQUIRE(c && dst && src, PFX_EINVAL, "null argument");
    HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, S(stream)));
    HIPCHECK(hipStreamSynchronize(S(stream)));
    return PFX_OK;
}

pfx_status pfx_memcpy_dtoh(pfx_ctx *c, void *dst, const void *src, size_t bytes, void *stream) {
    REQUIRE(c && dst && src, PFX_EINVAL, "null argument");
    HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, S(stream)));
    HIPCHECK(hipStreamSynchronize(S(stream)));
    return PFX_OK;
}

pfx_status pfx_stream_create(pfx_ctx *c, void **out) {
    REQUIRE(c && out, PFX_EINVAL, "null argument");
    HIPCHECK(hipSetDevice(c->device));
    hipStream_t st;
    HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    *out = st;
    return PFX_OK;
}

pfx_status pfx_event_create(pfx_ctx *c, void **out) {
    REQUIRE(c && out, PFX_EINVAL, "null argument");
    HIPCHECK(hipSetDevice(c->device));
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    *out = e;
    return PFX_OK;
}

pfx_status pfx_event_record(pfx_ctx *c, void *event, void *stream) {
    REQUIRE(c && event, PFX_EINVAL, "null argument");
    HIPCHECK(hipEventRecord((hipEvent_t)event, S(stream)));
    return PFX_OK;
}

pfx_status pfx_stream_wait_event(pfx_ctx *c, void *stream, void *event) {
    REQUIRE(c && event, PFX_EINVAL, "null argument");
    HIPCHECK(hipStreamWaitEvent(S(stream), (hipEvent_t)event, 0));
    return PFX_OK;
}

pfx_status pfx_event_elapsed(pfx_ctx *c, void *start, void *end, float *ms) {
    REQUIRE(c && start && end && ms, PFX_EINVAL, "null argument");
    HIPCHECK(hipEventSynchronize((hipEvent_t)end));
    HIPCHECK(hipEventElapsedTime(ms, (hipEvent_t)start, (hipEvent_t)end));
    return PFX_OK;
}

pfx_status pfx_event_destroy(pfx_ctx *c, void *event) {
    REQUIRE(c && event, PFX_EINVAL, "null argument");
    HIPCHECK(hipEventDestroy((hipEvent_t)event));
    return PFX_OK;
}

pfx_status pfx_stream_destroy(pfx_ctx *c, void *stream) {
    REQUIRE(c && stream, PFX_EINVAL, "null argument");
    HIPCHECK(hipStreamSynchronize(S(stream)));
    {
        std::lock_guard<std::mutex> g(c->mu);
        auto it = c->ws.find(S(stream));
        if (it != c->ws.end()) {
            bump_scratch_epoch();
            dfree(it->second->buf);
            dfree(it->second->bbuf);
            dfree(it->second->rbuf);
            dfree(it->second->pbuf);
            delete it->second;
            c->ws.erase(it);
        }
    }
    HIPCHECK(hipStreamDestroy(S(stream)));
    return PFX_OK;
}

// ------------------------------------------------------------------ profiling
pfx_status pfx_profile_enable(pfx_ctx *c, int on) {
    REQUIRE(c, PFX_EINVAL, "null context");
    c->prof_on = on != 0;
    return PFX_OK;
}

static void prof_drain(pfx_ctx *c) {
    for (auto &e : c->prof_pending) {
        (void)hipEventSynchronize(e.stop);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e.start, e.stop);
        ProfTotal &t = c->prof_done[e.name];
        t.launches += 1;
        t.ms += ms;
        t.bytes += e.bytes;
        c->prof_pool.push_back(e.start);
        c->prof_pool.push_back(e.stop);
    }
    c->prof_pending.clear();
}

pfx_status pfx_profile_get(pfx_ctx *c, const char *kernel, uint64_t *launches, double *total_ms, double *bytes) {
    REQUIRE(c && kernel, PFX_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(c->mu);
    prof_drain(c);
    auto it = c->prof_done.find(kernel);
    const bool have = it != c->prof_done.end();
    if (launches) *launches = have ? it->second.launches : 0;
    if (total_ms) *total_ms = have ? it->second.ms : 0.0;
    if (bytes) *bytes = have ? it->second.bytes : 0.0;
    return PFX_OK;
}

pfx_status pfx_profile_names(pfx_ctx *c, char *buf, size_t cap) {
    REQUIRE(c && buf && cap, PFX_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(c->mu);
    prof_drain(c);
    std::string s;
    for (auto &kv : c->prof_done) s += kv.first + "\n";
    std::strncpy(buf, s.c_str(), cap - 1);
    buf[cap - 1] = 0;
    return PFX_OK;
}

pfx_status pfx_profile_reset(pfx_ctx *c) {
    REQUIRE(c, PFX_EINVAL, "null context");
    std::lock_guard<std::mutex> g(c->mu);
    prof_drain(c);
    c->prof_done.clear();
    return PFX_OK;
}

}  // extern "C"

namespace pfx {

static hipEvent_t pool_event(pfx_ctx *c) {
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void prof_begin(const Launch &L, const char *, hipEvent_t *ev) {
    *ev = nullptr;
    if (!L.ctx->prof_on || L.ctx->capturing) return;
    *ev = pool_event(L.ctx);
    (void)hipEventRecord(*ev, L.st);
}

void prof_end(const Launch &L, const char *name, hipEvent_t ev, double bytes) {
    if (!L.ctx->prof_on || L.ctx->capturing || !ev) return;
    hipEvent_t stop = pool_event(L.ctx);
    (void)hipEventRecord(stop, L.st);
    std::lock_guard<std::mutex> g(L.ctx->mu);
    L.ctx->prof_pending.push_back(ProfEntry{ev, stop, name, bytes});
}

}  // namespace pfx
