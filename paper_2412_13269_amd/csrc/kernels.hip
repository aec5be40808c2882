// HIP kernels for gfx950 (MI355X) and their host launchers.
//
// Residues live in HBM as exact FP64 integers (every prime is below 2^50, see
// modarith.h), limb-major: limb i of a polynomial is N contiguous doubles.
// Ciphertexts stay in the NTT domain on the device.
#include <algorithm>
#include <cstdio>

#include <cstring>

#include "internal.h"
#include "modarith.h"
#include "ntt_core.h"

namespace pfx {

#define HIP_LAUNCH_CHECK()                                                     \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

static inline unsigned grid_for(size_t total, unsigned threads = 256) {
    size_t b = (total + threads - 1) / threads;
    return (unsigned)std::min<size_t>(b, 1u << 20);
}


// ============================================================== NTT
// Plain batched NTT over a LimbMap: both passes of ntt_core.h with ordinary
// global loads and stores.  Workgroups are remapped so that the tiles of one
// limb (one prime's twiddle table) stay on one XCD.
struct NttArgs {
    double *dst;
    const double *src;
    const PrimeDev *primes;
    int logn;
    int C;
    int tiles;
    int nblk;
    size_t bstride;   // batch copies of the map, this many doubles apart
    LimbMap map;
};

template <int S, bool ROW, bool INV, int TH>
__global__ __launch_bounds__(TH) void k_ntt_pass(const NttArgs a) {
    __shared__ double lds[ROW ? NttTile<TH>::lds : col_lds<S, TH>()];
    const int id = xcd_slot(a.nblk);
    if (id >= a.nblk) return;
    const int bl = id / a.tiles;
    const int tile = id - bl * a.tiles;
    const int bi = bl / a.map.n, limb = bl - bi * a.map.n;
    const PrimeDev &P = a.primes[a.map.pid[limb]];
    const size_t loff = ((size_t)a.map.off[limb] << a.logn) + bi * a.bstride;
    double *dst = a.dst + loff;
    const double *src = a.src + loff;
    auto ld = [&](int j, int) { return src[j]; };
    auto st = [&](int j, double v, int) { dst[j] = v; };
    if (ROW) row_pass<S, INV, TH>(P, a.logn, a.C, tile * a.C, lds, ld, st);
    else col_pass<S, INV, TH>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

template <bool ROW, bool INV, int TH>
static void dispatch_pass(int S, dim3 grid, hipStream_t st, const NttArgs &a) {
    switch (S) {
#define PFX_CASE(s) case s: k_ntt_pass<s, ROW, INV, TH><<<grid, TH, 0, st>>>(a); break;
        PFX_CASE(2) PFX_CASE(3) PFX_CASE(4) PFX_CASE(5) PFX_CASE(6) PFX_CASE(7) PFX_CASE(8)
#undef PFX_CASE
        default: set_error("unsupported NTT pass size");
    }
}

template <int TH>
static void dispatch_th(bool row, bool inverse, int S, dim3 grid, hipStream_t st, const NttArgs &a) {
    if (row) {
        if (inverse) dispatch_pass<true, true, TH>(S, grid, st, a);
        else dispatch_pass<true, false, TH>(S, grid, st, a);
    } else {
        if (inverse) dispatch_pass<false, true, TH>(S, grid, st, a);
        else dispatch_pass<false, false, TH>(S, grid, st, a);
    }
}

void launch_ntt_pass(const Launch &L, double *base, const double *src, const LimbMap &map, bool row, bool inverse,
                     int nb, size_t bstride) {
    if (map.n <= 0 || nb <= 0) return;
    pfx_ctx *ctx = L.ctx;
    const int logn = ctx->logn;
    NttArgs a;
    a.dst = base;
    a.primes = ctx->d_primes;
    a.logn = logn;
    a.map = map;
    const int th = pass_threads(logn, nb * map.n, row);
    PassShape ps = row ? row_shape(logn, th * kSlots) : col_shape(logn, th * kSlots);
    // very small batches: narrower row tiles (idle threads) so that the launch
    // still covers the CUs; column tiles stay >= 16 columns (128-byte rows:
    // 8-column tiles measured 17.0 us against 11.0 us for a 48-limb pass)
    const PassTuning &tu = pass_tuning(logn);
    const int minC = row ? 1 : tu.min_col;
    while (nb * map.n * ps.tiles < tu.widen_wg && ps.C / 2 >= minC) {
        ps.C /= 2;
        ps.tiles *= 2;
    }
    a.C = ps.C;
    a.tiles = ps.tiles;
    a.nblk = nb * map.n * ps.tiles;
    a.bstride = bstride;
    a.src = src ? src : base;
    dim3 grid(xcd_grid(a.nblk));
    hipEvent_t ev;
    char nm[32];
    std::snprintf(nm, sizeof nm, "%s/%d", inverse ? (row ? "intt_row" : "intt_col") : (row ? "ntt_row" : "ntt_col"),
                  nb * map.n);
    prof_begin(L, nm, &ev);
    PFX_SWITCH_TH(th, (dispatch_th<TH>(row, inverse, ps.S, grid, L.st, a)));
    HIP_LAUNCH_CHECK();
    prof_end(L, nm, ev, 16.0 * (double)ctx->N * map.n * nb);
}

// Transform of canonical uint64 words in place (the standalone entry point):
// the first pass reads words and converts them as it loads, the last pass
// stores canonical words; the intermediate is FP64 residues in the same
// memory (8 bytes per element either way; every block reads its whole tile
// before it writes it).  Limb l of the launch uses prime first + l % nl.
template <int S, bool ROW, bool INV, int TH, bool IN_WORDS, bool OUT_WORDS>
__global__ __launch_bounds__(TH) void k_ntt_words(uint64_t *words, const PrimeDev *primes, int logn, int C,
                                                  int tiles, int nblk, int first, int nl) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(nblk);
    if (id >= nblk) return;
    const int limb = id / tiles;
    const int tile = id - limb * tiles;
    const PrimeDev &P = primes[first + limb % nl];
    uint64_t *wl = words + ((size_t)limb << logn);
    double *dl = reinterpret_cast<double *>(wl);
    auto ld = [&](int j, int) { return IN_WORDS ? (double)wl[(unsigned)j] : dl[(unsigned)j]; };
    auto st = [&](int j, double v, int) {
        if (OUT_WORDS) wl[(unsigned)j] = (uint64_t)v;
        else dl[(unsigned)j] = v;
    };
    if (ROW) row_pass<S, INV, TH>(P, logn, C, tile * C, lds, ld, st);
    else col_pass<S, INV, TH>(P, logn, C, tile * C, lds, ld, st);
}

template <bool ROW, bool INV, bool IW, bool OW>
static void words_pass(uint64_t *words, pfx_ctx *ctx, size_t limbs, int first, int nl, hipStream_t st,
                       const char *name, const Launch &L) {
    const int logn = ctx->logn;
    const int th = pass_threads(logn, (int)limbs, ROW);
    const PassShape ps = ROW ? row_shape(logn, th * kSlots) : col_shape(logn, th * kSlots);
    const int nblk = (int)limbs * ps.tiles;
    hipEvent_t ev;
    prof_begin(L, name, &ev);
    PFX_SWITCH_TH(th, PFX_SWITCH_S(ps.S, (k_ntt_words<SS, ROW, INV, TH, IW, OW><<<xcd_grid(nblk), TH, 0, st>>>(
                                           words, ctx->d_primes, logn, ps.C, ps.tiles, nblk, first, nl))));
    HIP_LAUNCH_CHECK();
    prof_end(L, name, ev, 16.0 * (double)ctx->N * (double)limbs);
}

void launch_ntt_words(const Launch &L, uint64_t *words, size_t limbs, int first, int nl, bool inverse) {
    if (limbs == 0) return;
    if (!inverse) {
        words_pass<false, false, true, false>(words, L.ctx, limbs, first, nl, L.st, "ntt_words_col", L);
        words_pass<true, false, false, true>(words, L.ctx, limbs, first, nl, L.st, "ntt_words_row", L);
    } else {
        words_pass<true, true, true, false>(words, L.ctx, limbs, first, nl, L.st, "intt_words_row", L);
        words_pass<false, true, false, true>(words, L.ctx, limbs, first, nl, L.st, "intt_words_col", L);
    }
}

void launch_ntt(const Launch &L, double *base, const double *src, const LimbMap &map, bool inverse) {
    if (!inverse) {
        launch_ntt_pass(L, base, src, map, false, false);
        launch_ntt_pass(L, base, nullptr, map, true, false);
    } else {
        launch_ntt_pass(L, base, src, map, true, true);
        launch_ntt_pass(L, base, nullptr, map, false, true);
    }
}

// ============================================================== conversions
__global__ void k_u64_to_f64(double *out, const uint64_t *in, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}
__global__ void k_f64_to_u64(uint64_t *out, const double *in, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (uint64_t)in[i];
}
// out[i][c] = in[c] mod prime i  (|in| < 2^50)
__global__ void k_int_to_rns(double *out, const int64_t *in, int n_limbs, int logn, const PrimeDev *pr) {
    const size_t total = (size_t)n_limbs << logn;
    const size_t mask = ((size_t)1 << logn) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int l = (int)(i >> logn);
        const double q = pr[l].q;
        const int64_t v = in[i & mask];
        const uint64_t m = (uint64_t)q;
        const uint64_t r = v >= 0 ? (uint64_t)v % m : (m - ((uint64_t)(-v) % m)) % m;
        out[i] = (double)r;
    }
}
__global__ void k_s8_to_rns(double *out, const int8_t *in, int n_limbs, int logn, const PrimeDev *pr) {
    const size_t total = (size_t)n_limbs << logn;
    const size_t mask = ((size_t)1 << logn) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int l = (int)(i >> logn);
        const int v = in[i & mask];
        out[i] = v >= 0 ? (double)v : pr[l].q + (double)v;
    }
}

void launch_u64_to_f64(const Launch &L, double *out, const uint64_t *in, size_t n) {
    k_u64_to_f64<<<grid_for(n), 256, 0, L.st>>>(out, in, n);
    HIP_LAUNCH_CHECK();
}
void launch_f64_to_u64(const Launch &L, uint64_t *out, const double *in, size_t n) {
    k_f64_to_u64<<<grid_for(n), 256, 0, L.st>>>(out, in, n);
    HIP_LAUNCH_CHECK();
}
void launch_int_to_rns(const Launch &L, double *out, const int64_t *in, int n_limbs, int, int, int) {
    size_t total = (size_t)n_limbs << L.ctx->logn;
    k_int_to_rns<<<grid_for(total), 256, 0, L.st>>>(out, in, n_limbs, L.ctx->logn, L.ctx->d_primes);
    HIP_LAUNCH_CHECK();
}
void launch_s8_to_rns(const Launch &L, double *out, const int8_t *in, int n_limbs) {
    size_t total = (size_t)n_limbs << L.ctx->logn;
    k_s8_to_rns<<<grid_for(total), 256, 0, L.st>>>(out, in, n_limbs, L.ctx->logn, L.ctx->d_primes);
    HIP_LAUNCH_CHECK();
}

struct LimbConsts {
    double w[PFX_MAX_PRIMES];
    double wq[PFX_MAX_PRIMES];
};

// ============================================================== collected launches
// While a collector is active on the calling thread for a stream, the
// elementwise, constant and tensor launchers above record their launches
// instead of issuing them; ew_collect_end issues every record of one kernel
// variant (same operation, same per-limb constants) as one launch over up to
// kMaxBatch records (grid z).  The records of one collection must be
// independent of each other (the op-list executor collects runs of
// independent elementwise ops).
struct EwRec {
    double *out;
    const double *a, *b;
    size_t so, sa, sb;
    int rows, nl;
    uint32_t k;            // EW_MONO: the exponent
};
struct TensorRec {
    double *d0, *d1, *d2;
    const double *a0, *a1, *b0, *b1;
    int nl;
};
namespace {

struct EwGroup {
    int op;              // EwOp, or EW_MULC / EW_MULC_ACC / EW_ADDC
    LimbConsts k;
    int nk;              // constants in use (0: none)
    std::vector<EwRec> recs;
};

struct Collector {
    pfx_ctx *ctx = nullptr;
    hipStream_t st = nullptr;
    std::vector<EwGroup> ew;
    std::vector<TensorRec> tensor[2];
};

thread_local Collector *t_collect = nullptr;

Collector *collecting(const Launch &L) {
    Collector *c = t_collect;
    return (c && c->ctx == L.ctx && c->st == L.st) ? c : nullptr;
}

void collect_ew(Collector *c, int op, const EwRec &r, const LimbConsts *k, int nk) {
    for (EwGroup &g : c->ew) {
        if (g.op != op || g.nk != nk) continue;
        if (nk && (std::memcmp(g.k.w, k->w, nk * sizeof(double)) || std::memcmp(g.k.wq, k->wq, nk * sizeof(double))))
            continue;
        g.recs.push_back(r);
        return;
    }
    EwGroup g;
    g.op = op;
    g.nk = nk;
    if (nk) g.k = *k;
    g.recs.push_back(r);
    c->ew.push_back(g);
}

}  // namespace

// Records a launch when a collector is active for (ctx, stream); false if the
// caller should launch it itself.
static bool record_ew(const Launch &L, int op, double *out, const double *a, const double *b, size_t so, size_t sa,
                      size_t sb, int rows, int nl, const LimbConsts *k, int nk, uint32_t e = 0) {
    Collector *c = collecting(L);
    if (!c) return false;
    collect_ew(c, op, EwRec{out, a, b, so, sa, sb, rows, nl, e}, k, nk);
    return true;
}

static bool record_tensor(const Launch &L, const TensorRec &r, bool acc) {
    Collector *c = collecting(L);
    if (!c) return false;
    c->tensor[acc ? 1 : 0].push_back(r);
    return true;
}

// ============================================================== elementwise
// Grid: x over the N slots of a limb (a few per thread), y over polynomial x
// limb, so a block's prime and polynomial are uniform and no thread divides.
static inline dim3 ew_grid(int logn, int rows) {
    const int per_block = 256 * 4;
    return dim3((unsigned)std::max(1, (1 << logn) / per_block), (unsigned)rows);
}

template <int OP>
__global__ __launch_bounds__(256) void k_ew(double *out, const double *a, const double *b, size_t so, size_t sa,
                                            size_t sb, int nl, int logn, const PrimeDev *pr) {
    const int row = blockIdx.y;                 // polynomial k, limb i
    const int k = row / nl, i = row - k * nl;
    const size_t off = (size_t)i << logn;
    const double q = pr[i].q, qi = pr[i].qinv;
    const double *ap = a + k * sa + off;
    const double *bp = b + k * sb + off;
    double *op = out + k * so + off;
    const size_t N = (size_t)1 << logn;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const double x = ap[c];
        double r;
        if (OP == EW_ADD) r = madd(x, bp[c], q);
        else if (OP == EW_SUB) r = msub(x, bp[c], q);
        else if (OP == EW_MUL) r = mmul(x, bp[c], q, qi);
        else if (OP == EW_MAC) r = madd(op[c], mmul(x, bp[c], q, qi), q);
        else if (OP == EW_NEG) r = mneg(x, q);
        else r = x;
        op[c] = r;
    }
}

void launch_ew(const Launch &L, EwOp op, double *out, const double *a, const double *b, size_t so, size_t sa,
               size_t sb, int npoly, int nl) {
    const int logn = L.ctx->logn;
    const size_t total = ((size_t)npoly * nl) << logn;
    if (!total) return;
    if (record_ew(L, op, out, a, b, so, sa, sb, npoly * nl, nl, nullptr, 0)) return;
    const dim3 g = ew_grid(logn, npoly * nl);
    const PrimeDev *pr = L.ctx->d_primes;
    hipEvent_t ev;
    prof_begin(L, "elementwise", &ev);
    switch (op) {
        case EW_ADD: k_ew<EW_ADD><<<g, 256, 0, L.st>>>(out, a, b, so, sa, sb, nl, logn, pr); break;
        case EW_SUB: k_ew<EW_SUB><<<g, 256, 0, L.st>>>(out, a, b, so, sa, sb, nl, logn, pr); break;
        case EW_MUL: k_ew<EW_MUL><<<g, 256, 0, L.st>>>(out, a, b, so, sa, sb, nl, logn, pr); break;
        case EW_MAC: k_ew<EW_MAC><<<g, 256, 0, L.st>>>(out, a, b, so, sa, sb, nl, logn, pr); break;
        case EW_NEG: k_ew<EW_NEG><<<g, 256, 0, L.st>>>(out, a, b, so, sa, sb, nl, logn, pr); break;
        default: k_ew<EW_COPY><<<g, 256, 0, L.st>>>(out, a, b, so, sa, sb, nl, logn, pr); break;
    }
    HIP_LAUNCH_CHECK();
    const double words = (op == EW_NEG || op == EW_COPY) ? 2 : op == EW_MAC ? 4 : 3;
    prof_end(L, "elementwise", ev, 8.0 * (double)total * words);
}

template <bool ACC>
__global__ __launch_bounds__(256) void k_mulconst(double *out, const double *a, size_t so, size_t sa, int nl,
                                                   int logn, const PrimeDev *pr, const LimbConsts k) {
    const int row = blockIdx.y;
    const int kp = row / nl, i = row - kp * nl;
    const size_t off = (size_t)i << logn;
    const double *ap = a + kp * sa + off;
    double *op = out + kp * so + off;
    const double w = k.w[i], wq = k.wq[i], q = pr[i].q;
    const size_t N = (size_t)1 << logn;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const double r = mmulc(ap[c], w, wq, q);
        op[c] = ACC ? madd(op[c], r, q) : r;
    }
}

void launch_mulconst(const Launch &L, double *out, const double *a, size_t so, size_t sa, int npoly, int nl,
                     const uint64_t *cst, bool acc) {
    LimbConsts k;
    for (int i = 0; i < nl; ++i) {
        k.w[i] = (double)cst[i];
        k.wq[i] = (double)cst[i] / (double)L.ctx->primes[i];
    }
    if (record_ew(L, acc ? EW_MULC_ACC : EW_MULC, out, a, nullptr, so, sa, 0, npoly * nl, nl, &k, nl)) return;
    const size_t total = ((size_t)npoly * nl) << L.ctx->logn;
    hipEvent_t ev;
    prof_begin(L, "mulconst", &ev);
    const dim3 g = ew_grid(L.ctx->logn, npoly * nl);
    if (acc) k_mulconst<true><<<g, 256, 0, L.st>>>(out, a, so, sa, nl, L.ctx->logn, L.ctx->d_primes, k);
    else k_mulconst<false><<<g, 256, 0, L.st>>>(out, a, so, sa, nl, L.ctx->logn, L.ctx->d_primes, k);
    HIP_LAUNCH_CHECK();
    prof_end(L, "mulconst", ev, (acc ? 24.0 : 16.0) * (double)total);
}

// out[i][c] = a[i][c] + cst_i: a constant polynomial (coefficient 0 only) is the
// same value at every NTT slot.
__global__ void k_addconst(double *out, const double *a, int nl, int logn, const PrimeDev *pr, const LimbConsts k) {
    const size_t total = (size_t)nl << logn;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx >> logn);
        out[idx] = madd(a[idx], k.w[i], pr[i].q);
    }
}

void launch_addconst(const Launch &L, double *out, const double *a, int nl, const uint64_t *cst) {
    LimbConsts k;
    for (int i = 0; i < nl; ++i) {
        k.w[i] = (double)cst[i];
        k.wq[i] = 0.0;
    }
    if (record_ew(L, EW_ADDC, out, a, nullptr, 0, 0, 0, nl, nl, &k, nl)) return;
    const size_t total = (size_t)nl << L.ctx->logn;
    hipEvent_t ev;
    prof_begin(L, "addconst", &ev);
    k_addconst<<<grid_for(total), 256, 0, L.st>>>(out, a, nl, L.ctx->logn, L.ctx->d_primes, k);
    HIP_LAUNCH_CHECK();
    prof_end(L, "addconst", ev, 16.0 * (double)total);
}

// Monomial product (the lookup of a plaintext point, Sec. 3.4; the X^t of ring
// repacking, Alg. 1): a * X^k.
__global__ __launch_bounds__(256) void k_monomial(double *out, const double *a, size_t so, size_t sa, int nl,
                                                  int logn, const PrimeDev *pr, uint32_t k) {
    const int row = blockIdx.y;
    const int kp = row / nl, i = row - kp * nl;
    const size_t off = (size_t)i << logn;
    const double *ap = a + kp * sa + off;
    double *op = out + kp * so + off;
    const PrimeDev &P = pr[i];
    const size_t N = (size_t)1 << logn;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x)
        op[c] = monomial_mul(ap[c], (uint32_t)c, k, logn, P);
}

void launch_monomial(const Launch &L, double *out, const double *a, size_t so, size_t sa, int npoly, int nl,
                     uint32_t k) {
    if (record_ew(L, EW_MONO, out, a, nullptr, so, sa, 0, npoly * nl, nl, nullptr, 0, k)) return;
    const size_t total = ((size_t)npoly * nl) << L.ctx->logn;
    hipEvent_t ev;
    prof_begin(L, "monomial", &ev);
    k_monomial<<<ew_grid(L.ctx->logn, npoly * nl), 256, 0, L.st>>>(out, a, so, sa, nl, L.ctx->logn, L.ctx->d_primes,
                                                                     k);
    HIP_LAUNCH_CHECK();
    prof_end(L, "monomial", ev, 16.0 * (double)total);
}

// Score aggregation of the lookup tables (Sec. 3.4, Sec. 4.2): record r gets
// sum_l T_l X^(k_(r,l)), slot x of a limb being sum_l psi^(k_(r,l) e_x) T_l[x]
// (monomial_mul), times N^-1 when `ninv` is set (the pre-multiplication of
// ring repacking; (N^-1 mod q) times the reduced sum is the same residue as
// the sum of N^-1 T_l X^k).  Grid: x over the N slots, y over polynomial x
// limb rows, z over records r0 + z; records r >= n are written as zero.
__global__ __launch_bounds__(256) void k_mono_sum(double *out, size_t cs, size_t ps, const double *tables, size_t st,
                                                  size_t tps, int m, const int64_t *exps, int n, int r0, int lv,
                                                  int logn, const PrimeDev *pr, bool ninv) {
    const int row = blockIdx.y;
    const int u = row / lv, i = row - u * lv;
    const int r = r0 + (int)blockIdx.z;
    const size_t N = (size_t)1 << logn;
    const size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (x >= N) return;
    double *o = out + (size_t)r * cs + (size_t)u * ps + ((size_t)i << logn);
    if (r >= n) {
        o[x] = 0.0;
        return;
    }
    const PrimeDev &P = pr[i];
    const double q = P.q, qi = P.qinv;
    const int64_t *ke = exps + (size_t)r * m;
    const double *tb = tables + (size_t)u * tps + ((size_t)i << logn) + x;
    const uint32_t mask = (2u << logn) - 1u;
    // terms in [0, q), q < 2^50: seven of them and a reduced partial sum stay
    // below 8q < 2^53
    double s = 0.0;
    int pend = 0;
    for (int l = 0; l < m; ++l) {
        const uint32_t k = (uint32_t)((uint64_t)ke[l] & mask);   // k mod 2N, also for k < 0
        s += monomial_mul(tb[(size_t)l * st], (uint32_t)x, k, logn, P);
        if (++pend == 7) {
            s = mred(s, q, qi);
            pend = 0;
        }
    }
    s = mred(s, q, qi);
    o[x] = ninv ? mmulc(s, P.ninv, P.ninv_q, q) : s;
}

void launch_mono_sum(const Launch &L, double *out, size_t cs, size_t ps, const double *tables, size_t st,
                     size_t tps, int m, const int64_t *exps, int n, int n_slots, int lv, bool ninv) {
    if (n_slots <= 0) return;
    const int logn = L.ctx->logn;
    const size_t N = L.ctx->N;
    constexpr int kRecs = 32768;   // records per launch (grid z)
    hipEvent_t ev;
    prof_begin(L, "mono_sum", &ev);
    for (int r0 = 0; r0 < n_slots; r0 += kRecs) {
        const int nr = std::min(kRecs, n_slots - r0);
        const dim3 grid((unsigned)std::max<size_t>(1, (N + 255) / 256), (unsigned)(2 * lv), (unsigned)nr);
        k_mono_sum<<<grid, 256, 0, L.st>>>(out, cs, ps, tables, st, tps, m, exps, n, r0, lv, logn,
                                           L.ctx->d_primes, ninv);
        HIP_LAUNCH_CHECK();
    }
    // outputs written once, exponents read once (the tables stay in cache)
    prof_end(L, "mono_sum", ev, 16.0 * (double)N * lv * n_slots + 8.0 * (double)m * std::max(0, std::min(n, n_slots)));
}

// The same sums for 2^9 <= N <= 2^12 with the tables held in registers and
// the twiddles in LDS: a workgroup of 512 threads owns 512 consecutive slots x
// of one limb and a run of records; each thread loads T_l[x] of both
// polynomials for its slot once (at most MT tables), and per record and table
// reads psi^E, E = k e_x mod 2N, from an LDS table of psi^0 .. psi^(2N-1) in
// natural order with a pad entry every 128 (64.5 KiB: two groups, four waves
// per SIMD), so the tables are
// read once per workgroup instead of once per record.  Products are left
// signed in (-q, q) (the steps of mmul without the final correction) and the
// sums reduced every seven terms; the canonical result is the residue of the
// same integer as in k_mono_sum (the same words).  Grid: x over the slot
// blocks, y over the limbs, z over runs of `rpw` records.
template <int MT>
__global__ __launch_bounds__(512) void k_mono_sum_lds(double *out, size_t cs, size_t ps, const double *tables,
                                                      size_t st, size_t tps, int m, const int64_t *exps, int n,
                                                      int n_slots, int rpw, int logn, const PrimeDev *pr, bool ninv) {
    // psi^E at tws[E + E / 128]: one pad entry per 128, so that the 64 lanes'
    // exponents k e_x (e_x = 2 bitrev(x) + 1 for 64 consecutive slots x, which
    // are k + 128 k r: all one bank without the pad) spread over the banks
    __shared__ double tws[(2 << 12) + ((2 << 12) >> 7)];
    auto pidx = [](uint32_t e) { return e + (e >> 7); };
    const int i = blockIdx.y;
    const PrimeDev &P = pr[i];
    const double q = P.q, qi = P.qinv;
    const uint32_t N = 1u << logn;
    for (uint32_t j = threadIdx.x; j < N; j += blockDim.x) {
        const double w = P.tw[__brev(j) >> (32 - logn)].x;   // psi^j, and psi^(N + j) = -psi^j
        tws[pidx(j)] = w;
        tws[pidx(N + j)] = q - w;
    }
    __syncthreads();
    const uint32_t x = blockIdx.x * 512u + threadIdx.x;
    const uint32_t ex = 2u * (__brev(x) >> (32 - logn)) + 1u;
    const uint32_t mask = 2u * N - 1u;
    double t0[MT], t1[MT];
#pragma unroll
    for (int l = 0; l < MT; ++l) {
        const double *tl = tables + (size_t)l * st + ((size_t)i << logn) + x;
        t0[l] = l < m ? tl[0] : 0.0;
        t1[l] = l < m ? tl[tps] : 0.0;
    }
    // a * w - c q with c = rint(fl(a w) fl(1/q)): an integer in (-q, q) (mmul before its correction)
    auto mul_signed = [&](double a, double w) {
        const double h = a * w;
        const double lo = __builtin_fma(a, w, -h);
        const double c = __builtin_rint(h * qi);
        return __builtin_fma(-c, q, h) + lo;
    };
    const int r0 = (int)blockIdx.z * rpw, r1 = min(r0 + rpw, n_slots);
    for (int r = r0; r < r1; ++r) {
        double *o = out + (size_t)r * cs + ((size_t)i << logn) + x;
        if (r >= n) {
            o[0] = 0.0;
            o[ps] = 0.0;
            continue;
        }
        const int64_t *ke = exps + (size_t)r * m;
        // |term| < q, partial sums reduced to [-q/2, q/2] every seven terms: below 7.5q < 2^53
        double s0 = 0.0, s1 = 0.0;
        int pend = 0;
#pragma unroll
        for (int l = 0; l < MT; ++l) {
            if (l < m) {
                const uint32_t E = ((uint32_t)(uint64_t)ke[l] * ex) & mask;
                const double w = tws[pidx(E)];
                s0 += mul_signed(t0[l], w);
                s1 += mul_signed(t1[l], w);
                if (++pend == 7) {
                    s0 = mred_signed(s0, q, qi);
                    s1 = mred_signed(s1, q, qi);
                    pend = 0;
                }
            }
        }
        s0 = mcanon(mred_signed(s0, q, qi), q);
        s1 = mcanon(mred_signed(s1, q, qi), q);
        o[0] = ninv ? mmulc(s0, P.ninv, P.ninv_q, q) : s0;
        o[ps] = ninv ? mmulc(s1, P.ninv, P.ninv_q, q) : s1;
    }
}

bool mono_sum_lds_ok(const pfx_ctx *c, int m) { return c->logn >= 9 && c->logn <= 12 && m <= 16; }

void launch_mono_sum_lds(const Launch &L, double *out, size_t cs, size_t ps, const double *tables, size_t st,
                         size_t tps, int m, const int64_t *exps, int n, int n_slots, int lv, bool ninv) {
    if (n_slots <= 0) return;
    const int logn = L.ctx->logn;
    const size_t N = L.ctx->N;
    const int rpw = std::max(64, (n_slots + 32767) / 32768);      // records per workgroup
    const dim3 grid((unsigned)(N / 512), (unsigned)lv, (unsigned)((n_slots + rpw - 1) / rpw));
    hipEvent_t ev;
    prof_begin(L, "mono_sum_lds", &ev);
    k_mono_sum_lds<16><<<grid, 512, 0, L.st>>>(out, cs, ps, tables, st, tps, m, exps, n, n_slots, rpw, logn,
                                               L.ctx->d_primes, ninv);
    HIP_LAUNCH_CHECK();
    // outputs written once, exponents read once per slot block (from cache), tables once per workgroup
    prof_end(L, "mono_sum_lds", ev, 16.0 * (double)N * lv * n_slots + 8.0 * (double)m * std::max(0, std::min(n, n_slots)));
}

// Ring merging (Sec. 3.3, Sec. 4.3): the coefficient-domain polynomials of up
// to r = N / n small ciphertexts (stage: input i, polynomial u at (2i + u) n)
// placed in one of the large ring, coefficient j of input i at X^(j r + i):
// the embedding X -> X^r of each input times X^i, summed (disjoint supports).
// Coefficients of missing inputs (i >= n_in) are zero.  Grid: x over the N
// coefficients, y over the two polynomials.
__global__ void k_merge_gather(double *out, const double *stage, int n_in, int log_r, int logn_small) {
    const int u = blockIdx.y;
    const size_t N = (size_t)1 << (log_r + logn_small);
    const size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (x >= N) return;
    const int i = (int)(x & (((size_t)1 << log_r) - 1));
    const size_t j = x >> log_r;
    out[(size_t)u * N + x] = i < n_in ? stage[(((size_t)(2 * i + u)) << logn_small) + j] : 0.0;
}

void launch_merge_gather(const Launch &L, double *out, const double *stage, int n_in, int log_r, int logn_small) {
    const size_t N = (size_t)1 << (log_r + logn_small);
    hipEvent_t ev;
    prof_begin(L, "merge_gather", &ev);
    k_merge_gather<<<dim3((unsigned)((N + 255) / 256), 2), 256, 0, L.st>>>(out, stage, n_in, log_r, logn_small);
    HIP_LAUNCH_CHECK();
    prof_end(L, "merge_gather", ev, 16.0 * (double)N * 2);
}

// ModRaise (App. A.3): the coefficient-domain residues c of q_0 (one limb
// per polynomial, `in`, polynomials si apart) lifted to [-(q_0-1)/2, (q_0-1)/2]
// and reduced modulo each of the first nl primes (`out`, polynomials so
// apart).  |lift| < 2^49 < 2^50, so mred reduces its magnitude exactly.
// Grid: x over the N coefficients, y over polynomial x limb rows.
__global__ void k_mod_raise(double *out, size_t so, const double *in, size_t si, int nl, int logn,
                            const PrimeDev *pr) {
    const int row = blockIdx.y;
    const int u = row / nl, i = row - u * nl;
    const size_t N = (size_t)1 << logn;
    const size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (x >= N) return;
    const double q0 = pr[0].q;
    const double c = in[(size_t)u * si + x];
    const bool neg = c > 0.5 * (q0 - 1.0);                  // lift c - q_0
    const double mag = neg ? q0 - c : c;
    const double q = pr[i].q;
    const double r = mred(mag, q, pr[i].qinv);
    out[(size_t)u * so + ((size_t)i << logn) + x] = neg && r != 0.0 ? q - r : r;
}

void launch_mod_raise(const Launch &L, double *out, size_t so, const double *in, size_t si, int npoly, int nl) {
    const int logn = L.ctx->logn;
    const size_t N = L.ctx->N;
    hipEvent_t ev;
    prof_begin(L, "mod_raise", &ev);
    k_mod_raise<<<dim3((unsigned)((N + 255) / 256), (unsigned)(npoly * nl)), 256, 0, L.st>>>(out, so, in, si, nl, logn,
                                                                                          L.ctx->d_primes);
    HIP_LAUNCH_CHECK();
    prof_end(L, "mod_raise", ev, 8.0 * (double)N * npoly * (1 + nl));
}

// Tensor product in the NTT domain (Sec. 2.4.2): d0 = a0 b0, d1 = a0 b1 + a1 b0,
// d2 = a1 b1; ACC adds it to what d0, d1, d2 hold.
template <bool ACC>
__global__ __launch_bounds__(256) void k_tensor(double *d0, double *d1, double *d2, const double *a0, const double *a1,
                                                const double *b0, const double *b1, int logn, const PrimeDev *pr) {
    const int i = blockIdx.y;
    const double q = pr[i].q, qi = pr[i].qinv;
    const size_t N = (size_t)1 << logn;
    const size_t off = (size_t)i << logn;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const size_t idx = off + c;
        const double x0 = a0[idx], x1 = a1[idx], y0 = b0[idx], y1 = b1[idx];
        double r0 = mmul(x0, y0, q, qi);
        double r1 = madd(mmul(x0, y1, q, qi), mmul(x1, y0, q, qi), q);
        double r2 = mmul(x1, y1, q, qi);
        if (ACC) {
            r0 = madd(d0[idx], r0, q);
            r1 = madd(d1[idx], r1, q);
            r2 = madd(d2[idx], r2, q);
        }
        d0[idx] = r0;
        d1[idx] = r1;
        d2[idx] = r2;
    }
}

void launch_tensor(const Launch &L, double *d0, double *d1, double *d2, const double *a0, const double *a1,
                   const double *b0, const double *b1, int nl, bool acc) {
    if (record_tensor(L, TensorRec{d0, d1, d2, a0, a1, b0, b1, nl}, acc)) return;
    const size_t total = (size_t)nl << L.ctx->logn;
    const dim3 g = ew_grid(L.ctx->logn, nl);
    hipEvent_t ev;
    prof_begin(L, acc ? "tensor_acc" : "tensor", &ev);
    if (acc) k_tensor<true><<<g, 256, 0, L.st>>>(d0, d1, d2, a0, a1, b0, b1, L.ctx->logn, L.ctx->d_primes);
    else k_tensor<false><<<g, 256, 0, L.st>>>(d0, d1, d2, a0, a1, b0, b1, L.ctx->logn, L.ctx->d_primes);
    HIP_LAUNCH_CHECK();
    prof_end(L, acc ? "tensor_acc" : "tensor", ev, (acc ? 80.0 : 56.0) * (double)total);
}

// ---- multi-record launches of a collection
struct EwMultiArgs {
    EwRec e[kMaxBatch];
    int logn;
    const PrimeDev *pr;
};
struct TensorMultiArgs {
    TensorRec e[kMaxBatch];
    int logn;
    const PrimeDev *pr;
};

template <int OP>
__global__ __launch_bounds__(256) void k_ew_multi(const EwMultiArgs m, const LimbConsts k) {
    const EwRec &r = m.e[blockIdx.z];
    const int row = blockIdx.y;
    if (row >= r.rows) return;
    const int kp = row / r.nl, i = row - kp * r.nl;
    const int logn = m.logn;
    const size_t off = (size_t)i << logn;
    const double q = m.pr[i].q, qi = m.pr[i].qinv;
    const double *ap = r.a + kp * r.sa + off;
    const double *bp = r.b + kp * r.sb + off;
    double *op = r.out + kp * r.so + off;
    const size_t N = (size_t)1 << logn;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const double x = ap[c];
        double v;
        if (OP == EW_ADD) v = madd(x, bp[c], q);
        else if (OP == EW_SUB) v = msub(x, bp[c], q);
        else if (OP == EW_MUL) v = mmul(x, bp[c], q, qi);
        else if (OP == EW_MAC) v = madd(op[c], mmul(x, bp[c], q, qi), q);
        else if (OP == EW_NEG) v = mneg(x, q);
        else if (OP == EW_MULC) v = mmulc(x, k.w[i], k.wq[i], q);
        else if (OP == EW_MULC_ACC) v = madd(op[c], mmulc(x, k.w[i], k.wq[i], q), q);
        else if (OP == EW_ADDC) v = madd(x, k.w[i], q);
        else if (OP == EW_MONO) v = monomial_mul(x, (uint32_t)c, r.k, logn, m.pr[i]);
        else v = x;
        op[c] = v;
    }
}

template <bool ACC>
__global__ __launch_bounds__(256) void k_tensor_multi(const TensorMultiArgs m) {
    const TensorRec &r = m.e[blockIdx.z];
    const int i = blockIdx.y;
    if (i >= r.nl) return;
    const double q = m.pr[i].q, qi = m.pr[i].qinv;
    const size_t N = (size_t)1 << m.logn;
    const size_t off = (size_t)i << m.logn;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const size_t idx = off + c;
        const double x0 = r.a0[idx], x1 = r.a1[idx], y0 = r.b0[idx], y1 = r.b1[idx];
        double r0 = mmul(x0, y0, q, qi);
        double r1 = madd(mmul(x0, y1, q, qi), mmul(x1, y0, q, qi), q);
        double r2 = mmul(x1, y1, q, qi);
        if (ACC) {
            r0 = madd(r.d0[idx], r0, q);
            r1 = madd(r.d1[idx], r1, q);
            r2 = madd(r.d2[idx], r2, q);
        }
        r.d0[idx] = r0;
        r.d1[idx] = r1;
        r.d2[idx] = r2;
    }
}


void ew_collect_begin(const Launch &L) {
    Collector *c = new Collector;
    c->ctx = L.ctx;
    c->st = L.st;
    t_collect = c;
}

void ew_collect_end(const Launch &L) {
    Collector *c = t_collect;
    t_collect = nullptr;
    if (!c) return;
    const int logn = L.ctx->logn;
    const PrimeDev *pr = L.ctx->d_primes;
    hipEvent_t ev;
    for (const EwGroup &g : c->ew) {
        for (size_t s0 = 0; s0 < g.recs.size(); s0 += kMaxBatch) {
            const int n = (int)std::min<size_t>(kMaxBatch, g.recs.size() - s0);
            EwMultiArgs m;
            int rows = 0;
            double bytes = 0;
            const double words = (g.op == EW_NEG || g.op == EW_COPY || g.op == EW_MULC || g.op == EW_ADDC ||
                                  g.op == EW_MONO) ? 2
                                 : (g.op == EW_MAC) ? 4 : 3;
            for (int e = 0; e < kMaxBatch; ++e) {
                m.e[e] = e < n ? g.recs[s0 + e] : EwRec{};
                if (e < n) {
                    rows = std::max(rows, m.e[e].rows);
                    bytes += 8.0 * words * ((double)m.e[e].rows * (double)L.ctx->N);
                }
            }
            m.logn = logn;
            m.pr = pr;
            dim3 grid = ew_grid(logn, rows);
            grid.z = (unsigned)n;
            prof_begin(L, "elementwise_batch", &ev);
            switch (g.op) {
#define PFX_EWM(O) case O: k_ew_multi<O><<<grid, 256, 0, L.st>>>(m, g.k); break;
                PFX_EWM(EW_ADD) PFX_EWM(EW_SUB) PFX_EWM(EW_MUL) PFX_EWM(EW_MAC) PFX_EWM(EW_NEG) PFX_EWM(EW_MULC)
                PFX_EWM(EW_MULC_ACC) PFX_EWM(EW_ADDC) PFX_EWM(EW_MONO)
#undef PFX_EWM
                default: k_ew_multi<EW_COPY><<<grid, 256, 0, L.st>>>(m, g.k); break;
            }
            HIP_LAUNCH_CHECK();
            prof_end(L, "elementwise_batch", ev, bytes);
        }
    }
    for (int acc = 0; acc < 2; ++acc) {
        const std::vector<TensorRec> &v = c->tensor[acc];
        for (size_t s0 = 0; s0 < v.size(); s0 += kMaxBatch) {
            const int n = (int)std::min<size_t>(kMaxBatch, v.size() - s0);
            TensorMultiArgs m;
            int rows = 0;
            double bytes = 0;
            for (int e = 0; e < kMaxBatch; ++e) {
                m.e[e] = e < n ? v[s0 + e] : TensorRec{};
                if (e < n) {
                    rows = std::max(rows, m.e[e].nl);
                    bytes += (acc ? 80.0 : 56.0) * (double)m.e[e].nl * (double)L.ctx->N;
                }
            }
            m.logn = logn;
            m.pr = pr;
            dim3 grid = ew_grid(logn, rows);
            grid.z = (unsigned)n;
            prof_begin(L, "tensor_batch", &ev);
            if (acc) k_tensor_multi<true><<<grid, 256, 0, L.st>>>(m);
            else k_tensor_multi<false><<<grid, 256, 0, L.st>>>(m);
            HIP_LAUNCH_CHECK();
            prof_end(L, "tensor_batch", ev, bytes);
        }
    }
    delete c;
}

// ============================================================== automorphism
// phi_g in the NTT domain is the permutation galois_src (ntt_core.h).  Key
// switching reads its operand through the same map instead (no copy); this
// kernel serves callers that want the permuted polynomial itself.
__global__ void k_automorph(double *out, const double *in, size_t so, size_t si, int npoly, int nl, int logn,
                            uint32_t g) {
    const size_t total = ((size_t)npoly * nl) << logn;
    const uint32_t mask = (1u << logn) - 1;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)(idx & mask);
        const size_t li = idx >> logn;
        const int i = (int)(li % nl);
        const int k = (int)(li / nl);
        out[k * so + ((size_t)i << logn) + j] = in[k * si + ((size_t)i << logn) + galois_src(j, logn, g)];
    }
}

void launch_automorph(const Launch &L, double *out, const double *in, size_t so, size_t si, int npoly, int nl,
                      uint32_t g) {
    const size_t total = ((size_t)npoly * nl) << L.ctx->logn;
    hipEvent_t ev;
    prof_begin(L, "automorph", &ev);
    k_automorph<<<grid_for(total), 256, 0, L.st>>>(out, in, so, si, npoly, nl, L.ctx->logn, g);
    HIP_LAUNCH_CHECK();
    prof_end(L, "automorph", ev, 16.0 * (double)total);
}

// ============================================================== key switching (Sec. 2.4.1)
// Workspace layouts at level lv (E = lv + K limbs per extended polynomial):
//   ext[j][t][c]  digit j's fast conversion to the E - sz_j primes outside the
//                 digit, t in the order: q's below the digit, q's above, p's;
//   acc[u][m][c]  u in {0, 1}, m < E: q_0..q_{lv-1} then p_0..p_{K-1}.
// acc_u[m] = sum_j dtilde_j[m] * swk_{j,u}[m]   (NTT domain), for every entry
// of a key-switch batch: each key residue is loaded once and used by all
// entries.  The digit's own primes take d itself: phi_g(d_in) read through
// galois_src (KS_GALOIS), or a1 b1 formed from the product's operands
// (KS_PRODUCT).
struct InnerArgs {
    const double *ext, *key;
    double *acc;
    size_t sext, sacc;
    int nb, lv, logn, L, K, alpha;
    int hoisted;   // KS_GALOIS: ext holds the unpermuted decomposition, read through phi_g as well
    const PrimeDev *pr;
    const double *d[kMaxBatch], *d2[kMaxBatch];
    const double *keys[kMaxBatch];   // k_ks_inner_mk: entry b's own key (rotations by different steps)
    uint32_t g[kMaxBatch];
};

template <int MODE, int NB>
__global__ __launch_bounds__(256) void k_ks_inner(const InnerArgs a) {
    // digits whose loads are all in flight before any product: NB entries'
    // limbs plus two key residues per digit
    constexpr int kChunk = NB >= 4 ? 1 : 4 / NB;
    const int m = blockIdx.y;
    const int logn = a.logn;
    const size_t N = (size_t)1 << logn;
    const size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (c >= N) return;
    const int lv = a.lv, E = lv + a.K, alpha = a.alpha;
    const int beta = (lv + alpha - 1) / alpha;
    const int pid = m < lv ? m : a.L + (m - lv);
    const double q = a.pr[pid].q, qi = a.pr[pid].qinv;
    const size_t kstride = (size_t)(a.L + a.K) * N;
    const double *k0 = a.key + ((size_t)pid << logn) + c;
    const size_t lm = (size_t)m << logn;
    // products in [0, q) summed lazily, reduced once four digits have
    // accumulated: below q + 4q < 2^53, which mred reduces exactly (its
    // quotient estimate is off by at most one there)
    double a0[NB], a1[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) a0[b] = a1[b] = 0.0;
    int pend = 0;
    for (int jb = 0; jb < beta; jb += kChunk) {
        double x[kChunk][NB], w0[kChunk], w1[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            const int j = jb + t;
            if (j < beta) {
                const int j0 = j * alpha;
                const int sz = min(alpha, lv - j0);
                const bool own = m >= j0 && m < j0 + sz;
                const int tt = m < j0 ? m : m - sz;
                w0[t] = __builtin_nontemporal_load(k0 + (size_t)(2 * j) * kstride);
                w1[t] = __builtin_nontemporal_load(k0 + (size_t)(2 * j + 1) * kstride);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (b < a.nb) {
                        if (own) {
                            if (MODE == KS_GALOIS) x[t][b] = a.d[b][lm + galois_src((uint32_t)c, logn, a.g[b])];
                            else if (MODE == KS_PRODUCT) x[t][b] = mmul(a.d[b][lm + c], a.d2[b][lm + c], q, qi);
                            else x[t][b] = a.d[b][lm + c];
                        } else {
                            const size_t cc = MODE == KS_GALOIS && a.hoisted ? galois_src((uint32_t)c, logn, a.g[b]) : c;
                            x[t][b] = __builtin_nontemporal_load(a.ext + b * a.sext + ((size_t)j * E + tt) * N + cc);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            if (jb + t < beta) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (b < a.nb) {
                        a0[b] += mmul(x[t][b], w0[t], q, qi);
                        a1[b] += mmul(x[t][b], w1[t], q, qi);
                    }
                }
            }
        }
        pend += kChunk;
        if (pend >= 4) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                a0[b] = mred(a0[b], q, qi);
                a1[b] = mred(a1[b], q, qi);
            }
            pend = 0;
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b < a.nb) {
            a.acc[b * a.sacc + lm + c] = mred(a0[b], q, qi);
            a.acc[b * a.sacc + ((size_t)(E + m) << logn) + c] = mred(a1[b], q, qi);
        }
    }
}

// A batch whose entries have keys of their own (rotations by different
// steps): entry b = blockIdx.z, each workgroup streams one entry's key and
// ModUp limbs exactly as the one-entry kernel does (every key residue read
// once per entry; a larger grid, one launch).
template <int MODE>
__global__ __launch_bounds__(256) void k_ks_inner_mk(const InnerArgs a) {
    const int m = blockIdx.y, b = blockIdx.z;
    const int logn = a.logn;
    const size_t N = (size_t)1 << logn;
    const size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (c >= N) return;
    const int lv = a.lv, E = lv + a.K, alpha = a.alpha;
    const int beta = (lv + alpha - 1) / alpha;
    const int pid = m < lv ? m : a.L + (m - lv);
    const double q = a.pr[pid].q, qi = a.pr[pid].qinv;
    const size_t kstride = (size_t)(a.L + a.K) * N;
    const double *k0 = a.keys[b] + ((size_t)pid << logn) + c;
    const double *ext = a.ext + b * a.sext;
    const size_t lm = (size_t)m << logn;
    double a0 = 0.0, a1 = 0.0;
    for (int jb = 0; jb < beta; jb += 4) {
        double x[4], w0[4], w1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j = jb + t;
            if (j < beta) {
                const int j0 = j * alpha;
                const int sz = min(alpha, lv - j0);
                const bool own = m >= j0 && m < j0 + sz;
                const int tt = m < j0 ? m : m - sz;
                w0[t] = __builtin_nontemporal_load(k0 + (size_t)(2 * j) * kstride);
                w1[t] = __builtin_nontemporal_load(k0 + (size_t)(2 * j + 1) * kstride);
                if (own) {
                    if (MODE == KS_GALOIS) x[t] = a.d[b][lm + galois_src((uint32_t)c, logn, a.g[b])];
                    else x[t] = a.d[b][lm + c];
                } else {
                    x[t] = __builtin_nontemporal_load(ext + ((size_t)j * E + tt) * N + c);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (jb + t < beta) {
                a0 += mmul(x[t], w0[t], q, qi);
                a1 += mmul(x[t], w1[t], q, qi);
            }
        }
        a0 = mred(a0, q, qi);  // four products in [0, q) on a reduced sum: below 5q
        a1 = mred(a1, q, qi);
    }
    a.acc[b * a.sacc + lm + c] = mred(a0, q, qi);
    a.acc[b * a.sacc + ((size_t)(E + m) << logn) + c] = mred(a1, q, qi);
}

void launch_ks_inner(const Launch &L, const KsBatch &kb, const double *key, int lv) {
    pfx_ctx *ctx = L.ctx;
    InnerArgs a;
    a.ext = kb.ext;
    a.key = key;
    a.acc = kb.acc;
    a.sext = kb.sext;
    a.sacc = kb.sacc;
    a.nb = kb.nb;
    a.hoisted = kb.hoisted ? 1 : 0;
    a.lv = lv;
    a.logn = ctx->logn;
    a.L = ctx->L;
    a.K = ctx->K;
    a.alpha = ctx->alpha;
    a.pr = ctx->d_primes;
    for (int b = 0; b < kMaxBatch; ++b) {
        const KsOperand &o = kb.op[b];
        const bool on = b < kb.nb;
        a.d[b] = on ? (kb.mode == KS_PRODUCT ? o.a1 : o.d) : nullptr;
        a.d2[b] = on && kb.mode == KS_PRODUCT ? o.b1 : nullptr;
        a.g[b] = on ? o.galois : 0;
        a.keys[b] = on ? kb.keys[b] : nullptr;
    }
    const bool mk = kb.keys[0] != nullptr;
    dim3 grid((ctx->N + 255) / 256, lv + ctx->K);
    hipEvent_t ev;
    prof_begin(L, "ks_inner", &ev);
#define PFX_KS_INNER(NB_)                                                                        \
    do {                                                                                          \
        if (kb.mode == KS_GALOIS) k_ks_inner<KS_GALOIS, NB_><<<grid, 256, 0, L.st>>>(a);          \
        else if (kb.mode == KS_PRODUCT) k_ks_inner<KS_PRODUCT, NB_><<<grid, 256, 0, L.st>>>(a);   \
        else k_ks_inner<KS_PLAIN, NB_><<<grid, 256, 0, L.st>>>(a);                                \
    } while (0)
    if (mk) {
        grid.z = (unsigned)kb.nb;
        if (kb.mode == KS_GALOIS) k_ks_inner_mk<KS_GALOIS><<<grid, 256, 0, L.st>>>(a);
        else k_ks_inner_mk<KS_PLAIN><<<grid, 256, 0, L.st>>>(a);
    } else if (kb.nb <= 1) PFX_KS_INNER(1);
    else if (kb.nb <= 2) PFX_KS_INNER(2);
    else if (kb.nb <= 4) PFX_KS_INNER(4);
    else PFX_KS_INNER(kMaxBatch);
#undef PFX_KS_INNER
    HIP_LAUNCH_CHECK();
    // Algorithmic bytes of the inner product: the key once for the batch and
    // each entry's two accumulators.  The decomposition it also reads (the
    // ModUp limbs, written by the previous launches) is an intermediate of this
    // launch sequence, not an operand of the key switch, so its re-read counts
    // as traffic above the algorithmic bytes.
    const int beta = (lv + ctx->alpha - 1) / ctx->alpha;
    prof_end(L, "ks_inner", ev, 8.0 * (double)ctx->N * (lv + ctx->K) * (2.0 * kb.nb + 2.0 * beta * (mk ? kb.nb : 1)));
}

// ============================================================== keys, encryption
// b[m] = -a[m] s[m] + e[m] + g_m sfrom[m] over all L + K primes (NTT domain);
// g_m = [P]_{q_m} for the primes of digit `digit`, 0 elsewhere (P w_j reduced).
__global__ void k_keygen_b(double *b, const double *a, const double *e, const double *s, const double *sfrom,
                           int digit, int alpha, int L, int K, int logn, const PrimeDev *pr, const ModDownConst *md) {
    const size_t total = (size_t)(L + K) << logn;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(idx >> logn);
        const double q = pr[m].q, qi = pr[m].qinv;
        double x = msub(e[idx], mmul(a[idx], s[idx], q, qi), q);
        if (m < L && m >= digit * alpha && m < digit * alpha + alpha)
            x = madd(x, mmulc(sfrom[idx], md->pmod[m].x, md->pmod[m].y, q), q);
        b[idx] = x;
    }
}

void launch_keygen_b(const Launch &L, double *b, const double *a, const double *e, const double *s,
                     const double *sfrom, int digit) {
    pfx_ctx *ctx = L.ctx;
    const size_t total = (size_t)(ctx->L + ctx->K) << ctx->logn;
    k_keygen_b<<<grid_for(total), 256, 0, L.st>>>(b, a, e, s, sfrom, digit, ctx->alpha, ctx->L, ctx->K, ctx->logn,
                                                  ctx->d_primes, ctx->d_moddown);
    HIP_LAUNCH_CHECK();
}

// c0 = -a s + e + m  (NTT domain, lv limbs)
__global__ void k_encrypt(double *c0, const double *a, const double *e, const double *s, const double *m, int lv,
                          int logn, const PrimeDev *pr) {
    const size_t total = (size_t)lv << logn;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx >> logn);
        const double q = pr[i].q, qi = pr[i].qinv;
        c0[idx] = madd(msub(e[idx], mmul(a[idx], s[idx], q, qi), q), m[idx], q);
    }
}

void launch_encrypt(const Launch &L, double *c0, const double *a, const double *e, const double *s, const double *m,
                    int lv) {
    const size_t total = (size_t)lv << L.ctx->logn;
    k_encrypt<<<grid_for(total), 256, 0, L.st>>>(c0, a, e, s, m, lv, L.ctx->logn, L.ctx->d_primes);
    HIP_LAUNCH_CHECK();
}

// m = c0 + c1 s (+ c2 s^2)
__global__ void k_decrypt(double *m, const double *c0, const double *c1, const double *c2, const double *s, int lv,
                          int logn, const PrimeDev *pr) {
    const size_t total = (size_t)lv << logn;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx >> logn);
        const double q = pr[i].q, qi = pr[i].qinv;
        const double sv = s[idx];
        double x = madd(c0[idx], mmul(c1[idx], sv, q, qi), q);
        if (c2) x = madd(x, mmul(mmul(c2[idx], sv, q, qi), sv, q, qi), q);
        m[idx] = x;
    }
}

void launch_decrypt(const Launch &L, double *m, const double *c0, const double *c1, const double *c2, const double *s,
                    int lv) {
    const size_t total = (size_t)lv << L.ctx->logn;
    k_decrypt<<<grid_for(total), 256, 0, L.st>>>(m, c0, c1, c2, s, lv, L.ctx->logn, L.ctx->d_primes);
    HIP_LAUNCH_CHECK();
}

}  // namespace pfx
