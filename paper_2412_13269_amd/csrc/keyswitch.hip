// Fused hybrid key switching (Sec. 2.4.1 of the paper, SwitchKey):
//
//   KS(d) = ModDown( sum_j ModUp_j(d) * swk_j ),  d at lv limbs (NTT domain).
//
// Launch sequence (E = lv + K extended limbs, beta digits of alpha primes):
//   1. k_intt_scale:  INTT of d, each limb i of digit j scaled by (Q'_j/q_i)^-1
//                     on the way out: y_i = [d_i (Q'_j/q_i)^-1]_{q_i}  -> dcoef (lv limbs)
//   2. k_modup_col:   fast basis conversion sum_i y_i [Q'_j/q_i]_m, fed straight
//                     into the column pass of the forward NTT   -> ext     (one limb per (j, m))
//   3. k_row_inner:   row pass of ext_j[m] for every digit j, each result
//                     multiplied by swk_{j,0}[m], swk_{j,1}[m] and summed in
//                     registers (the digit's own primes take d itself) -> acc (2E limbs)
//   4. k_intt_special: INTT of the 2K special-prime limbs of acc, the last store
//                     giving z_k = [(x_k + floor(P/2)) (P/p_k)^-1]_{p_k}  (in place)
//   5. k_moddown_col: sum_k z_k [P/p_k]_{q_i} - floor(P/2), fed into the
//                     column pass                                -> tmp (2 lv limbs)
//   6. k_row_moddown: row pass of tmp, then (acc_Q - x) P^-1 (+ the polynomial
//                     the key switch is added to)                -> out
//
// The fusions remove the coefficient-domain ModUp output (beta * E limbs written
// and read back), the NTT-domain ModUp output (the same again) and the
// coefficient-domain ModDown conversion.  Workgroup ids are remapped so that
// blocks sharing input tiles (step 2, 5) or a prime's twiddle table (3, 6) run
// on one XCD (see xcd_slot in ntt_core.h).
#include <algorithm>
#include <cstdio>

#include "internal.h"
#include "ntt_core.h"

namespace pfx {

#define HIP_LAUNCH_CHECK_KS()                                                                    \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess) set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

struct KsArgs {
    const PrimeDev *primes;
    const ModUpConst *mu;
    const ModDownConst *md;
    int logn, lv, L, K, alpha, beta, E;
    int C, tiles;   // pass geometry (column or row, per kernel)
    int n;          // logical blocks
};

__device__ __forceinline__ int ks_ext_prime(int t, int j0, int sz, int lv, int L) {
    if (t < j0) return t;
    if (t < lv - sz) return t + sz;
    return L + (t - (lv - sz));
}

// ---- step 2: ModUp conversion into the forward column pass
template <int S>
__global__ __launch_bounds__(kNttThreads) void k_modup_col(const KsArgs a, double *__restrict__ ext,
                                                           const double *__restrict__ dcoef) {
    __shared__ double lds[kNttLds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int Tmax = a.E - 1;
    const int t = id % Tmax;
    const int pair = id / Tmax;
    const int tile = pair % a.tiles;
    const int j = pair / a.tiles;
    const int j0 = j * a.alpha;
    const int sz = min(a.alpha, a.lv - j0);
    if (t >= a.E - sz) return;
    const int m = ks_ext_prime(t, j0, sz, a.lv, a.L);
    const PrimeDev &P = a.primes[m];
    const double qm = P.q;
    const ModUpConst &cst = a.mu[j * a.alpha + (sz - 1)];
    double w[kMaxAlpha], wq[kMaxAlpha];
#pragma unroll
    for (int i = 0; i < kMaxAlpha; ++i) {
        if (i < sz) {
            w[i] = cst.hat[i][m].x;
            wq[i] = cst.hat[i][m].y;
        }
    }
    const size_t N = (size_t)1 << a.logn;
    const double *src = dcoef + (size_t)j0 * N;
    double *dst = ext + ((size_t)j * a.E + t) * N;
    auto ld = [&](int g, int) {
        // |each term| <= q_m < 2^50 (inputs below 2^50), at most alpha = 8 terms: < 2^53
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxAlpha; ++i)
            if (i < sz) acc += mmulc_lazy(src[(size_t)i * N + g], w[i], wq[i], qm);
        return mred_signed(acc, qm, P.qinv);
    };
    auto st = [&](int g, double v, int) { dst[g] = v; };
    col_pass<S, false>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

// global index of slot `slot` in the output layout of the forward row pass
// (coalesced: element e = thread + 256 * slot of the tile)
template <int S>
__device__ __forceinline__ bool row_fwd_out(int slot, int C, int cbase, int &gidx) {
    const int e = threadIdx.x + slot * kNttThreads;
    if (e >= (C << S)) return false;
    gidx = (cbase << S) + e;
    return true;
}

// ---- step 3: forward row pass of every digit's limb m, times the key, summed
template <int S>
__global__ __launch_bounds__(kNttThreads) void k_row_inner(const KsArgs a, double *__restrict__ acc,
                                                           const double *__restrict__ ext,
                                                           const double *__restrict__ d_ntt,
                                                           const double *__restrict__ key) {
    __shared__ double lds[kNttLds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int m = id / a.tiles;
    const int tile = id - m * a.tiles;
    const int pid = m < a.lv ? m : a.L + (m - a.lv);
    const PrimeDev &P = a.primes[pid];
    const double q = P.q, qinv = P.qinv;
    const size_t N = (size_t)1 << a.logn;
    const size_t kstride = (size_t)(a.L + a.K) * N;
    const int cbase = tile * a.C;
    double a0[kSlots], a1[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) a0[k] = a1[k] = 0.0;
    for (int j = 0; j < a.beta; ++j) {
        const int j0 = j * a.alpha;
        const int sz = min(a.alpha, a.lv - j0);
        const double *k0 = key + (size_t)(2 * j) * kstride + (size_t)pid * N;
        const double *k1 = k0 + kstride;
        auto mac = [&](int g, double x, int slot) {
            a0[slot] = madd(a0[slot], mmul(x, k0[g], q, qinv), q);
            a1[slot] = madd(a1[slot], mmul(x, k1[g], q, qinv), q);
        };
        if (m >= j0 && m < j0 + sz) {
            const double *x = d_ntt + (size_t)m * N;
#pragma unroll
            for (int slot = 0; slot < kSlots; ++slot) {
                int g;
                if (row_fwd_out<S>(slot, a.C, cbase, g)) mac(g, x[g], slot);
            }
        } else {
            const int t = m < j0 ? m : m - sz;
            const double *src = ext + ((size_t)j * a.E + t) * N;
            auto ld = [&](int g, int) { return src[g]; };
            row_pass<S, false>(P, a.logn, a.C, cbase, lds, ld, mac);
            __syncthreads();
        }
    }
    double *o0 = acc + (size_t)m * N, *o1 = acc + (size_t)(a.E + m) * N;
#pragma unroll
    for (int slot = 0; slot < kSlots; ++slot) {
        int g;
        if (row_fwd_out<S>(slot, a.C, cbase, g)) {
            o0[g] = a0[slot];
            o1[g] = a1[slot];
        }
    }
}

// ---- step 5: ModDown conversion into the forward column pass
template <int S>
__global__ __launch_bounds__(kNttThreads) void k_moddown_col(const KsArgs a, double *__restrict__ tmp,
                                                             const double *__restrict__ acc) {
    __shared__ double lds[kNttLds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int i = id % a.lv;
    const int rest = id / a.lv;
    const int tile = rest % a.tiles;
    const int u = rest / a.tiles;
    const PrimeDev &P = a.primes[i];
    const double q = P.q;
    const ModDownConst *md = a.md;
    const size_t N = (size_t)1 << a.logn;
    double w[kMaxSpecial], wq[kMaxSpecial];
#pragma unroll
    for (int k = 0; k < kMaxSpecial; ++k) {
        if (k < a.K) {
            w[k] = md->phat[k][i].x;
            wq[k] = md->phat[k][i].y;
        }
    }
    const double hi = md->half[i];
    const double *src = acc + ((size_t)u * a.E + a.lv) * N;
    double *dst = tmp + ((size_t)u * a.lv + i) * N;
    auto ld = [&](int g, int) {
        // src holds z_k = [(x_k + floor(P/2)) (P/p_k)^-1]_{p_k} (step 4).
        // |each term| <= q_i < 2^50, K <= 7 terms plus floor(P/2) mod q_i: < 2^53
        double s = -hi;
#pragma unroll
        for (int k = 0; k < kMaxSpecial; ++k)
            if (k < a.K) s += mmulc_lazy(src[(size_t)k * N + g], w[k], wq[k], q);
        return mred_signed(s, q, P.qinv);
    };
    auto st = [&](int g, double v, int) { dst[g] = v; };
    col_pass<S, false>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

// ---- step 6: forward row pass of the conversion, then (acc_Q - x) P^-1 (+ base)
template <int S>
__global__ __launch_bounds__(kNttThreads) void k_row_moddown(const KsArgs a, double *out0, double *out1,
                                                             const double *__restrict__ acc,
                                                             const double *__restrict__ tmp, const double *base0,
                                                             const double *base1) {
    __shared__ double lds[kNttLds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int tile = id % a.tiles;
    const int rest = id / a.tiles;
    const int u = rest % 2;
    const int i = rest / 2;
    const PrimeDev &P = a.primes[i];
    const double q = P.q;
    const double2 pinv = a.md->pinv[i];
    const size_t N = (size_t)1 << a.logn;
    const double *src = tmp + ((size_t)u * a.lv + i) * N;
    const double *ax = acc + ((size_t)u * a.E + i) * N;
    const double *base = u ? base1 : base0;
    double *out = (u ? out1 : out0) + (size_t)i * N;
    const double *bs = base ? base + (size_t)i * N : nullptr;
    auto ld = [&](int g, int) { return src[g]; };
    auto st = [&](int g, double v, int) {
        double x = mmulc(msub(ax[g], v, q), pinv.x, pinv.y, q);
        if (bs) x = madd(x, bs[g], q);
        out[g] = x;
    };
    row_pass<S, false>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

// ---- step 1: INTT of d with the ModUp scaling folded into the last stage's store
template <int S, bool ROW>
__global__ __launch_bounds__(kNttThreads) void k_intt_scale(const KsArgs a, double *__restrict__ dst,
                                                            const double *__restrict__ src) {
    __shared__ double lds[kNttLds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int i = id / a.tiles;
    const int tile = id - i * a.tiles;
    const PrimeDev &P = a.primes[i];
    const size_t N = (size_t)1 << a.logn;
    const double *s = src + (size_t)i * N;
    double *d = dst + (size_t)i * N;
    auto ld = [&](int g, int) { return s[g]; };
    if (ROW) {
        auto st = [&](int g, double v, int) { d[g] = v; };
        row_pass<S, true>(P, a.logn, a.C, tile * a.C, lds, ld, st);
    } else {
        const int j = i / a.alpha;
        const int sz = min(a.alpha, a.lv - j * a.alpha);
        const double2 inv = a.mu[j * a.alpha + (sz - 1)].inv[i - j * a.alpha];
        auto st = [&](int g, double v, int) { d[g] = mmulc(v, inv.x, inv.y, P.q); };
        col_pass<S, true>(P, a.logn, a.C, tile * a.C, lds, ld, st);
    }
}

// ---- step 4: INTT of the special-prime limbs of acc_0, acc_1 (in place); the
// last store adds floor(P/2) and multiplies by (P/p_k)^-1, so step 5 only sums.
template <int S, bool ROW>
__global__ __launch_bounds__(kNttThreads) void k_intt_special(const KsArgs a, double *__restrict__ acc) {
    __shared__ double lds[kNttLds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int limb = id / a.tiles;          // u * K + k
    const int tile = id - limb * a.tiles;
    const int u = limb / a.K, k = limb - u * a.K;
    const PrimeDev &P = a.primes[a.L + k];
    const size_t N = (size_t)1 << a.logn;
    double *x = acc + ((size_t)u * a.E + a.lv + k) * N;
    auto ld = [&](int g, int) { return x[g]; };
    if (ROW) {
        auto st = [&](int g, double v, int) { x[g] = v; };
        row_pass<S, true>(P, a.logn, a.C, tile * a.C, lds, ld, st);
    } else {
        const double h = a.md->half[a.L + k];
        const double2 iv = a.md->phat_inv[k];
        auto st = [&](int g, double v, int) { x[g] = mmulc(madd(v, h, P.q), iv.x, iv.y, P.q); };
        col_pass<S, true>(P, a.logn, a.C, tile * a.C, lds, ld, st);
    }
}

// ----------------------------------------------------------------- launchers
#define PFX_SWITCH_S(S_, CALL)                                   \
    switch (S_) {                                                \
        case 2: { constexpr int SS = 2; CALL; } break;           \
        case 3: { constexpr int SS = 3; CALL; } break;           \
        case 4: { constexpr int SS = 4; CALL; } break;           \
        case 5: { constexpr int SS = 5; CALL; } break;           \
        case 6: { constexpr int SS = 6; CALL; } break;           \
        case 7: { constexpr int SS = 7; CALL; } break;           \
        case 8: { constexpr int SS = 8; CALL; } break;           \
        default: set_error("unsupported NTT pass size"); break;  \
    }

static KsArgs ks_args(pfx_ctx *c, int lv) {
    KsArgs a;
    a.primes = c->d_primes;
    a.mu = c->d_modup;
    a.md = c->d_moddown;
    a.logn = c->logn;
    a.lv = lv;
    a.L = c->L;
    a.K = c->K;
    a.alpha = c->alpha;
    a.beta = (lv + c->alpha - 1) / c->alpha;
    a.E = lv + c->K;
    return a;
}

void launch_intt_scale(const Launch &L, double *dcoef, const double *d, int lv) {
    KsArgs a = ks_args(L.ctx, lv);
    const PassShape pr = row_shape(a.logn), pc = col_shape(a.logn);
    hipEvent_t ev;
    a.C = pr.C;
    a.tiles = pr.tiles;
    a.n = lv * a.tiles;
    prof_begin(L, "ks_intt_row", &ev);
    PFX_SWITCH_S(pr.S, (k_intt_scale<SS, true><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, dcoef, d)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_row", ev, 16.0 * (double)L.ctx->N * lv);
    a.C = pc.C;
    a.tiles = pc.tiles;
    a.n = lv * a.tiles;
    prof_begin(L, "ks_intt_col", &ev);
    PFX_SWITCH_S(pc.S, (k_intt_scale<SS, false><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, dcoef, dcoef)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_col", ev, 16.0 * (double)L.ctx->N * lv);
}

void launch_modup_col(const Launch &L, double *ext, const double *dcoef, int lv) {
    KsArgs a = ks_args(L.ctx, lv);
    const PassShape ps = col_shape(a.logn);
    a.C = ps.C;
    a.tiles = ps.tiles;
    a.n = a.beta * a.tiles * (a.E - 1);
    hipEvent_t ev;
    prof_begin(L, "ks_modup_col", &ev);
    PFX_SWITCH_S(ps.S, (k_modup_col<SS><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, ext, dcoef)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_modup_col", ev, 8.0 * (double)L.ctx->N * a.beta * a.E);
}

void launch_row_inner(const Launch &L, double *acc, const double *ext, const double *d_ntt, const double *key,
                      int lv) {
    KsArgs a = ks_args(L.ctx, lv);
    const PassShape ps = row_shape(a.logn);
    a.C = ps.C;
    a.tiles = ps.tiles;
    a.n = a.E * a.tiles;
    hipEvent_t ev;
    prof_begin(L, "ks_row_inner", &ev);
    PFX_SWITCH_S(ps.S, (k_row_inner<SS><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, acc, ext, d_ntt, key)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_row_inner", ev, 8.0 * (double)L.ctx->N * a.E * (3.0 * a.beta + 2.0));
}

void launch_intt_special(const Launch &L, double *acc, int lv) {
    KsArgs a = ks_args(L.ctx, lv);
    PassShape pr = row_shape(a.logn), pc = col_shape(a.logn);
    // 2K limbs only: narrower tiles for more workgroups
    while (2 * a.K * pr.tiles < 1024 && pr.C > 1) { pr.C /= 2; pr.tiles *= 2; }
    while (2 * a.K * pc.tiles < 1024 && pc.C / 2 >= 8) { pc.C /= 2; pc.tiles *= 2; }
    hipEvent_t ev;
    a.C = pr.C;
    a.tiles = pr.tiles;
    a.n = 2 * a.K * a.tiles;
    prof_begin(L, "ks_intt_special_row", &ev);
    PFX_SWITCH_S(pr.S, (k_intt_special<SS, true><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, acc)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_special_row", ev, 16.0 * (double)L.ctx->N * 2 * a.K);
    a.C = pc.C;
    a.tiles = pc.tiles;
    a.n = 2 * a.K * a.tiles;
    prof_begin(L, "ks_intt_special_col", &ev);
    PFX_SWITCH_S(pc.S, (k_intt_special<SS, false><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, acc)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_special_col", ev, 16.0 * (double)L.ctx->N * 2 * a.K);
}

void launch_moddown_col(const Launch &L, double *tmp, const double *acc, int lv) {
    KsArgs a = ks_args(L.ctx, lv);
    const PassShape ps = col_shape(a.logn);
    a.C = ps.C;
    a.tiles = ps.tiles;
    a.n = 2 * a.tiles * lv;
    hipEvent_t ev;
    prof_begin(L, "ks_moddown_col", &ev);
    PFX_SWITCH_S(ps.S, (k_moddown_col<SS><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, tmp, acc)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_moddown_col", ev, 8.0 * (double)L.ctx->N * (2.0 * a.K + 2.0 * lv));
}

void launch_row_moddown(const Launch &L, double *out0, double *out1, const double *acc, const double *tmp,
                        const double *base0, const double *base1, int lv) {
    KsArgs a = ks_args(L.ctx, lv);
    const PassShape ps = row_shape(a.logn);
    a.C = ps.C;
    a.tiles = ps.tiles;
    a.n = 2 * lv * a.tiles;
    hipEvent_t ev;
    prof_begin(L, "ks_row_moddown", &ev);
    PFX_SWITCH_S(ps.S, (k_row_moddown<SS><<<xcd_grid(a.n), kNttThreads, 0, L.st>>>(a, out0, out1, acc, tmp, base0,
                                                                                     base1)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_row_moddown", ev,
             8.0 * (double)L.ctx->N * lv * (6.0 + (base0 ? 1 : 0) + (base1 ? 1 : 0)));
}

}  // namespace pfx
