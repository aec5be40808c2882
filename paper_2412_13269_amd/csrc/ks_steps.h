// Device bodies of the fused key-switching steps (Sec. 2.4.1 of the paper,
// SwitchKey) shared by the per-step kernels of keyswitch.hip and the
// persistent batched kernel of persist.hip.  Each body runs one logical block
// (tile) of its step: `bi` is the batch entry of `a`, `id` the block within the
// entry, C and tiles the pass geometry, lds the caller's exchange area of a
// TH-thread tile.
#pragma once
#include "internal.h"
#include "ntt_core.h"

namespace pfx {

// One batch entry: its operand (KsOperand) and outputs, as plain pointers.
//   KS_GALOIS: the key-switched polynomial is phi_galois of d;
//   KS_PRODUCT: the operands of a ciphertext product (a0, a1) x (b0, b1):
//   d = a1 b1 and the bases a0 b0, a0 b1 + a1 b0 are formed where they are read.
struct KsEntry {
    const double *d, *base0, *base1, *a0, *a1, *b0, *b1;
    double *out0, *out1;
    uint32_t galois;
    const double *key;   // the entry's own key data, or null (the launch's key)
};

// Kernel arguments.  A launch covers nb batch entries (same level, key and
// mode): logical block id = entry * per + the entry's own block id, and the
// entry's scratch regions sit at the given strides (in doubles) from entry 0's.
struct KsArgs {
    const PrimeDev *primes;
    const ModUpConst *mu;
    const ModDownConst *md;
    int logn, lv, L, K, alpha, beta, E;
    int C, tiles;   // pass geometry (column or row, per kernel)
    int n;          // logical blocks
    int nb, per;    // batch entries, blocks per entry
    size_t sdc, sext, sacc, stmp;
    RepackDesc rp;  // KS_REPACK entries (op unused; nb may exceed kMaxBatch)
    KsEntry op[kMaxBatch];
};

// KS_REPACK: c_j (lo) and c_(j+t) (hi) of entry bi in the round's input array,
// and its slot in the output array.
struct RpPtrs {
    const double *lo, *hi;
    double *out;
    uint32_t t;
};
__device__ __forceinline__ RpPtrs rp_ptrs(const RepackDesc &r, int bi) {
    const unsigned e = (unsigned)(r.e0 + bi);
    const unsigned grp = e >> r.tlog, j = e & ((1u << r.tlog) - 1u);
    const uint32_t t = 1u << r.tlog;
    const double *lo = r.in + grp * r.in_gs + j * r.cs;
    return RpPtrs{lo, lo + t * r.cs, r.out + grp * r.out_gs + j * r.cs, t};
}
// lo[x] - X^t hi[x] (the difference that Alg. 1 rotates), slot x of one limb
__device__ __forceinline__ double rp_diff(const double *lo, const double *hi, uint32_t x, uint32_t t, int logn,
                                          const PrimeDev &P) {
    return msub(lo[x], monomial_mul(hi[x], x, t, logn, P), P.q);
}

__device__ __forceinline__ int ks_ext_prime(int t, int j0, int sz, int lv, int L) {
    if (t < j0) return t;
    if (t < lv - sz) return t + sz;
    return L + (t - (lv - sz));
}

// ---- step 2: ModUp conversion into the forward column pass
// NT is the digit size rounded up to a power of two; the terms of a shorter
// digit (the last one at some levels) beyond its size get weight 0 and read
// the digit's first limb again, so the sum has no data-dependent branches.
// Blocks: every (digit j, tile, target t) with t < E - sz_j, t fastest.
template <int S, int NT, int TH>
__device__ __forceinline__ void modup_col_body(const KsArgs &a, int C, int tiles, int bi, int id,
                                               double *__restrict__ ext, const double *__restrict__ dcoef, double *lds) {
    ext += bi * a.sext;
    dcoef += bi * a.sdc;
    const int Tf = a.E - a.alpha;                       // targets of a full digit
    const int full = (a.beta - 1) * Tf * tiles;
    int j, rem, T;
    if (id < full) {
        T = Tf;
        j = id / (Tf * tiles);
        rem = id - j * Tf * tiles;
    } else {
        j = a.beta - 1;
        T = a.E - (a.lv - j * a.alpha);
        rem = id - full;
    }
    const int t = rem % T;
    const int tile = rem / T;
    const int j0 = j * a.alpha;
    const int sz = min(a.alpha, a.lv - j0);
    const int m = ks_ext_prime(t, j0, sz, a.lv, a.L);
    const PrimeDev &P = a.primes[m];
    const double qm = P.q;
    const ModUpConst &cst = a.mu[j * a.alpha + (sz - 1)];
    const size_t N = (size_t)1 << a.logn;
    const double *src = dcoef + (size_t)j0 * N;
    const double *sp[NT];
    double w[NT], wq[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const bool on = i < sz;
        sp[i] = on ? src + (size_t)i * N : src;
        w[i] = on ? cst.hat[i][m].x : 0.0;
        wq[i] = on ? cst.hat[i][m].y : 0.0;
    }
    double *dst = ext + ((size_t)j * a.E + t) * N;
    auto ld = [&](int g, int) {
        // |each term| <= q_m < 2^50 (inputs below 2^50), at most 8 terms: < 2^53
        const unsigned ug = (unsigned)g;
        double acc = mmulc_lazy(sp[0][ug], w[0], wq[0], qm);
#pragma unroll
        for (int i = 1; i < NT; ++i) acc += mmulc_lazy(sp[i][ug], w[i], wq[i], qm);
        return mred_signed(acc, qm, P.qinv);
    };
    auto st = [&](int g, double v, int) { dst[(unsigned)g] = v; };
    col_pass<S, false, TH>(P, a.logn, C, tile * C, lds, ld, st);
}

// ---- step 5: ModDown conversion into the forward column pass
// NT is K rounded up to a power of two (terms beyond K: weight 0, limb 0 again).
template <int S, int NT, int TH>
__device__ __forceinline__ void moddown_col_body(const KsArgs &a, int C, int tiles, int bi, int id,
                                                 double *__restrict__ tmp, const double *__restrict__ acc, double *lds) {
    tmp += bi * a.stmp;
    acc += bi * a.sacc;
    const int i = id % a.lv;
    const int rest = id / a.lv;
    const int tile = rest % tiles;
    const int u = rest / tiles;
    const PrimeDev &P = a.primes[i];
    const double q = P.q;
    const ModDownConst *md = a.md;
    const size_t N = (size_t)1 << a.logn;
    const double *src = acc + ((size_t)u * a.E + a.lv) * N;
    const double *sp[NT];
    double w[NT], wq[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const bool on = k < a.K;
        sp[k] = on ? src + (size_t)k * N : src;
        w[k] = on ? md->phat[k][i].x : 0.0;
        wq[k] = on ? md->phat[k][i].y : 0.0;
    }
    const double hi = md->half[i];
    double *dst = tmp + ((size_t)u * a.lv + i) * N;
    auto ld = [&](int g, int) {
        // src holds z_k = [(x_k + floor(P/2)) (P/p_k)^-1]_{p_k} (step 4).
        // |each term| <= q_i < 2^50, at most 8 terms plus floor(P/2) mod q_i: < 2^53
        const unsigned ug = (unsigned)g;
        double s = -hi;
#pragma unroll
        for (int k = 0; k < NT; ++k) s += mmulc_lazy(sp[k][ug], w[k], wq[k], q);
        return mred_signed(s, q, P.qinv);
    };
    auto st = [&](int g, double v, int) { dst[(unsigned)g] = v; };
    col_pass<S, false, TH>(P, a.logn, C, tile * C, lds, ld, st);
}

// ---- step 6: forward row pass of the conversion, then (acc_Q - x) P^-1 (+ base)
// PREFETCH: the operands of the combination are loaded before the transform,
// so that their latency hides under it (slot k of this thread is element
// tid + k * TH of the tile, the row pass's output order); without it they are
// loaded where each output is stored (fewer registers; the same words).
template <int S, int MODE, int TH, bool PREFETCH = true>
__device__ __forceinline__ void row_moddown_body(const KsArgs &a, int C, int tiles, int bi, int id,
                                                 const double *__restrict__ acc, const double *__restrict__ tmp, double *lds) {
    const KsEntry &en = a.op[MODE == KS_REPACK ? 0 : bi];
    acc += bi * a.sacc;
    tmp += bi * a.stmp;
    double *out0, *out1;
    const double *base0, *base1;
    RpPtrs rp{};
    if constexpr (MODE == KS_REPACK) {
        rp = rp_ptrs(a.rp, bi);
        out0 = rp.out;
        out1 = rp.out + a.rp.ps;
        base0 = base1 = nullptr;
    } else {
        out0 = en.out0;
        out1 = en.out1;
        base0 = en.base0;
        base1 = en.base1;
    }
    const int tile = id % tiles;
    const int rest = id / tiles;
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
    const size_t li = (size_t)i * N;
    // KS_GALOIS: the base of output 0 (c0 of the rotated ciphertext) is read
    // through phi_g; KS_PRODUCT: the bases are the tensor terms of the inputs.
    const int g0 = (tile * C) << S, tot = C << S;
    // The accumulator and the base at element g of this limb (g < N).
    auto operands = [&](unsigned g, double &xa, double &xb) {
        xa = ax[g];
        xb = 0.0;
        if constexpr (MODE == KS_REPACK) {
            // c_j + X^t c_(j+t), plus phi_g(c_j - X^t c_(j+t)) for c0
            const double *lo = rp.lo + (size_t)u * a.rp.ps + li, *hi = rp.hi + (size_t)u * a.rp.ps + li;
            xb = madd(lo[g], monomial_mul(hi[g], g, rp.t, a.logn, P), q);
            if (u == 0) xb = madd(xb, rp_diff(lo, hi, galois_src(g, a.logn, a.rp.galois), rp.t, a.logn, P), q);
        } else if (MODE == KS_PRODUCT) {
            xb = u == 0 ? mmul(en.a0[li + g], en.b0[li + g], q, P.qinv)
                        : madd(mmul(en.a0[li + g], en.b1[li + g], q, P.qinv),
                               mmul(en.a1[li + g], en.b0[li + g], q, P.qinv), q);
        } else if (bs) {
            xb = bs[MODE == KS_GALOIS && u == 0 ? galois_src(g, a.logn, en.galois) : g];
        }
    };
    auto ld = [&](int g, int) { return src[g]; };
    if constexpr (PREFETCH) {
        double xa[kSlots], xb[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int e = threadIdx.x + k * TH;
            xa[k] = xb[k] = 0.0;
            if (e < tot) operands((unsigned)(g0 + e), xa[k], xb[k]);
        }
        auto st = [&](int g, double v, int k) {
            out[g] = madd(mmulc(msub(xa[k], v, q), pinv.x, pinv.y, q), xb[k], q);
        };
        row_pass<S, false, TH>(P, a.logn, C, tile * C, lds, ld, st);
    } else {
        auto st = [&](int g, double v, int) {
            double xa, xb;
            operands((unsigned)g, xa, xb);
            out[g] = madd(mmulc(msub(xa, v, q), pinv.x, pinv.y, q), xb, q);
        };
        row_pass<S, false, TH>(P, a.logn, C, tile * C, lds, ld, st);
    }
}

// ---- step 1: INTT of d with the ModUp scaling folded into the last stage's store
template <int S, bool ROW, int MODE, int TH>
__device__ __forceinline__ void intt_scale_body(const KsArgs &a, int C, int tiles, int bi, int id,
                                                double *__restrict__ dst, double *lds) {
    const KsEntry &en = a.op[MODE == KS_REPACK ? 0 : bi];
    dst += bi * a.sdc;
    // the row (first) pass reads the operand, the column pass dst in place
    RpPtrs rp{};
    if constexpr (MODE == KS_REPACK) rp = rp_ptrs(a.rp, bi);
    const double *src = ROW ? (MODE == KS_REPACK ? nullptr : en.d) : dst;
    const int i = id / tiles;
    const int tile = id - i * tiles;
    const PrimeDev &P = a.primes[i];
    const size_t N = (size_t)1 << a.logn;
    const double *s = src + (size_t)i * N;
    double *d = dst + (size_t)i * N;
    const size_t li = (size_t)i * N;
    auto ld = [&](int g, int) {
        const unsigned e = (unsigned)g;
        if constexpr (MODE == KS_REPACK)
            return rp_diff(rp.lo + a.rp.ps + li, rp.hi + a.rp.ps + li, galois_src(e, a.logn, a.rp.galois), rp.t,
                           a.logn, P);
        if (MODE == KS_PRODUCT) return mmul(en.a1[li + e], en.b1[li + e], P.q, P.qinv);
        return s[MODE == KS_GALOIS ? galois_src(e, a.logn, en.galois) : e];
    };
    if (ROW) {
        auto st = [&](int g, double v, int) { d[g] = v; };
        row_pass<S, true, TH>(P, a.logn, C, tile * C, lds, ld, st);
    } else {
        const int j = i / a.alpha;
        const int sz = min(a.alpha, a.lv - j * a.alpha);
        const double2 inv = a.mu[j * a.alpha + (sz - 1)].inv[i - j * a.alpha];
        auto st = [&](int g, double v, int) { d[g] = mmulc(v, inv.x, inv.y, P.q); };
        col_pass<S, true, TH>(P, a.logn, C, tile * C, lds, ld, st);
    }
}

// ---- step 4: INTT of the special-prime limbs of acc_0, acc_1 (in place); the
// last store adds floor(P/2) and multiplies by (P/p_k)^-1, so step 5 only sums.
template <int S, bool ROW, int TH>
__device__ __forceinline__ void intt_special_body(const KsArgs &a, int C, int tiles, int bi, int id,
                                                  double *__restrict__ acc, double *lds) {
    acc += bi * a.sacc;
    const int limb = id / tiles;          // u * K + k
    const int tile = id - limb * tiles;
    const int u = limb / a.K, k = limb - u * a.K;
    const PrimeDev &P = a.primes[a.L + k];
    const size_t N = (size_t)1 << a.logn;
    double *x = acc + ((size_t)u * a.E + a.lv + k) * N;
    auto ld = [&](int g, int) { return x[g]; };
    if (ROW) {
        auto st = [&](int g, double v, int) { x[g] = v; };
        row_pass<S, true, TH>(P, a.logn, C, tile * C, lds, ld, st);
    } else {
        const double h = a.md->half[a.L + k];
        const double2 iv = a.md->phat_inv[k];
        auto st = [&](int g, double v, int) { x[g] = mmulc(madd(v, h, P.q), iv.x, iv.y, P.q); };
        col_pass<S, true, TH>(P, a.logn, C, tile * C, lds, ld, st);
    }
}


}  // namespace pfx
