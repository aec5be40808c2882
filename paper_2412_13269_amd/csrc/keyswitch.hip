// Fused hybrid key switching (Sec. 2.4.1 of the paper, SwitchKey):
//
//   KS(d) = ModDown( sum_j ModUp_j(d) * swk_j ),  d at lv limbs (NTT domain).
//
// Launch sequence (E = lv + K extended limbs, beta digits of alpha primes):
//   1. k_intt_scale:  INTT of d, each limb i of digit j scaled by (Q'_j/q_i)^-1
//                     on the way out: y_i = [d_i (Q'_j/q_i)^-1]_{q_i}  -> dcoef (lv limbs)
//   2. k_modup_col:   fast basis conversion sum_i y_i [Q'_j/q_i]_m, fed straight
//                     into the column pass of the forward NTT   -> ext     (one limb per (j, m))
//   3. row pass of ext (plain NTT pass), then k_ks_inner: acc_u[m] =
//                     sum_j ext_j[m] swk_{j,u}[m] (the digit's own primes take
//                     d itself)                                  -> acc (2E limbs)
//   4. k_intt_special: INTT of the 2K special-prime limbs of acc, the last store
//                     giving z_k = [(x_k + floor(P/2)) (P/p_k)^-1]_{p_k}  (in place)
//   5. k_moddown_col: sum_k z_k [P/p_k]_{q_i} - floor(P/2), fed into the
//                     column pass                                -> tmp (2 lv limbs)
//   6. k_row_moddown: row pass of tmp, then (acc_Q - x) P^-1 (+ the polynomial
//                     the key switch is added to)                -> out
//
// The fusions remove the coefficient-domain ModUp output (beta * E limbs written
// and read back) and the coefficient-domain ModDown conversion.  The operand
// is read where it is needed (KsMode): for a rotation steps 1 and 3 read d
// through the NTT-domain permutation of phi_g and step 6 reads the polynomial
// it adds (c0) through it, so no permuted copy is made; for HMult + relin the
// tensor product is never stored: steps 1 and 3 form d2 = a1 b1 and step 6
// the bases d0 = a0 b0, d1 = a0 b1 + a1 b0 from the input ciphertexts.  Workgroup ids are remapped so that
// blocks sharing input tiles (step 2, 5) or a prime's twiddle table (3, 6) run
// on one XCD (see xcd_slot in ntt_core.h).
#include <algorithm>
#include <cstdio>

#include "internal.h"
#include "ks_steps.h"
#include "ntt_core.h"

namespace pfx {

#define HIP_LAUNCH_CHECK_KS()                                                                    \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess) set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

template <int S, int NT, int TH>
__global__ __launch_bounds__(TH) void k_modup_col(const KsArgs a, double *__restrict__ ext,
                                                           const double *__restrict__ dcoef) {
    __shared__ double lds[col_lds<S, TH>()];
    const int gid = xcd_slot(a.n);
    if (gid >= a.n) return;
    const int bi = gid / a.per, id = gid - bi * a.per;
    modup_col_body<S, NT, TH>(a, a.C, a.tiles, bi, id, ext, dcoef, lds);
}

template <int S, int NT, int TH>
__global__ __launch_bounds__(TH) void k_moddown_col(const KsArgs a, double *__restrict__ tmp,
                                                             const double *__restrict__ acc) {
    __shared__ double lds[col_lds<S, TH>()];
    const int gid = xcd_slot(a.n);
    if (gid >= a.n) return;
    const int bi = gid / a.per, id = gid - bi * a.per;
    moddown_col_body<S, NT, TH>(a, a.C, a.tiles, bi, id, tmp, acc, lds);
}

template <int S, int MODE, int TH>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(3))) void k_row_moddown(const KsArgs a, const double *__restrict__ acc,
                                                    const double *__restrict__ tmp) {
    __shared__ double lds[NttTile<TH>::lds];
    const int gid = xcd_slot(a.n);
    if (gid >= a.n) return;
    const int bi = gid / a.per, id = gid - bi * a.per;
    row_moddown_body<S, MODE, TH>(a, a.C, a.tiles, bi, id, acc, tmp, lds);
}

template <int S, bool ROW, int MODE, int TH>
__global__ __launch_bounds__(TH) void k_intt_scale(const KsArgs a, double *__restrict__ dst) {
    __shared__ double lds[ROW ? NttTile<TH>::lds : col_lds<S, TH>()];
    const int gid = xcd_slot(a.n);
    if (gid >= a.n) return;
    const int bi = gid / a.per, id = gid - bi * a.per;
    intt_scale_body<S, ROW, MODE, TH>(a, a.C, a.tiles, bi, id, dst, lds);
}

template <int S, bool ROW, int TH>
__global__ __launch_bounds__(TH) void k_intt_special(const KsArgs a, double *__restrict__ acc) {
    __shared__ double lds[ROW ? NttTile<TH>::lds : col_lds<S, TH>()];
    const int gid = xcd_slot(a.n);
    if (gid >= a.n) return;
    const int bi = gid / a.per, id = gid - bi * a.per;
    intt_special_body<S, ROW, TH>(a, a.C, a.tiles, bi, id, acc, lds);
}

// ---- steps 3 and 4a fused (KS_PLAIN, KS_GALOIS, KS_PRODUCT; not hoisted):
// one workgroup per (target limb m, row tile, batch entry), entries fastest so
// that the entries of a batch read one key tile from the same XCD's L2.  For
// every digit j it takes the digit's limb m in the NTT domain, either the
// forward row pass of the column-pass output in ext (left signed in
// [-q/2, q/2]) or, for the digit's own primes, the operand itself (d, phi_g(d)
// through the permutation, or a1 b1), and adds its products with the two key
// residues to accumulators held in registers (signed lazy products,
// |r| <= 0.875 q, reduced every fourth digit: below 4 q < 2^53).  Only the
// accumulators reach HBM: canonical for the q limbs; a special-prime limb
// first runs the first (row) pass of its inverse transform, whose input is the
// accumulator in the pass's own element order, so step 4's row launch is not
// needed.  The ModUp limbs and d are read once, the key once per launch.
template <int S, int MODE, int TH>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(2))) void k_row_inner(const KsArgs a, const double *__restrict__ ext,
                                                  const double *__restrict__ key, double *__restrict__ acc) {
    __shared__ double lds[NttTile<TH>::lds];
    const int gid = xcd_slot(a.n);
    if (gid >= a.n) return;
    const int bi = gid % a.nb, id = gid / a.nb;
    const int tile = id % a.tiles, m = id / a.tiles;
    const KsEntry &en = a.op[bi];
    const int lv = a.lv, E = a.E;
    const int pid = m < lv ? m : a.L + (m - lv);
    const PrimeDev &P = a.primes[pid];
    const double q = P.q, qi = P.qinv;
    const int logn = a.logn;
    const size_t N = (size_t)1 << logn;
    const size_t kstride = (size_t)(a.L + a.K) * N;
    const int C = a.C, g0 = (tile * C) << S, tot = C << S;
    const double *kq = (en.key ? en.key : key) + ((size_t)pid << logn);
    const size_t lm = (size_t)m << logn;
    ext += bi * a.sext;
    acc += bi * a.sacc;
    double s0[kSlots], s1[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) s0[k] = s1[k] = 0.0;
    for (int j = 0; j < a.beta; ++j) {
        const int j0 = j * a.alpha, sz = min(a.alpha, lv - j0);
        const double *w0 = kq + (size_t)(2 * j) * kstride, *w1 = w0 + kstride;
        if (m >= j0 && m < j0 + sz) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                const int e = threadIdx.x + k * TH;
                if (e < tot) {
                    const unsigned c = (unsigned)(g0 + e);
                    double x;
                    if constexpr (MODE == KS_GALOIS) x = en.d[lm + galois_src(c, logn, en.galois)];
                    else if constexpr (MODE == KS_PRODUCT) x = mmul(en.a1[lm + c], en.b1[lm + c], q, qi);
                    else x = en.d[lm + c];
                    s0[k] += mmul_lazy(x, __builtin_nontemporal_load(w0 + c), q, qi);
                    s1[k] += mmul_lazy(x, __builtin_nontemporal_load(w1 + c), q, qi);
                }
            }
        } else {
            const double *src = ext + ((size_t)j * E + (m < j0 ? m : m - sz)) * N;
            auto ld = [&](int g, int) { return __builtin_nontemporal_load(src + (unsigned)g); };
            auto st = [&](int g, double v, int k) {
                s0[k] += mmul_lazy(v, __builtin_nontemporal_load(w0 + (unsigned)g), q, qi);
                s1[k] += mmul_lazy(v, __builtin_nontemporal_load(w1 + (unsigned)g), q, qi);
            };
            __syncthreads();                 // the previous pass's last LDS reads are done
            row_pass<S, false, TH, false>(P, logn, C, tile * C, lds, ld, st);
        }
        if ((j & 3) == 3) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                s0[k] = mred_signed(s0[k], q, qi);
                s1[k] = mred_signed(s1[k], q, qi);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        s0[k] = mred_signed(s0[k], q, qi);
        s1[k] = mred_signed(s1[k], q, qi);
    }
    if (m < lv) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int e = threadIdx.x + k * TH;
            if (e < tot) {
                acc[lm + g0 + e] = mcanon(s0[k], q);
                acc[((size_t)(E + m) << logn) + g0 + e] = mcanon(s1[k], q);
            }
        }
    } else {
        // the first pass of the special limb's inverse transform, per polynomial
        double *x0 = acc + lm, *x1 = acc + ((size_t)(E + m) << logn);
        __syncthreads();
        row_pass<S, true, TH>(P, logn, C, tile * C, lds, [&](int, int k) { return s0[k]; },
                              [&](int g, double v, int) { x0[(unsigned)g] = v; });
        __syncthreads();
        row_pass<S, true, TH>(P, logn, C, tile * C, lds, [&](int, int k) { return s1[k]; },
                              [&](int g, double v, int) { x1[(unsigned)g] = v; });
    }
}

// ---- step 3 for KS_REPACK: the inner product of one entry per blockIdx.z (a
// batch of any size); the entry's own digit reads phi_g(c_j - X^t c_(j+t)) of
// the round's input array where the other entries' kernel reads d.
__global__ __launch_bounds__(256) void k_ks_inner_repack(const KsArgs a, const double *__restrict__ key,
                                                         const double *__restrict__ ext, double *__restrict__ acc) {
    const int m = blockIdx.y, bi = blockIdx.z;
    const int logn = a.logn;
    const size_t N = (size_t)1 << logn;
    const size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (c >= N) return;
    const int lv = a.lv, E = a.E, alpha = a.alpha, beta = a.beta;
    const int pid = m < lv ? m : a.L + (m - lv);
    const PrimeDev &P = a.primes[pid];
    const double q = P.q, qi = P.qinv;
    const size_t kstride = (size_t)(a.L + a.K) * N;
    const double *k0 = key + ((size_t)pid << logn) + c;
    const RpPtrs rp = rp_ptrs(a.rp, bi);
    ext += bi * a.sext;
    acc += bi * a.sacc;
    const size_t lm = (size_t)m << logn;
    // products in [0, q), reduced after every fourth digit (sums below 5q < 2^53)
    double a0 = 0.0, a1 = 0.0;
    int pend = 0;
    for (int j = 0; j < beta; ++j) {
        const int j0 = j * alpha;
        const int sz = min(alpha, lv - j0);
        const bool own = m >= j0 && m < j0 + sz;
        const int tt = m < j0 ? m : m - sz;
        const double x = own ? rp_diff(rp.lo + a.rp.ps + lm, rp.hi + a.rp.ps + lm,
                                       galois_src((uint32_t)c, logn, a.rp.galois), rp.t, logn, P)
                             : ext[((size_t)j * E + tt) * N + c];
        a0 += mmul(x, k0[(size_t)(2 * j) * kstride], q, qi);
        a1 += mmul(x, k0[(size_t)(2 * j + 1) * kstride], q, qi);
        if (++pend == 4) {
            a0 = mred(a0, q, qi);
            a1 = mred(a1, q, qi);
            pend = 0;
        }
    }
    acc[lm + c] = mred(a0, q, qi);
    acc[((size_t)(E + m) << logn) + c] = mred(a1, q, qi);
}

// ---- ring repacking, fused (KS_REPACK at N = 2^12 with one ciphertext prime
// and one special prime): one workgroup per entry runs the whole key switch
// with the arithmetic of the step kernels above (the same words): the INTT of
// d = phi_g(c_j - X^t c_(j+t)) over q and its scaling (step 1), the ModUp to p
// and NTT over p (steps 2, 3), and per output polynomial u the product with
// the key's p residue, its INTT and ModDown conversion (steps 3-5), the NTT
// over q and (acc_q - x) P^-1 + base (step 6).  A 4096-point transform is one
// tile of both passes; the passes exchange through one LDS buffer, and the
// NTT_p output, read by both products, through a per-entry global slot (32
// KiB, `scr`).  LDS: the pass exchange area of a 4096-element tile and the
// buffer, 66 KiB, so two groups share a CU; with 512 threads (8 elements per
// thread and register round, half the registers of 256) that is four waves
// per SIMD.
template <int TH>
__global__ __launch_bounds__(TH) void k_repack_fused(const KsArgs a, const double *__restrict__ key,
                                                     double *__restrict__ scr) {
    constexpr int S = 6, C = 64;                 // N = 2^12: 64 x 64 in both passes
    constexpr int N = C << S;
    __shared__ double lds[NttTile<N / kSlots>::lds];   // exchange area of one N-element tile
    __shared__ double buf[N];
    const int bi = blockIdx.x;
    if (bi >= a.nb) return;
    const int logn = a.logn;
    const RpPtrs rp = rp_ptrs(a.rp, bi);
    const PrimeDev &Pq = a.primes[0], &Pp = a.primes[a.L];
    const double q = Pq.q, p = Pp.q;
    const uint32_t g = a.rp.galois, t = rp.t;
    const double *lo0 = rp.lo, *hi0 = rp.hi, *lo1 = rp.lo + a.rp.ps, *hi1 = rp.hi + a.rp.ps;
    const size_t kst = (size_t)(a.L + a.K) * N;          // key: (b, a) of digit 0, L + K limbs each
    double *ext = scr + (size_t)bi * N;
    auto to_buf = [&](int e, double v, int) { buf[e] = v; };
    auto from_buf = [&](int e, int) { return buf[e]; };

    // step 1: INTT over q of d, scaled by (Q'/q)^-1; step 2: ModUp to p
    row_pass<S, true, TH>(Pq, logn, C, 0, lds,
                          [&](int e, int) { return rp_diff(lo1, hi1, galois_src((uint32_t)e, logn, g), t, logn, Pq); },
                          to_buf);
    __syncthreads();
    const double2 inv = a.mu[0].inv[0], hat = a.mu[0].hat[0][a.L];
    col_pass<S, true, TH>(Pq, logn, C, 0, lds, from_buf, [&](int e, double v, int) {
        const double y = mmulc(v, inv.x, inv.y, q);
        buf[e] = mred_signed(mmulc_lazy(y, hat.x, hat.y, p), p, Pp.qinv);
    });
    __syncthreads();
    // step 3: NTT over p
    col_pass<S, false, TH>(Pp, logn, C, 0, lds, from_buf, to_buf);
    __syncthreads();
    row_pass<S, false, TH>(Pp, logn, C, 0, lds, from_buf, [&](int e, double v, int) { ext[e] = v; });
    __syncthreads();
    const double hp = a.md->half[a.L], hq = a.md->half[0];
    const double2 piv = a.md->phat_inv[0], ph = a.md->phat[0][0], pinv = a.md->pinv[0];
#pragma unroll 1
    for (int u = 0; u < 2; ++u) {
        const double *kp = key + (size_t)u * kst + (size_t)a.L * N, *kq = key + (size_t)u * kst;
        // steps 3-5: acc_u over p = ext * key_u, its INTT with floor(P/2) and
        // (P/p)^-1 on the last store, the conversion to q
        row_pass<S, true, TH>(Pp, logn, C, 0, lds, [&](int e, int) { return mmul(ext[e], kp[e], p, Pp.qinv); },
                              to_buf);
        __syncthreads();
        col_pass<S, true, TH>(Pp, logn, C, 0, lds, from_buf, [&](int e, double v, int) {
            const double z = mmulc(madd(v, hp, p), piv.x, piv.y, p);
            buf[e] = mred_signed(-hq + mmulc_lazy(z, ph.x, ph.y, q), q, Pq.qinv);
        });
        __syncthreads();
        // step 6: NTT over q, then (acc_q - x) P^-1 plus c_j + X^t c_(j+t)
        // (and phi_g(c_j - X^t c_(j+t)) for c0), combined after the transform
        // two slots at a time (every slot's gathered operands at once would not
        // fit the registers)
        col_pass<S, false, TH>(Pq, logn, C, 0, lds, from_buf, to_buf);
        __syncthreads();
        row_pass<S, false, TH>(Pq, logn, C, 0, lds, from_buf, to_buf);
        __syncthreads();
        const double *lo = u ? lo1 : lo0, *hi = u ? hi1 : hi0;
        double *out = rp.out + (size_t)u * a.rp.ps;
#pragma unroll 2
        for (int k = 0; k < N / TH; ++k) {
            const uint32_t e = threadIdx.x + k * TH;
            const double xa = mmul(rp_diff(lo1, hi1, galois_src(e, logn, g), t, logn, Pq), kq[e], q, Pq.qinv);
            double xb = madd(lo[e], monomial_mul(hi[e], e, t, logn, Pq), q);
            if (u == 0) xb = madd(xb, rp_diff(lo0, hi0, galois_src(e, logn, g), t, logn, Pq), q);
            out[e] = madd(mmulc(msub(xa, buf[e], q), pinv.x, pinv.y, q), xb, q);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- launchers
// Term count of a conversion kernel: n rounded up to 1, 2, 4 or 8.
#define PFX_SWITCH_NT(n_, CALL)                                          \
    switch ((n_) <= 1 ? 1 : (n_) <= 2 ? 2 : (n_) <= 4 ? 4 : 8) {         \
        case 1: { constexpr int NT = 1; CALL; } break;                  \
        case 2: { constexpr int NT = 2; CALL; } break;                  \
        case 4: { constexpr int NT = 4; CALL; } break;                  \
        default: { constexpr int NT = 8; CALL; } break;                 \
    }

#define PFX_SWITCH_KS(m_, CALL)                                        \
    switch (m_) {                                                      \
        case KS_GALOIS: { constexpr int MD = KS_GALOIS; CALL; } break;  \
        case KS_PRODUCT: { constexpr int MD = KS_PRODUCT; CALL; } break; \
        case KS_REPACK: { constexpr int MD = KS_REPACK; CALL; } break;   \
        default: { constexpr int MD = KS_PLAIN; CALL; } break;          \
    }

static KsArgs ks_args(pfx_ctx *c, int lv, const KsBatch &kb) {
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
    a.nb = kb.nb;
    a.sdc = kb.sdc;
    a.sext = kb.sext;
    a.sacc = kb.sacc;
    a.stmp = kb.stmp;
    a.rp = kb.rp;
    for (int b = 0; b < kMaxBatch; ++b) {
        KsEntry &e = a.op[b];
        if (b < kb.nb && kb.mode != KS_REPACK) {
            const KsOperand &o = kb.op[b];
            e = KsEntry{o.d, o.base0, o.base1, o.a0, o.a1, o.b0, o.b1, kb.out0[b], kb.out1[b], o.galois, kb.keys[b]};
        } else {
            e = KsEntry{};
        }
    }
    return a;
}

static void set_blocks(KsArgs &a, int per) {
    a.per = per;
    a.n = a.nb * per;
}

// Narrower tiles (idle threads) until a launch over `limbs` limbs has at least
// widen_wg workgroups (1024 by default): the transforms of the special-prime
// limbs (2K of them) are too small to fill the chip even with 128-thread
// groups.  Column tiles keep min_col_special columns (8: 64-byte rows).
static void widen_grid(PassShape &pr, PassShape &pc, int limbs, int logn) {
    const PassTuning &tu = pass_tuning(logn);
    while (limbs * pr.tiles < tu.widen_wg && pr.C > 1) { pr.C /= 2; pr.tiles *= 2; }
    while (limbs * pc.tiles < tu.widen_wg && pc.C / 2 >= tu.min_col_special) { pc.C /= 2; pc.tiles *= 2; }
}

void launch_intt_scale(const Launch &L, const KsBatch &kb, int lv) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    double *dcoef = kb.dcoef;
    const int limbs = kb.nb * lv;
    const int th = pass_threads(a.logn, limbs, true), tc = pass_threads(a.logn, limbs, false);
    const PassShape pr = row_shape(a.logn, th * kSlots), pc = col_shape(a.logn, tc * kSlots);
    hipEvent_t ev;
    a.C = pr.C;
    a.tiles = pr.tiles;
    set_blocks(a, lv * a.tiles);
    prof_begin(L, "ks_intt_row", &ev);
    PFX_SWITCH_TH(th, PFX_SWITCH_KS(kb.mode, PFX_SWITCH_S(pr.S, (k_intt_scale<SS, true, MD, TH><<<xcd_grid(a.n), TH, 0,
                                                                                             L.st>>>(a, dcoef)))));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_row", ev, (kb.mode == KS_PRODUCT ? 24.0 : 16.0) * (double)L.ctx->N * limbs);
    a.C = pc.C;
    a.tiles = pc.tiles;
    set_blocks(a, lv * a.tiles);
    prof_begin(L, "ks_intt_col", &ev);
    PFX_SWITCH_TH(tc, PFX_SWITCH_S(pc.S, (k_intt_scale<SS, false, KS_PLAIN, TH><<<xcd_grid(a.n), TH, 0, L.st>>>(
                                              a, dcoef))));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_col", ev, 16.0 * (double)L.ctx->N * limbs);
}

void launch_modup_col(const Launch &L, const KsBatch &kb, int lv) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    const int th = pass_threads(a.logn, kb.nb * (a.beta * a.E - lv), false);
    const PassShape ps = col_shape(a.logn, th * kSlots);
    a.C = ps.C;
    a.tiles = ps.tiles;
    set_blocks(a, (a.beta * a.E - lv) * a.tiles);      // sum over digits of E - sz_j targets
    double *ext = kb.ext;
    const double *dcoef = kb.dcoef;
    hipEvent_t ev;
    prof_begin(L, "ks_modup_col", &ev);
    PFX_SWITCH_TH(th, PFX_SWITCH_NT(a.alpha, PFX_SWITCH_S(ps.S, (k_modup_col<SS, NT, TH><<<xcd_grid(a.n), TH, 0,
                                                                                           L.st>>>(a, ext, dcoef)))));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_modup_col", ev, 8.0 * (double)L.ctx->N * a.beta * a.E * kb.nb);
}

bool row_inner_ok(const pfx_ctx *c, const KsBatch &kb) {
    return pass_tuning(c->logn).ks_fuse != 0 && !kb.hoisted &&
           (kb.mode == KS_PLAIN || kb.mode == KS_GALOIS || kb.mode == KS_PRODUCT);
}

void launch_row_inner(const Launch &L, const KsBatch &kb, const double *key, int lv) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    const int th = pass_tuning(a.logn).ks_fuse == 256 ? 256 : 128;
    const PassShape pr = row_shape(a.logn, th * kSlots);
    a.C = pr.C;
    a.tiles = pr.tiles;
    a.per = a.E * a.tiles;
    a.n = a.nb * a.per;
    hipEvent_t ev;
    prof_begin(L, "ks_row_inner", &ev);
    PFX_SWITCH_TH(th, PFX_SWITCH_KS(kb.mode, PFX_SWITCH_S(pr.S, (k_row_inner<SS, MD == KS_REPACK ? KS_PLAIN : MD, TH>
                                                                 <<<xcd_grid(a.n), TH, 0, L.st>>>(a, kb.ext, key, kb.acc)))));
    HIP_LAUNCH_CHECK_KS();
    // the ModUp limbs and d (a1 and b1 for a product) read, the key read, the
    // accumulators written
    const double own = kb.mode == KS_PRODUCT ? 2.0 * lv : (double)lv;
    const double keys = kb.keys[0] ? kb.nb : 1.0;
    prof_end(L, "ks_row_inner", ev,
             8.0 * (double)L.ctx->N * kb.nb * ((a.beta * a.E - lv) + own + 2.0 * a.E) +
                 16.0 * (double)L.ctx->N * a.beta * a.E * keys);
}

void launch_intt_special(const Launch &L, const KsBatch &kb, int lv, bool col_only) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    double *acc = kb.acc;
    const int limbs = kb.nb * 2 * a.K;
    const int th = pass_threads(a.logn, limbs, true);
    constexpr int tc = 256;
    PassShape pr = row_shape(a.logn, th * kSlots), pc = col_shape(a.logn, tc * kSlots);
    widen_grid(pr, pc, limbs, a.logn);
    hipEvent_t ev;
    if (!col_only) {
        a.C = pr.C;
        a.tiles = pr.tiles;
        set_blocks(a, 2 * a.K * a.tiles);
        prof_begin(L, "ks_intt_special_row", &ev);
        PFX_SWITCH_TH(th, PFX_SWITCH_S(pr.S, (k_intt_special<SS, true, TH><<<xcd_grid(a.n), TH, 0, L.st>>>(a, acc))));
        HIP_LAUNCH_CHECK_KS();
        prof_end(L, "ks_intt_special_row", ev, 16.0 * (double)L.ctx->N * limbs);
    }
    a.C = pc.C;
    a.tiles = pc.tiles;
    set_blocks(a, 2 * a.K * a.tiles);
    prof_begin(L, "ks_intt_special_col", &ev);
    PFX_SWITCH_S(pc.S, (k_intt_special<SS, false, tc><<<xcd_grid(a.n), tc, 0, L.st>>>(a, acc)));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_intt_special_col", ev, 16.0 * (double)L.ctx->N * limbs);
}

void launch_moddown_col(const Launch &L, const KsBatch &kb, int lv) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    const int th = pass_threads(a.logn, kb.nb * 2 * lv, false);
    const PassShape ps = col_shape(a.logn, th * kSlots);
    a.C = ps.C;
    a.tiles = ps.tiles;
    set_blocks(a, 2 * a.tiles * lv);
    double *tmp = kb.tmp;
    const double *acc = kb.acc;
    hipEvent_t ev;
    prof_begin(L, "ks_moddown_col", &ev);
    PFX_SWITCH_TH(th, PFX_SWITCH_NT(a.K, PFX_SWITCH_S(ps.S, (k_moddown_col<SS, NT, TH><<<xcd_grid(a.n), TH, 0,
                                                                                       L.st>>>(a, tmp, acc)))));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_moddown_col", ev, 8.0 * (double)L.ctx->N * (2.0 * a.K + 2.0 * lv) * kb.nb);
}

void launch_row_moddown(const Launch &L, const KsBatch &kb, int lv) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    const int th = pass_threads(a.logn, kb.nb * 2 * lv, true);
    const PassShape ps = row_shape(a.logn, th * kSlots);
    a.C = ps.C;
    a.tiles = ps.tiles;
    set_blocks(a, 2 * lv * a.tiles);
    const double *acc = kb.acc, *tmp = kb.tmp;
    const int nbases = kb.mode == KS_PRODUCT ? 4 : kb.mode == KS_REPACK ? 3
                                                 : (kb.op[0].base0 ? 1 : 0) + (kb.op[0].base1 ? 1 : 0);
    hipEvent_t ev;
    prof_begin(L, "ks_row_moddown", &ev);
    PFX_SWITCH_TH(th, PFX_SWITCH_KS(kb.mode, PFX_SWITCH_S(ps.S, (k_row_moddown<SS, MD, TH><<<xcd_grid(a.n), TH, 0,
                                                                                          L.st>>>(a, acc, tmp)))));
    HIP_LAUNCH_CHECK_KS();
    prof_end(L, "ks_row_moddown", ev, 8.0 * (double)L.ctx->N * lv * (6.0 + nbases) * kb.nb);
}

void launch_ks_inner_repack(const Launch &L, const KsBatch &kb, const double *key, int lv) {
    KsArgs a = ks_args(L.ctx, lv, kb);
    const dim3 grid((unsigned)((L.ctx->N + 255) / 256), (unsigned)(lv + L.ctx->K), (unsigned)kb.nb);
    hipEvent_t ev;
    prof_begin(L, "ks_inner_repack", &ev);
    k_ks_inner_repack<<<grid, 256, 0, L.st>>>(a, key, kb.ext, kb.acc);
    HIP_LAUNCH_CHECK_KS();
    // per entry: ext or the two input limbs, the accumulators and the key residues
    prof_end(L, "ks_inner_repack", ev, 8.0 * (double)L.ctx->N * (lv + L.ctx->K) * (a.beta + 2.0 + 2.0 * a.beta) * kb.nb);
}

bool repack_fused_ok(const pfx_ctx *c, int lv) { return c->logn == 12 && lv == 1 && c->K == 1 && c->alpha == 1; }

void launch_repack_fused(const Launch &L, const KsBatch &kb, const double *key, double *scr) {
    KsArgs a = ks_args(L.ctx, 1, kb);
    a.C = 64;
    a.tiles = 1;
    set_blocks(a, 1);
    hipEvent_t ev;
    prof_begin(L, "repack_fused", &ev);
    k_repack_fused<512><<<kb.nb, 512, 0, L.st>>>(a, key, scr);
    HIP_LAUNCH_CHECK_KS();
    // per entry: c_j and c_(j+t) (4 limbs, read twice), the output (2 limbs),
    // the NTT_p scratch limb written once and read twice; the key (4 limbs) once
    prof_end(L, "repack_fused", ev, 8.0 * (double)L.ctx->N * ((8.0 + 2.0 + 3.0) * kb.nb + 4.0));
}

}  // namespace pfx
