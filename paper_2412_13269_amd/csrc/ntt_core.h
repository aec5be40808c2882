// Device building blocks of the negacyclic NTT (gfx950).
//
// Order: NTT(a)[j] = a(psi^(2 bitrev(j) + 1)).  Stage s (0 <= s < log N)
// pairs index j with j + N/2^(s+1); its twiddle is tw[2^s + (j >> (log N - s))]
// with tw[k] = psi^bitrev(k) (forward, Cooley-Tukey butterfly) or
// psi^-bitrev(k) (inverse, Gentleman-Sande butterfly).
//
// A limb of N = 2^16 doubles (512 KiB) does not fit one CU's LDS, so a
// transform is two passes over the limb:
//   column pass: global stages [0, S_col), sub-transforms of stride
//                2^(log N - S_col); a tile is C consecutive columns, so every
//                row of the tile is C contiguous doubles;
//   row pass:    global stages [S_col, log N), contiguous blocks of
//                2^S_row; a tile is C consecutive blocks.
// Inside a pass the S stages run as two register rounds (R1 = ceil(S/2), then
// R2 = S - R1 stages) with one LDS exchange between them.  The first round
// reads its operands through a caller-supplied `load(global_index, slot)`
// and the last round hands results to `store(global_index, value, slot)`,
// so a pass can be fused with what produces its input (a basis conversion)
// or consumes its output (a key inner product).  `slot` in [0, 16) numbers
// the elements a thread owns in that round; for a full tile of 4096 elements
// and 256 threads it is a compile-time index, so per-element accumulators of a
// fused consumer stay in registers.
//
// Element/thread layouts (chosen for coalesced global access):
//   column pass: thread group (c, m') with c fastest; row r of the tile is C
//                consecutive doubles, read/written by consecutive threads;
//   row pass, forward round 1 / inverse round B: (c, m_lo) with m_lo fastest
//                (consecutive threads touch consecutive doubles);
//   row pass, forward output / inverse input: through LDS, element e of the
//                tile to thread e mod 256 (consecutive threads, consecutive
//                doubles).
#pragma once
#include "internal.h"
#include "modarith.h"

namespace pfx {

// A workgroup of TH threads (256 or 128) works on a tile of TH * kSlots
// elements, kSlots per thread in each register round, through an LDS buffer of
// the tile plus 1/16 padding.  Launches over few limbs take 128-thread groups
// so that they still spread over every CU.
constexpr int kNttThreads = 256;
constexpr int kSlots = 16;                       // elements per thread per round
constexpr int kNttTile = kNttThreads * kSlots;
template <int TH>
struct NttTile {
    static constexpr int n = TH * kSlots;
    static constexpr int lds = n + n / 16;
};
constexpr int kNttLds = NttTile<kNttThreads>::lds;
// When both rounds of a column pass are one kSlots-point group per thread
// (2^S = kSlots^2), the pass exchanges its tile through LDS in two halves
// (rows below 2^(S-1), then the rest): a block that runs only column passes
// needs half a tile of LDS, so twice as many blocks fit on a CU.
template <int S>
constexpr bool col_half_exchange() { return (1 << ((S + 1) / 2)) == kSlots && (1 << (S / 2)) == kSlots; }
template <int S, int TH>
constexpr int col_lds() { return col_half_exchange<S>() ? NttTile<TH>::n / 2 : NttTile<TH>::lds; }

// Twiddle tables live in device global memory; their pointers are read from
// the PrimeDev records, so without this the compiler would emit generic (flat)
// loads for them.
typedef const __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ const gdouble *as_global(const double *p) { return (const gdouble *)p; }
// A table of (w, fl(w/q)) pairs in global memory.
struct GTw {
    const gdouble *p;
    __device__ __forceinline__ double2 operator[](int i) const { return make_double2(p[2 * i], p[2 * i + 1]); }
};
__device__ __forceinline__ GTw as_global(const double2 *p) { return GTw{(const gdouble *)p}; }

// Automorphism phi_g: X -> X^g (g odd) in the NTT domain.  Slot j holds
// a(psi^e) with e = 2 bitrev(j) + 1, and phi_g(a)(psi^e) = a(psi^(g e)), so
// phi_g(a)[j] = a[galois_src(j)] with 2 bitrev(galois_src(j)) + 1 = g e mod 2N.
__device__ __forceinline__ uint32_t galois_src(uint32_t j, int logn, uint32_t g) {
    const uint32_t e = 2u * (__brev(j) >> (32 - logn)) + 1u;
    const uint32_t e2 = (e * g) & ((2u << logn) - 1u);
    return __brev((e2 - 1u) >> 1) >> (32 - logn);
}

// Product with the monomial X^k in the NTT domain: slot j holds a(psi^e),
// e = 2 bitrev(j) + 1, so (X^k a)[j] = psi^(k e) a[j].  The exponent is taken
// mod 2N; psi^E comes from the bit-reversed table (tw[bitrev(E)] = psi^E for
// E < N) and is negated for E >= N (psi^N = -1).
__device__ __forceinline__ double monomial_mul(double x, uint32_t j, uint32_t k, int logn, const PrimeDev &P) {
    const uint32_t N = 1u << logn;
    const uint32_t ej = 2u * (__brev(j) >> (32 - logn)) + 1u;
    const uint32_t E = (uint32_t)(((uint64_t)k * ej) & (2ull * N - 1));
    const double2 w = P.tw[__brev(E & (N - 1)) >> (32 - logn)];
    const double r = mmulc(x, w.x, w.y, P.q);
    return (E >= N && r != 0.0) ? P.q - r : r;
}

// Arithmetic inside a transform is signed and lazy: a twiddle product returns
// a representative in [-q, q] (mmulc_lazy), sums and differences are left
// unreduced, and values are brought back to [-q/2, q/2] (mred_signed) often
// enough that every lazy product's input stays within 2^51.  Wide primes
// (2^47 <= q < 2^50, inputs |x| <= q): after every second forward stage (two
// stages take |x| <= 0.51q to at most 2.75q) and after every inverse stage's
// sum (sums and differences stay below 2q).  Narrow primes (q < 2^47, the
// `narrow` flag, uniform per launch tile): only at the end of a register group
// of at most 4 stages: forward values grow by at most 1.25q per stage (|x| <=
// q + 5q), inverse sums double per stage (at most 16q, differences 16q <
// 2^51).  Every intermediate is an integer below 2^52 in magnitude, so each
// step is exact.  Group outputs are reduced to [-q/2, q/2]; the last pass of a
// transform canonicalises to [0, q).
constexpr double kNarrowPrime = 140737488355328.0;   // 2^47

// Forward butterflies of NST consecutive stages on the E = 2^NST elements of
// one register group.  At stage kk of the group the butterflies come in 2^kk
// runs x = u >> (NST - kk) that share one twiddle; twf(kk, x) returns it (w,
// fl(w/q)), each exactly once per group.  The pass code below gives twf in
// closed form (for the first round of a column pass the index is a
// compile-time constant, so the twiddles are uniform scalar loads).
template <int NST, class Twf>
__device__ __forceinline__ void fwd_group(double *v, double q, double qinv, bool narrow, Twf &&twf) {
    constexpr int E = 1 << NST;
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int h = 1 << (NST - 1 - kk);
#pragma unroll
        for (int x = 0; x < (1 << kk); ++x) {
            const double2 w = twf(kk, x);
#pragma unroll
            for (int lo = 0; lo < h; ++lo) {
                const int u = (x << (NST - kk)) | lo;
                const double T = mmulc_lazy(v[u + h], w.x, w.y, q);
                const double U = v[u];
                v[u] = U + T;
                v[u + h] = U - T;
            }
        }
        if (kk == NST - 1 || ((kk & 1) && !narrow)) {
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = mred_signed(v[u], q, qinv);
        }
    }
}

// The sums of inverse group stage kk (the lower element of each pair) back to
// [-q/2, q/2]; called behind a uniform branch, so narrow primes skip it.
template <int NST>
__device__ __forceinline__ void inv_reduce_sums(double *v, int kk, double q, double qinv) {
    const int h = 1 << (NST - 1 - kk);
#pragma unroll
    for (int u = 0; u < (1 << NST); ++u)
        if (!(u & h)) v[u] = mred_signed(v[u], q, qinv);
}

// Inverse butterflies, group stages NST - 1 down to 0 (twiddles as above).
// With `last` the group's stage 0 is global stage 0 and N^-1 is folded into it.
template <int NST, class Twf>
__device__ __forceinline__ void inv_group(double *v, const PrimeDev &P, bool last, bool narrow, Twf &&twf) {
    constexpr int E = 1 << NST;
    const double q = P.q, qinv = P.qinv;
#pragma unroll
    for (int kk = NST - 1; kk >= 0; --kk) {
        const int h = 1 << (NST - 1 - kk);
#pragma unroll
        for (int x = 0; x < (1 << kk); ++x) {
            double2 w = make_double2(0.0, 0.0);
            if (!(last && kk == 0)) w = twf(kk, x);
#pragma unroll
            for (int lo = 0; lo < h; ++lo) {
                const int u = (x << (NST - kk)) | lo;
                const double U = v[u], V = v[u + h];
                if (last && kk == 0) {
                    v[u] = mmulc_lazy(U + V, P.ninv, P.ninv_q, q);
                    v[u + h] = mmulc_lazy(U - V, P.ninv_w1, P.ninv_w1_q, q);
                } else {
                    v[u] = U + V;
                    v[u + h] = mmulc_lazy(U - V, w.x, w.y, q);
                }
            }
        }
        if (!narrow && !(last && kk == 0)) inv_reduce_sums<NST>(v, kk, q, qinv);
    }
#pragma unroll
    for (int u = 0; u < E; ++u) v[u] = mred_signed(v[u], q, qinv);
}

// The last R2 stages of the row pass with twiddles generated in registers
// instead of read from the 2^logn-entry table (which would cost as many bytes
// as the data).  For the thread's group j = (P << R2) | u the stage-(T + k)
// twiddle is rc[2^k - 1 + x] * B_k, x = u >> (R2 - k), with B_{R2-1} =
// rtw[P] and B_{k-1} = B_k^2: 2^R2 - 1 + R2 - 1 modular products per group,
// each left signed in (-q, q) (mmul_lazy: |w| <= 0.875 q; the bases stay below
// q in magnitude, which is all the next square needs).  Generated twiddles
// come with wq = fl(w * fl(1/q)), so a lazy product with one is within 1.25 q
// (|a| <= 2^51) or 0.875 q (|a| <= q); the two-stage growth stays below
// 3.2 q < 2^52, the narrow-prime growth over a group below 6 q.
template <int NST>
__device__ __forceinline__ void row_twiddle_bases(double *B, double top, double q, double qinv) {
    B[NST - 1] = top;
#pragma unroll
    for (int k = NST - 1; k > 0; --k) B[k - 1] = mmul_lazy(B[k], B[k], q, qinv);
}

template <int NST>
__device__ __forceinline__ void fwd_group_gen(double *v, const double *B, const double *rc, double q, double qinv,
                                              bool narrow) {
    constexpr int E = 1 << NST;
#pragma unroll
    for (int kk = 0; kk < NST; ++kk) {
        const int h = 1 << (NST - 1 - kk);
#pragma unroll
        for (int x = 0; x < (1 << kk); ++x) {
            const double w = mmul_lazy(rc[(1 << kk) - 1 + x], B[kk], q, qinv);
            const double wq = w * qinv;
#pragma unroll
            for (int lo = 0; lo < h; ++lo) {
                const int u = (x << (NST - kk)) | lo;
                const double T = mmulc_lazy(v[u + h], w, wq, q);
                const double U = v[u];
                v[u] = U + T;
                v[u + h] = U - T;
            }
        }
        if (kk == NST - 1 || ((kk & 1) && !narrow)) {
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = mred_signed(v[u], q, qinv);
        }
    }
}

template <int NST>
__device__ __forceinline__ void inv_group_gen(double *v, const double *B, const double *rc, double q, double qinv,
                                              bool narrow) {
    constexpr int E = 1 << NST;
#pragma unroll
    for (int kk = NST - 1; kk >= 0; --kk) {
        const int h = 1 << (NST - 1 - kk);
#pragma unroll
        for (int x = 0; x < (1 << kk); ++x) {
            const double w = mmul_lazy(rc[(1 << kk) - 1 + x], B[kk], q, qinv);
            const double wq = w * qinv;
#pragma unroll
            for (int lo = 0; lo < h; ++lo) {
                const int u = (x << (NST - kk)) | lo;
                const double U = v[u], V = v[u + h];
                v[u] = U + V;
                v[u + h] = mmulc_lazy(U - V, w, wq, q);
            }
        }
        if (!narrow) inv_reduce_sums<NST>(v, kk, q, qinv);
    }
#pragma unroll
    for (int u = 0; u < E; ++u) v[u] = mred_signed(v[u], q, qinv);
}

// Column pass: global stages [0, S) on the tile of columns [cbase, cbase + C),
// run by TH threads.
// Inputs |x| <= q.  Forward: the first pass of a transform, outputs in
// [-q/2, q/2] for the row pass.  Inverse: the last pass, outputs in [0, q).
template <int S, bool INV, int TH, class Load, class Store>
__device__ __forceinline__ void col_pass(const PrimeDev &P, int logn, int C, int cbase, double *lds, Load &&load,
                                         Store &&store) {
    constexpr int R1 = (S + 1) / 2, R2 = S - R1, E1 = 1 << R1, E2 = 1 << R2;
    constexpr int IT1 = kSlots / E1, IT2 = kSlots / E2;
    const int lo = logn - S;
    const double q = P.q;
    const bool narrow = q < kNarrowPrime;
    const GTw tw = as_global(INV ? P.itw : P.tw);
    const int n1 = C << (S - R1), n2 = C << R1;
    auto gidx = [&](int c, int mid) { return (mid << lo) | (cbase + c); };
    if constexpr (col_half_exchange<S>()) {
        // One group per thread in each round (E1 = E2 = kSlots).  Round-1
        // group g = (c, m) holds rows (u << R2) | m and round-2 group g holds
        // rows (m << R2) | u, so the exchange splits on the row's top bit: u
        // below H in the first half, m below H reads only the first half.
        // LDS rows are local to the half (C * 2^(S-1) doubles).
        constexpr int H = kSlots / 2;
        constexpr int NTW = E1 * (E2 - 1);   // round-2 table twiddles, staged in LDS
        __shared__ double2 twl[NTW];
        const int g = threadIdx.x, c = g % C, m = g / C;
        const bool on1 = g < n1, on2 = g < n2;
        auto lrow1 = [&](int u) { return ((u & (H - 1)) << (S - R1)) | m; };   // round-1 slot u, local row
        auto lrow2 = [&](int u) { return ((m & (H - 1)) << R2) | u; };         // round-2 slot u, local row
        double v[kSlots], w[kSlots];
        if (!INV) {
            if (on1) {
#pragma unroll
                for (int u = 0; u < kSlots; ++u) v[u] = load(gidx(c, (u << (S - R1)) | m), u);
            }
            for (int t = g; t < NTW; t += TH) {
                const int mh = t / (E2 - 1), j = t - mh * (E2 - 1);
                const int kk = 31 - __clz(j + 1), x = j + 1 - (1 << kk);
                twl[t] = tw[(1 << (R1 + kk)) + ((mh << kk) | x)];
            }
            if (on1) {
                fwd_group<R1>(v, q, P.qinv, narrow, [&](int kk, int x) { return tw[(1 << kk) + x]; });
#pragma unroll
                for (int u = 0; u < H; ++u) lds[lrow1(u) * C + c] = v[u];
            }
            __syncthreads();
            if (on2 && m < H) {
#pragma unroll
                for (int u = 0; u < kSlots; ++u) w[u] = lds[lrow2(u) * C + c];
            }
            __syncthreads();
            if (on1) {
#pragma unroll
                for (int u = H; u < kSlots; ++u) lds[lrow1(u) * C + c] = v[u];
            }
            __syncthreads();
            if (on2) {
                if (m >= H) {
#pragma unroll
                    for (int u = 0; u < kSlots; ++u) w[u] = lds[lrow2(u) * C + c];
                }
                fwd_group<R2>(w, q, P.qinv, narrow,
                              [&](int kk, int x) { return twl[m * (E2 - 1) + (1 << kk) - 1 + x]; });
#pragma unroll
                for (int u = 0; u < kSlots; ++u) store(gidx(c, (m << R2) | u), w[u], u);
            }
        } else {
            if (on2) {
#pragma unroll
                for (int u = 0; u < kSlots; ++u) v[u] = load(gidx(c, (m << R2) | u), u);
            }
            for (int t = g; t < NTW; t += TH) {
                const int m2 = t / (E2 - 1), j = t - m2 * (E2 - 1);
                const int kk = 31 - __clz(j + 1), x = j + 1 - (1 << kk);
                twl[t] = tw[(1 << (R1 + kk)) + ((m2 << kk) | x)];
            }
            __syncthreads();
            if (on2) {
                inv_group<R2>(v, P, false, narrow, [&](int kk, int x) { return twl[m * (E2 - 1) + (1 << kk) - 1 + x]; });
                if (m < H) {
#pragma unroll
                    for (int u = 0; u < kSlots; ++u) lds[lrow2(u) * C + c] = v[u];
                }
            }
            __syncthreads();
            if (on1) {
#pragma unroll
                for (int u = 0; u < H; ++u) w[u] = lds[lrow1(u) * C + c];
            }
            __syncthreads();
            if (on2 && m >= H) {
#pragma unroll
                for (int u = 0; u < kSlots; ++u) lds[lrow2(u) * C + c] = v[u];
            }
            __syncthreads();
            if (on1) {
#pragma unroll
                for (int u = H; u < kSlots; ++u) w[u] = lds[lrow1(u) * C + c];
                inv_group<R1>(w, P, true, narrow, [&](int kk, int x) { return tw[(1 << kk) + x]; });
#pragma unroll
                for (int u = 0; u < kSlots; ++u) store(gidx(c, (u << (S - R1)) | m), mcanon(w[u], q), u);
            }
        }
    } else {
        if (!INV) {
            // The second round's table twiddles depend only on mh (E1 groups of
            // E2 - 1): staged once per block in LDS, one load per thread, and read
            // there (16 lanes of a wave share each) instead of 2^R2 - 1 vector
            // loads per thread after the barrier.
            constexpr int NTW = E1 * (E2 - 1);
            constexpr bool STAGE = IT2 == 1 && NTW <= TH;
            __shared__ double2 twl[STAGE ? NTW : 1];
            if (STAGE && (int)threadIdx.x < NTW) {
                const int t = threadIdx.x, mh = t / (E2 - 1), j = t - mh * (E2 - 1);
                const int kk = 31 - __clz(j + 1), x = j + 1 - (1 << kk);
                twl[t] = tw[(1 << (R1 + kk)) + ((mh << kk) | x)];
            }
#pragma unroll
            for (int gi = 0; gi < IT1; ++gi) {
                const int g = threadIdx.x + gi * TH;
                if (g < n1) {
                    const int c = g % C, ml = g / C;
                    auto gu = [&](int u) { return gidx(c, (u << (S - R1)) | ml); };
                    double v[E1];
#pragma unroll
                    for (int u = 0; u < E1; ++u) v[u] = load(gu(u), gi * E1 + u);
                    // stage kk < R1: index 2^kk + (mid >> (S - kk)) = 2^kk + x (ml shifts out)
                    fwd_group<R1>(v, q, P.qinv, narrow, [&](int kk, int x) { return tw[(1 << kk) + x]; });
#pragma unroll
                    for (int u = 0; u < E1; ++u) lds[((u << (S - R1)) | ml) * C + c] = v[u];
                }
            }
            __syncthreads();
#pragma unroll
            for (int gi = 0; gi < IT2; ++gi) {
                const int g = threadIdx.x + gi * TH;
                if (g < n2) {
                    const int c = g % C, mh = g / C;
                    auto gu = [&](int u) { return gidx(c, (mh << R2) | u); };
                    double v[E2];
#pragma unroll
                    for (int u = 0; u < E2; ++u) v[u] = lds[((mh << R2) | u) * C + c];
                    // stage R1 + kk: mid >> (R2 - kk) = (mh << kk) | x
                    fwd_group<R2>(v, q, P.qinv, narrow, [&](int kk, int x) {
                        return STAGE ? twl[mh * (E2 - 1) + (1 << kk) - 1 + x] : tw[(1 << (R1 + kk)) + ((mh << kk) | x)];
                    });
#pragma unroll
                    for (int u = 0; u < E2; ++u) store(gu(u), v[u], gi * E2 + u);
                }
            }
        } else {
            // the first round's table twiddles, staged in LDS as in the forward
            // pass's second round (data loads first, one barrier for both)
            constexpr int NTW = E1 * (E2 - 1);
            constexpr bool STAGE = IT2 == 1 && NTW <= TH;
            if constexpr (STAGE) {
                __shared__ double2 twl[NTW];
                const int g = threadIdx.x;
                const bool on = g < n2;
                const int c = g % C, mh = g / C;
                auto gu = [&](int u) { return gidx(c, (mh << R2) | u); };
                double v[E2];
                if (on) {
#pragma unroll
                    for (int u = 0; u < E2; ++u) v[u] = load(gu(u), u);
                }
                if (g < NTW) {
                    const int m2 = g / (E2 - 1), j = g - m2 * (E2 - 1);
                    const int kk = 31 - __clz(j + 1), x = j + 1 - (1 << kk);
                    twl[g] = tw[(1 << (R1 + kk)) + ((m2 << kk) | x)];
                }
                __syncthreads();
                if (on) {
                    inv_group<R2>(v, P, false, narrow, [&](int kk, int x) { return twl[mh * (E2 - 1) + (1 << kk) - 1 + x]; });
#pragma unroll
                    for (int u = 0; u < E2; ++u) lds[((mh << R2) | u) * C + c] = v[u];
                }
            } else {
#pragma unroll
                for (int gi = 0; gi < IT2; ++gi) {
                    const int g = threadIdx.x + gi * TH;
                    if (g < n2) {
                        const int c = g % C, mh = g / C;
                        auto gu = [&](int u) { return gidx(c, (mh << R2) | u); };
                        double v[E2];
#pragma unroll
                        for (int u = 0; u < E2; ++u) v[u] = load(gu(u), gi * E2 + u);
                        inv_group<R2>(v, P, false, narrow,
                                      [&](int kk, int x) { return tw[(1 << (R1 + kk)) + ((mh << kk) | x)]; });
#pragma unroll
                        for (int u = 0; u < E2; ++u) lds[((mh << R2) | u) * C + c] = v[u];
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int gi = 0; gi < IT1; ++gi) {
                const int g = threadIdx.x + gi * TH;
                if (g < n1) {
                    const int c = g % C, ml = g / C;
                    auto gu = [&](int u) { return gidx(c, (u << (S - R1)) | ml); };
                    double v[E1];
#pragma unroll
                    for (int u = 0; u < E1; ++u) v[u] = lds[((u << (S - R1)) | ml) * C + c];
                    inv_group<R1>(v, P, true, narrow, [&](int kk, int x) { return tw[(1 << kk) + x]; });
#pragma unroll
                    for (int u = 0; u < E1; ++u) store(gu(u), mcanon(v[u], q), gi * E1 + u);
                }
            }
        }
    }
}

// Row pass: global stages [logn - S, logn) on the tile of blocks [cbase, cbase + C).
// Inputs |x| <= q.  Forward: the last pass, outputs in [0, q) (in [-q/2, q/2]
// with CANON = false, for a consumer that reduces anyway).  Inverse: the first
// pass, outputs in [-q/2, q/2] for the column pass.
// The tile is C * 2^S contiguous doubles; the side of the pass that would own
// 2^R2 consecutive doubles per thread (forward output, inverse input) goes
// through LDS in coalesced order instead: element e of the tile belongs to
// thread e mod TH as slot e / TH.
template <int S, bool INV, int TH, bool CANON = true, class Load, class Store>
__device__ __forceinline__ void row_pass(const PrimeDev &P, int logn, int C, int cbase, double *lds, Load &&load,
                                         Store &&store) {
    constexpr int R = 1 << S;
    constexpr int R1 = (S + 1) / 2, R2 = S - R1, E1 = 1 << R1, E2 = 1 << R2;
    constexpr int IT1 = kSlots / E1, IT2 = kSlots / E2;
    constexpr int PAD = R + R / 16;
    const int s0 = logn - S;
    const double q = P.q;
    const bool narrow = q < kNarrowPrime;
    const GTw tw = as_global(INV ? P.itw : P.tw);
    const int n1 = C << (S - R1), n2 = C << R1;
    const int tot = C * R;
    const int base = cbase << S;
    auto gidx = [&](int c, int mid) { return ((cbase + c) << S) | mid; };
    auto lidx = [&](int c, int mid) { return c * PAD + mid + (mid >> 4); };
    // Twiddle operands of the rounds after the first barrier are loaded before
    // it when each thread owns one group per round (IT == 1, the 2^16 shape),
    // so that their latency hides under the first round.
    const gdouble *rt = as_global(INV ? P.irtw : P.rtw);
    double rtop = 0.0;
    if (IT2 == 1 && (int)threadIdx.x < n2) rtop = rt[((cbase + ((int)threadIdx.x >> R1)) << R1) | ((int)threadIdx.x & (E1 - 1))];
    if (!INV) {
        // The first round's table twiddles depend only on the row c of the
        // tile (C groups of E1 - 1): when each thread owns one group they are
        // staged once per block in LDS, one load per thread, and read there
        // (the lanes of one row share them) instead of 2^R1 - 1 vector loads
        // per thread.
        constexpr int NTW = (kSlots * TH >> S) * (E1 - 1);
        constexpr bool STAGE = IT1 == 1 && NTW <= TH;
        if constexpr (STAGE) {
            // one group per thread: its data loads go out first, then the
            // block's twiddle loads, and one barrier covers both
            __shared__ double2 twl[NTW];
            const int g = threadIdx.x;
            const bool on = g < n1;
            const int ml = g & ((1 << (S - R1)) - 1), c = g >> (S - R1);
            auto gu = [&](int u) { return gidx(c, (u << (S - R1)) | ml); };
            double v[E1];
            if (on) {
#pragma unroll
                for (int u = 0; u < E1; ++u) v[u] = load(gu(u), u);
            }
            if (g < C * (E1 - 1)) {
                const int cc = g / (E1 - 1), j = g - cc * (E1 - 1);
                const int kk = 31 - __clz(j + 1), x = j + 1 - (1 << kk);
                twl[g] = tw[(1 << (s0 + kk)) + (((cbase + cc) << kk) | x)];
            }
            __syncthreads();
            if (on) {
                fwd_group<R1>(v, q, P.qinv, narrow, [&](int kk, int x) { return twl[c * (E1 - 1) + (1 << kk) - 1 + x]; });
#pragma unroll
                for (int u = 0; u < E1; ++u) lds[lidx(c, (u << (S - R1)) | ml)] = v[u];
            }
        } else {
#pragma unroll
            for (int gi = 0; gi < IT1; ++gi) {
                const int g = threadIdx.x + gi * TH;
                if (g < n1) {
                    const int ml = g & ((1 << (S - R1)) - 1), c = g >> (S - R1);
                    auto gu = [&](int u) { return gidx(c, (u << (S - R1)) | ml); };
                    double v[E1];
#pragma unroll
                    for (int u = 0; u < E1; ++u) v[u] = load(gu(u), gi * E1 + u);
                    // stage s0 + kk: gidx >> (S - kk) = ((cbase + c) << kk) | x
                    fwd_group<R1>(v, q, P.qinv, narrow,
                                  [&](int kk, int x) { return tw[(1 << (s0 + kk)) + (((cbase + c) << kk) | x)]; });
#pragma unroll
                    for (int u = 0; u < E1; ++u) lds[lidx(c, (u << (S - R1)) | ml)] = v[u];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int gi = 0; gi < IT2; ++gi) {
            const int g = threadIdx.x + gi * TH;
            if (g < n2) {
                const int mh = g & (E1 - 1), c = g >> R1;
                double v[E2], B[R2];
#pragma unroll
                for (int u = 0; u < E2; ++u) v[u] = lds[lidx(c, (mh << R2) | u)];
                row_twiddle_bases<R2>(B, IT2 == 1 ? rtop : rt[((cbase + c) << R1) | mh], q, P.qinv);
                fwd_group_gen<R2>(v, B, P.rc, q, P.qinv, narrow);
#pragma unroll
                for (int u = 0; u < E2; ++u) lds[lidx(c, (mh << R2) | u)] = v[u];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int e = threadIdx.x + k * TH;
            if (e < tot) {
                const double x = lds[lidx(e >> S, e & (R - 1))];
                store(base + e, CANON ? mcanon(x, q) : x, k);
            }
        }
    } else {
        // the second round's table twiddles (C groups of E1 - 1, by row),
        // staged in LDS before the first barrier when each thread owns one
        // group there
        constexpr int NTW = (kSlots * TH >> S) * (E1 - 1);
        constexpr bool STAGE = IT1 == 1 && NTW <= TH;
        __shared__ double2 twl[STAGE ? NTW : 1];
        if (STAGE && (int)threadIdx.x < C * (E1 - 1)) {
            const int t = threadIdx.x, cc = t / (E1 - 1), j = t - cc * (E1 - 1);
            const int kk = 31 - __clz(j + 1), x = j + 1 - (1 << kk);
            twl[t] = tw[(1 << (s0 + kk)) + (((cbase + cc) << kk) | x)];
        }
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int e = threadIdx.x + k * TH;
            if (e < tot) lds[lidx(e >> S, e & (R - 1))] = load(base + e, k);
        }
        __syncthreads();
#pragma unroll
        for (int gi = 0; gi < IT2; ++gi) {
            const int g = threadIdx.x + gi * TH;
            if (g < n2) {
                const int mh = g & (E1 - 1), c = g >> R1;
                double v[E2], B[R2];
#pragma unroll
                for (int u = 0; u < E2; ++u) v[u] = lds[lidx(c, (mh << R2) | u)];
                row_twiddle_bases<R2>(B, IT2 == 1 ? rtop : rt[((cbase + c) << R1) | mh], q, P.qinv);
                inv_group_gen<R2>(v, B, P.irc, q, P.qinv, narrow);
#pragma unroll
                for (int u = 0; u < E2; ++u) lds[lidx(c, (mh << R2) | u)] = v[u];
            }
        }
        __syncthreads();
#pragma unroll
        for (int gi = 0; gi < IT1; ++gi) {
            const int g = threadIdx.x + gi * TH;
            if (g < n1) {
                const int ml = g & ((1 << (S - R1)) - 1), c = g >> (S - R1);
                auto gu = [&](int u) { return gidx(c, (u << (S - R1)) | ml); };
                double v[E1];
#pragma unroll
                for (int u = 0; u < E1; ++u) v[u] = lds[lidx(c, (u << (S - R1)) | ml)];
                inv_group<R1>(v, P, false, narrow, [&](int kk, int x) {
                    return STAGE ? twl[c * (E1 - 1) + (1 << kk) - 1 + x]
                                 : tw[(1 << (s0 + kk)) + (((cbase + c) << kk) | x)];
                });
#pragma unroll
                for (int u = 0; u < E1; ++u) store(gu(u), v[u], gi * E1 + u);
            }
        }
    }
}

// Pass geometry shared by host launchers and kernels.
struct PassShape {
    int S;       // stages in the pass
    int C;       // sub-transforms per tile
    int tiles;   // tiles per limb
};

inline PassShape col_shape(int logn, int tile = kNttTile) {
    PassShape p;
    p.S = logn / 2;
    const int subs = 1 << (logn - p.S);
    p.C = std::min(tile >> p.S, subs);
    p.tiles = subs / p.C;
    return p;
}

inline PassShape row_shape(int logn, int tile = kNttTile) {
    PassShape p;
    p.S = logn - logn / 2;
    const int subs = 1 << (logn - p.S);
    p.C = std::min(tile >> p.S, subs);
    p.tiles = subs / p.C;
    return p;
}

// Workgroup size of a pass launch over `limbs` limbs (PassTuning).

inline int pass_threads(int logn, int limbs, bool row) {
    const PassTuning &t = pass_tuning(logn);
    return limbs * col_shape(logn).tiles >= (row ? t.row_wg256 : t.col_wg256) ? 256 : 128;
}

// Stages of a pass (log N / 2 or the rest) as a compile-time constant SS.
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

#define PFX_SWITCH_TH(th_, CALL)                                   \
    switch (th_) {                                                 \
        case 128: { constexpr int TH = 128; CALL; } break;         \
        default: { constexpr int TH = 256; CALL; } break;          \
    }

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8).  xcd_slot() turns the hardware id into a logical id such that
// each XCD works through a contiguous range of logical ids, so logical
// neighbours (tiles of one limb, targets of one digit) share that XCD's L2.
// The grid is padded to a multiple of 8; ids >= `n` exit.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_slot(int n) {
    const int per = (n + kXcds - 1) / kXcds;
    const int b = blockIdx.x;
    return (b % kXcds) * per + b / kXcds;
}

inline unsigned xcd_grid(int n) { return (unsigned)(((n + kXcds - 1) / kXcds) * kXcds); }

}  // namespace pfx
