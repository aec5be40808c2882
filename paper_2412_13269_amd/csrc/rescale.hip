// Fused rescale (Sec. 2.5 of the paper): drop the last prime q_l of a
// ciphertext in the NTT domain,
//
//   c'_i = (c_i + h - [c_l + h]_{q_l}) q_l^-1 mod q_i,   h = floor(q_l / 2),
//
// the division of the [0, Q) lift by q_l rounded half up.  h sits on every
// coefficient, so it joins the correction t_i = [c_l + h]_{q_l} - h, which is
// built in the coefficient domain and taken to the NTT domain of q_i:
// c'_i = (c_i - NTT_i(t_i)) q_l^-1.  Four launches over np = degree + 1
// polynomials:
//   1. k_rs_intt_row: first (row) pass of the INTT of each last limb -> last
//   2. k_rs_intt_col: second (column) pass in place, storing [c_l + h]_{q_l}
//   3. k_rs_col:      t_i = [x]_{q_i} - [h]_{q_i} fed straight into the forward
//                     column pass for every i < l                      -> tmp
//   4. k_rs_row:      forward row pass of tmp, then (c_i - v) q_l^-1   -> out
// Nothing between the correction and its NTT, or between the NTT and the
// combination, goes through HBM.
#include "internal.h"
#include "ntt_core.h"

namespace pfx {

// A launch covers nb ciphertexts of one level and degree: polynomial index
// k = entry * np + p runs over all of them; `last` and `tmp` hold every
// polynomial's scratch back to back.
struct RsArgs {
    const PrimeDev *primes;
    const RescaleConst *rc;
    int logn, lv, np;
    int C, tiles, n;
    RsEntry e[kMaxBatch];
};

__device__ __forceinline__ const double *rs_in(const RsArgs &a, int k) {
    const int b = k / a.np;
    return a.e[b].in + (size_t)(k - b * a.np) * a.e[b].si;
}

__device__ __forceinline__ double *rs_out(const RsArgs &a, int k) {
    const int b = k / a.np;
    return a.e[b].out + (size_t)(k - b * a.np) * a.e[b].so;
}

template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_intt_row(const RsArgs a, double *__restrict__ last) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int k = id / a.tiles, tile = id - k * a.tiles;
    const PrimeDev &P = a.primes[a.lv - 1];
    const size_t N = (size_t)1 << a.logn;
    const double *src = rs_in(a, k) + (size_t)(a.lv - 1) * N;
    double *dst = last + (size_t)k * N;
    auto ld = [&](int g, int) { return src[(unsigned)g]; };
    auto st = [&](int g, double v, int) { dst[(unsigned)g] = v; };
    row_pass<S, true, TH>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_intt_col(const RsArgs a, double *__restrict__ last) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int k = id / a.tiles, tile = id - k * a.tiles;
    const PrimeDev &P = a.primes[a.lv - 1];
    const double h = __builtin_floor(P.q * 0.5);
    double *x = last + ((size_t)k << a.logn);
    auto ld = [&](int g, int) { return x[(unsigned)g]; };
    auto st = [&](int g, double v, int) { x[(unsigned)g] = madd(v, h, P.q); };
    col_pass<S, true, TH>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

// blocks: (poly k, tile, prime i), i fastest so that the blocks reading one
// tile of `last` run together
template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_col(const RsArgs a, double *__restrict__ tmp,
                                               const double *__restrict__ last) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int nout = a.lv - 1;
    const int i = id % nout, rest = id / nout;
    const int tile = rest % a.tiles, k = rest / a.tiles;
    const PrimeDev &P = a.primes[i];
    const double half = a.rc[(a.lv - 1) * PFX_MAX_PRIMES + i].half;
    const size_t N = (size_t)1 << a.logn;
    const double *src = last + (size_t)k * N;
    double *dst = tmp + ((size_t)k * nout + i) * N;
    // x < q_l < 2^50: mred takes it to [0, q_i); the difference stays in [0, q_i)
    auto ld = [&](int g, int) { return msub(mred(src[(unsigned)g], P.q, P.qinv), half, P.q); };
    auto st = [&](int g, double v, int) { dst[(unsigned)g] = v; };
    col_pass<S, false, TH>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

// blocks: (poly k, prime i, tile), tile fastest (one twiddle table per run of blocks)
template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_row(const RsArgs a, const double *__restrict__ tmp) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    const int nout = a.lv - 1;
    const int tile = id % a.tiles, rest = id / a.tiles;
    const int i = rest % nout, k = rest / nout;
    const PrimeDev &P = a.primes[i];
    const double2 inv = a.rc[(a.lv - 1) * PFX_MAX_PRIMES + i].inv;
    const size_t N = (size_t)1 << a.logn;
    const double *src = tmp + ((size_t)k * nout + i) * N;
    const double *c = rs_in(a, k) + (size_t)i * N;
    double *o = rs_out(a, k) + (size_t)i * N;
    // c is loaded before the transform (its latency hides under it); slot k of
    // this thread is element tid + k * TH of the tile, the row pass's output
    // order.  out may alias in: each element is read and then written by the
    // same thread.
    const int g0 = (tile * a.C) << S, tot = a.C << S;
    double xc[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int e = threadIdx.x + k * TH;
        xc[k] = e < tot ? c[(unsigned)(g0 + e)] : 0.0;
    }
    auto ld = [&](int g, int) { return src[(unsigned)g]; };
    auto st = [&](int g, double v, int k) { o[(unsigned)g] = mmulc(msub(xc[k], v, P.q), inv.x, inv.y, P.q); };
    row_pass<S, false, TH>(P, a.logn, a.C, tile * a.C, lds, ld, st);
}

#define HIP_LAUNCH_CHECK_RS()                                                                    \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess) set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

void launch_rescale(const Launch &L, const RsEntry *ents, int nb, int np, int lv, double *last, double *tmp) {
    pfx_ctx *c = L.ctx;
    RsArgs a;
    a.primes = c->d_primes;
    a.rc = c->d_rescale;
    a.logn = c->logn;
    a.lv = lv;
    a.np = np;
    for (int b = 0; b < kMaxBatch; ++b) a.e[b] = b < nb ? ents[b] : RsEntry{};
    const double N = (double)c->N;
    const int polys = nb * np;
    hipEvent_t ev;
    // 1-2: INTT of the last limbs (narrow launches)
    {
        const int th = pass_threads(a.logn, polys, true), tc = pass_threads(a.logn, polys, false);
        PassShape pr = row_shape(a.logn, th * kSlots), pc = col_shape(a.logn, tc * kSlots);
        while (polys * pr.tiles < 256 && pr.C > 1) { pr.C /= 2; pr.tiles *= 2; }
        while (polys * pc.tiles < 256 && pc.C / 2 >= 8) { pc.C /= 2; pc.tiles *= 2; }
        a.C = pr.C;
        a.tiles = pr.tiles;
        a.n = polys * pr.tiles;
        prof_begin(L, "rs_intt_row", &ev);
        PFX_SWITCH_TH(th, PFX_SWITCH_S(pr.S, (k_rs_intt_row<SS, TH><<<xcd_grid(a.n), TH, 0, L.st>>>(a, last))));
        HIP_LAUNCH_CHECK_RS();
        prof_end(L, "rs_intt_row", ev, 16.0 * N * polys);
        a.C = pc.C;
        a.tiles = pc.tiles;
        a.n = polys * pc.tiles;
        prof_begin(L, "rs_intt_col", &ev);
        PFX_SWITCH_TH(tc, PFX_SWITCH_S(pc.S, (k_rs_intt_col<SS, TH><<<xcd_grid(a.n), TH, 0, L.st>>>(a, last))));
        HIP_LAUNCH_CHECK_RS();
        prof_end(L, "rs_intt_col", ev, 16.0 * N * polys);
    }
    const int limbs = polys * (lv - 1);
    {
        const int tc = pass_threads(a.logn, limbs, false);
        const PassShape pc = col_shape(a.logn, tc * kSlots);
        a.C = pc.C;
        a.tiles = pc.tiles;
        a.n = limbs * pc.tiles;
        prof_begin(L, "rs_col", &ev);
        PFX_SWITCH_TH(tc, PFX_SWITCH_S(pc.S, (k_rs_col<SS, TH><<<xcd_grid(a.n), TH, 0, L.st>>>(a, tmp, last))));
        HIP_LAUNCH_CHECK_RS();
        prof_end(L, "rs_col", ev, 8.0 * N * (polys + limbs));
    }
    {
        const int th = pass_threads(a.logn, limbs, true);
        const PassShape pr = row_shape(a.logn, th * kSlots);
        a.C = pr.C;
        a.tiles = pr.tiles;
        a.n = limbs * pr.tiles;
        prof_begin(L, "rs_row", &ev);
        PFX_SWITCH_TH(th, PFX_SWITCH_S(pr.S, (k_rs_row<SS, TH><<<xcd_grid(a.n), TH, 0, L.st>>>(a, tmp))));
        HIP_LAUNCH_CHECK_RS();
        prof_end(L, "rs_row", ev, 24.0 * N * limbs);
    }
}

}  // namespace pfx
