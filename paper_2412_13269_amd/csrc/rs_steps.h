// Device bodies of the fused rescale (Sec. 2.5 of the paper) shared by the
// per-step kernels of rescale.hip and the persistent batched kernel of
// persist.hip.  Each body runs one logical block (tile) `id` of its step, with
// the pass geometry C, tiles and the caller's LDS exchange area.
#pragma once
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
__device__ __forceinline__ void rs_intt_row_body(const RsArgs &a, int C, int tiles, int id,
                                                 double *__restrict__ last, double *lds) {
    const int k = id / tiles, tile = id - k * tiles;
    const PrimeDev &P = a.primes[a.lv - 1];
    const size_t N = (size_t)1 << a.logn;
    const double *src = rs_in(a, k) + (size_t)(a.lv - 1) * N;
    double *dst = last + (size_t)k * N;
    auto ld = [&](int g, int) { return src[(unsigned)g]; };
    auto st = [&](int g, double v, int) { dst[(unsigned)g] = v; };
    row_pass<S, true, TH>(P, a.logn, C, tile * C, lds, ld, st);
}

template <int S, int TH>
__device__ __forceinline__ void rs_intt_col_body(const RsArgs &a, int C, int tiles, int id,
                                                 double *__restrict__ last, double *lds) {
    const int k = id / tiles, tile = id - k * tiles;
    const PrimeDev &P = a.primes[a.lv - 1];
    const double h = __builtin_floor(P.q * 0.5);
    double *x = last + ((size_t)k << a.logn);
    auto ld = [&](int g, int) { return x[(unsigned)g]; };
    auto st = [&](int g, double v, int) { x[(unsigned)g] = madd(v, h, P.q); };
    col_pass<S, true, TH>(P, a.logn, C, tile * C, lds, ld, st);
}

// blocks: (poly k, tile, prime i), i fastest so that the blocks reading one
// tile of `last` run together
template <int S, int TH>
__device__ __forceinline__ void rs_col_body(const RsArgs &a, int C, int tiles, int id,
                                            double *__restrict__ tmp, const double *__restrict__ last, double *lds) {
    const int nout = a.lv - 1;
    const int i = id % nout, rest = id / nout;
    const int tile = rest % tiles, k = rest / tiles;
    const PrimeDev &P = a.primes[i];
    const double half = a.rc[(a.lv - 1) * PFX_MAX_PRIMES + i].half;
    const size_t N = (size_t)1 << a.logn;
    const double *src = last + (size_t)k * N;
    double *dst = tmp + ((size_t)k * nout + i) * N;
    // x < q_l < 2^50: mred takes it to [0, q_i); the difference stays in [0, q_i)
    auto ld = [&](int g, int) { return msub(mred(src[(unsigned)g], P.q, P.qinv), half, P.q); };
    auto st = [&](int g, double v, int) { dst[(unsigned)g] = v; };
    col_pass<S, false, TH>(P, a.logn, C, tile * C, lds, ld, st);
}

// blocks: (poly k, prime i, tile), tile fastest (one twiddle table per run of blocks)
template <int S, int TH>
__device__ __forceinline__ void rs_row_body(const RsArgs &a, int C, int tiles, int id,
                                            const double *__restrict__ tmp, double *lds) {
    const int nout = a.lv - 1;
    const int tile = id % tiles, rest = id / tiles;
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
    const int g0 = (tile * C) << S, tot = C << S;
    double xc[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int e = threadIdx.x + k * TH;
        xc[k] = e < tot ? c[(unsigned)(g0 + e)] : 0.0;
    }
    auto ld = [&](int g, int) { return src[(unsigned)g]; };
    auto st = [&](int g, double v, int k) { o[(unsigned)g] = mmulc(msub(xc[k], v, P.q), inv.x, inv.y, P.q); };
    row_pass<S, false, TH>(P, a.logn, C, tile * C, lds, ld, st);
}

}  // namespace pfx
