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
#include "rs_steps.h"

namespace pfx {

template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_intt_row(const RsArgs a, double *__restrict__ last) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    rs_intt_row_body<S, TH>(a, a.C, a.tiles, id, last, lds);
}

template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_intt_col(const RsArgs a, double *__restrict__ last) {
    __shared__ double lds[col_lds<S, TH>()];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    rs_intt_col_body<S, TH>(a, a.C, a.tiles, id, last, lds);
}

template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_col(const RsArgs a, double *__restrict__ tmp,
                                               const double *__restrict__ last) {
    __shared__ double lds[col_lds<S, TH>()];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    rs_col_body<S, TH>(a, a.C, a.tiles, id, tmp, last, lds);
}

template <int S, int TH>
__global__ __launch_bounds__(TH) void k_rs_row(const RsArgs a, const double *__restrict__ tmp) {
    __shared__ double lds[NttTile<TH>::lds];
    const int id = xcd_slot(a.n);
    if (id >= a.n) return;
    rs_row_body<S, TH>(a, a.C, a.tiles, id, tmp, lds);
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
        const PassTuning &tu = pass_tuning(a.logn);
        while (polys * pr.tiles < tu.rs_widen_wg && pr.C > 1) { pr.C /= 2; pr.tiles *= 2; }
        while (polys * pc.tiles < tu.rs_widen_wg && pc.C / 2 >= tu.min_col_special) { pc.C /= 2; pc.tiles *= 2; }
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
