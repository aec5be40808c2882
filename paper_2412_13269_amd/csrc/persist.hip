// Batched HMult + relinearisation + rescale of ciphertexts of uneven ring
// degree and level in ONE persistent launch (the batched form of the key
// switch, Sec. 2.4.1, and rescale, Sec. 2.5).
//
// The work of every entry is cut into the thirteen steps of the per-entry path
// (INTT of d = a1 b1 in two passes, the ModUp conversion into the column pass,
// the row pass of the ModUp limbs, the inner product with the relinearisation
// key, the INTT of the special-prime limbs in two passes, the ModDown
// conversion into the column pass, the row pass with the combination into the
// output, and the four rescale steps) and each step into tiles, as the step
// kernels cut them.  A cooperative grid of as many workgroups as fit on the
// device at once walks the steps in order: within a step the tiles of all
// entries (any ring degree, any level) are dealt to the workgroups, each
// tile running the same device body as the step kernel, then the grid meets
// at a barrier before the next step.  No step waits for a launch, and a step
// of a small entry shares the device with the same step of every other entry.
//
// Tiles are dealt XCD by XCD: the tiles of a step are split into eight
// contiguous ranges, and the workgroups of one XCD (hardware id mod 8) walk one
// range, so neighbouring tiles (one limb, one ModUp digit) share that XCD's L2.
//
// The barrier waits are bounded: a workgroup that has waited past the limit
// sets the error word and leaves, and so do the others after it; the host
// reports PFX_EDEVICE.  With a cooperative launch every workgroup is resident,
// so the limit is never reached in a correct run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.h"
#include "ks_steps.h"
#include "ntt_core.h"
#include "rs_steps.h"

namespace pfx {

constexpr int kPersistThreads = 256;
constexpr int kPersistSteps = 13;
constexpr int kMaxStepEntries = 1024;   // entries per step-major launch (owner table in LDS)

// One entry: its key switch (KsArgs with one batch entry, KS_PRODUCT), its
// rescale (RsArgs of the output, in place), key and scratch, pass geometry.
struct PersistEntry {
    KsArgs ks;
    RsArgs rs;
    const double *key;
    double *dcoef, *ext, *acc, *tmp;    // key-switch scratch (one entry of each region)
    double *rs_last, *rs_tmp;
    int s_col, s_row;           // stages of the column and row passes
    int c_col, t_col, c_row, t_row;
};

struct PersistCtl {
    unsigned count, gen, err, pad;
};

struct PersistArgs {
    const PersistEntry *ents;
    const int *prefix;          // [step][n + 1] tile offsets of the entries
    PersistCtl *ctl;
    int n;
};

__device__ __forceinline__ bool grid_barrier(PersistCtl *ctl, unsigned nblocks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned g = __hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = atomicAdd(&ctl->count, 1u);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins > (1u << 24) ||
                    __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __threadfence();
    }
    __syncthreads();
    return __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// The entry that owns tile t of a step (prefix[0] = 0, prefix[n] = all tiles).
__device__ __forceinline__ int owner(const int *prefix, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Row pass of one ModUp limb of one entry in place (the step after the ModUp
// conversion): limb k of the entry's ext limbs, digit j first, target t next.
template <int S>
__device__ __forceinline__ void ext_row_body(const KsArgs &a, double *ext, int C, int tiles, int id, double *lds) {
    const int k = id / tiles, tile = id - k * tiles;
    const int Tf = a.E - a.alpha;
    int j, t;
    if (k < (a.beta - 1) * Tf) {
        j = k / Tf;
        t = k - j * Tf;
    } else {
        j = a.beta - 1;
        t = k - (a.beta - 1) * Tf;
    }
    const int j0 = j * a.alpha, sz = min(a.alpha, a.lv - j0);
    const PrimeDev &P = a.primes[ks_ext_prime(t, j0, sz, a.lv, a.L)];
    double *x = ext + (((size_t)j * a.E + t) << a.logn);
    auto ld = [&](int g, int) { return x[(unsigned)g]; };
    auto st = [&](int g, double v, int) { x[(unsigned)g] = v; };
    row_pass<S, false, kPersistThreads>(P, a.logn, C, tile * C, lds, ld, st);
}

// Inner product of one entry (KS_PRODUCT): limb m, kInnerPer coefficients per
// tile (each thread kInnerPer / 256 of them, 256 apart, all their loads of a
// digit in flight together).  Products in [0, q) summed exactly (below 5q <
// 2^53) and reduced every four digits: the canonical sum, as the
// inner-product kernel forms it.
constexpr int kInnerVec = 8;
constexpr int kInnerPer = kPersistThreads * kInnerVec;

__device__ __forceinline__ void inner_body(const KsArgs &a, const double *__restrict__ key,
                                           const double *__restrict__ ext, double *__restrict__ acc, int id) {
    const int logn = a.logn;
    const size_t N = (size_t)1 << logn;
    const int per = (int)(N / kInnerPer);
    const int m = id / per;
    const size_t c0 = (size_t)(id - m * per) * kInnerPer + threadIdx.x;
    const int lv = a.lv, E = a.E, alpha = a.alpha, beta = a.beta;
    const int pid = m < lv ? m : a.L + (m - lv);
    const double q = a.primes[pid].q, qi = a.primes[pid].qinv;
    const size_t kstride = (size_t)(a.L + a.K) * N;
    const double *k0 = key + ((size_t)pid << logn) + c0;
    const size_t lm = (size_t)m << logn;
    const KsEntry &en = a.op[0];
    double a0[kInnerVec], a1[kInnerVec];
#pragma unroll
    for (int v = 0; v < kInnerVec; ++v) a0[v] = a1[v] = 0.0;
    int pend = 0;
    for (int j = 0; j < beta; ++j) {
        const int j0 = j * alpha, sz = min(alpha, lv - j0);
        const bool own = m >= j0 && m < j0 + sz;
        const int tt = m < j0 ? m : m - sz;
        const double *x0 = ext + ((size_t)j * E + tt) * N + c0;
        double w0[kInnerVec], w1[kInnerVec], x[kInnerVec];
#pragma unroll
        for (int v = 0; v < kInnerVec; ++v) {
            const size_t o = (size_t)v * kPersistThreads;
            w0[v] = __builtin_nontemporal_load(k0 + (size_t)(2 * j) * kstride + o);
            w1[v] = __builtin_nontemporal_load(k0 + (size_t)(2 * j + 1) * kstride + o);
            x[v] = own ? mmul(en.a1[lm + c0 + o], en.b1[lm + c0 + o], q, qi) : __builtin_nontemporal_load(x0 + o);
        }
#pragma unroll
        for (int v = 0; v < kInnerVec; ++v) {
            a0[v] += mmul(x[v], w0[v], q, qi);
            a1[v] += mmul(x[v], w1[v], q, qi);
        }
        if (++pend == 4) {
#pragma unroll
            for (int v = 0; v < kInnerVec; ++v) {
                a0[v] = mred(a0[v], q, qi);
                a1[v] = mred(a1[v], q, qi);
            }
            pend = 0;
        }
    }
#pragma unroll
    for (int v = 0; v < kInnerVec; ++v) {
        const size_t c = c0 + (size_t)v * kPersistThreads;
        acc[lm + c] = mred(a0[v], q, qi);
        acc[((size_t)(E + m) << logn) + c] = mred(a1[v], q, qi);
    }
}

template <int S>
__device__ __forceinline__ bool run_col(int step, const PersistEntry &pe, int id, double *lds) {
    constexpr int TH = kPersistThreads;
    const KsArgs &a = pe.ks;
    switch (step) {
        case 1: intt_scale_body<S, false, KS_PLAIN, TH>(a, pe.c_col, pe.t_col, 0, id, pe.dcoef, lds); return true;
        case 2: modup_col_body<S, 4, TH>(a, pe.c_col, pe.t_col, 0, id, pe.ext, pe.dcoef, lds); return true;
        case 6: intt_special_body<S, false, TH>(a, pe.c_col, pe.t_col, 0, id, pe.acc, lds); return true;
        case 7: moddown_col_body<S, 4, TH>(a, pe.c_col, pe.t_col, 0, id, pe.tmp, pe.acc, lds); return true;
        case 10: rs_intt_col_body<S, TH>(pe.rs, pe.c_col, pe.t_col, id, pe.rs_last, lds); return true;
        case 11: rs_col_body<S, TH>(pe.rs, pe.c_col, pe.t_col, id, pe.rs_tmp, pe.rs_last, lds); return true;
        default: return false;
    }
}

template <int S>
__device__ __forceinline__ bool run_row(int step, const PersistEntry &pe, int id, double *lds) {
    constexpr int TH = kPersistThreads;
    const KsArgs &a = pe.ks;
    switch (step) {
        case 0: intt_scale_body<S, true, KS_PRODUCT, TH>(a, pe.c_row, pe.t_row, 0, id, pe.dcoef, lds); return true;
        case 3: ext_row_body<S>(a, pe.ext, pe.c_row, pe.t_row, id, lds); return true;
        case 5: intt_special_body<S, true, TH>(a, pe.c_row, pe.t_row, 0, id, pe.acc, lds); return true;
        case 8: row_moddown_body<S, KS_PRODUCT, TH, false>(a, pe.c_row, pe.t_row, 0, id, pe.acc, pe.tmp, lds); return true;
        case 9: rs_intt_row_body<S, TH>(pe.rs, pe.c_row, pe.t_row, id, pe.rs_last, lds); return true;
        case 12: rs_row_body<S, TH>(pe.rs, pe.c_row, pe.t_row, id, pe.rs_tmp, lds); return true;
        default: return false;
    }
}

// Steps 0, 3, 5, 8, 9, 12 are row passes, 1, 2, 6, 7, 10, 11 column passes, 4
// the inner product.
__device__ __forceinline__ void run_tile(int step, const PersistEntry &pe, int id, double *lds) {
    if (step == 4) {
        inner_body(pe.ks, pe.key, pe.ext, pe.acc, id);
        return;
    }
    const bool row = step == 0 || step == 3 || step == 5 || step == 8 || step == 9 || step == 12;
    const int S = row ? pe.s_row : pe.s_col;
    if (row) {
        if (S == 6) run_row<6>(step, pe, id, lds);
        else if (S == 7) run_row<7>(step, pe, id, lds);
        else run_row<8>(step, pe, id, lds);
    } else {
        if (S == 6) run_col<6>(step, pe, id, lds);
        else if (S == 7) run_col<7>(step, pe, id, lds);
        else run_col<8>(step, pe, id, lds);
    }
}

__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_persistent(const PersistArgs p) {
    __shared__ double lds[NttTile<kPersistThreads>::lds];
    const unsigned nblocks = gridDim.x;
    const int per_xcd = (int)nblocks / kXcds;           // the grid is a multiple of 8
    const int xcd = (int)blockIdx.x % kXcds, lane = (int)blockIdx.x / kXcds;
    for (int step = 0; step < kPersistSteps; ++step) {
        const int *pre = p.prefix + (size_t)step * (p.n + 1);
        const int total = pre[p.n];
        const int range = (total + kXcds - 1) / kXcds;
        const int t0 = xcd * range, t1 = min(total, t0 + range);
        // tiles come in increasing order: the owning entry is found once and
        // then advanced
        int e = -1, e_lo = 0, e_hi = 0;
        for (int t = t0 + lane; t < t1; t += per_xcd) {
            if (e < 0) {
                e = owner(pre, p.n, t);
                e_lo = pre[e];
                e_hi = pre[e + 1];
            }
            while (t >= e_hi) {
                ++e;
                e_lo = e_hi;
                e_hi = pre[e + 1];
            }
            run_tile(step, p.ents[e], t - e_lo, lds);
            __syncthreads();            // the next tile reuses the exchange area
        }
        if (step + 1 < kPersistSteps && !grid_barrier(p.ctl, nblocks)) return;
    }
}

// Step-major form of the same batch: one launch per step over the tiles of
// every entry (one workgroup per tile, grid remapped by XCD as the step
// kernels are), so each step's body gets the registers and occupancy it needs
// on its own; the steps follow in stream order.  The entries' tile offsets of
// the step are staged in LDS for the owner search.
template <int STEP>
__global__ __launch_bounds__(kPersistThreads) void k_batch_step(const PersistArgs p, int total) {
    __shared__ double lds[NttTile<kPersistThreads>::lds];
    __shared__ int pre[kMaxStepEntries + 1];
    const int t = xcd_slot(total);
    if (t >= total) return;
    const int *src = p.prefix + (size_t)STEP * (p.n + 1);
    for (int i = threadIdx.x; i <= p.n; i += kPersistThreads) pre[i] = src[i];
    __syncthreads();
    const int e = owner(pre, p.n, t);
    run_tile(STEP, p.ents[e], t - pre[e], lds);
}

// ------------------------------------------------------------------ host
namespace {

struct PersistCache {
    int grid = 0;
};

}  // namespace

bool persist_shape_ok(const pfx_ctx *c) { return c->logn >= 12 && c->logn <= 16 && c->alpha <= 4 && c->K <= 4; }

size_t persist_entry_doubles(const pfx_ctx *c, int lv) {
    const size_t N = c->N, E = (size_t)lv + c->K, beta = (size_t)(lv + c->alpha - 1) / c->alpha;
    // dcoef, ext, acc, ModDown tmp, rescale last and tmp
    return N * ((size_t)lv + beta * E + 2 * E + 2 * (size_t)lv + 2 + 2 * (size_t)(lv - 1));
}

size_t persist_tail_bytes(size_t n) {
    return n * sizeof(PersistEntry) + (size_t)kPersistSteps * (n + 1) * sizeof(int) + 64 + sizeof(PersistCtl);
}

// Tiles of each step for one entry (see run_tile).
static void step_tiles(const PersistEntry &pe, int out[kPersistSteps]) {
    const KsArgs &a = pe.ks;
    const int lv = a.lv, ext_limbs = a.beta * a.E - lv;
    const int inner = (a.lv + a.K) * ((1 << a.logn) / kInnerPer);
    const int counts[kPersistSteps] = {lv * pe.t_row,        lv * pe.t_col,        ext_limbs * pe.t_col,
                                       ext_limbs * pe.t_row, inner,                2 * a.K * pe.t_row,
                                       2 * a.K * pe.t_col,   2 * lv * pe.t_col,    2 * lv * pe.t_row,
                                       2 * pe.t_row,         2 * pe.t_col,         2 * (lv - 1) * pe.t_col,
                                       2 * (lv - 1) * pe.t_row};
    std::memcpy(out, counts, sizeof counts);
}

pfx_status launch_batch_persistent(pfx_ctx *const *ctxs, const pfx_ct *const *a, const pfx_ct *const *b,
                                   const pfx_swk *const *rlk, pfx_ct *const *out, const std::vector<size_t> &idx,
                                   double *region, size_t region_doubles, hipStream_t st, bool step_major) {
    const int n = (int)idx.size();
    if (n == 0) return PFX_OK;
    if (step_major && n > kMaxStepEntries) return fail(PFX_EINVAL, "too many entries for one step-major batch");
    std::vector<PersistEntry> ents(n);
    std::vector<int> prefix((size_t)kPersistSteps * (n + 1), 0);
    double *next = region;
    for (int e = 0; e < n; ++e) {
        const size_t i = idx[e];
        pfx_ctx *c = ctxs[i];
        const int lv = (int)std::min(a[i]->n_limbs, b[i]->n_limbs);
        PersistEntry &pe = ents[e];
        std::memset(&pe, 0, sizeof pe);
        KsArgs &k = pe.ks;
        k.primes = c->d_primes;
        k.mu = c->d_modup;
        k.md = c->d_moddown;
        k.logn = c->logn;
        k.lv = lv;
        k.L = c->L;
        k.K = c->K;
        k.alpha = c->alpha;
        k.beta = (lv + c->alpha - 1) / c->alpha;
        k.E = lv + c->K;
        k.nb = 1;
        k.op[0] = KsEntry{nullptr, nullptr, nullptr, a[i]->poly(0), a[i]->poly(1), b[i]->poly(0), b[i]->poly(1),
                          out[i]->poly(0), out[i]->poly(1), 0};
        const size_t N = c->N, E = (size_t)k.E;
        pe.dcoef = next;
        pe.ext = pe.dcoef + (size_t)lv * N;
        pe.acc = pe.ext + (size_t)k.beta * E * N;
        pe.tmp = pe.acc + 2 * E * N;
        pe.rs_last = pe.tmp + 2 * (size_t)lv * N;
        pe.rs_tmp = pe.rs_last + 2 * N;
        next = pe.rs_tmp + 2 * (size_t)(lv - 1) * N;
        if ((size_t)(next - region) > region_doubles) return fail(PFX_EINVAL, "persistent batch region too small");
        RsArgs &r = pe.rs;
        r.primes = c->d_primes;
        r.rc = c->d_rescale;
        r.logn = c->logn;
        r.lv = lv;
        r.np = 2;
        r.e[0] = RsEntry{out[i]->d, out[i]->d, (size_t)out[i]->cap_limbs * N, (size_t)out[i]->cap_limbs * N};
        pe.key = rlk[i]->d_k;
        const PassShape pr = row_shape(c->logn, kPersistThreads * kSlots), pc = col_shape(c->logn, kPersistThreads * kSlots);
        pe.s_row = pr.S;
        pe.c_row = pr.C;
        pe.t_row = pr.tiles;
        pe.s_col = pc.S;
        pe.c_col = pc.C;
        pe.t_col = pc.tiles;
        int cnt[kPersistSteps];
        step_tiles(pe, cnt);
        for (int s = 0; s < kPersistSteps; ++s) prefix[(size_t)s * (n + 1) + e + 1] = prefix[(size_t)s * (n + 1) + e] + cnt[s];
    }
    // descriptors, offsets and the barrier words after the entries' scratch
    // (8-byte aligned: PersistEntry holds doubles and pointers)
    char *tail = reinterpret_cast<char *>(next);
    const size_t ebytes = ents.size() * sizeof(PersistEntry), pbytes = prefix.size() * sizeof(int);
    const size_t need = (size_t)(tail - reinterpret_cast<char *>(region)) + ebytes + pbytes + 64 + sizeof(PersistCtl);
    if (need > region_doubles * sizeof(double)) return fail(PFX_EINVAL, "persistent batch region too small");
    PersistEntry *d_ents = reinterpret_cast<PersistEntry *>(tail);
    int *d_prefix = reinterpret_cast<int *>(tail + ebytes);
    PersistCtl *d_ctl = reinterpret_cast<PersistCtl *>(
        (reinterpret_cast<uintptr_t>(tail + ebytes + pbytes) + 63) & ~(uintptr_t)63);
    if (hipMemcpyAsync(d_ents, ents.data(), ebytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_prefix, prefix.data(), pbytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(d_ctl, 0, sizeof(PersistCtl), st) != hipSuccess)
        return fail(PFX_EDEVICE, "persistent batch: descriptor upload failed");
    Launch L{ctxs[idx[0]], st};
    hipEvent_t ev;
    PersistArgs pa;
    pa.ents = d_ents;
    pa.prefix = d_prefix;
    pa.ctl = d_ctl;
    pa.n = n;
    if (step_major) {
        prof_begin(L, "batch_steps", &ev);
        auto launch = [&](auto kern, int step) {
            const int total = prefix[(size_t)step * (n + 1) + n];
            if (total) kern<<<xcd_grid(total), kPersistThreads, 0, st>>>(pa, total);
        };
        launch(k_batch_step<0>, 0);
        launch(k_batch_step<1>, 1);
        launch(k_batch_step<2>, 2);
        launch(k_batch_step<3>, 3);
        launch(k_batch_step<4>, 4);
        launch(k_batch_step<5>, 5);
        launch(k_batch_step<6>, 6);
        launch(k_batch_step<7>, 7);
        launch(k_batch_step<8>, 8);
        launch(k_batch_step<9>, 9);
        launch(k_batch_step<10>, 10);
        launch(k_batch_step<11>, 11);
        launch(k_batch_step<12>, 12);
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess) return fail(PFX_EDEVICE, std::string("step-major batch launch: ") + hipGetErrorString(le));
        prof_end(L, "batch_steps", ev, 0.0);
    } else {
        static PersistCache cache;
        if (!cache.grid) {
            int per_cu = 0, dev = 0;
            hipDeviceProp_t prop;
            if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent, kPersistThreads, 0) !=
                    hipSuccess || per_cu < 1)
                return fail(PFX_EDEVICE, "persistent batch: occupancy query failed");
            cache.grid = (per_cu * prop.multiProcessorCount) / kXcds * kXcds;
        }
        void *args[] = {&pa};
        prof_begin(L, "batch_persistent", &ev);
        const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_batch_persistent),
                                                        dim3((unsigned)cache.grid), dim3(kPersistThreads), args, 0, st);
        if (e != hipSuccess) return fail(PFX_EDEVICE, std::string("persistent batch launch: ") + hipGetErrorString(e));
        prof_end(L, "batch_persistent", ev, 0.0);
    }
    unsigned err = 0;
    if (hipMemcpyAsync(&err, &d_ctl->err, sizeof err, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(PFX_EDEVICE, "persistent batch: synchronisation failed");
    if (err) return fail(PFX_EDEVICE, "persistent batch: a grid barrier timed out");
    for (int e2 = 0; e2 < n; ++e2) {
        const size_t i = idx[e2];
        out[i]->n_limbs = (uint32_t)(ents[e2].ks.lv - 1);
        out[i]->degree = 1;
        out[i]->scale = a[i]->scale * b[i]->scale / (double)ctxs[i]->primes[ents[e2].ks.lv - 1];
    }
    return PFX_OK;
}

}  // namespace pfx
