// HMult + relinearisation that allocates nothing: the key-switch scratch lives
// in a fixed device array of this file instead of the stream's workspace, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array is a device symbol: in host code its name is only a stand-in, so
// its device address is taken once per device (noalloc_init, called by
// pfx_ctx_create with that device current) and only that address is used.
// Every call on one device shares the array: calls that overlap on one GPU
// (two streams, two threads) race on it and must be ordered by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "internal.h"

namespace pfx {

// 64 MiB: one key switch at N = 2^14 and 24 + 4 primes (4.85 Mi doubles, 6.03
// Mi with room for the tensor product of an aliased output).
constexpr size_t kNoAllocDoubles = (size_t)8 << 20;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};   // device address of `scratch` per device, once taken

}  // namespace

// Takes the device address of `scratch` on `device` (the current device) once.
pfx_status noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(PFX_EDEVICE, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return PFX_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(PFX_EDEVICE, std::string("no-allocation scratch: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_ptr[device] = static_cast<double *>(p);
    return PFX_OK;
}

}  // namespace pfx

using namespace pfx;

extern "C" {

size_t pfx_noalloc_scratch_bytes(void) { return kNoAllocDoubles * sizeof(double); }

pfx_status pfx_mul_relin_noalloc(pfx_ctx *c, const pfx_ct *a, const pfx_ct *b, const pfx_swk *rlk, pfx_ct *out,
                                 void *stream) {
    pfx_status r = mul_relin_check(c, a, b, rlk, out);
    if (r) return r;
    if (c->prof_on) return fail(PFX_EINVAL, "the library's profiler creates events: disable it for this call");
    double *base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (c->device >= 0 && c->device < kMaxDevices) base = g_ptr[c->device];
    }
    if (!base) return fail(PFX_EDEVICE, "no-allocation scratch was not set up on this device");
    // regions for this level: d's coefficients, the ModUp limbs, the two
    // accumulators over Q and P, the ModDown temporary, and a tensor product
    // when the output aliases an operand
    const size_t N = c->N;
    const size_t lv = std::min(a->n_limbs, b->n_limbs);
    const size_t E = lv + c->K, beta = (lv + c->alpha - 1) / c->alpha;
    const bool alias = out->d == a->d || out->d == b->d;
    const size_t need = N * (lv + beta * E + 2 * E + 2 * lv + (alias ? 3 * lv : 0));
    if (need > kNoAllocDoubles)
        return fail(PFX_ENOMEM, "no-allocation scratch holds " + std::to_string(kNoAllocDoubles * 8) +
                                    " bytes; this product needs " + std::to_string(need * 8));
    KsScratch s;
    s.dcoef = base;
    s.ext = s.dcoef + lv * N;
    s.acc = s.ext + beta * E * N;
    s.tmp = s.acc + 2 * E * N;
    s.t3 = s.tmp + 2 * lv * N;
    s.t3_stride = lv * N;
    if (hipSetDevice(c->device) != hipSuccess) return fail(PFX_EDEVICE, "hipSetDevice failed");
    mul_relin_run(c, a, b, rlk, out, (hipStream_t)stream, s);
    return PFX_OK;
}

}  // extern "C"
