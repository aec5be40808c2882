// Group sums of the BSGS plaintext-matrix product (App. A.4): for one giant
// step j the terms phi_g(d_k) (.) rot(z, i_k) are summed in one pass, each
// thread owning one coefficient of one limb and reading every term's residue
// there, instead of a plaintext automorphism and a product launch per term.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "linear.h"
#include "modarith.h"
#include "ntt_core.h"

namespace pfx {

// Block: kGroups term groups x 64 coefficients.  Group u sums the terms
// t = u, u + kGroups, ... for its lane's coefficient; the partial sums meet in
// LDS and group 0 writes.  Splitting the terms gives a launch kGroups times the
// waves of one thread per coefficient, which at N = 2^12 would leave most SIMDs
// without a second wave to hide the loads' latency.
constexpr int kGroups = 4;

__global__ void __launch_bounds__(256) k_diag_mac(double *out, size_t so, const MacTerms m, int n_terms, int nl,
                                                  int logn, uint32_t g, int accumulate, const PrimeDev *pr) {
    __shared__ double part[2][kGroups - 1][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const size_t idx = blockIdx.x * (size_t)64 + lane;
    const bool live = idx < ((size_t)nl << logn);
    double s0 = 0.0, s1 = 0.0;
    double q = 1.0;
    if (live) {
        const uint32_t x = (uint32_t)(idx & ((1u << logn) - 1));
        const size_t row = idx - x;                   // i N
        const int i = (int)(idx >> logn);
        q = pr[i].q;
        const double qi = pr[i].qinv;
        const uint32_t src = g == 1 ? x : galois_src(x, logn, g);
        if (grp == 0 && accumulate) {
            s0 = out[idx];
            s1 = out[so + idx];
        }
        for (int t = grp; t < n_terms; t += kGroups) {
            const double w = m.pt[t][row + src];
            const double *c = m.ct[t];
            s0 = madd(s0, mmul(c[idx], w, q, qi), q);
            s1 = madd(s1, mmul(c[m.cs[t] + idx], w, q, qi), q);
        }
    }
    if (grp > 0) {
        part[0][grp - 1][lane] = s0;
        part[1][grp - 1][lane] = s1;
    }
    __syncthreads();
    if (grp == 0 && live) {
#pragma unroll
        for (int u = 0; u < kGroups - 1; ++u) {
            s0 = madd(s0, part[0][u][lane], q);
            s1 = madd(s1, part[1][u][lane], q);
        }
        out[idx] = s0;
        out[so + idx] = s1;
    }
}

void launch_diag_mac(const Launch &L, double *out, size_t so, const MacTerms &m, int n_terms, int nl, uint32_t g,
                     bool accumulate) {
    const size_t total = (size_t)nl << L.ctx->logn;
    hipEvent_t ev;
    prof_begin(L, "diag_mac", &ev);
    const unsigned blocks = (unsigned)((total + 63) / 64);
    k_diag_mac<<<blocks, 64 * kGroups, 0, L.st>>>(out, so, m, n_terms, nl, L.ctx->logn, g, accumulate ? 1 : 0,
                                                  L.ctx->d_primes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) set_error(std::string("kernel launch: ") + hipGetErrorString(e));
    prof_end(L, "diag_mac", ev, 8.0 * (double)total * (3.0 * n_terms + (accumulate ? 4.0 : 2.0)));
}

}  // namespace pfx
