// Host-side parameter generation: primes, 2N-th roots, modular helpers.
//
// The paper fixes only the bit sizes of its moduli (Tab. 1).  The rule here:
// every prime is 1 mod 2^mod_log2 so that a primitive 2N-th root exists for
// every ring degree N <= 2^(mod_log2-1); a 50-bit prime is the next unused
// prime below 2^50, a smaller one the next unused prime nearest 2^bits,
// alternating above and below.  All primes stay below 2^50, which the FP64
// modular arithmetic of the kernels requires.
#include <string>
#include <vector>

#include "internal.h"

namespace pfx {

typedef unsigned __int128 u128;

uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod_u64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod_u64(r, a, m);
        a = mulmod_u64(a, a, m);
    }
    return r;
}

uint64_t invmod_u64(uint64_t a, uint64_t m) {
    // extended Euclid (m need not be prime)
    __int128 t = 0, nt = 1, r = m, nr = a % m;
    while (nr) {
        __int128 qq = r / nr, tmp;
        tmp = t - qq * nt; t = nt; nt = tmp;
        tmp = r - qq * nr; r = nr; nr = tmp;
    }
    if (t < 0) t += m;
    return (uint64_t)t;
}

static bool miller_rabin(uint64_t n) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t b : bases)
        if (n % b == 0) return n == b;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t b : bases) {
        uint64_t x = powmod_u64(b, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod_u64(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

static uint64_t find_root(uint64_t q, uint64_t n) {
    // first g = 2, 3, ... whose power g^((q-1)/2N) has order exactly 2N
    for (uint64_t g = 2;; ++g) {
        uint64_t x = powmod_u64(g, (q - 1) / (2 * n), q);
        if (powmod_u64(x, n, q) == q - 1) return x;
    }
}

bool build_primes(const pfx_params *prm, std::vector<uint64_t> &q, std::vector<uint64_t> &p,
                  std::vector<uint64_t> &psi, std::string &err) {
    if (!prm) { err = "null params"; return false; }
    if (prm->log_n < PFX_MIN_LOGN || prm->log_n > PFX_MAX_LOGN) { err = "log_n out of range"; return false; }
    if (prm->n_q < 1 || prm->n_p < 1 || prm->n_q + prm->n_p > PFX_MAX_PRIMES) {
        err = "need 1..64 primes in total with n_q >= 1 and n_p >= 1";
        return false;
    }
    if (prm->alpha < 1 || prm->alpha > (uint32_t)kMaxAlpha) { err = "alpha must be in [1, 8]"; return false; }
    uint32_t ml = prm->mod_log2 ? prm->mod_log2 : prm->log_n + 1;
    if (ml < prm->log_n + 1 || ml > 40) { err = "mod_log2 must be in [log_n + 1, 40]"; return false; }
    const uint64_t step = 1ull << ml;
    std::vector<uint64_t> all;
    auto used = [&](uint64_t c) {
        for (uint64_t x : all)
            if (x == c) return true;
        return false;
    };
    for (uint32_t t = 0; t < prm->n_q + prm->n_p; ++t) {
        uint32_t b = t < prm->n_q ? prm->q_bits[t] : prm->p_bits[t - prm->n_q];
        if (b < 20 || b > 50) { err = "prime bit sizes must be in [20, 50]"; return false; }
        if (b <= ml + 1) { err = "prime bit size too small for mod_log2"; return false; }
        uint64_t c = 0;
        if (b == 50) {
            for (uint64_t k = 1;; ++k) {
                c = (1ull << b) + 1 - k * step;
                if (!used(c) && miller_rabin(c)) break;
            }
        } else {
            for (uint64_t i = 0;; ++i) {
                int64_t k = (i & 1) ? (int64_t)((i + 1) / 2) : -(int64_t)(i / 2);
                c = (uint64_t)((int64_t)(1ull << b) + 1 + k * (int64_t)step);
                if (!used(c) && miller_rabin(c)) break;
            }
        }
        if (c >= (1ull << 50)) { err = "prime above 2^50"; return false; }
        all.push_back(c);
    }
    q.assign(all.begin(), all.begin() + prm->n_q);
    p.assign(all.begin() + prm->n_q, all.end());
    psi.clear();
    for (uint64_t x : all) psi.push_back(find_root(x, 1ull << prm->log_n));
    return true;
}

}  // namespace pfx
