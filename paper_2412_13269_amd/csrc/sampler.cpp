// Seeded sampling of the scheme's random inputs (host side of the scientist's
// calls): the secret key, the uniform polynomials a and the errors e of key
// generation and encryption (Sec. 2.3, Sec. 2.4.1).  The paper fixes no
// generator; every draw here comes from a SHAKE-256 stream (FIPS 202) keyed by
// seed (32 bytes) || tag || index || limb (little-endian uint32 each):
//   uniform below m: 8-byte little-endian words masked to bitlen(m - 1) bits,
//     rejected while >= m;
//   uniform ternary: bytes b, v = b & 3 rejected while 3, 0/1/2 -> 0/+1/-1;
//   h-sparse ternary: positions 0..N-1; for i < h swap entry i with entry
//     i + u, u uniform below N - i; then one byte per chosen position, in
//     order, bit 0 the sign (0: +1, 1: -1);
//   discrete Gaussian, sigma 3.2, |e| <= 19: cumulative table T[k] =
//     floor(2^63 P(|X| <= k)) for k < 19 (weights exp(-k^2 / 2 sigma^2),
//     doubled for k > 0, summed in order in FP64), T[19] = 2^63; u = word >> 1,
//     |e| the least k with u < T[k], and for |e| > 0 a sign byte (bit 0).
// Tags: 1 secret, 2 switching-key a (index 256 g + digit, limb = prime index
// over Q then P), 3 its error (index as a), 4 encryption a (limb = prime
// index), 5 encryption error.
//
// Keccak-f[1600] below is written from FIPS 202: the round constants come
// from the rc(t) linear-feedback shift register and the rotation offsets from
// the (x, y) -> (y, 2x + 3y) walk, both computed at first use.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace pfx {
namespace {

struct KeccakTables {
    uint64_t rc[24];
    int rot[5][5];
    KeccakTables() {
        // rc(t): the output bit of an 8-bit LFSR (FIPS 202, Algorithm 5)
        auto rcbit = [](int t) -> int {
            if (t % 255 == 0) return 1;
            unsigned R = 1;                 // R[0] is bit 0
            for (int i = 1; i <= t % 255; ++i) {
                R <<= 1;                    // R = 0 || R
                const unsigned r8 = (R >> 8) & 1u;
                R ^= r8 | (r8 << 4) | (r8 << 5) | (r8 << 6);
                R &= 0xffu;
            }
            return (int)(R & 1u);
        };
        for (int ir = 0; ir < 24; ++ir) {
            uint64_t v = 0;
            for (int j = 0; j <= 6; ++j)
                if (rcbit(j + 7 * ir)) v |= 1ull << ((1 << j) - 1);
            rc[ir] = v;
        }
        std::memset(rot, 0, sizeof rot);
        int x = 1, y = 0;
        for (int t = 0; t < 24; ++t) {
            rot[x][y] = ((t + 1) * (t + 2) / 2) % 64;
            const int nx = y, ny = (2 * x + 3 * y) % 5;
            x = nx;
            y = ny;
        }
    }
};

const KeccakTables &ktab() {
    static const KeccakTables t;
    return t;
}

inline uint64_t rotl(uint64_t v, int s) { return s ? (v << s) | (v >> (64 - s)) : v; }

// Lane (x, y) is A[x + 5 y].
void keccak_f(uint64_t A[25]) {
    const KeccakTables &T = ktab();
    for (int ir = 0; ir < 24; ++ir) {
        uint64_t C[5], D[5], B[25];
        for (int x = 0; x < 5; ++x) C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];
        for (int x = 0; x < 5; ++x) D[x] = C[(x + 4) % 5] ^ rotl(C[(x + 1) % 5], 1);
        for (int i = 0; i < 25; ++i) A[i] ^= D[i % 5];
        // rho and pi: B[y, 2x + 3y] = rot(A[x, y]), i.e. A'[x, y] = A[x + 3y, x]
        for (int x = 0; x < 5; ++x)
            for (int y = 0; y < 5; ++y) B[y + 5 * ((2 * x + 3 * y) % 5)] = rotl(A[x + 5 * y], T.rot[x][y]);
        for (int y = 0; y < 5; ++y)
            for (int x = 0; x < 5; ++x)
                A[x + 5 * y] = B[x + 5 * y] ^ (~B[(x + 1) % 5 + 5 * y] & B[(x + 2) % 5 + 5 * y]);
        A[0] ^= T.rc[ir];
    }
}

// SHAKE-256: rate 136 bytes, domain bits 1111 then pad10*1.
class Shake256 {
public:
    explicit Shake256(const uint8_t *msg, size_t n) {
        std::memset(A_, 0, sizeof A_);
        std::vector<uint8_t> m(msg, msg + n);
        m.push_back(0x1f);
        while (m.size() % kRate) m.push_back(0);
        m.back() |= 0x80;
        for (size_t off = 0; off < m.size(); off += kRate) {
            for (size_t i = 0; i < kRate; ++i) A_[i / 8] ^= (uint64_t)m[off + i] << (8 * (i % 8));
            keccak_f(A_);
        }
        pos_ = 0;
    }
    uint8_t byte() {
        if (pos_ == kRate) {
            keccak_f(A_);
            pos_ = 0;
        }
        const uint8_t b = (uint8_t)(A_[pos_ / 8] >> (8 * (pos_ % 8)));
        ++pos_;
        return b;
    }
    uint64_t word() {
        uint64_t v = 0;
        for (int i = 0; i < 8; ++i) v |= (uint64_t)byte() << (8 * i);
        return v;
    }

private:
    static constexpr size_t kRate = 136;
    uint64_t A_[25];
    size_t pos_;
};

Shake256 stream(const uint8_t seed[32], uint32_t tag, uint32_t index, uint32_t limb) {
    uint8_t m[44];
    std::memcpy(m, seed, 32);
    const uint32_t f[3] = {tag, index, limb};
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 4; ++i) m[32 + 4 * k + i] = (uint8_t)(f[k] >> (8 * i));
    return Shake256(m, sizeof m);
}

uint64_t below(Shake256 &s, uint64_t m) {
    int bits = 0;
    while (bits < 64 && ((m - 1) >> bits)) ++bits;
    const uint64_t mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
    for (;;) {
        const uint64_t v = s.word() & mask;
        if (v < m) return v;
    }
}

constexpr double kSigma = 3.2;
constexpr int kBound = 19;

struct Cdt {
    uint64_t t[kBound + 1];
    Cdt() {
        double rho[kBound + 1];
        for (int k = 0; k <= kBound; ++k) rho[k] = std::exp(-(double)(k * k) / (2.0 * kSigma * kSigma));
        double total = rho[0];
        for (int k = 1; k <= kBound; ++k) total += 2.0 * rho[k];
        double acc = 0.0;
        for (int k = 0; k < kBound; ++k) {
            acc += (k == 0 ? rho[k] : 2.0 * rho[k]) / total;
            t[k] = (uint64_t)std::floor(acc * 9223372036854775808.0);
        }
        t[kBound] = 1ull << 63;
    }
};

}  // namespace

void sample_uniform(const uint8_t seed[32], uint32_t tag, uint32_t index, uint32_t limb, uint64_t q, size_t n,
                    uint64_t *out) {
    Shake256 s = stream(seed, tag, index, limb);
    for (size_t i = 0; i < n; ++i) out[i] = below(s, q);
}

void sample_secret(const uint8_t seed[32], size_t n, int32_t h, int8_t *out) {
    Shake256 s = stream(seed, kTagSecret, 0, 0);
    if (h < 0) {
        for (size_t i = 0; i < n; ++i) {
            unsigned v;
            do v = s.byte() & 3u;
            while (v == 3u);
            out[i] = v == 0 ? 0 : (v == 1 ? 1 : -1);
        }
        return;
    }
    std::vector<uint32_t> pos(n);
    for (size_t i = 0; i < n; ++i) pos[i] = (uint32_t)i;
    for (size_t i = 0; i < (size_t)h; ++i)
        if (n - i > 1) std::swap(pos[i], pos[i + below(s, n - i)]);
    std::memset(out, 0, n);
    for (size_t i = 0; i < (size_t)h; ++i) out[pos[i]] = (s.byte() & 1u) ? -1 : 1;
}

void sample_gaussian(const uint8_t seed[32], uint32_t tag, uint32_t index, size_t n, int64_t *out) {
    static const Cdt cdt;
    Shake256 s = stream(seed, tag, index, 0);
    for (size_t i = 0; i < n; ++i) {
        const uint64_t u = s.word() >> 1;
        int k = 0;
        while (u >= cdt.t[k]) ++k;
        if (k && (s.byte() & 1u)) k = -k;
        out[i] = k;
    }
}

void shake256(const uint8_t *msg, size_t n, uint8_t *out, size_t outlen) {
    Shake256 s(msg, n);
    for (size_t i = 0; i < outlen; ++i) out[i] = s.byte();
}

}  // namespace pfx

// ------------------------------------------------------------------ C-ABI
using namespace pfx;

extern "C" {

pfx_status pfx_shake256(const uint8_t *msg, size_t n, uint8_t *out, size_t outlen) {
    if ((!msg && n) || (!out && outlen)) return fail(PFX_EINVAL, "null argument");
    shake256(msg, n, out, outlen);
    return PFX_OK;
}

pfx_status pfx_sample_uniform(const uint8_t *seed, uint32_t tag, uint32_t index, uint32_t limb, uint64_t q,
                              size_t n, uint64_t *out) {
    if (!seed || (!out && n)) return fail(PFX_EINVAL, "null argument");
    if (q < 2) return fail(PFX_EINVAL, "modulus below 2");
    sample_uniform(seed, tag, index, limb, q, n, out);
    return PFX_OK;
}

pfx_status pfx_sample_secret(const uint8_t *seed, size_t n, int32_t h, int8_t *out) {
    if (!seed || (!out && n)) return fail(PFX_EINVAL, "null argument");
    if (h > 0 && (size_t)h > n) return fail(PFX_EINVAL, "more non-zero coefficients than coefficients");
    sample_secret(seed, n, h, out);
    return PFX_OK;
}

pfx_status pfx_sample_gaussian(const uint8_t *seed, uint32_t tag, uint32_t index, size_t n, int64_t *out) {
    if (!seed || (!out && n)) return fail(PFX_EINVAL, "null argument");
    sample_gaussian(seed, tag, index, n, out);
    return PFX_OK;
}

pfx_status pfx_keygen_secret(pfx_ctx *c, const uint8_t *seed, int32_t h, pfx_sk **out) {
    if (!c || !seed || !out) return fail(PFX_EINVAL, "null argument");
    if (h > c->N) return fail(PFX_EINVAL, "more non-zero coefficients than coefficients");
    std::vector<int8_t> s((size_t)c->N);
    sample_secret(seed, s.size(), h, s.data());
    return pfx_sk_create(c, s.data(), out);
}

namespace {

pfx_status keygen_one(pfx_ctx *c, const pfx_sk *sk, uint32_t g, const uint8_t *seed, pfx_swk **out) {
    const size_t N = c->N, NP = (size_t)c->L + c->K;
    std::vector<uint64_t> a((size_t)c->beta * NP * N);
    std::vector<int64_t> e((size_t)c->beta * N);
    for (int j = 0; j < c->beta; ++j) {
        const uint32_t idx = 256u * g + (uint32_t)j;
        for (size_t m = 0; m < NP; ++m)
            sample_uniform(seed, kTagKeyA, idx, (uint32_t)m, c->primes[m], N, a.data() + ((size_t)j * NP + m) * N);
        sample_gaussian(seed, kTagKeyE, idx, N, e.data() + (size_t)j * N);
    }
    return pfx_swk_create(c, sk, g, a.data(), e.data(), out);
}

}  // namespace

pfx_status pfx_keygen_relin(pfx_ctx *c, const pfx_sk *sk, const uint8_t *seed, pfx_swk **out) {
    if (!c || !sk || !seed || !out) return fail(PFX_EINVAL, "null argument");
    return keygen_one(c, sk, 0, seed, out);
}

pfx_status pfx_keygen_galois(pfx_ctx *c, const pfx_sk *sk, const int32_t *steps, size_t n, int conj,
                             const uint8_t *seed, pfx_swk **out) {
    if (!c || !sk || !seed || !out || (n && !steps)) return fail(PFX_EINVAL, "null argument");
    const int64_t half = c->N / 2;
    const size_t total = n + (conj ? 1 : 0);
    std::vector<pfx_swk *> made;
    for (size_t i = 0; i < total; ++i) {
        uint32_t g;
        if (i < n) {
            const int64_t st = (((int64_t)steps[i] % half) + half) % half;
            g = (uint32_t)powmod_u64(5, (uint64_t)st, 2ull * c->N);
        } else {
            g = (uint32_t)(2 * c->N - 1);
        }
        pfx_swk *k = nullptr;
        pfx_status r = keygen_one(c, sk, g, seed, &k);
        if (r) {
            for (pfx_swk *x : made) pfx_swk_destroy(x);
            return r;
        }
        made.push_back(k);
    }
    for (size_t i = 0; i < total; ++i) out[i] = made[i];
    return PFX_OK;
}

pfx_status pfx_encrypt_seeded(pfx_ctx *c, const pfx_sk *sk, const pfx_pt *m, const uint8_t *seed, pfx_ct *out,
                              void *stream) {
    if (!c || !sk || !m || !seed || !out) return fail(PFX_EINVAL, "null argument");
    if (m->n_limbs == 0 || m->ctx != c) return fail(PFX_EINVAL, "bad plaintext");
    const size_t N = c->N, lv = m->n_limbs;
    std::vector<uint64_t> a(lv * N);
    std::vector<int64_t> e(N);
    for (size_t i = 0; i < lv; ++i) sample_uniform(seed, kTagEncA, 0, (uint32_t)i, c->primes[i], N, a.data() + i * N);
    sample_gaussian(seed, kTagEncE, 0, N, e.data());
    return pfx_encrypt(c, sk, m, a.data(), e.data(), out, stream);
}

}  // extern "C"
