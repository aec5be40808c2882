// Slot encoding and decoding on the host (App. A.1 of the paper, canonical
// embedding), FP64.
//
// n complex slots live in the subring Y = X^(N/2n).  Slot j is p(zeta_j) for
// the real polynomial p of degree < 2n, zeta_j = w^(5^j mod 4n), w = e^(i pi/2n).
// Since 5^j = 1 mod 4, write 5^j mod 4n = 4 t_j + 1; with u_k = p_k + i p_{k+n}
// (and zeta_j^n = i) the slots are z_j = sum_{k<n} (u_k w^k) rho^(k t_j) with
// rho = e^(2 pi i / n): an n-point DFT of the twisted vector, read at t_j.
// Encoding runs it backwards: scatter z to t_j, inverse DFT, untwist, split
// real and imaginary parts into p_k and p_{k+n}, scale, round half away from
// zero, reduce modulo each prime.  Decoding lifts the residues by Garner's
// mixed-radix CRT to centred integers first.
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace pfx {

typedef std::complex<double> cd;

// In-place radix-2 DFT, X[k] = sum_t x[t] e^(sign 2 pi i t k / n).
static void fft(std::vector<cd> &a, int sign) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = sign * 2.0 * M_PI / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                cd w(std::cos(ang * k), std::sin(ang * k));
                cd u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

static std::vector<size_t> slot_index(size_t n) {
    std::vector<size_t> t(n);
    uint64_t e = 1;
    for (size_t j = 0; j < n; ++j) {
        t[j] = (size_t)((e - 1) / 4);
        e = (e * 5) % (4 * n);
    }
    return t;
}

// Exact residue of an integral double v modulo m (any magnitude).
static uint64_t double_mod(double v, uint64_t m) {
    bool neg = v < 0;
    double a = std::fabs(v);
    uint64_t r;
    if (a < 9007199254740992.0) {
        r = (uint64_t)a % m;
    } else {
        int ex;
        double fr = std::frexp(a, &ex);           // a = fr * 2^ex, fr in [0.5, 1)
        uint64_t mant = (uint64_t)std::ldexp(fr, 53);
        r = mulmod_u64(mant % m, powmod_u64(2, (uint64_t)(ex - 53), m), m);
    }
    return (neg && r) ? m - r : r;
}

bool encode_coeffs(int logn, const double *re, const double *im, size_t n, double scale,
                   const std::vector<uint64_t> &mods, std::vector<uint64_t> &words, std::string &err) {
    const size_t N = (size_t)1 << logn;
    if (n == 0 || (n & (n - 1)) || n > N / 2) { err = "n_slots must be a power of two <= N/2"; return false; }
    std::vector<size_t> t = slot_index(n);
    std::vector<cd> u(n);
    for (size_t j = 0; j < n; ++j) u[t[j]] = cd(re[j], im ? im[j] : 0.0);
    fft(u, -1);
    std::vector<double> coeff(2 * n);
    for (size_t k = 0; k < n; ++k) {
        double ang = -M_PI * (double)k / (2.0 * (double)n);
        cd v = u[k] * cd(std::cos(ang), std::sin(ang)) / (double)n;
        coeff[k] = v.real();
        coeff[k + n] = v.imag();
    }
    const size_t gap = N / (2 * n);
    words.assign(mods.size() * N, 0);
    for (size_t k = 0; k < 2 * n; ++k) {
        double x = coeff[k] * scale;
        if (!std::isfinite(x)) { err = "non-finite value after scaling"; return false; }
        double r = std::copysign(std::floor(std::fabs(x) + 0.5), x);
        for (size_t i = 0; i < mods.size(); ++i) words[i * N + k * gap] = double_mod(r, mods[i]);
    }
    return true;
}

void decode_words(int logn, const uint64_t *words, int n_limbs, const std::vector<uint64_t> &mods,
                  double scale, size_t n, double *re, double *im) {
    const size_t N = (size_t)1 << logn;
    const size_t gap = N / (2 * n);
    const int l = n_limbs;
    // Garner: x = sum_i v_i prod_{j<i} q_j with v_i in [0, q_i).
    std::vector<std::vector<uint64_t>> inv(l, std::vector<uint64_t>(l));
    for (int i = 0; i < l; ++i)
        for (int j = 0; j < i; ++j) inv[i][j] = invmod_u64(mods[j] % mods[i], mods[i]);
    // mixed-radix digits of (Q-1)/2, whose residues are (q_i - 1)/2
    std::vector<uint64_t> half(l);
    for (int i = 0; i < l; ++i) {
        uint64_t tv = (mods[i] - 1) / 2;
        for (int j = 0; j < i; ++j) {
            uint64_t d = half[j] % mods[i];
            tv = mulmod_u64((tv + mods[i] - d) % mods[i], inv[i][j], mods[i]);
        }
        half[i] = tv;
    }
    std::vector<double> p(2 * n);
    std::vector<uint64_t> v(l);
    for (size_t k = 0; k < 2 * n; ++k) {
        const size_t c = k * gap;
        for (int i = 0; i < l; ++i) {
            uint64_t tv = words[(size_t)i * N + c];
            for (int j = 0; j < i; ++j) {
                uint64_t d = v[j] % mods[i];
                tv = mulmod_u64((tv + mods[i] - d) % mods[i], inv[i][j], mods[i]);
            }
            v[i] = tv;
        }
        bool negative = false;
        for (int i = l - 1; i >= 0; --i) {
            if (v[i] != half[i]) { negative = v[i] > half[i]; break; }
        }
        double val = 0.0;
        if (!negative) {
            for (int i = l - 1; i >= 0; --i) val = val * (double)mods[i] + (double)v[i];
        } else {   // Q - x = sum (q_i - 1 - v_i) prod q_j + 1
            for (int i = l - 1; i >= 0; --i) val = val * (double)mods[i] + (double)(mods[i] - 1 - v[i]);
            val = -(val + 1.0);
        }
        p[k] = val / scale;
    }
    std::vector<cd> u(n);
    for (size_t k = 0; k < n; ++k) {
        double ang = M_PI * (double)k / (2.0 * (double)n);
        u[k] = cd(p[k], p[k + n]) * cd(std::cos(ang), std::sin(ang));
    }
    fft(u, +1);
    std::vector<size_t> t = slot_index(n);
    for (size_t j = 0; j < n; ++j) {
        re[j] = u[t[j]].real();
        if (im) im[j] = u[t[j]].imag();
    }
}

}  // namespace pfx
