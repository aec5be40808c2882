/*
 * CPU oracle for RNS-CKKS: exact integer loops.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * path.
 *
 * Every routine here is a plain textbook loop with 128-bit products and the C
 * `%` operator, written for reading, not for speed.  Residues are canonical
 * (in [0, q)), moduli are odd and below 2^62.
 *
 * Paper anchors (arXiv 2412.13269):
 *   - ring R_Q^N = Z_Q[X]/(X^N + 1), products are negacyclic convolutions
 *     (Sec. 2.2, "Plaintexts and Ciphertexts Domain");
 *   - automorphisms phi_g : X -> X^g for odd g (Sec. 2.2);
 *   - the RNS split of Q, the NTT and the fast basis conversion are not
 *     described in the paper; the oracle follows the plain definitions that
 *     the test suite pins (schoolbook convolution, O(N^2) transform, big-integer
 *     CRT).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;

static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 submod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - b) % q); }

static u64 powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); } /* q prime */

static unsigned bitrev(unsigned x, int bits) {
    unsigned r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

/* ---------------------------------------------------------------------- */
/* Negacyclic NTT.                                                          */
/* Definition used throughout:                                              */
/*   NTT(a)[j] = sum_k a[k] * psi^(k * (2*bitrev(j) + 1))  (mod q)          */
/* i.e. the evaluation of a(X) at the odd powers of a primitive 2N-th root  */
/* psi, listed in bit-reversed order of the exponent.                       */
/* ---------------------------------------------------------------------- */

/* The definition itself, O(N^2). */
void pfo_ntt_naive(u64 q, u64 psi, int logn, const u64 *a, u64 *out) {
    const unsigned n = 1u << logn;
    for (unsigned j = 0; j < n; j++) {
        u64 root = powmod(psi, 2ull * bitrev(j, logn) + 1, q);
        u64 acc = 0, x = 1;
        for (unsigned k = 0; k < n; k++) {
            acc = addmod(acc, mulmod(a[k], x, q), q);
            x = mulmod(x, root, q);
        }
        out[j] = acc;
    }
}

/* Textbook radix-2 Cooley-Tukey with the powers psi^bitrev(i) (in place). */
void pfo_ntt(u64 q, u64 psi, int logn, u64 *a) {
    const unsigned n = 1u << logn;
    u64 *tw = (u64 *)malloc(sizeof(u64) * n);
    for (unsigned i = 0; i < n; i++) tw[i] = powmod(psi, bitrev(i, logn), q);
    unsigned t = n;
    for (unsigned m = 1; m < n; m <<= 1) {
        t >>= 1;
        for (unsigned i = 0; i < m; i++) {
            const u64 w = tw[m + i];
            for (unsigned j = 2 * i * t; j < 2 * i * t + t; j++) {
                u64 u = a[j];
                u64 v = mulmod(a[j + t], w, q);
                a[j] = addmod(u, v, q);
                a[j + t] = submod(u, v, q);
            }
        }
    }
    free(tw);
}

/* Inverse: Gentleman-Sande with psi^-bitrev(i), then multiply by N^-1. */
void pfo_intt(u64 q, u64 psi, int logn, u64 *a) {
    const unsigned n = 1u << logn;
    const u64 psi_inv = invmod(psi, q);
    u64 *tw = (u64 *)malloc(sizeof(u64) * n);
    for (unsigned i = 0; i < n; i++) tw[i] = powmod(psi_inv, bitrev(i, logn), q);
    unsigned t = 1;
    for (unsigned m = n >> 1; m >= 1; m >>= 1) {
        for (unsigned i = 0; i < m; i++) {
            const u64 w = tw[m + i];
            for (unsigned j = 2 * i * t; j < 2 * i * t + t; j++) {
                u64 u = a[j], v = a[j + t];
                a[j] = addmod(u, v, q);
                a[j + t] = mulmod(submod(u, v, q), w, q);
            }
        }
        t <<= 1;
    }
    const u64 ninv = invmod(n % q, q);
    for (unsigned j = 0; j < n; j++) a[j] = mulmod(a[j], ninv, q);
    free(tw);
}

/* Schoolbook negacyclic product, O(N^2): X^N = -1. */
void pfo_negacyclic_mul_naive(u64 q, int logn, const u64 *a, const u64 *b, u64 *out) {
    const unsigned n = 1u << logn;
    for (unsigned i = 0; i < n; i++) out[i] = 0;
    for (unsigned i = 0; i < n; i++)
        for (unsigned j = 0; j < n; j++) {
            u64 p = mulmod(a[i], b[j], q);
            unsigned k = i + j;
            if (k < n) out[k] = addmod(out[k], p, q);
            else out[k - n] = submod(out[k - n], p, q);
        }
}

/* ---------------------------------------------------------------------- */
/* RNS polynomial helpers: a polynomial over nl moduli is nl rows of N.     */
/* ---------------------------------------------------------------------- */

void pfo_ntt_rns(int nl, const u64 *q, const u64 *psi, int logn, u64 *a) {
    const size_t n = (size_t)1 << logn;
#pragma omp parallel for schedule(dynamic)
    for (int l = 0; l < nl; l++) pfo_ntt(q[l], psi[l], logn, a + (size_t)l * n);
}

void pfo_intt_rns(int nl, const u64 *q, const u64 *psi, int logn, u64 *a) {
    const size_t n = (size_t)1 << logn;
#pragma omp parallel for schedule(dynamic)
    for (int l = 0; l < nl; l++) pfo_intt(q[l], psi[l], logn, a + (size_t)l * n);
}

/* Ring product in the coefficient domain: forward transforms, pointwise
 * product, inverse transform (convolution theorem for X^N + 1). */
void pfo_polymul_rns(int nl, const u64 *q, const u64 *psi, int logn,
                     const u64 *a, const u64 *b, u64 *out) {
    const size_t n = (size_t)1 << logn;
#pragma omp parallel for schedule(dynamic)
    for (int l = 0; l < nl; l++) {
        u64 *ta = (u64 *)malloc(sizeof(u64) * n);
        u64 *tb = (u64 *)malloc(sizeof(u64) * n);
        memcpy(ta, a + l * n, sizeof(u64) * n);
        memcpy(tb, b + l * n, sizeof(u64) * n);
        pfo_ntt(q[l], psi[l], logn, ta);
        pfo_ntt(q[l], psi[l], logn, tb);
        for (size_t i = 0; i < n; i++) ta[i] = mulmod(ta[i], tb[i], q[l]);
        pfo_intt(q[l], psi[l], logn, ta);
        memcpy(out + l * n, ta, sizeof(u64) * n);
        free(ta);
        free(tb);
    }
}

/* out[l][i] = a[l][i] * b[l][i] mod q[l] */
void pfo_pmul_rns(int nl, const u64 *q, size_t n, const u64 *a, const u64 *b, u64 *out) {
#pragma omp parallel for
    for (int l = 0; l < nl; l++)
        for (size_t i = 0; i < n; i++) out[l * n + i] = mulmod(a[l * n + i], b[l * n + i], q[l]);
}

/* out[l][i] = a[l][i] * k[l] mod q[l] */
void pfo_smul_rns(int nl, const u64 *q, size_t n, const u64 *a, const u64 *k, u64 *out) {
#pragma omp parallel for
    for (int l = 0; l < nl; l++)
        for (size_t i = 0; i < n; i++) out[l * n + i] = mulmod(a[l * n + i], k[l], q[l]);
}

/*
 * Fast (uncorrected) basis conversion of x from the moduli qin[0..nin) to the
 * moduli qout[0..nout):
 *   y_i     = [x_i * (Q'/q_i)^-1]_{q_i}
 *   out_m   = sum_i y_i * [Q'/q_i]_{m}    (mod m)
 * which is x' = sum_i y_i (Q'/q_i) reduced mod m, an integer congruent to x
 * mod Q' and equal to [x]_{Q'} + u Q' with 0 <= u < nin.
 *   qhat_inv[i]        = (Q'/q_i)^-1 mod q_i
 *   qhat_mod[i*nout+m] = (Q'/q_i) mod qout[m]
 */
void pfo_bconv(size_t n, int nin, const u64 *qin, const u64 *x, const u64 *qhat_inv,
               int nout, const u64 *qout, const u64 *qhat_mod, u64 *out) {
    u64 *y = (u64 *)malloc(sizeof(u64) * n * nin);
    for (int i = 0; i < nin; i++)
        for (size_t c = 0; c < n; c++) y[i * n + c] = mulmod(x[i * n + c], qhat_inv[i], qin[i]);
#pragma omp parallel for
    for (int m = 0; m < nout; m++)
        for (size_t c = 0; c < n; c++) {
            u64 acc = 0;
            for (int i = 0; i < nin; i++)
                acc = addmod(acc, mulmod(y[i * n + c] % qout[m], qhat_mod[i * nout + m], qout[m]), qout[m]);
            out[m * n + c] = acc;
        }
    free(y);
}

/*
 * Automorphism phi_g in the coefficient domain (g odd): X^i -> X^(i*g mod 2N),
 * with X^N = -1 turning exponents in [N, 2N) into a sign flip.
 */
void pfo_automorphism(int nl, const u64 *q, int logn, u64 g, const u64 *a, u64 *out) {
    const size_t n = (size_t)1 << logn;
    for (int l = 0; l < nl; l++)
        for (size_t i = 0; i < n; i++) {
            u64 e = (u64)(((u128)i * g) % (2 * n));
            u64 v = a[l * n + i];
            if (e < n) out[l * n + e] = v;
            else out[l * n + (e - n)] = (v == 0) ? 0 : q[l] - v;
        }
}

/* Threads of the OpenMP loops above (plumbing for timing runs: the results
 * do not depend on it). */
int pfo_threads(void) { return omp_get_max_threads(); }
void pfo_set_threads(int n) { omp_set_num_threads(n); }
