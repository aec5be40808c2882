"""Oracle of the private lookup-table evaluation and ring repacking
(TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's
CPU baseline use it; the library shares no code with it).

Follows the paper's first phase (Sec. 3.4 "Large-Domain Private Function",
Sec. 3.2 "Ring Repacking", Alg. 1), on coefficient-encoded RLWE ciphertexts of
`oracle.ckks` (words in the coefficient domain):

  lookup table   u_f = f(0) - f(N-1) X - f(N-2) X^2 - ... - f(1) X^{N-1}, its
                 coefficients scaled by Delta and rounded, encrypted by the
                 scientist;
  evaluation     X^i * Enc(u_f) encrypts a polynomial whose constant
                 coefficient is f(i) (X^N = -1), for a plaintext point i;
  aggregation    record r of a database: sum_l X^(k_(r,l)) * Enc(u_(f_l)), whose
                 constant coefficient is sum_l f_l(k_(r,l)) (Sec. 4.2, the
                 encrypted scoring functions summed over the attributes);
  repacking      N ciphertexts -> one encrypting sum_i m_i[0] X^i: every
                 input times N^-1 mod Q, then for i = 0 .. log N - 1 with
                 t = N / 2^(i+1), g = 2N - 1 for i = 0 and 5^(2^(i-1)) mod 2N
                 after, c_j <- c_j + c_{j+t} X^t + phi_g(c_j - c_{j+t} X^t) for
                 j < t; the result is c_0 (Lemma 1).

Readings: the paper's Set I moduli (55 and 54 bits) are replaced by primes
below 2^50 (the library's residues are FP64 integers); its extra base-2^30
decomposition of the repacking keys is not used (hybrid key switching with
one special prime keeps the key-switching noise small).  Fewer than N inputs
are padded with zero ciphertexts, as the paper allows.
"""
from __future__ import annotations

import numpy as np

from oracle import ckks as O


def monomial(a: np.ndarray, k: int, mods, N: int) -> np.ndarray:
    """a(X) * X^k in Z_q[X]/(X^N + 1), row by row (k taken mod 2N): coefficient
    j moves to j + k, negated each time it wraps past X^N."""
    k %= 2 * N
    d = np.arange(N) + k                     # where coefficient j lands, before reduction
    neg = (d // N) % 2 == 1                  # an odd number of wraps past X^N
    out = np.empty_like(a)
    for r, q in enumerate(mods):
        v = a[r].copy()
        flip = neg & (v != 0)
        v[flip] = np.uint64(q) - v[flip]
        out[r, d % N] = v
    return out


def ct_monomial(P, x: O.Ct, k: int) -> O.Ct:
    mods = P.mods(x.level)
    return O.Ct(np.stack([monomial(c, k, mods, P.N) for c in x.c]), x.scale)


def ct_mul_inv_n(P, x: O.Ct) -> O.Ct:
    """Every residue times N^-1 mod q_i; the scale is left as it is (the
    repacking multiplies by N again)."""
    mods = P.mods(x.level)
    ks = [pow(P.N, -1, q) for q in mods]
    return O.Ct(np.stack([O.smul(c, ks, mods) for c in x.c]), x.scale)


def repack_galois(P, i: int) -> int:
    """Galois element of round i of Alg. 1."""
    return 2 * P.N - 1 if i == 0 else pow(5, 1 << (i - 1), 2 * P.N)


def repack(P, cts: list, gks: dict) -> O.Ct:
    """Alg. 1 on len(cts) <= N ciphertexts of one level (zeros beyond)."""
    N = P.N
    assert 1 <= len(cts) <= N
    lv, sc = cts[0].level, cts[0].scale
    zero = O.Ct(np.zeros((2, lv, N), dtype=np.uint64), sc)
    c = [ct_mul_inv_n(P, x) for x in cts] + [zero] * (N - len(cts))
    for i in range(P.logn):
        t = N >> (i + 1)
        g = repack_galois(P, i)
        for j in range(t):
            u = ct_monomial(P, c[j + t], t)
            w = O.apply_galois(P, O.ct_sub(P, c[j], u), g, gks[g])
            c[j] = O.ct_add(P, O.ct_add(P, c[j], u), w)
    return c[0]


def lut_poly(f_values, delta: float) -> np.ndarray:
    """Integer coefficients of round(delta * u_f), u_f = f(0) - sum_k f(N-k) X^k."""
    f = np.asarray(f_values, dtype=np.float64)
    N = len(f)
    u = np.empty(N, dtype=np.float64)
    u[0] = f[0]
    u[1:] = -f[N - np.arange(1, N)]
    return O.round_half_away(delta * u).astype(np.int64)


def evaluate(P, U: O.Ct, points) -> list:
    """X^i * U for each point i: the lookup of f at i in the constant coefficient."""
    return [ct_monomial(P, U, int(i)) for i in points]


def score_records(P, tables: list, exps) -> list:
    """Record r: sum over the tables l of X^(exps[r][l]) * tables[l] (Sec. 4.2)."""
    out = []
    for row in np.asarray(exps, dtype=np.int64):
        acc = ct_monomial(P, tables[0], int(row[0]))
        for U, k in zip(tables[1:], row[1:]):
            acc = O.ct_add(P, acc, ct_monomial(P, U, int(k)))
        out.append(acc)
    return out


def repack_groups(P, cts: list, gks: dict) -> list:
    """Alg. 1 on consecutive groups of N ciphertexts (the last one zero-padded)."""
    return [repack(P, cts[g:g + P.N], gks) for g in range(0, len(cts), P.N)]


def packed_values(P, s, ct: O.Ct, n: int) -> np.ndarray:
    """Decrypted coefficients 0..n-1 over the scale (centred lift)."""
    m = O.decrypt(P, s, ct)
    return O.crt_centered(m, P.mods(ct.level))[:n].astype(np.float64) / ct.scale
