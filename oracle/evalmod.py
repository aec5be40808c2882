"""Oracle of EvalMod, the modular-reduction step of bootstrapping (TEST
INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU
baseline use it; the library shares no code with it).

App. A.3: after ModRaise and CoeffsToSlots the slots hold t = m'/q_0 = I + m/q_0
with I a small integer; EvalMod evaluates a polynomial approximation of the
reduction modulo 1 there.  Reading (the paper uses Lattigo's EvalMod without
printing it): the scaled sine sin(2 pi t) / (2 pi), which equals t - I up to
O((t - I)^3), computed as

    u  = ((t - 1/4) / 2^r) / a                      a = (K + 1/4) / 2^r, |t| <= K
    c  = sum_k c_k T_k(u)                           Chebyshev approximation of
                                                    cos(2 pi a u) on [-1, 1]
    c <- 2 c^2 - 1, r times                         double angle: cos(2 pi (t - 1/4))
    out = c / (2 pi)                                = sin(2 pi t) / (2 pi)

(times an optional factor f folded into the last constant, out_factor, e.g.
q_0 / Delta to return the message at its own scale)

with T_1 = u, T_2k = 2 T_k^2 - 1, T_2k+1 = 2 T_k T_k+1 - T_1 (relinearised and
rescaled products, the factor 2 an integer product), c_0 added last, the
coefficients c_k an input (the caller interpolates them).

Scales.  A sum of two ciphertexts decrypts to x_a + (s_b / s_a) x_b when their
scales s_a, s_b differ, and rescaling by primes that are only near a power of
two lets the scales of the T_k drift apart by ~1e-6 relative, which is far
more than bootstrapping tolerates (the message is the small fraction m / q_0 of
t).  So every term meets its partner at one scale exactly, and every sum is
formed before its one rescale: a constant factor is encoded at the scale
c = s_target / s_x, which brings the term to the sum's scale before the
rescale exactly (mul_const_like; the sum sits at the level of its lowest
term, the others' extra primes dropped).  T_1 enters each odd T_k that way:
T_k = rescale(2 T_i T_j - T_1 c) with the relinearised product not yet
rescaled; the highest term c_d T_d is taken at the next prime's scale, the
other c_k T_k are brought to its scale, summed from k = d down and rescaled
once.  Constants added with add_const are encoded at the ciphertext's own
scale and need nothing.
Reading (App. A.3 does not place the rescales): one rescale per sum, not one
per term; both give the same scale and level, the first with fewer
rescalings (one rounding per sum).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ckks as O
from oracle.query import _mr, add_const, mul_const_like, mul_const_next


def cheb_index_pair(k: int):
    """T_k = 2 T_a T_b - T_(a-b) with a = ceil(k/2), b = floor(k/2)."""
    return (k + 1) // 2, k // 2


def evalmod(P, x: O.Ct, coeffs, r: int, K: float, rlk, out_factor: float = 1.0) -> O.Ct:
    a = (K + 0.25) / 2 ** r
    d = len(coeffs) - 1
    t = add_const(P, x, -0.25)
    u = O.rescale(P, mul_const_next(P, t, 1.0 / (2 ** r * a)))
    T = {1: u}
    for k in range(2, d + 1):
        i, j = cheb_index_pair(k)
        if i == j:
            T[k] = add_const(P, O.ct_mul_int(P, _mr(P, T[i], T[j], rlk), 2), -1.0)
        else:
            p = O.ct_mul_int(P, O.mul_relin(P, T[i], T[j], rlk), 2)
            T[k] = O.rescale(P, O.ct_sub(P, p, mul_const_like(P, T[1], 1.0, p.scale)))
    acc = mul_const_next(P, T[d], float(coeffs[d]))
    for k in range(d - 1, 0, -1):
        acc = O.ct_add(P, acc, mul_const_like(P, T[k], float(coeffs[k]), acc.scale))
    c = add_const(P, O.rescale(P, acc), float(coeffs[0]))
    for _ in range(r):
        c = add_const(P, O.ct_mul_int(P, _mr(P, c, c, rlk), 2), -1.0)
    return O.rescale(P, mul_const_next(P, c, out_factor / (2 * math.pi)))


def evalmod_fp64(t, coeffs, r: int, K: float, out_factor: float = 1.0):
    """The same steps on plain FP64 values."""
    a = (K + 0.25) / 2 ** r
    u = (np.asarray(t) - 0.25) / (2 ** r * a)
    d = len(coeffs) - 1
    T = {0: np.ones_like(u), 1: u}
    for k in range(2, d + 1):
        i, j = cheb_index_pair(k)
        T[k] = 2 * T[i] * T[j] - (1.0 if i == j else T[1])
    c = float(coeffs[d]) * T[d]
    for k in range(d - 1, 0, -1):
        c = c + float(coeffs[k]) * T[k]
    c = c + float(coeffs[0])
    for _ in range(r):
        c = 2 * c * c - 1
    return c * (out_factor / (2 * math.pi))
