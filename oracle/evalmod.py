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

with T_1 = u, T_2k = 2 T_k^2 - 1, T_2k+1 = 2 T_k T_k+1 - T_1 (relinearised and
rescaled products, the factor 2 an integer product), each c_k T_k a constant
product at the scale of the next prime, rescaled, the terms summed in order of
k (scale of the first), c_0 added last.  The coefficients c_k are an input (the
caller interpolates them).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ckks as O
from oracle.query import _mr, add_const, mul_const_next


def cheb_index_pair(k: int):
    """T_k = 2 T_a T_b - T_(a-b) with a = ceil(k/2), b = floor(k/2)."""
    return (k + 1) // 2, k // 2


def evalmod(P, x: O.Ct, coeffs, r: int, K: float, rlk) -> O.Ct:
    a = (K + 0.25) / 2 ** r
    d = len(coeffs) - 1
    t = add_const(P, x, -0.25)
    u = O.rescale(P, mul_const_next(P, t, 1.0 / (2 ** r * a)))
    T = {1: u}
    for k in range(2, d + 1):
        i, j = cheb_index_pair(k)
        p = O.ct_mul_int(P, _mr(P, T[i], T[j], rlk), 2)
        T[k] = add_const(P, p, -1.0) if i == j else O.ct_sub(P, p, T[1])
    c = None
    for k in range(1, d + 1):
        term = O.rescale(P, mul_const_next(P, T[k], float(coeffs[k])))
        c = term if c is None else O.ct_add(P, c, term)
    c = add_const(P, c, float(coeffs[0]))
    for _ in range(r):
        c = add_const(P, O.ct_mul_int(P, _mr(P, c, c, rlk), 2), -1.0)
    return O.rescale(P, mul_const_next(P, c, 1.0 / (2 * math.pi)))


def evalmod_fp64(t, coeffs, r: int, K: float):
    """The same steps on plain FP64 values."""
    a = (K + 0.25) / 2 ** r
    u = (np.asarray(t) - 0.25) / (2 ** r * a)
    d = len(coeffs) - 1
    T = {0: np.ones_like(u), 1: u}
    for k in range(2, d + 1):
        i, j = cheb_index_pair(k)
        T[k] = 2 * T[i] * T[j] - (1.0 if i == j else T[1])
    c = sum(float(coeffs[k]) * T[k] for k in range(d + 1))
    for _ in range(r):
        c = 2 * c * c - 1
    return c / (2 * math.pi)
