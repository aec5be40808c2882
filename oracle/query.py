"""Oracle of the private-query circuit (TEST INFRASTRUCTURE ONLY).

The circuit follows the paper's private threshold and count (Alg. 2, lines
12-15; Sec. 5.3 "Private Threshold Functions"), with the slot-domain linear
score of the query in place of the paper's coefficient-encoded PFE phase:

  per record block b (2^(logN-1) records in the slots):
    S   = rescale( sum_a W[a] * X[b][a] )                    linear score
    Y_k = powers of S up to degree D <= 15 by the binary tree
          Y2 = Y1 Y1, Y3 = Y2 Y1, Y4 = Y2 Y2, Y5 = Y4 Y1, Y6 = Y4 Y2, Y7 = Y4 Y3,
          Y8 = Y4 Y4, Y(8+i) = Y8 Yi
    Z   = rescale(relin(sum_{k=1..D} C[k] (x) Y_k)) + C[0]   polynomial p(S): the
          tensor products (degree 2) are summed, at the level of the deepest
          Y_k, and relinearised and rescaled once
    U   = rescale(relin((Z - T) H))                          normalised threshold input
    3 times (composite sign, degree-7 stage f7(x) = (35x - 35x^3 + 21x^5 - 5x^7)/16):
        X2 = X X, X4 = X2 X2, X6 = X4 X2                     (relin + rescale each)
        P  = (-35) X2 + 21 X4 + (-5) X6 + 35                 integer products, constant add
        X' = rescale(X * round(q / 16))  (constant at the scale of the prime q that the
                                          rescale drops, so X' keeps X's scale)
        U  = rescale(relin(X' P))
    step_b = (U + 1) with the scale doubled                  step = (sign + 1) / 2
  W   = step_0 + step_1 + ...
  OUT = rotate-and-sum over all slots (InnerSum), on the first FINAL_LIMBS
        limbs of W only (dropping limbs is exact; Q_2 > 2^94 holds any count
        below 2^17 at a scale near 2^46 with room to spare)

Additions take the scale of their first operand (the rule of the library).
Every ct x ct product is relinearised and rescaled.

Readings: the paper's [15,15,15] minimax composite coefficients are not
printed (Tab. 2); f7 is the closed-form odd polynomial with f7(+-1) = +-1 and
f7'(+-1) = 0, and the degree-7 score polynomial and the attribute count come
from the query configuration (N = 2^16, 2^17 records x 8 attributes).  The
degree-15 stages of the paper's first threshold take the member of the same
closed-form family of degree 15, f15(x) = x P(x^2) / 2048 with
P(y) = sum_{i<=7} 4^(7-i) C(2i, i) (1 - y)^i / 4^7 * 2048 (f15(+-1) = +-1, its
first seven derivatives 0 at +-1), evaluated like f7: y = x^2, the powers of y
by the tree above, the integer combination, x / 2048 at the next prime's
scale, one product.

The paper's thresholds themselves (Tab. 2) are composite minimax
approximations whose coefficients it does not print; oracle/remez.py designs
them (stage by stage, Remez), and with `sign_coeffs` the query takes those
stages instead (minimax_stage: odd powers by ODD_TREE, each term's constant
at the scale that lands on the sum's).  global_threshold is the second,
global threshold on the count.
"""
from __future__ import annotations

import numpy as np

from oracle import ckks as O

# sign stages f(x) = x P(x^2) / den: integer coefficients of P (y^0, y^1, ...)
SIGN = {7: ((35, -35, 21, -5), 16),
        15: ((6435, -15015, 27027, -32175, 25025, -12285, 3465, -429), 2048)}
F7 = SIGN[7][0]


def f_sign(x, degree=7):
    c, den = SIGN[degree]
    y = x * x
    return x * sum(ck * y ** k for k, ck in enumerate(c)) / den


def f7(x):
    return f_sign(x, 7)


def fp64_query(x, w, c, t, eta, stages=3, sign_degree=7, sign_coeffs=None):
    """The circuit in plain FP64 on the records x (records, attributes)."""
    s = x @ w
    z = sum(c[k] * s ** k for k in range(len(c)))
    u = (z - t) * eta
    if sign_coeffs is not None:
        u = fp64_minimax(u, sign_coeffs)
    for _ in range(stages if sign_coeffs is None else 0):
        u = f_sign(u, sign_degree)
    step = (u + 1.0) / 2.0
    return step, float(step.sum())


def _mr(P, a, b, rlk):
    return O.rescale(P, O.mul_relin(P, a, b, rlk))


def _factors(k):
    """The two lower powers whose product gives y^k in the power tree."""
    if k == 2:
        return 1, 1
    if k == 3:
        return 2, 1
    if k == 4:
        return 2, 2
    if k <= 7:
        return 4, k - 4
    if k == 8:
        return 4, 4
    return 8, k - 8


def _powers(P, y1, D, rlk):
    """y^k for k <= D <= 15: y^2 = y y, y^3 = y^2 y, y^4 = y^2 y^2, y^5 = y^4 y,
    y^6 = y^4 y^2, y^7 = y^4 y^3, y^8 = y^4 y^4, and y^(8+i) = y^8 y^i."""
    assert 1 <= D <= 15
    Y = {1: y1}
    for k in range(2, D + 1):
        a, b = _factors(k)
        Y[k] = _mr(P, Y[a], Y[b], rlk)
    return Y


def add_const(P, x: O.Ct, value: float) -> O.Ct:
    """x + value, the constant encoded at x's scale: round(value * scale) on
    coefficient 0 (App. A.1: a constant has a single coefficient)."""
    k = int(O.round_half_away(np.array([value * x.scale]))[0])
    c = x.c.copy()
    for i, q in enumerate(P.mods(x.level)):
        c[0, i, 0] = (int(c[0, i, 0]) + k) % q
    return O.Ct(c, x.scale)


def mul_const_next(P, x: O.Ct, value: float) -> O.Ct:
    """x times the constant `value` encoded at the scale of x's last prime."""
    q = P.q[x.level - 1]
    k = int(O.round_half_away(np.array([value * q]))[0])
    return O.Ct(O.ct_mul_int(P, x, k).c, x.scale * q)


def sign_stage(P, x: O.Ct, rlk, degree=7) -> O.Ct:
    """f(x) = x P(x^2) / den: y = x^2, y^k by the power tree, P(y) as integer
    products summed (coefficient of y first) plus the constant, then
    rescale(x * round(q / den)) times P(y)."""
    c, den = SIGN[degree]
    Y = _powers(P, _mr(P, x, x, rlk), len(c) - 1, rlk)
    p = O.ct_mul_int(P, Y[1], c[1])
    for k in range(2, len(c)):
        p = O.ct_add(P, p, O.ct_mul_int(P, Y[k], c[k]))
    p = add_const(P, p, float(c[0]))
    xs = O.rescale(P, mul_const_next(P, x, 1.0 / den))
    return _mr(P, xs, p, rlk)


def mul_const_to(P, x: O.Ct, value: float, target_scale: float) -> O.Ct:
    """x times `value` encoded at the scale c = target q / s_x (q the prime the
    next rescale drops): the rescaled product has scale `target_scale`."""
    q = P.q[x.level - 1]
    cs = target_scale * q / x.scale
    k = int(O.round_half_away(np.array([value * cs]))[0])
    return O.Ct(O.ct_mul_int(P, x, k).c, x.scale * cs)


def mul_const_like(P, x: O.Ct, value: float, target_scale: float) -> O.Ct:
    """x times `value` encoded at the scale c = target / s_x: the product has
    scale `target_scale` itself (a term of a sum formed before its rescale)."""
    cs = target_scale / x.scale
    k = int(O.round_half_away(np.array([value * cs]))[0])
    return O.Ct(O.ct_mul_int(P, x, k).c, x.scale * cs)


# odd powers of a minimax stage and the two lower powers each is the product of
ODD_TREE = {2: (1, 1), 3: (2, 1), 4: (2, 2), 5: (4, 1), 7: (4, 3), 8: (4, 4), 9: (8, 1), 11: (8, 3),
            13: (8, 5), 15: (8, 7)}


def minimax_stage(P, x: O.Ct, coeffs, rlk) -> O.Ct:
    """One stage p(x) = sum_k coeffs[k] x^(2k+1) of a composite minimax sign
    approximation (Tab. 2 thresholds; the coefficients an input, designed by
    oracle/remez.py): the odd powers x^3 .. x^d and their helpers x^2, x^4,
    x^8 by ODD_TREE (each relinearised and rescaled, depth 4 for d = 15); the
    highest term c_d x^d with the constant at the next prime's scale, every
    other term c_k x^k with its constant at the scale that brings it to the
    sum's scale before the rescale (mul_const_like), added from k = d - 2
    down, and the sum rescaled once (the reading of EvalMod's sums, App. A.3:
    one rescale per sum)."""
    d = 2 * len(coeffs) - 1
    Xp = {1: x}
    for k in sorted(ODD_TREE):
        if (k <= d) if k % 2 else (k + 1 <= d):       # an even power only as a factor
            a, b = ODD_TREE[k]
            Xp[k] = _mr(P, Xp[a], Xp[b], rlk)
    acc = mul_const_next(P, Xp[d], float(coeffs[-1]))
    for k in range(d - 2, 0, -2):
        acc = O.ct_add(P, acc, mul_const_like(P, Xp[k], float(coeffs[(k - 1) // 2]), acc.scale))
    return O.rescale(P, acc)


def fp64_minimax(u, sign_coeffs):
    for c in sign_coeffs:
        u = u * np.polynomial.polynomial.polyval(u * u, np.asarray(c, dtype=np.float64))
    return u


def global_threshold(P, count: O.Ct, T1: O.Ct, inv_p: float, sign_coeffs, rlk) -> O.Ct:
    """The global threshold on the count (Sec. 5.3, Threshold2 of Tab. 2):
    step((count - t1) p^-1) with t1 encrypted and p public: the difference,
    times p^-1 at the next prime's scale and rescaled, the minimax stages,
    then (u + 1) with the scale doubled."""
    u = O.ct_sub(P, count, T1)
    u = O.rescale(P, mul_const_next(P, u, inv_p))
    for c in sign_coeffs:
        u = minimax_stage(P, u, c, rlk)
    s = add_const(P, u, 1.0)
    return O.Ct(s.c, s.scale * 2.0)


def fp64_global_threshold(count, t1, inv_p, sign_coeffs):
    return (fp64_minimax((np.asarray(count, dtype=np.float64) - t1) * inv_p, sign_coeffs) + 1.0) / 2.0


FINAL_LIMBS = 2   # limbs the InnerSum runs on


def query_circuit(P, X, x_scale, W, C, T, H, rlk, gks, stages=3, log_slots=None, final_limbs=FINAL_LIMBS,
                  sign_degree=7, sign_coeffs=None):
    """X[b][a]: plaintext words at scale x_scale; W[a], C[k], T, H: oracle ciphertexts."""
    D = len(C) - 1
    total = None
    for b in range(len(X)):
        s = O.ct_mul_plain(P, W[0], X[b][0], x_scale)
        for a in range(1, len(W)):
            s = O.ct_add(P, s, O.ct_mul_plain(P, W[a], X[b][a], x_scale))
        s = O.rescale(P, s)
        Y = _powers(P, s, D, rlk)
        z2 = O.tensor(P, C[1], Y[1])
        for k in range(2, D + 1):
            z2 = O.ct_add(P, z2, O.tensor(P, C[k], Y[k]))
        z = O.ct_add(P, O.rescale(P, O.relinearize(P, z2, rlk)), C[0])
        u = _mr(P, O.ct_sub(P, z, T), H, rlk)
        if sign_coeffs is not None:          # composite minimax stages (their count replaces `stages`)
            for c in sign_coeffs:
                u = minimax_stage(P, u, c, rlk)
        else:
            for _ in range(stages):
                u = sign_stage(P, u, rlk, sign_degree)
        step = add_const(P, u, 1.0)
        step = O.Ct(step.c, step.scale * 2.0)
        total = step if total is None else O.ct_add(P, total, step)
    total = O.Ct(total.c[:, :min(final_limbs, total.level)], total.scale)
    return O.rotate_sum(P, total, log_slots if log_slots is not None else P.logn - 1, gks)
