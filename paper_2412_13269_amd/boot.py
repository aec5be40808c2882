"""Half-BTS (Sec. 4.3, App. A.3-A.4): a coefficient-encoded ciphertext of one
limb -> one whose slots hold its coefficients, as calls of the C-ABI.

    y   = ModRaise(x) to n_limbs, read at scale q_0      pfx_mod_raise, pfx_ct_set_scale
    w/2 = CoeffsToSlots(y): the dense matrix B/2 by the   pfx_linear_transform
          BSGS diagonal method (before its rescale)
    then the op list HalfBootPlan (pfx_run_circuit):
    z   = rescale(w/2)
    re  = z + conj(z),  im = X^(3N/2) (z - conj(z))      conj: Galois element 2N - 1;
                                                         X^(3N/2) multiplies slots by -i
    re, im <- EvalMod(re), EvalMod(im)                   two lanes side by side
    out = re + X^(N/2) im

After ModRaise the coefficients read at scale q_0 are t = I + m/q_0; the slots
of re and im are t_j and t_(j+N/2), EvalMod's last constant carries q_0 / Delta,
so slot j of out holds m_j / Delta + i m_(j+N/2) / Delta.  Its depth is one
level for CoeffsToSlots plus EvalMod's.
"""
from __future__ import annotations

import numpy as np

from . import pfx as X
from .evalmod import EvalModPlan


def c2s_half_diagonals(N: int):
    """The N/2 generalised diagonals of B/2, B[j, l] = (2/N) zeta_l^(-j) with
    zeta_l = exp(i pi 5^l / N) the slot roots (App. A.4: B maps the slots to
    w_j = m_j + i m_(j+N/2)); diagonal k holds B[j, (j + k) mod N/2] / 2 at slot
    j, so B z / 2 = sum_k d_k (.) rot(z, k)."""
    n = N // 2
    five = np.empty(n, dtype=np.int64)
    five[0] = 1
    for l in range(1, n):
        five[l] = five[l - 1] * 5 % (2 * N)
    j = np.arange(n)
    out = []
    for k in range(n):
        l = (j + k) % n
        # zeta_l^(-j) = exp(-i pi 5^l j / N), the exponent reduced mod 2N
        e = (five[l] * j) % (2 * N)
        out.append(np.exp(-1j * np.pi * e / N) / N)
    return out


class HalfBootPlan:
    """Op list from the CoeffsToSlots product (register 0, read-only) to the
    slots; `out` names the result, `evalmod` is the two-lane EvalMod list."""

    def __init__(self, N: int, coeffs, r: int = 3, K: float = 8.0, out_factor: float = 1.0):
        n = N // 2
        em = EvalModPlan(list(coeffs), r, K, out_factor, lanes=2)
        self.evalmod = em
        z, zc, re, diff, im = 1, 2, 3, 4, 5
        ops = [(X.OP_RESCALE, z, 0, -1, 0, 0.0),
               (X.OP_GALOIS, zc, z, -1, 2 * N - 1, 0.0),
               (X.OP_ADD, re, z, zc, 0, 0.0),
               (X.OP_SUB, diff, z, zc, 0, 0.0),
               (X.OP_MONO, im, diff, -1, 3 * n, 0.0)]
        base = im + 1

        def reg(e):                      # EvalMod's registers after the ones above
            return (re, im)[e] if e < 2 else base + e - 2
        for code, dst, a, b, k, value in em.ops:
            ops.append((code, reg(dst), reg(a), reg(b) if b >= 0 else b, k, value))
        top = base + em.n_regs - 2
        ops.append((X.OP_MONO, top, reg(em.outs[1]), -1, n, 0.0))
        ops.append((X.OP_ADD, top + 1, reg(em.outs[0]), top, 0, 0.0))
        self.ops = ops
        self.out = top + 1
        self.n_regs = top + 2
        self.n_inputs = 1
        self.reg_degree = [1] * self.n_regs
        self.galois = [2 * N - 1]
        self.depth = 1 + em.depth


def half_bootstrap(ctx, x, n_limbs: int, q0: float, diags, n1: int, gks, rlk, plan: HalfBootPlan, regs, stream=None,
                   mode: int = X.RUN_EAGER):
    """x: one limb, coefficient-encoded; diags: the N/2 plaintext diagonals of
    B/2; gks: the Galois keys of the BSGS steps and of 2N - 1; regs: plan.n_regs
    ciphertexts of n_limbs limbs (register 0 receives the CoeffsToSlots
    product); mode: how pfx_run_circuit runs the op list (RUN_GRAPH captures
    it on the first call for these registers and replays it after).  Returns
    regs[plan.out]."""
    half = len(diags)
    X.pfx_mod_raise(ctx, x, n_limbs, regs[1], stream)
    X.pfx_ct_set_scale(regs[1], q0)
    X.pfx_linear_transform(ctx, regs[1], diags, list(range(half)), n1, gks, regs[0], stream)
    X.pfx_run_circuit(ctx, plan.ops, regs, plan.n_inputs, [], rlk, gks, mode, stream)
    return regs[plan.out]
