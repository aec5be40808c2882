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

Factorised CoeffsToSlots (App. A.4, for the paper's ring): B = A^-1 with A the
slot transform, and A = F_L ... F_1 R (R the bit reversal of the n = N/2
packed coefficients, F_s the radix-2 butterfly stage of length 2^s, twiddle of
pair j: exp(2 pi i (5^j mod 2^(s+2)) / 2^(s+2))).  So F_1^-1 ... F_L^-1 = R B
needs no permutation and leaves slot p holding w_rev(p): every stage has three
generalised diagonals (steps 0, +-2^(s-1)), and `levels` groups of consecutive
stages, each one BSGS transform and one rescale, replace the dense product
(N/2 diagonals) at a cost of levels - 1 extra levels.  The slots of the result
are then in bit-reversed order, which EvalMod (slot-wise) and what follows
Half-BTS (thresholds, InnerSum) do not see.

Sparse packing (App. A.3-A.4, n = N/2r slots): a message on the powers of
Y = X^r has n slots, each repeated r times among the N/2, and its packed
coefficients w_j = m_(jr) + i m_((j+n)r) are B' z for the n-slot matrix B'
(roots exp(i pi 5^l / 2n)).  The trace-like map after ModRaise
(pfx_subring_trace, log r automorphisms) leaves r times the subring part, so
the stages are those of R B' / (2r) on n slots: their steps are below n and
their diagonals have length n (encoded with n slots, hence repeated), and a
rotation of the full ring by k rotates every period of n slots by k mod n.
The op list is unchanged: conjugation and the monomials act slot by slot.
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


def _inverse_stage(n: int, s: int) -> dict:
    """F_s^-1 as {step: diagonal}: a lower row p of a pair takes (u + v) / 2,
    the upper row (u - v) / (2 w_j)."""
    lh = 1 << (s - 1)
    ln = lh << 1
    p = np.arange(n)
    j = p % ln
    lower = j < lh
    jj = np.where(lower, j, j - lh)
    pw = np.empty(lh, dtype=np.int64)            # 5^t mod 4 ln, t < lh
    pw[0] = 1
    for t in range(1, lh):
        pw[t] = pw[t - 1] * 5 % (4 * ln)
    w = np.exp(2j * np.pi * pw[jj] / (4 * ln))
    out = {0: np.where(lower, 0.5, -0.5 / w)}
    for step, d in ((lh % n, np.where(lower, 0.5, 0.0)), ((n - lh) % n, np.where(lower, 0.0, 0.5 / w))):
        out[step] = out.get(step, 0) + d
    return out


def _after(m2: dict, m1: dict, n: int) -> dict:
    """Diagonals of m2 applied after m1: d_k[p] = sum_a m2_a[p] m1_(k-a)[p + a]."""
    out = {}
    for a, d2 in m2.items():
        for b, d1 in m1.items():
            k = (a + b) % n
            out[k] = out.get(k, 0) + d2 * np.roll(d1, -a)
    return out


def c2s_factor_stages(N: int, levels: int, factor: float = 0.5, n_slots: int | None = None) -> list:
    """[(steps, diagonals)] of the merged stages of factor * R B in the order
    they apply (F_L^-1 first; ceil(L / levels) radix-2 stages per group); for
    n_slots < N/2 those of the n-slot matrix B' (steps below n_slots,
    diagonals of length n_slots)."""
    n = n_slots or N // 2
    assert n & (n - 1) == 0 and 1 <= n <= N // 2
    L = n.bit_length() - 1
    k = -(-L // levels)
    order = list(range(L, 0, -1))
    out = []
    for g in range(0, L, k):
        acc = None
        for s in order[g:g + k]:
            st = _inverse_stage(n, s)
            acc = st if acc is None else _after(st, acc, n)
        if not out:
            acc = {o: factor * d for o, d in acc.items()}
        steps = sorted(o for o, d in acc.items() if np.any(d != 0))
        out.append((steps, [acc[o] for o in steps]))
    return out


def bsgs_n1(steps) -> int:
    """Baby-step count for a stage's steps: the stride times the power of two
    nearest the square root of their number."""
    stride = min([s for s in steps if s] or [1])
    return stride * (1 << max(0, (len(steps).bit_length() + 1) // 2))


def bsgs_rotations(N: int, steps, n1: int) -> set:
    """Slot rotations (mod N/2, non-zero) of the baby and giant steps of one
    BSGS transform."""
    half = N // 2
    return {r % half for s in steps for r in (s % n1, n1 * (s // n1)) if r % half}


def bsgs_galois(N: int, steps, n1: int) -> set:
    """Galois elements of the baby and giant steps of one BSGS transform."""
    return {pow(5, r, 2 * N) for r in bsgs_rotations(N, steps, n1)}


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
        # the two real ciphertexts the paper's Half-BTS returns (Sec. 4.3): the
        # scores of the real and of the imaginary parts (ctL, ctR), each real
        # in every slot, before they are recombined into `out`
        self.out_lr = (reg(em.outs[0]), reg(em.outs[1]))
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


def trace_rotations(N: int, log_r: int) -> list:
    """Slot rotations k whose Galois elements 5^k mod 2N are the trace-like
    map's, N/2^t + 1 for t < log_r (each is 1 mod 4, so a power of 5, for
    log_r <= log2(N) - 2)."""
    assert 0 <= log_r <= N.bit_length() - 3
    want = {N // (1 << t) + 1: t for t in range(log_r)}
    out = [0] * log_r
    g = 1
    for k in range(N // 2):
        if g in want:
            out[want[g]] = k
        g = g * 5 % (2 * N)
    return out


def half_bootstrap_factorised(ctx, x, n_limbs: int, q0: float, stages, gks, rlk, plan: HalfBootPlan, regs,
                              stream=None, mode: int = X.RUN_EAGER, log_r: int = 0):
    """Half-BTS with the factorised CoeffsToSlots: stages = [(steps, diagonal
    plaintexts, n1)] of factor-1/2 R B (c2s_factor_stages), each a BSGS
    transform; every stage but the last is rescaled here, the last one's
    product goes to regs[0] for the op list (whose first op rescales it).
    regs[1] and regs[2] hold the stages' intermediates before the op list
    reuses them.  Slot p of regs[plan.out] holds m_rev(p) / Delta +
    i m_(rev(p) + N/2) / Delta.
    Sparse packing (log_r > 0): the trace-like map runs after ModRaise (its
    keys, trace_rotations, among gks) and the stages are c2s_factor_stages(N,
    levels, 0.5 / 2^log_r, N / 2^(log_r + 1)); slot p, and every slot p + k n,
    then holds m_(rev(p) r) / Delta + i m_((rev(p) + n) r) / Delta (n =
    N / 2r slots, r = 2^log_r, rev over log2(n) bits)."""
    X.pfx_mod_raise(ctx, x, n_limbs, regs[1], stream)
    if log_r:
        X.pfx_subring_trace(ctx, regs[1], log_r, gks, regs[1], stream)
    X.pfx_ct_set_scale(regs[1], q0)
    cur, other = 1, 2
    for i, (steps, pts, n1) in enumerate(stages):
        last = i == len(stages) - 1
        dst = 0 if last else other
        X.pfx_linear_transform(ctx, regs[cur], pts, steps, n1, gks, regs[dst], stream)
        if not last:
            X.pfx_rescale(ctx, regs[dst], regs[cur], stream)
    X.pfx_run_circuit(ctx, plan.ops, regs, plan.n_inputs, [], rlk, gks, mode, stream)
    return regs[plan.out]
