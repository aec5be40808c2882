"""EvalMod, the modular-reduction step of bootstrapping (App. A.3), as an op
list for pfx_run_circuit.

The slots hold t = I + m/q_0 (I a small integer, |t| <= K); the list computes
the scaled sine sin(2 pi t) / (2 pi), the reduction of t modulo 1 up to a cubic
term:

    u   = ((t - 1/4) / 2^r) / a                  a = (K + 1/4) / 2^r
    T_1 = u, T_2k = 2 T_k^2 - 1, T_2k+1 = 2 T_k T_k+1 - T_1
    c   = sum_k c_k T_k + c_0                    Chebyshev approximation of
                                                 cos(2 pi a u) on [-1, 1]
    c  <- 2 c^2 - 1, r times                     double angle
    out = c * f / (2 pi)                         f = out_factor (1 by default)

Every ciphertext product is relinearised (MUL_RELIN) and rescaled, the
factors 2 are integer products (MUL_INT), constants added with ADD_CONST.
Terms that are added meet at one scale exactly, and a sum is rescaled once,
after its last term: T_1 enters each odd T_k as MUL_CONST_LIKE(T_1, 1, the
product before its rescale), T_k = RESCALE(2 T_i T_j - that); c_d T_d is a
constant product at the next prime's scale (MUL_CONST), the other c_k T_k are
brought to that scale (MUL_CONST_LIKE) and summed from k = d down, then one
RESCALE (the sum sits at the level of T_d; ADD drops the others' extra
primes).  Per lane that is 30 rescales for d = 24, r = 4 instead of 64 with
one per term.
The coefficients are an input (the caller interpolates cos(2 pi a x), e.g. at
Chebyshev points).  Depth: 1 + ceil(log2 d) + 1 + r + 1 levels for
d = len(coeffs) - 1.

Register 0 is the input (read-only); `out` names the result.  With lanes = n
the list evaluates n inputs (registers 0 .. n-1) side by side, each op issued
for every lane in turn, so the lanes' products form runs of independent
HMult + relin ops that the executor batches into one key switch; `outs` names
the n results.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

from . import pfx as X


@dataclass
class EvalModPlan:
    coeffs: list
    r: int = 3
    K: float = 8.0
    out_factor: float = 1.0
    lanes: int = 1
    ops: list = field(default_factory=list)
    n_regs: int = 0
    n_inputs: int = 1
    out: int = -1
    outs: list = field(default_factory=list)

    def __post_init__(self):
        assert self.lanes >= 1
        self._next = 1
        self._build()
        n = self.lanes
        one, self.ops = self.ops, []

        def reg(r, i):                   # register r of the one-lane list, lane i
            return i if r == 0 else n + (r - 1) * n + i
        for code, dst, a, b, k, value in one:
            for i in range(n):
                self.ops.append((code, reg(dst, i), reg(a, i), reg(b, i) if b >= 0 else b, k, value))
        self.outs = [reg(self.out, i) for i in range(n)]
        self.out = self.outs[0]
        self.n_inputs = n
        self.n_regs = n + (self._next - 1) * n
        self.reg_degree = [1] * self.n_regs

    def _new(self) -> int:
        r = self._next
        self._next += 1
        return r

    def _op(self, code, dst, a, b=-1, k=0, value=0.0):
        self.ops.append((code, dst, a, b, k, value))

    def _build(self):
        d = len(self.coeffs) - 1
        assert d >= 1 and self.r >= 0
        a = (self.K + 0.25) / 2 ** self.r
        t = self._new()
        self._op(X.OP_ADD_CONST, t, 0, value=-0.25)
        T = {1: self._new()}
        self._op(X.OP_MUL_CONST, T[1], t, value=1.0 / (2 ** self.r * a))
        self._op(X.OP_RESCALE, T[1], T[1])
        for k in range(2, d + 1):
            i, j = (k + 1) // 2, k // 2              # T_k = 2 T_i T_j - T_(i-j)
            T[k] = self._new()
            self._op(X.OP_MUL_RELIN, T[k], T[i], T[j])
            if i == j:
                self._op(X.OP_RESCALE, T[k], T[k])
                self._op(X.OP_MUL_INT, T[k], T[k], k=2)
                self._op(X.OP_ADD_CONST, T[k], T[k], value=-1.0)
            else:
                self._op(X.OP_MUL_INT, T[k], T[k], k=2)
                t1 = self._new()                     # T_1 at the unrescaled product's scale
                self._op(X.OP_MUL_CONST_LIKE, t1, T[1], T[k], value=1.0)
                self._op(X.OP_SUB, T[k], T[k], t1)
                self._op(X.OP_RESCALE, T[k], T[k])
        c, term = self._new(), self._new()
        self._op(X.OP_MUL_CONST, c, T[d], value=float(self.coeffs[d]))
        for k in range(d - 1, 0, -1):
            self._op(X.OP_MUL_CONST_LIKE, term, T[k], c, value=float(self.coeffs[k]))
            self._op(X.OP_ADD, c, c, term)
        self._op(X.OP_RESCALE, c, c)
        self._op(X.OP_ADD_CONST, c, c, value=float(self.coeffs[0]))
        for _ in range(self.r):
            sq = self._new()
            self._op(X.OP_MUL_RELIN, sq, c, c)
            self._op(X.OP_RESCALE, sq, sq)
            self._op(X.OP_MUL_INT, sq, sq, k=2)
            self._op(X.OP_ADD_CONST, sq, sq, value=-1.0)
            c = sq
        self.out = self._new()
        self._op(X.OP_MUL_CONST, self.out, c, value=self.out_factor / (2 * math.pi))
        self._op(X.OP_RESCALE, self.out, self.out)

    @property
    def depth(self) -> int:
        d = len(self.coeffs) - 1
        return 1 + math.ceil(math.log2(d)) + 1 + self.r + 1 if d > 1 else 3 + self.r
