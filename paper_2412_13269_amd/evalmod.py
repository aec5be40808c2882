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
    out = c / (2 pi)

Every ciphertext product is relinearised and rescaled (MUL_RELIN, RESCALE),
the factors 2 are integer products (MUL_INT), each c_k T_k a constant product
at the scale of the next prime (MUL_CONST, RESCALE), the terms summed in order
of k, constants added with ADD_CONST.  The coefficients are an input (the
caller interpolates cos(2 pi a x), e.g. at Chebyshev points).  Depth:
1 + ceil(log2 d) + 1 + r + 1 levels for d = len(coeffs) - 1.

Register 0 is the input (read-only); `out` names the result.
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
    ops: list = field(default_factory=list)
    n_regs: int = 0
    n_inputs: int = 1
    out: int = -1

    def __post_init__(self):
        self._next = 1
        self._build()
        self.n_regs = self._next
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
            self._op(X.OP_RESCALE, T[k], T[k])
            self._op(X.OP_MUL_INT, T[k], T[k], k=2)
            if i == j:
                self._op(X.OP_ADD_CONST, T[k], T[k], value=-1.0)
            else:
                self._op(X.OP_SUB, T[k], T[k], T[1])
        c, term = self._new(), self._new()
        for k in range(1, d + 1):
            dst = c if k == 1 else term
            self._op(X.OP_MUL_CONST, dst, T[k], value=float(self.coeffs[k]))
            self._op(X.OP_RESCALE, dst, dst)
            if k > 1:
                self._op(X.OP_ADD, c, c, term)
        self._op(X.OP_ADD_CONST, c, c, value=float(self.coeffs[0]))
        for _ in range(self.r):
            sq = self._new()
            self._op(X.OP_MUL_RELIN, sq, c, c)
            self._op(X.OP_RESCALE, sq, sq)
            self._op(X.OP_MUL_INT, sq, sq, k=2)
            self._op(X.OP_ADD_CONST, sq, sq, value=-1.0)
            c = sq
        self.out = self._new()
        self._op(X.OP_MUL_CONST, self.out, c, value=1.0 / (2 * math.pi))
        self._op(X.OP_RESCALE, self.out, self.out)

    @property
    def depth(self) -> int:
        d = len(self.coeffs) - 1
        return 1 + math.ceil(math.log2(d)) + 1 + self.r + 1 if d > 1 else 3 + self.r
