"""The private query as a native op list (pfx_run_circuit).

Circuit (the threshold-and-count phase of the paper's Alg. 2, with a
slot-domain linear score): for each block b of 2^(logN-1) records

    S   = rescale(sum_a W[a] * X[b][a])     (products accumulated in place)
    Y_k = S^k by the binary power tree (Y2 = Y1 Y1, Y3 = Y2 Y1, Y4 = Y2 Y2,
          Y5 = Y4 Y1, Y6 = Y4 Y2, Y7 = Y4 Y3, Y8 = Y4 Y4, Y(8+i) = Y8 Yi;
          each relinearised and rescaled), degree D <= 15
    Z   = rescale(relin(sum_{k=1..D} C[k] (x) Y_k)) + C[0]   (tensor products
          summed at degree 2, one relinearisation)
    U   = rescale(relin((Z - T) H))
    3 stages of f(x) = x P(x^2) / den, f7 (sign_degree 7: P = 35 - 35y + 21y^2
    - 5y^3, den 16) or its degree-15 sibling (sign_degree 15: P of degree 7,
    den 2048, the paper's first-threshold degree):
        Y1 = X^2, Y_k = powers of Y1 by the tree above (k <= deg P)
        P  = c1 Y1 + c2 Y2 + ... + c0            (integer products, constant)
        U  = rescale(relin(rescale(X * round(q/den)) * P))
  or, with sign_coeffs (the composite minimax thresholds of Tab. 2, one
  tuple of coefficients c_1, c_3, .., c_d per stage, their count replacing
  `stages`), per stage p(x) = sum c_k x^k:
        x^2, x^3, x^4, x^5, x^7, x^8, x^9, .. x^d by ODD_TREE (relinearised,
        rescaled; depth 4 for d = 15)
        acc = x^d * c_d at the next prime's scale
        acc = acc + x^k * c_k at acc's scale, k = d - 2 down to 1
                                                           (MUL_CONST_LIKE)
        acc = rescale(acc)                                 (one per sum)
    step_b = (U + 1) with the scale doubled
  OUT = InnerSum(step_0 + step_1 + ...) on the first final_limbs limbs

Inputs (registers, read-only): W[0..A), C[0..D], T, H.  Plaintexts: X[b][a]
at index b * A + a.  The op list and the register allocation are built here;
the library executes them (eagerly, or captured once into a HIP graph; on one
stream, or scheduled over its lane streams by register dependencies).  The
registers that hold the degree-2 sum need capacity for degree 2: reg_degree
gives the capacity degree of every register (1 or 2).

Register allocation: temporaries are recycled through a free list.  With
parallel=False and interleave=False one list serves the whole circuit (fewest
registers: the smallest HBM footprint, the natural choice on one stream).
Otherwise every record block recycles only its own registers (more registers):
  parallel=True   the blocks of lane l (b mod lanes == l) follow a LANE l marker
                  and the sum of the blocks a LANE -1 marker, so that with
                  PFX_RUN_LANES the lanes run concurrently on the library's lane
                  streams; without it the markers are ignored;
  interleave=True the op lists of the blocks of one lane (of the whole circuit
                  without parallel) are interleaved op by op: the blocks' i-th
                  ops sit side by side, so their HMult + relin ops form runs of
                  independent ops that the library executes as one batched key
                  switch;
  interleave=G    (an int >= 2, without parallel) the blocks are interleaved in
                  groups of G, one group after the other; block i of a group
                  reuses the registers of block i of the previous group, so the
                  footprint is that of G blocks whatever the database size.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import pfx as X

# composite-sign stages f(x) = x P(x^2) / den: integer coefficients of P
# (y^0, y^1, ...) and den, for stage degree 7 (f7) and 15
SIGN = {7: ((35, -35, 21, -5), 16),
        15: ((6435, -15015, 27027, -32175, 25025, -12285, 3465, -429), 2048)}

# minimax stages: the odd powers x^3 .. x^15 and the even helpers x^2, x^4,
# x^8, each the product of the two lower powers listed
ODD_TREE = {2: (1, 1), 3: (2, 1), 4: (2, 2), 5: (4, 1), 7: (4, 3), 8: (4, 4), 9: (8, 1), 11: (8, 3),
            13: (8, 5), 15: (8, 7)}


class _OpList:
    """Op-list building blocks shared by the plans: registers (free lists by
    capacity degree, inputs never recycled) and the op sequences of an
    HMult + relin + rescale and of one minimax sign stage."""

    # register allocation: free lists by capacity degree
    def _new(self, degree: int = 1) -> int:
        if self._free[degree]:
            return self._free[degree].pop()
        r = self._next
        self._next += 1
        if degree == 2:
            self._deg2.add(r)
        return r

    def _drop(self, *regs):
        for r in regs:
            if r >= self.n_inputs:
                self._free[2 if r in self._deg2 else 1].append(r)

    def _op(self, code, dst, a, b=-1, k=0, value=0.0):
        self.ops.append((code, dst, a, b, k, value))

    def _mr(self, dst, a, b):
        if dst in (a, b):      # the product goes to a temporary: the library then
            t = self._new()    # never stores the tensor product (its output may
            self._op(X.OP_MUL_RELIN, t, a, b)   # not alias an operand for that)
            self._op(X.OP_RESCALE, dst, t)
            self._drop(t)
        else:
            self._op(X.OP_MUL_RELIN, dst, a, b)
            self._op(X.OP_RESCALE, dst, dst)

    def _minimax_stage(self, u: int, c) -> int:
        d = 2 * len(c) - 1
        xp = {1: u}
        for k in sorted(ODD_TREE):
            if (k <= d) if k % 2 else (k + 1 <= d):      # an even power only as a factor
                xp[k] = self._new()
                self._mr(xp[k], xp[ODD_TREE[k][0]], xp[ODD_TREE[k][1]])
        acc = self._new()
        self._op(X.OP_MUL_CONST, acc, xp[d], value=c[-1])
        t = self._new()
        for k in range(d - 2, 0, -2):
            self._op(X.OP_MUL_CONST_LIKE, t, xp[k], acc, value=c[(k - 1) // 2])
            self._op(X.OP_ADD, acc, acc, t)
        self._op(X.OP_RESCALE, acc, acc)
        self._drop(t, *xp.values())
        return acc


@dataclass
class QueryPlan(_OpList):
    n_blocks: int
    attributes: int = 8
    degree: int = 7
    stages: int = 3
    log_slots: int = 15
    parallel: bool = False
    lanes: int = 4
    interleave: bool | int = False
    final_limbs: int = 2
    sign_degree: int = 7      # 7 or 15: the degree of each composite-sign stage
    sign_coeffs: tuple | None = None   # minimax stages (c_1, c_3, .., c_d) instead
    ops: list = field(default_factory=list)
    n_regs: int = 0
    out: int = -1

    def __post_init__(self):
        A, D = self.attributes, self.degree
        assert 1 <= D <= 15 and A >= 1 and self.n_blocks >= 1
        assert self.sign_degree in SIGN
        if self.sign_coeffs is not None:
            self.sign_coeffs = tuple(tuple(float(v) for v in c) for c in self.sign_coeffs)
            assert self.sign_coeffs and all(1 <= len(c) <= 8 for c in self.sign_coeffs)
        self.W = list(range(A))
        self.C = list(range(A, A + D + 1))
        self.T = A + D + 1
        self.H = A + D + 2
        self.n_inputs = A + D + 3
        self._free: dict = {1: [], 2: []}
        self._next = self.n_inputs
        self._deg2: set = set()
        self._build()
        self.n_regs = self._next
        self.reg_degree = [2 if r in self._deg2 else 1 for r in range(self.n_regs)]



    def _block(self, b: int) -> int:
        A, D = self.attributes, self.degree
        s = self._new()
        self._op(X.OP_MUL_PLAIN, s, self.W[0], b * A)
        for a in range(1, A):
            self._op(X.OP_MUL_PLAIN_ACC, s, self.W[a], b * A + a)
        self._op(X.OP_RESCALE, s, s)
        Y = {1: s}
        tree = {2: (1, 1), 3: (2, 1), 4: (2, 2), 5: (4, 1), 6: (4, 2), 7: (4, 3), 8: (4, 4)}
        tree.update({8 + i: (8, i) for i in range(1, 8)})
        for k in range(2, D + 1):
            Y[k] = self._new()
            self._mr(Y[k], Y[tree[k][0]], Y[tree[k][1]])
        z2 = self._new(2)
        self._op(X.OP_MUL, z2, self.C[1], Y[1])
        for k in range(2, D + 1):
            self._op(X.OP_MUL_ACC, z2, self.C[k], Y[k])
        z = self._new()
        self._op(X.OP_RELIN, z, z2)
        self._op(X.OP_RESCALE, z, z)
        self._drop(z2)
        self._op(X.OP_ADD, z, z, self.C[0])
        self._drop(*Y.values())
        u = self._new()
        self._op(X.OP_SUB, u, z, self.T)
        self._mr(u, u, self.H)
        self._drop(z)
        if self.sign_coeffs is not None:
            for c in self.sign_coeffs:
                u = self._minimax_stage(u, c)
        cs, den = SIGN[self.sign_degree]
        for _ in range(self.stages if self.sign_coeffs is None else 0):
            ys = {1: self._new()}
            self._mr(ys[1], u, u)                       # y = x^2
            for k in range(2, len(cs)):
                ys[k] = self._new()
                self._mr(ys[k], ys[tree[k][0]], ys[tree[k][1]])
            p = self._new()
            self._op(X.OP_MUL_INT, p, ys[1], k=cs[1])
            for k in range(2, len(cs)):
                self._op(X.OP_MUL_INT_ACC, p, ys[k], k=cs[k])
            self._op(X.OP_ADD_CONST, p, p, value=float(cs[0]))
            self._op(X.OP_MUL_CONST, ys[1], u, value=1.0 / den)     # x / den at the next prime's scale
            self._op(X.OP_RESCALE, ys[1], ys[1])
            self._mr(u, ys[1], p)
            self._drop(*ys.values(), p)
        self._op(X.OP_ADD_CONST, u, u, value=1.0)
        self._op(X.OP_SCALE_MUL, u, u, value=2.0)
        return u

    def _build(self):
        if self.parallel or self.interleave is True:
            lanes = self.lanes if self.parallel else 1
            us = []
            for lane in range(lanes):
                blocks = [b for b in range(self.n_blocks) if b % lanes == lane]
                if not blocks:
                    continue
                if self.parallel:
                    self._op(X.OP_LANE, 0, 0, k=lane)
                lists = []
                for b in blocks:
                    self._free = {1: [], 2: []}     # every block recycles only its own registers
                    start = len(self.ops)
                    us.append(self._block(b))
                    lists.append(self.ops[start:])
                    del self.ops[start:]
                if self.interleave:
                    assert len({len(ops) for ops in lists}) == 1
                    for step in zip(*lists):
                        self.ops.extend(step)
                else:
                    for ops in lists:
                        self.ops.extend(ops)
            if self.parallel:
                self._op(X.OP_LANE, 0, 0, k=-1)
            self._free = {1: [], 2: []}
            total = us[0]
            for u in us[1:]:
                self._op(X.OP_ADD, total, total, u)
        elif self.interleave is not False and int(self.interleave) >= 2:
            G = int(self.interleave)
            pools = [{1: [], 2: []} for _ in range(G)]   # block i of every group recycles pools[i]
            total = None
            for g0 in range(0, self.n_blocks, G):
                lists, us = [], []
                for i, b in enumerate(range(g0, min(g0 + G, self.n_blocks))):
                    self._free = pools[i]
                    start = len(self.ops)
                    us.append(self._block(b))
                    lists.append(self.ops[start:])
                    del self.ops[start:]
                assert len({len(ops) for ops in lists}) == 1
                for step in zip(*lists):
                    self.ops.extend(step)
                for i, u in enumerate(us):
                    if total is None:
                        total = u
                    else:
                        self._op(X.OP_ADD, total, total, u)
                        pools[i][1].append(u)
            self._free = {d: [r for pool in pools for r in pool[d]] for d in (1, 2)}
        else:
            total = None
            for b in range(self.n_blocks):
                u = self._block(b)
                if total is None:
                    total = u
                else:
                    self._op(X.OP_ADD, total, total, u)
                    self._drop(u)
        self._op(X.OP_DROP, total, total, k=self.final_limbs)   # InnerSum on the lowest limbs that hold the count
        self.out = self._new()
        self._op(X.OP_ROTATE_SUM, self.out, total, k=self.log_slots)
        self._drop(total)

    @property
    def key_switches(self) -> int:
        return sum(1 for o in self.ops if o[0] in (X.OP_MUL_RELIN, X.OP_RELIN)) + self.log_slots


@dataclass
class GlobalThresholdPlan(_OpList):
    """The global threshold on the count (Sec. 5.3, Threshold2 of Tab. 2):
    step((count - t1) p^-1) with t1 encrypted and p public, by the minimax
    stages `sign_coeffs`:

        U   = rescale((COUNT - T1) * p^-1 at the next prime's scale)
        U   = minimax stage (as in QueryPlan) for each tuple of coefficients
        OUT = (U + 1) with the scale doubled

    Inputs (registers, read-only): 0 the count (every slot), 1 t1.  Depth
    1 + 5 per stage of degree 15: with six stages a fresh ciphertext of at
    least 32 limbs (the count after a bootstrapping, in the paper)."""
    sign_coeffs: tuple
    inv_p: float
    ops: list = field(default_factory=list)
    n_regs: int = 0
    out: int = -1

    def __post_init__(self):
        self.sign_coeffs = tuple(tuple(float(v) for v in c) for c in self.sign_coeffs)
        assert self.sign_coeffs and all(1 <= len(c) <= 8 for c in self.sign_coeffs) and self.inv_p > 0
        self.n_inputs = 2
        self._free: dict = {1: [], 2: []}
        self._next = self.n_inputs
        self._deg2: set = set()
        u = self._new()
        self._op(X.OP_SUB, u, 0, 1)
        self._op(X.OP_MUL_CONST, u, u, value=self.inv_p)
        self._op(X.OP_RESCALE, u, u)
        for c in self.sign_coeffs:
            u = self._minimax_stage(u, c)
        self._op(X.OP_ADD_CONST, u, u, value=1.0)
        self._op(X.OP_SCALE_MUL, u, u, value=2.0)
        self.out = u
        self.n_regs = self._next
        self.reg_degree = [1] * self.n_regs

    @property
    def depth(self) -> int:
        return 1 + sum(1 + (2 * len(c) - 2).bit_length() for c in self.sign_coeffs)   # x^d, then c_d x^d
