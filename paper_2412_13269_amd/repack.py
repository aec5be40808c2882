"""Op lists of the private lookup-table evaluation and ring repacking
(pfx_run_circuit).

Lookup (Sec. 3.4): with the encrypted table U = Enc(u_f), u_f = f(0) -
f(N-1) X - ... - f(1) X^{N-1}, the ciphertext X^i * U holds f(i) in its
constant coefficient for a plaintext point i (op MONO).

Repacking (Sec. 3.2, Alg. 1) of n <= N ciphertexts c_0 .. c_{n-1} (zeros
beyond n): every input times N^-1 mod Q (op INV_N), then for round i < log N,
t = N / 2^(i+1), g = 2N - 1 for i = 0 and 5^(2^(i-1)) mod 2N after,

    c_j <- c_j + c_{j+t} X^t + phi_g(c_j - c_{j+t} X^t)      (j < t)

and c_0 is the result, an encryption of sum_j m_j[0] X^j (Lemma 1).  The
zero ciphertexts are not materialised: the inputs are c_0 .. c_{n-1}, so a
pair whose c_{j+t} is zero takes c_j + phi_g(c_j) (the same words as
c_j + 0 + phi_g(c_j - 0)) and a pair of zeros stays zero.

Within a round the pairs are independent, so the ops are emitted kind by kind
(all monomial products, then all differences, all automorphisms, all sums):
the executor collects the elementwise runs into multi-record launches and
runs the automorphisms, which share one Galois key, as batched key switches.

Registers: 0 .. n_inputs - 1 are the inputs (the table U for a lookup plan,
else the n ciphertexts); every work register is of degree 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import pfx as X


def repack_galois(logn: int, i: int) -> int:
    """Galois element of round i of the repacking."""
    N = 1 << logn
    return 2 * N - 1 if i == 0 else pow(5, 1 << (i - 1), 2 * N)


def repack_keys_needed(logn: int) -> list:
    """Galois elements whose keys the repacking uses (log N of them)."""
    return [repack_galois(logn, i) for i in range(logn)]


@dataclass
class RepackPlan:
    logn: int
    n: int                       # ciphertexts to repack (<= N)
    points: list | None = None   # lookup points: inputs = [U]; else inputs = the n ciphertexts
    ops: list = field(default_factory=list)
    n_regs: int = 0
    n_inputs: int = 0
    out: int = -1

    def __post_init__(self):
        N = 1 << self.logn
        assert 1 <= self.n <= N
        if self.points is not None:
            assert len(self.points) == self.n
        self.n_inputs = 1 if self.points is not None else self.n
        self._next = self.n_inputs
        self._free: list = []
        self._build()
        self.n_regs = self._next
        self.reg_degree = [1] * self.n_regs

    def _new(self) -> int:
        if self._free:
            return self._free.pop()
        r = self._next
        self._next += 1
        return r

    def _op(self, code, dst, a, b=-1, k=0, value=0.0):
        self.ops.append((code, dst, a, b, k, value))

    def _build(self):
        N, n = 1 << self.logn, self.n
        c = {}
        if self.points is not None:
            # N^-1 (U X^i) = (N^-1 U) X^i: one pre-multiplication for all points
            t = self._new()
            self._op(X.OP_INV_N, t, 0)
            for j, p in enumerate(self.points):
                c[j] = self._new()
                self._op(X.OP_MONO, c[j], t, k=int(p) % (2 * N))
            self._free.append(t)
        else:
            for j in range(n):
                c[j] = self._new()
                self._op(X.OP_INV_N, c[j], j)
        for i in range(self.logn):
            t = N >> (i + 1)
            g = repack_galois(self.logn, i)
            both = [j for j in range(t) if j + t in c]               # inputs are c_0 .. c_{n-1}
            low = [j for j in range(t) if j in c and j + t not in c]  # c_{j+t} = 0
            u, v, w = {}, {}, {}
            for j in both:                              # u = c_{j+t} X^t
                u[j] = self._new()
                self._op(X.OP_MONO, u[j], c[j + t], k=t)
            for j in both:                              # v = c_j - u
                v[j] = self._new()
                self._op(X.OP_SUB, v[j], c[j], u[j])
            for j in both:                              # w = phi_g(v)
                w[j] = self._new()
                self._op(X.OP_GALOIS, w[j], v[j], k=g)
            for j in low:                               # c_{j+t} = 0: w = phi_g(c_j)
                w[j] = self._new()
                self._op(X.OP_GALOIS, w[j], c[j], k=g)
            for j in both:                              # c_j + u
                self._op(X.OP_ADD, c[j], c[j], u[j])
            for j in both + low:                        # ... + w
                self._op(X.OP_ADD, c[j], c[j], w[j])
            for j in range(t, N):                       # the upper half is no longer read
                if j in c:
                    self._free.append(c.pop(j))
            self._free += list(u.values()) + list(v.values()) + list(w.values())
        self.out = c[0]

    @property
    def key_switches(self) -> int:
        return sum(1 for o in self.ops if o[0] == X.OP_GALOIS)
