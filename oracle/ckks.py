"""CPU oracle for the RNS-CKKS evaluation path (arXiv 2412.13269).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the HIP library: the primes, roots, constants, encoder and every
scheme operation below are computed here from their definitions, with Python
big integers for the constants and the plain C loops of ``ckks_ref.c`` for the
O(N log N) work.  Words are canonical residues in the coefficient domain.

What each function follows in the paper:

* ring and automorphisms ............ Sec. 2.2 (R_Q^N, phi_g : X -> X^g)
* RLWE encryption / decryption ...... Sec. 2.3 (c = (-a s + e + m, a))
* SwitchKeyGen / SwitchKey .......... Sec. 2.4.1 (swk_i = RLWE_{s'}(0) + w_i P s;
                                      output round(P^-1 <d, swk>))
* relinearisation, automorphism ..... Sec. 2.4.2 and App. A.2
* scale and rescale ................. Sec. 2.5 (round(c / Delta), modulus Q/Delta)
* slot encoding / decoding .......... App. A.1, "In the Canonical Embedding"
* rotation / conjugation ............ App. A.1 (phi_(0,k) rotates left by k,
                                      phi_(1,0) conjugates)

Readings where the paper is silent or garbled (each is pinned by tests):

* RNS primes: every prime is 1 mod 2^mod_log2; a prime of 50 bits or more is
  the next unused prime below 2^bits, a smaller one the next unused prime
  nearest 2^bits (offsets 0, +1, -1, +2, ... steps of 2^mod_log2).
* psi: the first g = 2, 3, ... with x = g^((q-1)/2N), x^N = -1 gives psi = x.
* hybrid gadget: digit j holds primes [alpha j, alpha j + alpha); w_j is the
  CRT idempotent of digit j over the full Q; ModUp is the fast (uncorrected)
  basis conversion; ModDown adds floor(P/2) before the fast conversion, so it
  rounds, as the paper's round(P^-1 ...) asks.
* rescale divides by the last prime with round-half-up of the [0, Q) lift.
* slots: n complex slots live in Y = X^(N/2n); slot j is p(zeta_j) with
  zeta_j = exp(i pi (5^j mod 4n) / 2n).  Encoding rounds half away from zero.

Parity unpinned: encoding at exact rounding ties (an FP64 tie can round either
way under a different FFT); the tests compare encodings within one unit.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_ref.c")
_SO = os.path.join(_HERE, "libpfo.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)


def build() -> str:
    """Compile the C loops (gcc, OpenMP).  Returns the shared-object path."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO, _SRC])
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        i, u, sz = ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
        L.pfo_ntt_naive.argtypes = [u, u, i, _u64p, _u64p]
        L.pfo_ntt.argtypes = [u, u, i, _u64p]
        L.pfo_intt.argtypes = [u, u, i, _u64p]
        L.pfo_negacyclic_mul_naive.argtypes = [u, i, _u64p, _u64p, _u64p]
        L.pfo_ntt_rns.argtypes = [i, _u64p, _u64p, i, _u64p]
        L.pfo_intt_rns.argtypes = [i, _u64p, _u64p, i, _u64p]
        L.pfo_polymul_rns.argtypes = [i, _u64p, _u64p, i, _u64p, _u64p, _u64p]
        L.pfo_pmul_rns.argtypes = [i, _u64p, sz, _u64p, _u64p, _u64p]
        L.pfo_smul_rns.argtypes = [i, _u64p, sz, _u64p, _u64p, _u64p]
        L.pfo_bconv.argtypes = [sz, i, _u64p, _u64p, _u64p, i, _u64p, _u64p, _u64p]
        L.pfo_automorphism.argtypes = [i, _u64p, i, u, _u64p, _u64p]
        L.pfo_threads.restype = i
        L.pfo_set_threads.argtypes = [i]
        _lib = L
    return _lib


def threads() -> int:
    """Threads the oracle's OpenMP loops use (results do not depend on it)."""
    return int(lib().pfo_threads())


def set_threads(n: int) -> None:
    lib().pfo_set_threads(int(n))


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def _u64(xs) -> np.ndarray:
    return np.ascontiguousarray(np.array([int(x) for x in xs], dtype=np.uint64))


# --------------------------------------------------------------------------
# Primes and roots
# --------------------------------------------------------------------------
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve prime bases (deterministic below 3e23)."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for b in _MR_BASES:
        x = pow(b, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def gen_primes(mod_log2: int, q_bits, p_bits):
    """Chain primes, in order q_0.. then p_0.. (rule in the module docstring)."""
    step = 1 << mod_log2
    used: set[int] = set()
    out = []
    for b in list(q_bits) + list(p_bits):
        if b >= 50:
            k = 1
            while True:
                c = (1 << b) + 1 - k * step
                if c not in used and is_prime(c):
                    break
                k += 1
        else:
            t = 0
            while True:
                k = (t + 1) // 2 if t % 2 == 1 else -(t // 2)
                c = (1 << b) + 1 + k * step
                if c > 2 and c not in used and is_prime(c):
                    break
                t += 1
        used.add(c)
        out.append(c)
    nq = len(q_bits)
    return out[:nq], out[nq:]


def find_psi(q: int, n: int) -> int:
    """Primitive 2N-th root of unity mod q (rule in the module docstring)."""
    assert (q - 1) % (2 * n) == 0
    g = 2
    while True:
        x = pow(g, (q - 1) // (2 * n), q)
        if pow(x, n, q) == q - 1:
            return x
        g += 1


def bitrev(x: int, bits: int) -> int:
    r = 0
    for i in range(bits):
        r |= ((x >> i) & 1) << (bits - 1 - i)
    return r


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
@dataclass
class Params:
    logn: int
    q_bits: list
    p_bits: list
    alpha: int
    mod_log2: int = 0
    q: list = field(default_factory=list)
    p: list = field(default_factory=list)

    def __post_init__(self):
        if not self.mod_log2:
            self.mod_log2 = self.logn + 1
        assert self.mod_log2 >= self.logn + 1
        self.q, self.p = gen_primes(self.mod_log2, self.q_bits, self.p_bits)
        self.N = 1 << self.logn
        self.L = len(self.q)
        self.K = len(self.p)
        self.psi_q = [find_psi(x, self.N) for x in self.q]
        self.psi_p = [find_psi(x, self.N) for x in self.p]

    @property
    def beta(self) -> int:
        return -(-self.L // self.alpha)

    def digits(self, level: int):
        """Prime indices of each key-switching digit active at `level` limbs."""
        return [list(range(j * self.alpha, min((j + 1) * self.alpha, level)))
                for j in range(-(-level // self.alpha))]

    def mods(self, level: int):
        return self.q[:level]

    def psis(self, level: int):
        return self.psi_q[:level]

    def ext_mods(self, level: int):
        return self.q[:level] + self.p

    def ext_psis(self, level: int):
        return self.psi_q[:level] + self.psi_p


def params_n12_three_50bit() -> Params:
    """N = 2^12, three 50-bit ciphertext primes and one 50-bit special prime."""
    return Params(12, [50, 50, 50], [50], alpha=1)


def params_50_45_chain(logn: int = 16, level: int = 24) -> Params:
    """N = 2^16, 24 ciphertext primes (one 50-bit, then 45-bit), 4 special
    primes of 50 bits, digits of 4 primes (dnum = 6).  Primes are 1 mod 2^17
    so the same chain serves every ring degree up to 2^16."""
    return Params(logn, [50] + [45] * (level - 1), [50] * 4, alpha=4, mod_log2=17)


# --------------------------------------------------------------------------
# Polynomial helpers over lists of moduli (rows = limbs)
# --------------------------------------------------------------------------
def ntt(a: np.ndarray, mods, psis, logn) -> np.ndarray:
    out = np.ascontiguousarray(a.copy())
    lib().pfo_ntt_rns(len(mods), _p(_u64(mods)), _p(_u64(psis)), logn, _p(out))
    return out


def intt(a: np.ndarray, mods, psis, logn) -> np.ndarray:
    out = np.ascontiguousarray(a.copy())
    lib().pfo_intt_rns(len(mods), _p(_u64(mods)), _p(_u64(psis)), logn, _p(out))
    return out


def polymul(a, b, mods, psis, logn) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().pfo_polymul_rns(len(mods), _p(_u64(mods)), _p(_u64(psis)), logn, _p(a), _p(b), _p(out))
    return out


def pmul(a, b, mods) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().pfo_pmul_rns(len(mods), _p(_u64(mods)), a.shape[1], _p(a), _p(b), _p(out))
    return out


def smul(a, ks, mods) -> np.ndarray:
    """Row l times the integer ks[l] (any Python int), mod mods[l]."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    kk = _u64([int(k) % int(m) for k, m in zip(ks, mods)])
    lib().pfo_smul_rns(len(mods), _p(_u64(mods)), a.shape[1], _p(a), _p(kk), _p(out))
    return out


def _col(mods) -> np.ndarray:
    return np.array([int(m) for m in mods], dtype=np.uint64)[:, None]


def add(a, b, mods) -> np.ndarray:
    return (a + b) % _col(mods)          # residues < 2^62: the sum cannot wrap


def sub(a, b, mods) -> np.ndarray:
    m = _col(mods)
    return (a + (m - b)) % m


def neg(a, mods) -> np.ndarray:
    m = _col(mods)
    return (m - a) % m


def add_int(a, vals, mods) -> np.ndarray:
    """Add the integer vals[l] (any Python int) to every coefficient of row l."""
    m = _col(mods)
    c = np.array([int(v) % int(q) for v, q in zip(vals, mods)], dtype=np.uint64)[:, None]
    return (a + c) % m


def from_ints(vals, mods) -> np.ndarray:
    """Integer polynomial (Python ints or an int64 array) -> residues."""
    vals = np.asarray(vals)
    out = np.empty((len(mods), len(vals)), dtype=np.uint64)
    if vals.dtype != object and np.issubdtype(vals.dtype, np.integer):
        v = vals.astype(np.int64)
        for i, q in enumerate(mods):
            out[i] = (v % np.int64(q)).astype(np.uint64)
    else:
        for i, q in enumerate(mods):
            out[i] = np.array([int(x) % int(q) for x in vals], dtype=np.uint64)
    return out


def bconv(x, mods_in, mods_out) -> np.ndarray:
    """Fast basis conversion of the residues x (rows over mods_in) to mods_out."""
    Qp = math.prod(int(m) for m in mods_in)
    qhat_inv = [pow(Qp // int(qi), -1, int(qi)) for qi in mods_in]
    qhat_mod = [[(Qp // int(qi)) % int(m) for m in mods_out] for qi in mods_in]
    x = np.ascontiguousarray(x, dtype=np.uint64)
    n = x.shape[1]
    out = np.empty((len(mods_out), n), dtype=np.uint64)
    lib().pfo_bconv(n, len(mods_in), _p(_u64(mods_in)), _p(x), _p(_u64(qhat_inv)),
                    len(mods_out), _p(_u64(mods_out)), _p(_u64(sum(qhat_mod, []))), _p(out))
    return out


def automorphism(a, g, mods, logn) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    lib().pfo_automorphism(len(mods), _p(_u64(mods)), logn, int(g), _p(a), _p(out))
    return out


def crt_centered(words: np.ndarray, mods) -> np.ndarray:
    """Centred integers in [-(Q-1)/2, (Q-1)/2] from residues (object array of
    ints).  Sec. 2.2 centres coefficients around 0; Q is odd, so the symmetric
    range holds exactly one lift of every residue."""
    mods = [int(m) for m in mods]
    Q = math.prod(mods)
    acc = np.zeros(words.shape[1], dtype=object)
    for i, q in enumerate(mods):
        Qi = Q // q
        acc = acc + words[i].astype(object) * (Qi * pow(Qi, -1, q))
    acc = acc % Q
    half = Q // 2
    return np.where(acc > half, acc - Q, acc)


# --------------------------------------------------------------------------
# Slot encoding (App. A.1, canonical embedding)
# --------------------------------------------------------------------------
def _slot_exponents(n: int) -> np.ndarray:
    return np.array([pow(5, j, 4 * n) for j in range(n)], dtype=np.int64)


def round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def encode_real_coeffs(z, N: int) -> np.ndarray:
    """Real coefficients p_k (k < 2n) of the polynomial with p(zeta_j) = z_j.

    The 2n primitive 4n-th roots are zeta_j and their conjugates, so by
    orthogonality p_k = (1/n) Re(sum_j z_j zeta_j^-k).  The sum is one
    length-4n DFT of the vector holding z_j at position 5^j mod 4n.
    """
    z = np.asarray(z, dtype=np.complex128)
    n = len(z)
    assert n & (n - 1) == 0 and 1 <= n <= N // 2
    v = np.zeros(4 * n, dtype=np.complex128)
    v[_slot_exponents(n)] = z
    return np.fft.fft(v)[: 2 * n].real / n


def encode(P: Params, z, scale: float, level: int) -> np.ndarray:
    """round(Delta * tau^-1(z)) placed on X^(k N/2n), as residues (level, N)."""
    N = P.N
    coeff = encode_real_coeffs(z, N)
    n = len(coeff) // 2
    gap = N // (2 * n)
    r = round_half_away(coeff * scale)
    if np.max(np.abs(r)) < 2.0 ** 62:
        ints = r.astype(np.int64)
    else:
        ints = np.array([int(x) for x in r], dtype=object)
    full = np.zeros(N, dtype=object if ints.dtype == object else np.int64)
    full[::gap] = ints
    return from_ints(full, P.mods(level))


def decode(P: Params, words: np.ndarray, scale: float, n: int) -> np.ndarray:
    """Slots z_j = p(zeta_j) with p_k = (centred coefficient of X^(k N/2n)) / Delta."""
    level = words.shape[0]
    gap = P.N // (2 * n)
    vals = crt_centered(words[:, ::gap], P.mods(level))
    p = np.array([float(v) for v in vals]) / scale
    w = np.zeros(4 * n, dtype=np.complex128)
    w[: 2 * n] = p
    G = np.fft.ifft(w) * (4 * n)
    return G[_slot_exponents(n)]


# --------------------------------------------------------------------------
# Keys, encryption (Sec. 2.3-2.4)
# --------------------------------------------------------------------------
@dataclass
class Ct:
    c: np.ndarray          # (degree + 1, level, N) residues, coefficient domain
    scale: float

    @property
    def level(self) -> int:
        return self.c.shape[1]


@dataclass
class SwitchKey:
    b: np.ndarray          # (beta, L + K, N)
    a: np.ndarray          # (beta, L + K, N)
    galois: int = 0        # 0: s^2 -> s; otherwise phi_g(s) -> s


def secret_rns(P: Params, s, mods) -> np.ndarray:
    return from_ints(np.asarray(s, dtype=np.int64), mods)


def swk_gen(P: Params, s, s_from_ext: np.ndarray, a: np.ndarray, e: np.ndarray, galois: int) -> SwitchKey:
    """swk_j = (-a_j s + e_j + P w_j s_from, a_j) over Q*P, w_j the CRT
    idempotent of digit j (1 mod its primes, 0 mod the other primes of Q)."""
    mods = P.ext_mods(P.L)
    psis = P.ext_psis(P.L)
    s_ext = secret_rns(P, s, mods)
    Qb = math.prod(P.q)
    Pb = math.prod(P.p)
    bs = []
    for j, D in enumerate(P.digits(P.L)):
        Qj = math.prod(P.q[i] for i in D)
        w_j = (Qb // Qj) * pow(Qb // Qj, -1, Qj)
        gadget = [(Pb * w_j) % m for m in mods]
        a_j = np.ascontiguousarray(a[j], dtype=np.uint64)
        e_j = from_ints(np.asarray(e[j], dtype=np.int64), mods)
        b_j = add(neg(polymul(a_j, s_ext, mods, psis, P.logn), mods), e_j, mods)
        b_j = add(b_j, smul(s_from_ext, gadget, mods), mods)
        bs.append(b_j)
    return SwitchKey(np.stack(bs), np.ascontiguousarray(a, dtype=np.uint64), galois)


def relin_key(P: Params, s, a, e) -> SwitchKey:
    mods = P.ext_mods(P.L)
    s_ext = secret_rns(P, s, mods)
    s2 = polymul(s_ext, s_ext, mods, P.ext_psis(P.L), P.logn)
    return swk_gen(P, s, s2, a, e, 0)


def galois_element(P: Params, step: int) -> int:
    """5^step mod 2N; rotation to the left by `step` slots."""
    return pow(5, step % (P.N // 2), 2 * P.N)


def galois_key(P: Params, s, g: int, a, e) -> SwitchKey:
    mods = P.ext_mods(P.L)
    s_g = automorphism(secret_rns(P, s, mods), g, mods, P.logn)
    return swk_gen(P, s, s_g, a, e, g)


def encrypt(P: Params, s, m: np.ndarray, a: np.ndarray, e, scale: float) -> Ct:
    """(c0, c1) = (-a s + e + m, a) at the level of m."""
    level = m.shape[0]
    mods, psis = P.mods(level), P.psis(level)
    s_r = secret_rns(P, s, mods)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    c0 = add(add(neg(polymul(a, s_r, mods, psis, P.logn), mods),
                 from_ints(np.asarray(e, dtype=np.int64), mods), mods), m, mods)
    return Ct(np.stack([c0, a]), scale)


def decrypt(P: Params, s, ct: Ct) -> np.ndarray:
    """c0 + c1 s (+ c2 s^2): residues of m + e at the ciphertext's level."""
    mods, psis = P.mods(ct.level), P.psis(ct.level)
    s_r = secret_rns(P, s, mods)
    acc = ct.c[0].copy()
    s_pow = s_r
    for k in range(1, ct.c.shape[0]):
        acc = add(acc, polymul(ct.c[k], s_pow, mods, psis, P.logn), mods)
        s_pow = polymul(s_pow, s_r, mods, psis, P.logn)
    return acc


# --------------------------------------------------------------------------
# Evaluation (Sec. 2.4-2.5, App. A.1-A.2)
# --------------------------------------------------------------------------
def _drop(ct: Ct, level: int) -> np.ndarray:
    return ct.c[:, :level]


def ct_add(P, x: Ct, y: Ct) -> Ct:
    lv = min(x.level, y.level)
    return Ct(np.stack([add(a, b, P.mods(lv)) for a, b in zip(_drop(x, lv), _drop(y, lv))]), x.scale)


def ct_sub(P, x: Ct, y: Ct) -> Ct:
    lv = min(x.level, y.level)
    return Ct(np.stack([sub(a, b, P.mods(lv)) for a, b in zip(_drop(x, lv), _drop(y, lv))]), x.scale)


def ct_add_plain(P, x: Ct, m: np.ndarray) -> Ct:
    lv = min(x.level, m.shape[0])
    c = _drop(x, lv).copy()
    c[0] = add(c[0], m[:lv], P.mods(lv))
    return Ct(c, x.scale)


def ct_mul_plain(P, x: Ct, m: np.ndarray, m_scale: float) -> Ct:
    lv = min(x.level, m.shape[0])
    mods, psis = P.mods(lv), P.psis(lv)
    return Ct(np.stack([polymul(c, m[:lv], mods, psis, P.logn) for c in _drop(x, lv)]), x.scale * m_scale)


def ct_mul_int(P, x: Ct, k: int) -> Ct:
    mods = P.mods(x.level)
    return Ct(np.stack([smul(c, [k] * x.level, mods) for c in x.c]), x.scale)


def tensor(P, x: Ct, y: Ct) -> Ct:
    """(a0 b0, a0 b1 + a1 b0, a1 b1): the degree-2 product before relinearisation."""
    lv = min(x.level, y.level)
    mods, psis = P.mods(lv), P.psis(lv)
    a0, a1 = _drop(x, lv)
    b0, b1 = _drop(y, lv)
    mul = lambda u, v: polymul(u, v, mods, psis, P.logn)
    return Ct(np.stack([mul(a0, b0), add(mul(a0, b1), mul(a1, b0), mods), mul(a1, b1)]), x.scale * y.scale)


def mod_up(P: Params, d: np.ndarray, level: int):
    """Per digit j: fast conversion of [d]_{Q'_j} to every modulus of Q_level * P."""
    ext = P.ext_mods(level)
    return [bconv(d[D], [P.q[i] for i in D], ext) for D in P.digits(level)]


def mod_down(P: Params, x: np.ndarray, level: int) -> np.ndarray:
    """round(x / P) up to the fast-conversion slack: (y - FastBConv([y]_P)) P^-1
    with y = x + floor(P/2); x has rows Q_level then P."""
    Pb = math.prod(P.p)
    ext = P.ext_mods(level)
    y = add_int(x, [Pb // 2] * len(ext), ext)
    r = bconv(y[level:], P.p, P.mods(level))
    qs = P.mods(level)
    return smul(sub(y[:level], r, qs), [pow(Pb, -1, q) for q in qs], qs)


def key_switch(P: Params, d: np.ndarray, key: SwitchKey):
    """SwitchKey(d, swk) = round(P^-1 <decomp(d), swk>) over Q_level."""
    level = d.shape[0]
    ext = P.ext_mods(level)
    psis = P.ext_psis(level)
    rows = list(range(level)) + list(range(P.L, P.L + P.K))
    acc0 = np.zeros((len(ext), P.N), dtype=np.uint64)
    acc1 = np.zeros((len(ext), P.N), dtype=np.uint64)
    for j, dj in enumerate(mod_up(P, d, level)):
        acc0 = add(acc0, polymul(dj, np.ascontiguousarray(key.b[j][rows]), ext, psis, P.logn), ext)
        acc1 = add(acc1, polymul(dj, np.ascontiguousarray(key.a[j][rows]), ext, psis, P.logn), ext)
    return mod_down(P, acc0, level), mod_down(P, acc1, level)


def relinearize(P, x: Ct, rlk: SwitchKey) -> Ct:
    mods = P.mods(x.level)
    k0, k1 = key_switch(P, x.c[2], rlk)
    return Ct(np.stack([add(x.c[0], k0, mods), add(x.c[1], k1, mods)]), x.scale)


def mul_relin(P, x: Ct, y: Ct, rlk: SwitchKey) -> Ct:
    return relinearize(P, tensor(P, x, y), rlk)


def rescale(P, x: Ct) -> Ct:
    """c' = floor((c + floor(q_l/2)) / q_l) over Q_{l-1}, q_l the last prime."""
    lv = x.level
    assert lv >= 2
    ql = P.q[lv - 1]
    h = ql // 2
    qs = P.mods(lv - 1)
    out = []
    for c in x.c:
        last = (c[lv - 1] + np.uint64(h)) % np.uint64(ql)
        last_r = np.stack([last % np.uint64(q) for q in qs])
        t = sub(add_int(c[: lv - 1], [h] * (lv - 1), qs), last_r, qs)
        out.append(smul(t, [pow(ql, -1, q) for q in qs], qs))
    return Ct(np.stack(out), x.scale / ql)


def apply_galois(P, x: Ct, g: int, key: SwitchKey) -> Ct:
    """(phi_g(c0) + KS_0(phi_g(c1)), KS_1(phi_g(c1))) with swk_{phi_g(s) -> s}."""
    assert key.galois == g
    mods = P.mods(x.level)
    c0 = automorphism(x.c[0], g, mods, P.logn)
    c1 = automorphism(x.c[1], g, mods, P.logn)
    k0, k1 = key_switch(P, c1, key)
    return Ct(np.stack([add(c0, k0, mods), k1]), x.scale)


def rotate(P, x: Ct, step: int, keys: dict) -> Ct:
    g = galois_element(P, step)
    return apply_galois(P, x, g, keys[g])


def conjugate(P, x: Ct, keys: dict) -> Ct:
    g = 2 * P.N - 1
    return apply_galois(P, x, g, keys[g])


def rotate_sum(P, x: Ct, log_steps: int, keys: dict) -> Ct:
    """x <- x + rot(x, 2^k) for k < log_steps: every slot gets the sum of all."""
    for k in range(log_steps):
        x = ct_add(P, x, rotate(P, x, 1 << k, keys))
    return x
