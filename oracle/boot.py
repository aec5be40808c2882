"""Oracle of ModRaise, the first step of bootstrapping (TEST INFRASTRUCTURE
ONLY: only tests/, the smoke check and the benchmark's CPU baseline use it;
the library shares no code with it).

App. A.3: a ciphertext modulo q_0 is read modulo the larger Q_L: each
coefficient's residue is lifted to an integer and reduced modulo every prime
of Q_L, so the ciphertext decrypts modulo Q_L to m + q_0 I(X) with I(X) a small
integer polynomial (O(sqrt(h)): c0 + c1 s without the reduction mod q_0).

Reading: the lift is the centred one, (-q_0/2, q_0/2] (q_0 odd: [-(q_0-1)/2,
(q_0-1)/2]), which keeps |I| at most (h + 1)/2 for a secret of h non-zeros.

The trace-like map that follows ModRaise when 2n != N (App. A.3) keeps the
coefficients of degree a multiple of r = N/2n and cancels the others with
log r automorphisms: x <- x + phi_g(x) for g = N/2^t + 1, t = 0 .. log r - 1
(phi_{N/2^t + 1} fixes X^j for j = 0 mod 2^(t+1) and negates it for
j = 2^t mod 2^(t+1), so after the steps for t < T only multiples of 2^T are
left, each times 2^T).

CoeffsToSlots and SlotsToCoeffs (App. A.4) with all N/2 slots: for the
message m(X) = sum_k m_k X^k (real m_k) the slots are z_l = m(zeta_l),
zeta_l = exp(i pi 5^l / N); since zeta_l^(N/2) = i, the complex vector
w_j = m_j + i m_(j+N/2) (j < N/2) gives z = A w with A[l, j] = zeta_l^j, and
w = B z with B[j, l] = (2/N) zeta_l^(-j) (the conjugate terms cancel).  Both
are evaluated as dense matrix-vector products on the slots by the BSGS
diagonal method (oracle.linear), diagonal k of M being M[j, (j + k) mod N/2].

Sparse packing (App. A.3-A.4, n slots, 2n < N): a message in the subring of
Y = X^r, r = N/2n, has n slots xi_l = exp(i pi 5^l / 2n), l < n, each repeated
r times among the N/2 slots of the full ring (zeta_l^r = xi_(l mod n)).  The
same packing holds with n in place of N/2: w_j = m'_j + i m'_(j+n) for the
subring coefficients m'_k = m_(k r), z = A' w with A'[l, j] = xi_l^j and
w = B' z with B'[j, l] = (1/n) xi_l^(-j); a slot rotation by k of the full ring
rotates every period of n slots by k mod n, so the diagonal method on n
diagonals of length n (each repeated r times) applies B' to the periodic slot
vector.  After ModRaise the trace-like map leaves r times the subring part.

Half-BTS (Sec. 4.3, App. A.3-A.4): a coefficient-encoded ciphertext of one limb
-> one at a higher level whose slots hold its coefficients, i.e. ModRaise,
CoeffsToSlots and EvalMod without the SlotsToCoeffs of a full bootstrapping.
Reading: after ModRaise the ciphertext is read at scale q_0, so its
coefficients are t = m'/q_0 = I + m/q_0; CoeffsToSlots applies B/2 (diagonals
an input, at scale d_scale) and rescales, so the slots hold w/2 with
w_j = t_j + i t_(j+N/2); re = w/2 + conj(w/2) and im = -i (w/2 - conj(w/2))
(conjugation: the automorphism 2N - 1; -i: the monomial X^(3N/2)) are the real
vectors t_j and t_(j+N/2); EvalMod on each (oracle.evalmod, its last constant
times out_factor = q_0 / Delta) returns m / Delta; the result is
re + i im (i: X^(N/2)), slot j holding m_j / Delta + i m_(j+N/2) / Delta.
"""
from __future__ import annotations

import numpy as np

from oracle import ckks as O


def lift(words: np.ndarray, q0: int) -> np.ndarray:
    """Residues modulo q_0 as integers in [-(q_0-1)/2, (q_0-1)/2]."""
    w = words.astype(np.int64)
    return np.where(w > (q0 - 1) // 2, w - q0, w)


def mod_raise(P, x: O.Ct, level: int) -> O.Ct:
    """x at one limb (q_0) -> the same integers at `level` limbs."""
    assert x.level == 1 and 1 <= level <= P.L
    mods = P.mods(level)
    return O.Ct(np.stack([O.from_ints(lift(c[0], P.q[0]), mods) for c in x.c]), x.scale)


def trace_galois(P, t: int) -> int:
    """Galois element of step t of the trace-like map."""
    return P.N // (1 << t) + 1


def subring_trace(P, x: O.Ct, log_r: int, keys: dict) -> O.Ct:
    """prod_t (1 + phi_{N/2^t + 1}) applied to x, t < log_r."""
    for t in range(log_r):
        g = trace_galois(P, t)
        x = O.ct_add(P, x, O.apply_galois(P, x, g, keys[g]))
    return x


def slot_roots(P, n: int | None = None) -> np.ndarray:
    """exp(i pi 5^l / 2n), l < n (n slots; n = N/2: the full ring's zeta_l)."""
    n = n or P.N // 2
    e = np.array([pow(5, l, 4 * n) for l in range(n)], dtype=np.float64)
    return np.exp(1j * np.pi * e / (2 * n))


def s2c_matrix(P, n: int | None = None) -> np.ndarray:
    """A[l, j] = zeta_l^j: slots of the message whose coefficients are w (packed)."""
    n = n or P.N // 2
    return slot_roots(P, n)[:, None] ** np.arange(n)[None, :]


def c2s_matrix(P, n: int | None = None) -> np.ndarray:
    """B[j, l] = (1/n) zeta_l^-j: packed coefficients w_j = m_j + i m_(j+n) from
    the n slots (n = N/2: the factor is 2/N)."""
    n = n or P.N // 2
    return (1.0 / n) * np.conj(slot_roots(P, n)[None, :] ** np.arange(n)[:, None])


def bit_reverse(n: int) -> np.ndarray:
    L = n.bit_length() - 1
    return np.array([int(format(j, f"0{L}b")[::-1], 2) if L else 0 for j in range(n)])


def fft_stage_inverse(P, s: int, n: int | None = None):
    """F_s^-1 as a sparse n x n matrix (n slots, N/2 by default): rows j
    (lower) (u + v) / 2, rows j + 2^(s-1) (upper) (u - v) / (2 w_j) of the pair
    (u, v)."""
    from scipy import sparse
    n = n or P.N // 2
    ln, lh = 1 << s, 1 << (s - 1)
    rows, cols, vals = [], [], []
    for i in range(0, n, ln):
        for j in range(lh):
            w = np.exp(2j * np.pi * (pow(5, j, 4 * ln)) / (4 * ln))
            lo, hi = i + j, i + j + lh
            rows += [lo, lo, hi, hi]
            cols += [lo, hi, lo, hi]
            vals += [0.5, 0.5, 0.5 / w, -0.5 / w]
    return sparse.csr_matrix((vals, (rows, cols)), shape=(n, n), dtype=complex)


def c2s_factor_matrices(P, levels: int, factor: float = 1.0, n: int | None = None) -> list:
    """The merged stages of R B (times `factor`), in the order they apply:
    the L = log2(n) inverse stages F_L^-1 (first) .. F_1^-1 split into
    `levels` consecutive groups of ceil(L / levels) stages (the last group
    takes what is left); n slots, N/2 by default."""
    n = n or P.N // 2
    L = n.bit_length() - 1
    k = -(-L // levels)
    order = list(range(L, 0, -1))                   # F_L^-1 applies first
    mats = []
    for g in range(0, L, k):
        M = None
        for s in order[g:g + k]:
            F = fft_stage_inverse(P, s, n)
            M = F if M is None else F @ M
        mats.append(M)
    mats[0] = mats[0] * factor
    return mats


def sparse_diagonals(M) -> tuple:
    """(steps, diagonals) of the non-zero generalised diagonals of a sparse
    matrix: d_k[j] = M[j, (j + k) mod n]."""
    n = M.shape[0]
    C = M.tocoo()
    k = (C.col - C.row) % n
    steps = sorted(set(int(x) for x in k))
    out = []
    for st in steps:
        d = np.zeros(n, dtype=complex)
        sel = k == st
        d[C.row[sel]] = C.data[sel]
        out.append(d)
    return steps, out


def diagonals(M: np.ndarray) -> list:
    """Diagonal k of M: d_k[j] = M[j, (j + k) mod n], so M z = sum_k d_k (.) rot(z, k)."""
    n = M.shape[0]
    j = np.arange(n)
    return [M[j, (j + k) % n] for k in range(n)]



def half_bootstrap(P, x: O.Ct, c2s_words: list, d_scale: float, n1: int, keys: dict, rlk, coeffs, r: int,
                   K: float, out_factor: float) -> O.Ct:
    """x: one limb, coefficient-encoded; c2s_words: the N/2 diagonals of B/2
    encoded at d_scale (coefficient domain, at least P.L limbs); keys: the
    Galois keys of the BSGS steps and of 2N - 1."""
    from oracle import evalmod as EM
    from oracle import linear as LT
    from oracle import repack as RP
    n = P.N // 2
    y = mod_raise(P, x, P.L)
    y = O.Ct(y.c, float(P.q[0]))
    z = O.rescale(P, LT.linear_transform(P, y, c2s_words, d_scale, list(range(n)), n1, keys))
    zc = O.conjugate(P, z, keys)
    re = O.ct_add(P, z, zc)
    im = RP.ct_monomial(P, O.ct_sub(P, z, zc), 3 * n)
    re = EM.evalmod(P, re, coeffs, r, K, rlk, out_factor)
    im = EM.evalmod(P, im, coeffs, r, K, rlk, out_factor)
    return O.ct_add(P, re, RP.ct_monomial(P, im, n))


def half_bootstrap_factorised(P, x: O.Ct, stages: list, keys: dict, rlk, coeffs, r: int, K: float,
                              out_factor: float, log_r: int = 0) -> O.Ct:
    """Half-BTS with the factorised CoeffsToSlots: stages[i] = (steps, words,
    n1, d_scale) of merged stage i (words: its diagonals of R B / 2, the factor
    1/2 in the first stage, encoded at d_scale), each a BSGS transform followed
    by a rescale; then the conjugate split and EvalMod as in half_bootstrap.
    Slot p of the result holds m_rev(p) / Delta + i m_(rev(p) + N/2) / Delta.
    Reading (scales): the first stage's diagonals take the dense transform's
    scale, every later stage's the prime its rescale drops, so the scale after
    CoeffsToSlots is the dense one's times the ratio of the dropped primes (each
    later stage keeps the scale it receives exactly).
    Sparse packing (log_r > 0, n = N / 2^(log_r + 1) slots): the trace-like
    map follows ModRaise (keys of N/2^t + 1 among `keys`) and the stages are
    those of R B' for n slots with the factor 1/(2 * 2^log_r) in the first
    (the trace multiplies the subring part by 2^log_r); slot p (and every
    slot p + k n) of the result holds m'_rev(p) / Delta + i m'_(rev(p) + n) /
    Delta, m'_k = m_(k 2^log_r), rev over log2(n) bits."""
    from oracle import evalmod as EM
    from oracle import linear as LT
    from oracle import repack as RP
    n = P.N // 2
    y = mod_raise(P, x, P.L)
    if log_r:
        y = subring_trace(P, y, log_r, keys)
    z = O.Ct(y.c, float(P.q[0]))
    for steps, words, n1, d_scale in stages:
        z = O.rescale(P, LT.linear_transform(P, z, words, d_scale, steps, n1, keys))
    zc = O.conjugate(P, z, keys)
    re = O.ct_add(P, z, zc)
    im = RP.ct_monomial(P, O.ct_sub(P, z, zc), 3 * n)
    re = EM.evalmod(P, re, coeffs, r, K, rlk, out_factor)
    im = EM.evalmod(P, im, coeffs, r, K, rlk, out_factor)
    return O.ct_add(P, re, RP.ct_monomial(P, im, n))
