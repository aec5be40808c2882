"""Oracle of ring merging and ring switching (TEST INFRASTRUCTURE ONLY: only
tests/, the smoke check and the benchmark's CPU baseline use it; the library
shares no code with it).

Follows Sec. 3.3 ("Ring Merging and Schemes Switching") and Sec. 4.3 ("Ring
Merging"), with the subring isomorphism of Sec. 3.1: for r = N/n the map
X -> X^r sends Z_Q[X]/(X^n + 1) into Z_Q[X]/(X^N + 1) as a ring homomorphism
((X^r)^n = X^N = -1), so a small ciphertext (b, a) with b + a s = m + e maps to
a large one (b(X^r), a(X^r)) that decrypts under the embedded secret s(X^r) to
m(X^r) + e(X^r).  Up to r such ciphertexts, shifted by X^i and summed, give a
ciphertext of sum_i X^i m_i(X^r) (coefficient j of input i at X^(j r + i):
disjoint supports), still under s(X^r); a key switch with a key from s(X^r)
to the large ring's secret S finishes the ring switching.

Readings: the merged exponent printed as "X^{N/n}" inside the sum is read as
X^(j N/n) (coefficient j of input i at j N/n + i); both rings share their
first prime, and the merged ciphertext keeps one limb (the paper's R^N_{Q_0});
missing inputs are zero ciphertexts.
"""
from __future__ import annotations

import numpy as np

from oracle import ckks as O
from oracle import repack as RP


def embed_poly(a: np.ndarray, r: int) -> np.ndarray:
    """Rows of a(X) -> a(X^r): coefficient j moves to j r."""
    out = np.zeros((a.shape[0], a.shape[1] * r), dtype=a.dtype)
    out[:, ::r] = a
    return out


def embed(Ps, Pb, ct: O.Ct) -> O.Ct:
    r = Pb.N // Ps.N
    return O.Ct(np.stack([embed_poly(c, r) for c in ct.c]), ct.scale)


def embedded_secret(s_small, r: int) -> np.ndarray:
    s = np.zeros(len(s_small) * r, dtype=np.int64)
    s[::r] = np.asarray(s_small, dtype=np.int64)
    return s


def merge_key(Pb, S, s_small, a, e) -> O.SwitchKey:
    """Switching key from the embedded small secret s(X^r) to S (Sec. 2.4.1)."""
    r = Pb.N // len(s_small)
    mods = Pb.ext_mods(Pb.L)
    return O.swk_gen(Pb, S, O.secret_rns(Pb, embedded_secret(s_small, r), mods), a, e, 0)


def merge(Ps, Pb, cts: list, key: O.SwitchKey) -> O.Ct:
    """sum_i X^i embed(ct_i), then (c0, 0) + SwitchKey(c1) to the large secret."""
    r = Pb.N // Ps.N
    assert 1 <= len(cts) <= r and all(c.level == 1 for c in cts)
    mods = Pb.mods(1)
    acc = np.zeros((2, 1, Pb.N), dtype=np.uint64)
    for i, ct in enumerate(cts):
        e = embed(Ps, Pb, ct)
        for u in range(2):
            acc[u] = O.add(acc[u], RP.monomial(e.c[u], i, mods, Pb.N), mods)
    k0, k1 = O.key_switch(Pb, acc[1], key)
    return O.Ct(np.stack([O.add(acc[0], k0, mods), k1]), cts[0].scale)
