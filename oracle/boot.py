"""Oracle of ModRaise, the first step of bootstrapping (TEST INFRASTRUCTURE
ONLY: only tests/, the smoke check and the benchmark's CPU baseline use it;
the library shares no code with it).

App. A.3: a ciphertext modulo q_0 is read modulo the larger Q_L: each
coefficient's residue is lifted to an integer and reduced modulo every prime
of Q_L, so the ciphertext decrypts modulo Q_L to m + q_0 I(X) with I(X) a small
integer polynomial (O(sqrt(h)): c0 + c1 s without the reduction mod q_0).

Reading: the lift is the centred one, (-q_0/2, q_0/2] (q_0 odd: [-(q_0-1)/2,
(q_0-1)/2]), which keeps |I| at most (h + 1)/2 for a secret of h non-zeros.
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
