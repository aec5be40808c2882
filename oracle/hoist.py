"""Oracle of hoisted automorphisms (TEST INFRASTRUCTURE ONLY: only tests/, the
smoke check and the benchmark's CPU baseline use it; the library shares no
code with it).

The baby steps of the BSGS linear transforms of bootstrapping (App. A.4,
after Halevi and Shoup) rotate one ciphertext by many Galois elements.  Each
rotation is a key switch of phi_g(c1) (Sec. 2.4.1, App. A.2); hoisting
decomposes c1 once, D_j = ModUp_j(c1), and switches phi_g(D_j) for every g:
the automorphism is a ring homomorphism applied limb by limb to the same
integer polynomial D_j, so phi_g(D_j) is a decomposition of phi_g(c1) (its
digit parts reduce to phi_g(c1) modulo each digit) and the result

    (phi_g(c0) + ModDown(sum_j phi_g(D_j) swk_j,0), ModDown(sum_j phi_g(D_j) swk_j,1))

decrypts to phi_g(m) like apply_galois.  It is not the same words as
apply_galois: ModUp(phi_g(c1)) lifts each negated residue to [0, q) while
phi_g(D_j) negates the lifted integer, so the two decompositions differ by
multiples of the digit's modulus (a different, equally small key-switching
error).  With g = 1 both are the plain key switch.
"""
from __future__ import annotations

import numpy as np

from oracle import ckks as O


def apply_galois_hoisted(P, x: O.Ct, gs: list, keys: dict) -> list:
    level = x.level
    ext = P.ext_mods(level)
    psis = P.ext_psis(level)
    mods = P.mods(level)
    rows = list(range(level)) + list(range(P.L, P.L + P.K))
    D = O.mod_up(P, x.c[1], level)                      # once for every g
    outs = []
    for g in gs:
        key = keys[g]
        assert key.galois == g
        acc0 = acc1 = None
        for j, dj in enumerate(D):
            dg = O.automorphism(dj, g, ext, P.logn)
            t0 = O.polymul(dg, np.ascontiguousarray(key.b[j][rows]), ext, psis, P.logn)
            t1 = O.polymul(dg, np.ascontiguousarray(key.a[j][rows]), ext, psis, P.logn)
            acc0 = t0 if acc0 is None else O.add(acc0, t0, ext)
            acc1 = t1 if acc1 is None else O.add(acc1, t1, ext)
        k0, k1 = O.mod_down(P, acc0, level), O.mod_down(P, acc1, level)
        c0 = O.automorphism(x.c[0], g, mods, P.logn)
        outs.append(O.Ct(np.stack([O.add(c0, k0, mods), k1]), x.scale))
    return outs
