"""Oracle of the plaintext-matrix linear transform in slots (TEST
INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU
baseline use it; the library shares no code with it).

CoeffsToSlots and SlotsToCoeffs of bootstrapping are plaintext matrix-vector
products on the slots (App. A.4), evaluated by the diagonal method with the
baby-step giant-step split of Halevi and Shoup: with the matrix's non-zero
generalised diagonals d_k at rotation steps s_k = n1 j_k + i_k,

    M z = sum_k d_k (.) rot(z, s_k)
        = sum_j rot( sum_{k: j_k = j} rot(d_k, -n1 j) (.) rot(z, i_k), n1 j ),

so only the distinct baby steps i (hoisted: one decomposition, oracle.hoist)
and the distinct giant steps n1 j are key switches; rot(d_k, -n1 j) is a
plaintext automorphism (no key).  Steps are taken mod N/2 (slot rotations
form a cyclic group of that order).
"""
from __future__ import annotations

from oracle import ckks as O
from oracle import hoist as H


def giant_back(P, n1: int, j: int) -> int:
    """Galois element of rot(., -n1 j), applied to the diagonals of giant step j."""
    half = P.N // 2
    return O.galois_element(P, (half - n1 * j) % half)


def linear_transform(P, x: O.Ct, diags: list, d_scale: float, steps: list, n1: int, keys: dict) -> O.Ct:
    """diags: plaintext words (coefficient domain, at least x.level limbs), one per step."""
    half = P.N // 2
    lv = x.level
    mods = P.mods(lv)
    st = [int(s) % half for s in steps]
    babies = sorted({s % n1 for s in st} - {0})
    rot = dict(zip(babies, H.apply_galois_hoisted(P, x, [O.galois_element(P, i) for i in babies], keys)))
    rot[0] = x
    out = None
    for j in sorted({s // n1 for s in st}):
        g_back = giant_back(P, n1, j)
        acc = None
        for k, s in enumerate(st):
            if s // n1 != j:
                continue
            d = O.automorphism(diags[k][:lv], g_back, mods, P.logn)
            term = O.ct_mul_plain(P, rot[s % n1], d, d_scale)
            acc = term if acc is None else O.ct_add(P, acc, term)
        if j:
            acc = O.rotate(P, acc, n1 * j, keys)
        out = acc if out is None else O.ct_add(P, out, acc)
    return out
