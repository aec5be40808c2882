"""Pins of the hoisted-automorphism oracle (CPU only): with g = 1 it is the
plain key switch (apply_galois with the key of g = 1), word for word; for
rotations and conjugation it decrypts to the rotated (conjugated) slots, as
the FP64 roll of the input slots, and its difference to apply_galois
decrypts to a small error."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import hoist as H
from paper_2412_13269_amd import inputs as I

DELTA = 2.0 ** 40


@pytest.fixture(scope="module")
def setup():
    P = O.Params(6, [50, 45, 45, 45], [50, 50], alpha=2, mod_log2=17)
    s = I.ternary_secret(P.N, None, 1)
    ext = P.ext_mods(P.L)
    gs = [1, O.galois_element(P, 1), O.galois_element(P, 5), 2 * P.N - 1]
    keys = {g: O.galois_key(P, s, g, I.uniform_residues(ext, P.N, 10 + i, lead=(P.beta,)),
                            I.gaussian_error((P.beta, P.N), 20 + i)) for i, g in enumerate(gs)}
    z = I.uniform_slots(P.N // 2, 2) + 1j * I.uniform_slots(P.N // 2, 3)
    lv = 3                                              # below the top level: a partial last digit
    m = O.encode(P, z, DELTA, lv)
    x = O.encrypt(P, s, m, I.uniform_residues(P.mods(lv), P.N, 4), I.gaussian_error(P.N, 5), DELTA)
    return P, s, gs, keys, z, x


def test_identity_element_is_the_plain_key_switch(setup):
    P, s, gs, keys, z, x = setup
    got = H.apply_galois_hoisted(P, x, [1], keys)[0]
    assert np.array_equal(got.c, O.apply_galois(P, x, 1, keys[1]).c)


def test_hoisted_rotations_decrypt_to_the_rotated_slots(setup):
    P, s, gs, keys, z, x = setup
    outs = H.apply_galois_hoisted(P, x, gs, keys)
    for g, o in zip(gs, outs):
        got = O.decode(P, O.decrypt(P, s, o), DELTA, P.N // 2)
        if g == 2 * P.N - 1:
            want = np.conj(z)
        else:
            k = next(k for k in range(P.N // 2) if O.galois_element(P, k) == g)
            want = np.roll(z, -k)
        assert np.max(np.abs(got - want)) < 2 ** -20, g
        # the same message as the unhoisted automorphism, up to a small error
        ref = O.decode(P, O.decrypt(P, s, O.apply_galois(P, x, g, keys[g])), DELTA, P.N // 2)
        assert np.max(np.abs(got - ref)) < 2 ** -20, g
