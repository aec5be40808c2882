"""Pins of the BSGS linear-transform oracle (CPU only): the decrypted result
is the plaintext matrix-vector product sum_k d_k (.) roll(z, -s_k) computed in
FP64 on the slots, for several baby-step counts n1 (n1 = 1: every step a
giant step, no hoisting), with steps past N/2 and a zero step."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import linear as LT
from paper_2412_13269_amd import inputs as I

DELTA = 2.0 ** 40
STEPS = [0, 1, 2, 5, 7, 9, 13, 31, 34]          # 34 = 2 mod 32


@pytest.fixture(scope="module")
def setup():
    P = O.Params(6, [50, 45, 45], [50, 50], alpha=2, mod_log2=17)
    half = P.N // 2
    s = I.ternary_secret(P.N, None, 1)
    ext = P.ext_mods(P.L)
    keys = {}
    for k in range(1, half):
        g = O.galois_element(P, k)
        keys[g] = O.galois_key(P, s, g, I.uniform_residues(ext, P.N, 100 + k, lead=(P.beta,)),
                               I.gaussian_error((P.beta, P.N), 200 + k))
    z = I.uniform_slots(half, 2) + 1j * I.uniform_slots(half, 3)
    x = O.encrypt(P, s, O.encode(P, z, DELTA, P.L), I.uniform_residues(P.mods(P.L), P.N, 4),
                  I.gaussian_error(P.N, 5), DELTA)
    ds = [(I.uniform_slots(half, 10 + k) + 1j * I.uniform_slots(half, 30 + k)) / len(STEPS)
          for k in range(len(STEPS))]
    words = [O.encode(P, d, DELTA, P.L) for d in ds]
    want = sum(d * np.roll(z, -(st % half)) for d, st in zip(ds, STEPS))
    return P, s, keys, x, words, want


@pytest.mark.parametrize("n1", [1, 4, 8])
def test_transform_is_the_matrix_vector_product(setup, n1):
    P, s, keys, x, words, want = setup
    out = LT.linear_transform(P, x, words, DELTA, STEPS, n1, keys)
    assert out.scale == DELTA * DELTA
    got = O.decode(P, O.decrypt(P, s, out), out.scale, P.N // 2)
    assert np.max(np.abs(got - want)) < 2 ** -20
