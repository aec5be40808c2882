"""Pins of the ring-merging oracle (CPU only).

The embedding X -> X^r is checked as a ring homomorphism against schoolbook
negacyclic products over Python integers in both rings; an embedded
ciphertext decrypts under the embedded secret to the embedded plaintext plus
the embedded error, exactly; the merged ciphertext decrypts under the large
secret to coefficient j of input i at X^(j r + i) (Sec. 3.3, Sec. 4.3)."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import merge as M
from paper_2412_13269_amd import inputs as I
from tests.test_oracle_pins import schoolbook_negacyclic

DELTA = 2.0 ** 30


def rings():
    # shared first prime: both chains draw primes 1 mod 2^8
    Ps = O.Params(5, [50], [50], alpha=1, mod_log2=8)
    Pb = O.Params(7, [50, 45], [50, 50], alpha=2, mod_log2=8)
    assert Ps.q[0] == Pb.q[0]
    return Ps, Pb


def test_embedding_is_a_ring_homomorphism():
    Ps, Pb = rings()
    r = Pb.N // Ps.N
    q = Ps.q[0]
    a = I.uniform_residues([q], Ps.N, 1)
    b = I.uniform_residues([q], Ps.N, 2)
    small = schoolbook_negacyclic(a[0], b[0], q)
    big = schoolbook_negacyclic(M.embed_poly(a, r)[0], M.embed_poly(b, r)[0], q)
    assert big == [int(v) for v in M.embed_poly(np.array([small], dtype=np.uint64), r)[0]]


def test_embedded_ciphertext_decrypts_under_the_embedded_secret():
    Ps, Pb = rings()
    r = Pb.N // Ps.N
    s = I.ternary_secret(Ps.N, None, 3)
    m = O.from_ints(np.random.default_rng(4).integers(-2 ** 29, 2 ** 29, size=Ps.N), Ps.mods(1))
    e = I.gaussian_error(Ps.N, 5)
    ct = O.encrypt(Ps, s, m, I.uniform_residues(Ps.mods(1), Ps.N, 6), e, DELTA)
    got = O.decrypt(Pb, M.embedded_secret(s, r), M.embed(Ps, Pb, ct))
    want = O.from_ints(M.embed_poly(np.array([e]), r)[0], Pb.mods(1))
    want = O.add(want, M.embed_poly(m, r), Pb.mods(1))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n_in", [4, 3])
def test_merge_places_coefficient_j_of_input_i_at_j_r_plus_i(n_in):
    Ps, Pb = rings()
    r = Pb.N // Ps.N
    s = I.ternary_secret(Ps.N, None, 10)
    S = I.ternary_secret(Pb.N, None, 11)
    ext = Pb.ext_mods(Pb.L)
    key = M.merge_key(Pb, S, s, I.uniform_residues(ext, Pb.N, 12, lead=(Pb.beta,)),
                      I.gaussian_error((Pb.beta, Pb.N), 13))
    rng = np.random.default_rng(14)
    ms = [rng.integers(-2 ** 29, 2 ** 29, size=Ps.N) for _ in range(n_in)]
    cts = [O.encrypt(Ps, s, O.from_ints(m, Ps.mods(1)), I.uniform_residues(Ps.mods(1), Ps.N, 20 + i),
                     I.gaussian_error(Ps.N, 40 + i), DELTA) for i, m in enumerate(ms)]
    out = M.merge(Ps, Pb, cts, key)
    got = O.crt_centered(O.decrypt(Pb, S, out), Pb.mods(1)).astype(np.float64) / DELTA
    want = np.zeros(Pb.N)
    for i, m in enumerate(ms):
        want[i::r] = m / DELTA
    assert np.max(np.abs(got - want)) < 2 ** -12
