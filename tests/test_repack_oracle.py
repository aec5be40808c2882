"""Pins of the lookup-table evaluation and ring-repacking oracle (CPU only).

Each pin checks the oracle against something other than itself: the monomial
product against a schoolbook negacyclic product with X^k over Python
integers; the lookup identity (Sec. 3.4: the constant coefficient of
X^i * u_f is f(i)) after decryption; Lemma 1 (the repacked ciphertext decrypts
to sum_i m_i[0] X^i) on tiny rings, with N inputs and with fewer."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import repack as R
from paper_2412_13269_amd import inputs as I
from tests.test_oracle_pins import schoolbook_negacyclic

DELTA = 2.0 ** 30


def params(logn=5):
    return O.Params(logn, [50, 50], [50], alpha=1, mod_log2=logn + 1)


def keys(P, s, seed):
    ext = P.ext_mods(P.L)
    out = {}
    for i in range(P.logn):
        g = R.repack_galois(P, i)
        a = I.uniform_residues(ext, P.N, seed + 2 * i, lead=(P.beta,))
        e = I.gaussian_error((P.beta, P.N), seed + 2 * i + 1)
        out[g] = O.galois_key(P, s, g, a, e)
    return out


def enc_poly(P, s, coeffs, seed):
    m = O.from_ints(np.asarray(coeffs, dtype=np.int64), P.mods(P.L))
    return O.encrypt(P, s, m, I.uniform_residues(P.q, P.N, seed), I.gaussian_error(P.N, seed + 1), DELTA)


@pytest.mark.parametrize("k", [0, 1, 7, 31, 32, 33, 50, 63])
def test_monomial_is_the_negacyclic_product_with_x_to_the_k(k):
    P = params()
    a = I.uniform_residues(P.q, P.N, 3)
    got = R.monomial(a, k, P.q, P.N)
    for r, q in enumerate(P.q):
        xk = [0] * P.N
        kk = k % (2 * P.N)
        xk[kk % P.N] = (q - 1) if kk >= P.N else 1          # X^k = -X^(k-N) for N <= k < 2N
        assert [int(v) for v in got[r]] == schoolbook_negacyclic(a[r], xk, q), (k, r)


def test_lookup_constant_coefficient_is_f_of_the_point():
    P = params()
    s = I.ternary_secret(P.N, None, 11)
    f = I.uniform_slots(P.N, 12)
    U = enc_poly(P, s, R.lut_poly(f, DELTA), 13)
    for i, ct in zip(range(P.N), R.evaluate(P, U, range(P.N))):
        got = R.packed_values(P, s, ct, 1)[0]
        assert abs(got - f[i]) < 2 ** -20, i


@pytest.mark.parametrize("n", [32, 5])
def test_repack_decrypts_to_the_constant_coefficients(n):
    # Lemma 1: repack(c_0 .. c_{n-1}) encrypts sum_i m_i[0] X^i
    P = params()
    s = I.ternary_secret(P.N, None, 21)
    gks = keys(P, s, 300)
    rng = np.random.default_rng(22)
    ms = [rng.integers(-2 ** 29, 2 ** 29, size=P.N) for _ in range(n)]
    cts = [enc_poly(P, s, m, 400 + 2 * i) for i, m in enumerate(ms)]
    out = R.repack(P, cts, gks)
    got = R.packed_values(P, s, out, P.N)
    want = np.zeros(P.N)
    want[:n] = [m[0] / DELTA for m in ms]
    assert np.max(np.abs(got - want)) < 2 ** -16


def test_lookup_then_repack_gives_the_table_at_the_points():
    P = params(6)
    s = I.ternary_secret(P.N, None, 31)
    gks = keys(P, s, 500)
    f = I.uniform_slots(P.N, 32)
    U = enc_poly(P, s, R.lut_poly(f, DELTA), 33)
    points = np.random.default_rng(34).integers(0, P.N, size=P.N)
    out = R.repack(P, R.evaluate(P, U, points), gks)
    got = R.packed_values(P, s, out, P.N)
    assert np.max(np.abs(got - f[points])) < 2 ** -16
