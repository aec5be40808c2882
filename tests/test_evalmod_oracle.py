"""Pins of the EvalMod oracle (CPU only): its FP64 steps give sin(2 pi t)/(2 pi)
(the closed form) on [-K, K] and t - round(t) near integers; the homomorphic
oracle decrypts to its FP64 steps (App. A.3)."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import ckks as O
from oracle import evalmod as E
from paper_2412_13269_amd import inputs as I

K, R, DEG = 8.0, 3, 24


def coeffs(deg=DEG, K=K, r=R):
    a = (K + 0.25) / 2 ** r
    return C.chebinterpolate(lambda x: np.cos(2 * math.pi * a * x), deg)


def test_fp64_steps_are_the_scaled_sine():
    t = np.linspace(-K, K, 4001)
    got = E.evalmod_fp64(t, coeffs(), R, K)
    assert np.max(np.abs(got - np.sin(2 * math.pi * t) / (2 * math.pi))) < 1e-6
    # near an integer the scaled sine is the fractional part up to its cubic term
    rng = np.random.default_rng(1)
    ints = rng.integers(-7, 8, size=200)
    frac = rng.uniform(-0.01, 0.01, size=200)
    got = E.evalmod_fp64(ints + frac, coeffs(), R, K)
    assert np.max(np.abs(got - frac) - (2 * math.pi) ** 2 * np.abs(frac) ** 3 / 6) < 1e-6


def test_chebyshev_recurrence_indices():
    for k in range(2, 40):
        a, b = E.cheb_index_pair(k)
        assert a + b == k and a - b in (0, 1)
        x = np.linspace(-1, 1, 9)
        Tk = lambda n: np.cos(n * np.arccos(x))
        assert np.allclose(Tk(k), 2 * Tk(a) * Tk(b) - Tk(a - b))


def homomorphic_setup():
    P = O.Params(7, [50] + [45] * 13, [50] * 3, alpha=4, mod_log2=17)
    s = I.ternary_secret(P.N, None, 2)
    ext = P.ext_mods(P.L)
    rlk = O.relin_key(P, s, I.uniform_residues(ext, P.N, 3, lead=(P.beta,)), I.gaussian_error((P.beta, P.N), 4))
    rng = np.random.default_rng(5)
    t = rng.integers(-7, 8, size=P.N // 2) + rng.uniform(-0.05, 0.05, size=P.N // 2)
    x = O.encrypt(P, s, O.encode(P, t, 2.0 ** 45, P.L), I.uniform_residues(P.mods(P.L), P.N, 6),
                  I.gaussian_error(P.N, 7), 2.0 ** 45)
    return P, s, rlk, t, x


@pytest.fixture(scope="module")
def homomorphic():
    return homomorphic_setup()


def test_homomorphic_evalmod_decrypts_to_its_fp64_steps(homomorphic):
    # with every sum taken at one scale the error is the encryption noise's
    # (~1e-10 here); terms left at the scales the primes give drift by their
    # offsets from 2^45 (~1e-7 relative each) and land near 1e-5
    P, s, rlk, t, x = homomorphic
    out = E.evalmod(P, x, coeffs(), R, K, rlk)
    got = O.decode(P, O.decrypt(P, s, out), out.scale, P.N // 2).real
    assert np.max(np.abs(got - E.evalmod_fp64(t, coeffs(), R, K))) < 1e-8
    assert out.level == P.L - (1 + math.ceil(math.log2(DEG)) + 1 + R + 1)
