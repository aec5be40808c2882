"""The library's seeded sampler (its own Keccak-f[1600] and draws, host side,
no GPU) against the oracle's (Python's hashlib SHAKE-256 and the draws written
from their definitions), byte for byte and draw for draw."""
import hashlib

import numpy as np
import pytest

from oracle import ckks as O
from oracle import sampler as S

X = pytest.importorskip("paper_2412_13269_amd.pfx", reason="libpfx.so not built")

SEEDS = [bytes(32), bytes(range(32)), hashlib.sha256(b"cfg2").digest()]


@pytest.mark.parametrize("mlen", [0, 1, 43, 44, 135, 136, 137, 271, 272, 1000])
def test_shake256_matches_hashlib(mlen):
    msg = bytes((7 * i + 3) % 256 for i in range(mlen))
    for outlen in (1, 32, 135, 136, 137, 700):
        assert X.pfx_shake256(msg, outlen) == hashlib.shake_256(msg).digest(outlen), (mlen, outlen)


@pytest.mark.parametrize("seed", SEEDS)
def test_uniform_draws_match(seed):
    P = O.Params(16, [50] + [45] * 23, [50] * 4, alpha=4, mod_log2=17)
    for tag, index, limb, q in ((2, 0, 0, P.q[0]), (2, 256 * 5 + 3, 27, P.p[3]), (4, 0, 11, P.q[11]),
                                (4, 0, 0, 5), (2, 7, 1, 2), (3, 1, 2, (1 << 49) + 12345), (4, 2, 3, (1 << 61) - 1)):
        got = X.pfx_sample_uniform(seed, tag, index, limb, q, 3000)
        assert np.array_equal(got, S.uniform_poly(seed, tag, index, limb, q, 3000)), (tag, index, limb, q)


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("n,h", [(1 << 12, -1), (1 << 12, 64), (1 << 16, 192), (64, 64), (64, 0), (1, 1)])
def test_secret_draws_match(seed, n, h):
    assert np.array_equal(X.pfx_sample_secret(seed, n, h), S.secret(seed, n, h))


@pytest.mark.parametrize("seed", SEEDS)
def test_gaussian_draws_match(seed):
    for tag, index in ((3, 0), (3, 256 * 25 + 1), (5, 0)):
        assert np.array_equal(X.pfx_sample_gaussian(seed, tag, index, 5000), S.gaussian_poly(seed, tag, index, 5000))


def test_bad_sampling_arguments():
    with pytest.raises(X.PfxError):
        X.pfx_sample_uniform(bytes(32), 2, 0, 0, 1, 4)
    with pytest.raises(X.PfxError):
        X.pfx_sample_secret(bytes(32), 8, 9)
    with pytest.raises(ValueError):
        X.pfx_sample_secret(bytes(31), 8, 2)
