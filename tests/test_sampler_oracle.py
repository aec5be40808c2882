"""Pins of the oracle's seeded sampler (oracle/sampler.py) against what
FIPS 202 and the distributions' definitions fix: a SHAKE-256 known answer,
the stream framing, the rejection rules on tiny moduli, the support and
counts of the secrets, and the moments and tails of the discrete Gaussian
(sigma = 3.2 cut at 19).  The library implements the same reading with its
own Keccak; tests/test_lib_host.py compares the two byte for byte."""
import hashlib
import math
import struct

import numpy as np

from oracle import sampler as S

SEED = bytes(range(32))


def test_shake256_known_answer():
    # SHAKE256 of the empty message (FIPS 202 example value)
    assert hashlib.shake_256(b"").hexdigest(32) == \
        "46b9dd2b0ba88d13233b3feb743eeb243fcd52ea62b81b82b50c27646ed5762f"


def test_stream_framing_and_extension():
    st = S.Stream(SEED, 4, 7, 9)
    want = hashlib.shake_256(SEED + struct.pack("<III", 4, 7, 9)).digest(10000)
    got = b"".join(st.read(k) for k in (1, 7, 4096, 3, 5000, 889))
    assert got == want[:len(got)]
    assert S.Stream(SEED, 4, 7, 10).read(32) != want[:32]       # every field keys the stream


def test_uniform_rejection_rule_on_tiny_moduli():
    # q = 5: words masked to 3 bits, values 5..7 rejected (read back by hand)
    st = S.Stream(SEED, 2, 0, 0)
    words = [struct.unpack("<Q", st.read(8))[0] & 7 for _ in range(200)]
    want = [w for w in words if w < 5]
    got = S.uniform_poly(SEED, 2, 0, 0, 5, len(want))
    assert list(got) == want
    # q = 2: one bit, nothing rejected
    st = S.Stream(SEED, 2, 1, 0)
    bits = [struct.unpack("<Q", st.read(8))[0] & 1 for _ in range(64)]
    assert list(S.uniform_poly(SEED, 2, 1, 0, 2, 64)) == bits


def test_uniform_is_uniform():
    q = (1 << 49) + 12345            # just above a power of two: about half the words rejected
    x = S.uniform_poly(SEED, 4, 0, 3, q, 20000).astype(np.float64)
    assert x.max() < q
    assert abs(x.mean() / q - 0.5) < 0.01
    assert abs(x.std() / q - math.sqrt(1 / 12)) < 0.01
    small = S.uniform_poly(SEED, 4, 0, 4, 3, 30000)
    counts = np.bincount(small.astype(np.int64), minlength=3)
    assert counts.sum() == 30000 and np.all(np.abs(counts / 10000 - 1) < 0.05)


def test_ternary_secrets():
    u = S.secret(SEED, 1 << 14, -1)
    c = {v: int((u == v).sum()) for v in (-1, 0, 1)}
    assert sum(c.values()) == 1 << 14 and all(abs(k / (1 << 14) - 1 / 3) < 0.02 for k in c.values())
    for n, h in ((1 << 12, 192), (64, 64), (64, 0), (5, 3)):
        s = S.secret(SEED, n, h)
        assert int((s != 0).sum()) == h and set(np.unique(s)) <= {-1, 0, 1}
    s = S.secret(SEED, 1 << 16, 192)
    nz = np.nonzero(s)[0]
    assert abs(nz.mean() / (1 << 16) - 0.5) < 0.1                 # positions spread over the ring
    assert 60 < int((s > 0).sum()) < 132                           # signs about even
    assert not np.array_equal(s, S.secret(bytes(32), 1 << 16, 192))


def test_gaussian_table_and_moments():
    t = S.gaussian_table()
    assert len(t) == 20 and t[-1] == 1 << 63 and all(a < b for a, b in zip(t, t[1:]))
    # P(|X| = 0) = 1 / sum_k rho(k) over -19..19
    z = sum(math.exp(-k * k / (2 * 3.2 ** 2)) for k in range(-19, 20))
    assert abs(t[0] / 2.0 ** 63 - 1 / z) < 1e-12
    e = S.gaussian_poly(SEED, 3, 0, 40000)
    assert e.dtype == np.int64 and np.abs(e).max() <= 19
    assert abs(e.mean()) < 0.06
    assert abs(e.var() / 3.2 ** 2 - 1) < 0.03
    assert abs((e == 0).mean() - 1 / z) < 0.01


def test_key_and_encryption_inputs_shapes():
    mods = [97, 193, 257]
    a, e = S.key_inputs(SEED, mods, 16, 2, 5)
    assert a.shape == (2, 3, 16) and e.shape == (2, 16)
    assert all((a[:, m] < q).all() for m, q in enumerate(mods))
    a2, _ = S.key_inputs(SEED, mods, 16, 2, 25)
    assert not np.array_equal(a, a2)                               # the Galois element keys the streams
    ea, ee = S.encryption_inputs(SEED, mods[:2], 16)
    assert ea.shape == (2, 16) and ee.shape == (16,)
