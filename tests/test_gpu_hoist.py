"""GPU: hoisted automorphisms (one ModUp, every Galois element switched from
its permutation) against the oracle word for word, at the top level and at a
level with a partial last digit, over more elements than one batch holds;
and the argument checks."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import hoist as H
from tests.test_gpu_parity import CONFIGS, Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


@pytest.fixture(scope="module", params=["n12_3x50", "n13_9_limbs"])
def pair(request, X):
    cfg = CONFIGS[request.param]
    p = Pair(X, cfg["logn"], cfg["qb"], cfg["pb"], cfg["alpha"], cfg["ml"], cfg["h"], seed=23, scale=cfg["scale"])
    yield p
    p.close()


def test_hoisted_automorphisms_match_oracle(pair, X):
    P = pair.P
    gs = [1] + [O.galois_element(P, k) for k in (1, 2, 3, 5, 8, 13, 21, P.N // 2 - 1)] + [2 * P.N - 1]
    for g in gs:
        pair.key(g)
    for lv in (P.L, max(1, P.L - 3)):
        co, cx, z = pair.enc(lv)
        outs = [pair.ct(lv, deg=1) for _ in gs]
        X.pfx_apply_galois_hoisted(pair.ctx, cx, [pair.kx[g] for g in gs], outs)
        for o, w in zip(outs, H.apply_galois_hoisted(P, co, gs, pair.ko)):
            pair.same(w, o)
        # the identity element is the plain key switch
        one = pair.ct(lv, deg=1)
        X.pfx_apply_galois(pair.ctx, cx, pair.kx[1], one)
        assert np.array_equal(pair.words(one), pair.words(outs[0]))


def test_hoisted_argument_checks(pair, X):
    P = pair.P
    g = O.galois_element(P, 1)
    pair.key(g)
    pair.key(0)
    co, cx, z = pair.enc(P.L)
    out = pair.ct(P.L, deg=1)
    with pytest.raises(X.PfxError) as e:                        # output aliasing the input
        X.pfx_apply_galois_hoisted(pair.ctx, cx, [pair.kx[g]], [cx])
    assert e.value.status == X.PFX_EINVAL
    with pytest.raises(X.PfxError) as e:                        # a relinearisation key
        X.pfx_apply_galois_hoisted(pair.ctx, cx, [pair.kx[0]], [out])
    assert e.value.status == X.PFX_ENOKEY
    with pytest.raises(X.PfxError) as e:                        # two outputs in one place
        X.pfx_apply_galois_hoisted(pair.ctx, cx, [pair.kx[g], pair.kx[g]], [out, out])
    assert e.value.status == X.PFX_EINVAL
