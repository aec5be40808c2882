"""GPU: ModRaise (App. A.3) against the oracle word for word, to the top level
and to a middle one, out of place and in place."""
import numpy as np
import pytest

from oracle import boot as B
from tests.test_gpu_parity import CONFIGS, Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


@pytest.fixture(scope="module", params=["c1", "c2s"])
def pair(request, X):
    cfg = CONFIGS[request.param]
    p = Pair(X, cfg["logn"], cfg["qb"], cfg["pb"], cfg["alpha"], cfg["ml"], cfg["h"], seed=31, scale=cfg["scale"])
    yield p
    p.close()


def test_mod_raise_matches_oracle(pair, X):
    P = pair.P
    co, cx, z = pair.enc(1)
    for lv in sorted({P.L, max(2, P.L // 2)}):
        out = pair.ct(lv, deg=1)
        X.pfx_mod_raise(pair.ctx, cx, lv, out)
        pair.same(B.mod_raise(P, co, lv), out)
    X.pfx_mod_raise(pair.ctx, cx, P.L, cx)                      # in place (capacity L)
    pair.same(B.mod_raise(P, co, P.L), cx)
    with pytest.raises(X.PfxError) as e:                        # only from one limb
        X.pfx_mod_raise(pair.ctx, cx, P.L, pair.ct(P.L, deg=1))
    assert e.value.status == X.PFX_ELEVEL


def test_subring_trace_matches_oracle(pair, X):
    P = pair.P
    log_r = 3
    for t in range(log_r):
        pair.key(B.trace_galois(P, t))
    co, cx, z = pair.enc(P.L)
    out = pair.ct(P.L, deg=1)
    X.pfx_subring_trace(pair.ctx, cx, log_r, list(pair.kx.values()), out)
    pair.same(B.subring_trace(P, co, log_r, pair.ko), out)
    X.pfx_subring_trace(pair.ctx, cx, log_r, list(pair.kx.values()), cx)    # in place
    pair.same(B.subring_trace(P, co, log_r, pair.ko), cx)
