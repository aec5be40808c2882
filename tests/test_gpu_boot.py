"""GPU: ModRaise (App. A.3) against the oracle word for word, to the top level
and to a middle one, out of place and in place; the trace-like map; and
Half-BTS as a whole (ModRaise, dense CoeffsToSlots, EvalMod on both parts)."""
import numpy as np
import pytest

from oracle import boot as B
from oracle import ckks as O
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


def test_half_bootstrap_matches_oracle(X):
    # Half-BTS (Sec. 4.3, App. A.3-A.4) at N = 2^12 over the 50 + 13 x 45-bit
    # chain: ModRaise, dense CoeffsToSlots (2048 diagonals, n1 = 64), the
    # conjugate split and two EvalMod lanes, word for word against the oracle
    from paper_2412_13269_amd import boot as HB
    from tests.test_boot_oracle import half_boot_setup, run_half_boot
    d = half_boot_setup(12, 64, h=32, seed=900)
    P = d["P"]
    want = run_half_boot(d)
    ctx = X.pfx_ctx_create(X.make_params(P.logn, [50] + [45] * 13, [50] * 4, 4, 17), 0)
    sk = X.pfx_sk_create(ctx, d["s"])
    gks = [X.pfx_swk_create(ctx, sk, g, a, e) for g, (a, e) in d["key_inputs"].items()]
    rlk = X.pfx_swk_create(ctx, sk, 0, *d["rlk_inputs"])
    plan = HB.HalfBootPlan(P.N, d["coeffs"], 3, 8.0, d["out_factor"])
    handles = []
    try:
        m, a, e = d["enc"]
        x = X.pfx_ct_create(ctx, 1, 1)
        handles.append(x)
        pt = X.pfx_pt_import(ctx, m, d["delta"])
        X.pfx_encrypt(ctx, sk, pt, a, e, x)
        X.pfx_ct_destroy(pt)
        diags = []
        for w in d["c2s"]:
            diags.append(X.pfx_pt_import(ctx, w, d["sd"]))
            handles.append(diags[-1])
        regs = [X.pfx_ct_create(ctx, P.L, 1) for _ in range(plan.n_regs)]
        handles += regs
        out = HB.half_bootstrap(ctx, x, P.L, float(P.q[0]), diags, d["n1"], gks, rlk, plan, regs)
        assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c)
        assert X.pfx_ct_info(out).scale == want.scale
        # the op-list part captured into a HIP graph on the first call and
        # replayed, ModRaise and CoeffsToSlots run eagerly between replays
        gregs = [X.pfx_ct_create(ctx, P.L, 1) for _ in range(plan.n_regs)]
        handles += gregs
        stream = X.pfx_stream_create(ctx)
        try:
            for rep in range(3):
                out = HB.half_bootstrap(ctx, x, P.L, float(P.q[0]), diags, d["n1"], gks, rlk, plan, gregs, stream,
                                        X.RUN_GRAPH)
                X.pfx_sync(ctx, stream)
                assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c), rep
        finally:
            X.pfx_stream_destroy(ctx, stream)
        n = P.N // 2
        got = O.decode(P, O.decrypt(P, d["s"], want), want.scale, n)
        # the scaled sine's error (< 1e-6 on [-8, 8]) times q_0 / Delta = 2^10
        assert np.max(np.abs(got - (d["v"][:n] + 1j * d["v"][n:]))) < 2 ** -10
        assert want.level == P.L - plan.depth
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)
