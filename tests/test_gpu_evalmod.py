"""GPU: the EvalMod op list (App. A.3) through pfx_run_circuit against the
oracle word for word, eagerly and from a replayed HIP graph, at N = 2^12 with
the 24-limb chain; decrypted slots against the FP64 steps."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import evalmod as E
from paper_2412_13269_amd import inputs as I
from tests.test_evalmod_oracle import coeffs
from tests.test_gpu_query import ALPHA, DELTA, ML, PB, QB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def test_evalmod_plan_matches_oracle(X):
    from paper_2412_13269_amd.evalmod import EvalModPlan
    logn, K, r, deg = 12, 8.0, 3, 24
    P = O.Params(logn, QB, PB, alpha=ALPHA, mod_log2=ML)
    N = P.N
    ctx = X.pfx_ctx_create(X.make_params(logn, QB, PB, ALPHA, ML), 0)
    s = I.ternary_secret(N, 192, 71)
    sk = X.pfx_sk_create(ctx, s)
    ext = P.ext_mods(P.L)
    ka, ke = I.uniform_residues(ext, N, 72, lead=(P.beta,)), I.gaussian_error((P.beta, N), 73)
    rlk_o, rlk = O.relin_key(P, s, ka, ke), X.pfx_swk_create(ctx, sk, 0, ka, ke)
    rng = np.random.default_rng(74)
    t = rng.integers(-7, 8, size=N // 2) + rng.uniform(-0.05, 0.05, size=N // 2)
    m = O.encode(P, t, DELTA, P.L)
    a, e = I.uniform_residues(P.mods(P.L), N, 75), I.gaussian_error(N, 76)
    xo = O.encrypt(P, s, m, a, e, DELTA)
    plan = EvalModPlan(list(coeffs(deg, K, r)), r, K)
    regs = [X.pfx_ct_create(ctx, P.L, 1) for _ in range(plan.n_regs)]
    pt = X.pfx_pt_import(ctx, m, DELTA)
    X.pfx_encrypt(ctx, sk, pt, a, e, regs[0])
    X.pfx_ct_destroy(pt)
    stream = X.pfx_stream_create(ctx)
    try:
        want = E.evalmod(P, xo, coeffs(deg, K, r), r, K, rlk_o)
        for graph in (False, True, True):
            X.pfx_run_circuit(ctx, plan.ops, regs, 1, [], rlk, [], X.RUN_GRAPH if graph else X.RUN_EAGER, stream)
            X.pfx_sync(ctx, stream)
            words = X.pfx_ct_export(ctx, regs[plan.out], N)
            assert np.array_equal(words, want.c), graph
            assert X.pfx_ct_info(regs[plan.out]).scale == want.scale
        assert want.level == P.L - plan.depth
        got = O.decode(P, O.decrypt(P, s, want), want.scale, N // 2).real
        assert np.max(np.abs(got - E.evalmod_fp64(t, coeffs(deg, K, r), r, K))) < 2 ** -15
        assert np.max(np.abs(got - (t - np.round(t)))) < 1e-3       # the fractional part, up to its cubic term
    finally:
        for h in regs:
            X.pfx_ct_destroy(h)
        X.pfx_swk_destroy(rlk)
        X.pfx_sk_destroy(sk)
        X.pfx_stream_destroy(ctx, stream)
        X.pfx_ctx_destroy(ctx)


def test_mul_const_to_checks(X):
    # MUL_CONST_TO: the target register must exist, and a one-limb operand has
    # no prime left to rescale by; MUL_CONST_LIKE against the oracle
    logn = 12
    P = O.Params(logn, QB[:3], PB, alpha=ALPHA, mod_log2=ML)
    ctx = X.pfx_ctx_create(X.make_params(logn, QB[:3], PB, ALPHA, ML), 0)
    sk = X.pfx_sk_create(ctx, I.ternary_secret(P.N, 192, 81))
    regs = [X.pfx_ct_create(ctx, P.L, 1) for _ in range(3)]
    try:
        for lv, reg in ((P.L, regs[0]), (1, regs[1])):
            m = O.encode(P, I.uniform_slots(P.N // 2, 82), DELTA, lv)
            pt = X.pfx_pt_import(ctx, m, DELTA)
            X.pfx_encrypt(ctx, sk, pt, I.uniform_residues(P.mods(lv), P.N, 83), I.gaussian_error(P.N, 84), reg)
            X.pfx_ct_destroy(pt)
        with pytest.raises(X.PfxError) as e:
            X.pfx_run_circuit(ctx, [(X.OP_MUL_CONST_TO, 2, 0, 7, 0, 0.5)], regs, 2, [], None, [])
        assert e.value.status == X.PFX_EINVAL
        with pytest.raises(X.PfxError) as e:
            X.pfx_run_circuit(ctx, [(X.OP_MUL_CONST_TO, 2, 1, 0, 0, 0.5)], regs, 2, [], None, [])
        assert e.value.status == X.PFX_ELEVEL
        # the product of a full-level operand, rescaled, carries register 0's scale
        X.pfx_run_circuit(ctx, [(X.OP_MUL_CONST_TO, 2, 0, 0, 0, 0.5), (X.OP_RESCALE, 2, 2, -1, 0, 0.0)],
                          regs, 2, [], None, [])
        got, want = X.pfx_ct_info(regs[2]).scale, X.pfx_ct_info(regs[0]).scale
        assert abs(got / want - 1) < 1e-15 and X.pfx_ct_info(regs[2]).n_limbs == P.L - 1
        # the product's words before the rescale are the oracle's
        from oracle.query import mul_const_to
        X.pfx_run_circuit(ctx, [(X.OP_MUL_CONST_TO, 2, 0, 0, 0, 0.5)], regs, 2, [], None, [])
        x0 = O.Ct(X.pfx_ct_export(ctx, regs[0], P.N), X.pfx_ct_info(regs[0]).scale)
        assert np.array_equal(X.pfx_ct_export(ctx, regs[2], P.N), mul_const_to(P, x0, 0.5, x0.scale).c)
        # MUL_CONST_LIKE: the product carries register b's scale, at a's level,
        # with the constant round(value * scale_b / scale_a) (the oracle's)
        X.pfx_ct_set_scale(regs[1], DELTA * 2.0 ** 20)
        X.pfx_run_circuit(ctx, [(X.OP_MUL_CONST_LIKE, 2, 0, 1, 0, -0.75)], regs, 2, [], None, [])
        info = X.pfx_ct_info(regs[2])
        assert info.scale == X.pfx_ct_info(regs[0]).scale * (DELTA * 2.0 ** 20 / X.pfx_ct_info(regs[0]).scale)
        assert info.n_limbs == P.L
        from oracle.query import mul_const_like
        x0 = O.Ct(X.pfx_ct_export(ctx, regs[0], P.N), X.pfx_ct_info(regs[0]).scale)
        assert np.array_equal(X.pfx_ct_export(ctx, regs[2], P.N), mul_const_like(P, x0, -0.75, DELTA * 2.0 ** 20).c)
        with pytest.raises(X.PfxError) as e:
            X.pfx_run_circuit(ctx, [(X.OP_MUL_CONST_LIKE, 2, 0, 7, 0, 0.5)], regs, 2, [], None, [])
        assert e.value.status == X.PFX_EINVAL
    finally:
        for h in regs:
            X.pfx_ct_destroy(h)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)
