"""The fused ModUp row pass + key inner product (pass tuning ks_fuse = 128 or
256) against the separate launches (ks_fuse = 0, oracle-exact in the parity
tests): rotations, conjugation, HMult + relin, relinearisation and batched
HMult + relin give the same words at ring degrees 2^12, 2^14 and 2^16, at the
full level and at a partial one; at 2^12 also the oracle's words for a
rotation."""
import numpy as np
import pytest

from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu

QB, PB, ALPHA, ML = [50] + [45] * 23, [50] * 4, 4, 17


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def _ops(X, ctx, st, N, cts, rlk, gks, lv):
    """Words of every key-switching op on the operands cut to lv limbs."""
    out = {}
    a, b = cts
    if lv < len(QB):
        cut = []
        for x in (a, b):
            y = X.pfx_ct_create(ctx, len(QB), 1)
            X.pfx_drop_level(ctx, x, lv, y, st)
            cut.append(y)
        a, b = cut
    o = X.pfx_ct_create(ctx, len(QB), 1)
    t2 = X.pfx_ct_create(ctx, len(QB), 2)
    try:
        for step in (1, 5, -1):
            X.pfx_rotate(ctx, a, step, gks, o, st)
            out[f"rot{step}"] = X.pfx_ct_export(ctx, o, N, st)
        X.pfx_conjugate(ctx, a, gks, o, st)
        out["conj"] = X.pfx_ct_export(ctx, o, N, st)
        X.pfx_mul_relin(ctx, a, b, rlk, o, st)
        out["mul_relin"] = X.pfx_ct_export(ctx, o, N, st)
        X.pfx_mul(ctx, a, b, t2, st)
        X.pfx_relinearize(ctx, t2, rlk, o, st)
        out["relin"] = X.pfx_ct_export(ctx, o, N, st)
        outs = [X.pfx_ct_create(ctx, len(QB), 1) for _ in range(3)]
        try:
            X.pfx_mul_relin_batch(ctx, [a, b, a], [b, b, a], rlk, outs, st)
            for i, h in enumerate(outs):
                out[f"batch{i}"] = X.pfx_ct_export(ctx, h, N, st)
        finally:
            for h in outs:
                X.pfx_ct_destroy(h)
    finally:
        X.pfx_ct_destroy(o)
        X.pfx_ct_destroy(t2)
        if lv < len(QB):
            for y in (a, b):
                X.pfx_ct_destroy(y)
    return out


@pytest.mark.parametrize("logn", [12, 14, 16])
def test_fused_key_switch_words_equal_separate_launches(X, logn):
    N = 1 << logn
    saved = X.pfx_tuning_get(logn)
    ctx = X.pfx_ctx_create(X.make_params(logn, QB, PB, ALPHA, ML), 0)
    st = X.pfx_stream_create(ctx)
    seed = bytes([logn, 7]) * 16
    sk = X.pfx_keygen_secret(ctx, seed, 192 if logn >= 13 else 64)
    rlk = X.pfx_keygen_relin(ctx, sk, seed)
    gks = X.pfx_keygen_galois(ctx, sk, [1, 5, -1], True, seed)
    q, _, _ = X.pfx_ctx_moduli(ctx, len(QB), len(PB))
    cts = []
    try:
        for k in range(2):
            h = X.pfx_ct_create(ctx, len(QB), 1)
            X.pfx_ct_import(ctx, I.uniform_residues(q, N, 900 + 10 * logn + k, lead=(2,)), 2.0 ** 45, h, st)
            cts.append(h)
        for lv in (len(QB), 13):
            res = {}
            for fuse in (0, 128, 256):
                X.pfx_tuning_set(logn, ks_fuse=fuse)
                res[fuse] = _ops(X, ctx, st, N, cts, rlk, gks, lv)
            for fuse in (128, 256):
                for k, v in res[0].items():
                    assert np.array_equal(res[fuse][k], v), (logn, lv, fuse, k)
    finally:
        X.pfx_tuning_set(logn, **{f: getattr(saved, f) for f in X.TUNING_FIELDS})
        for h in cts:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_stream_destroy(ctx, st)
        X.pfx_ctx_destroy(ctx)


def test_fused_rotation_matches_oracle(X):
    from oracle import ckks as O
    logn, qb, pb, alpha = 12, [50] + [45] * 5, [50] * 2, 2
    N = 1 << logn
    P = O.Params(logn, qb, pb, alpha=alpha, mod_log2=ML)
    saved = X.pfx_tuning_get(logn)
    ctx = X.pfx_ctx_create(X.make_params(logn, qb, pb, alpha, ML), 0)
    try:
        s = I.ternary_secret(N, 64, 31)
        sk = X.pfx_sk_create(ctx, s)
        ext = P.ext_mods(P.L)
        g = pow(5, 3, 2 * N)
        ka, ke = I.uniform_residues(ext, N, 32, lead=(P.beta,)), I.gaussian_error((P.beta, N), 33)
        gk = X.pfx_swk_create(ctx, sk, g, ka, ke)
        words = I.uniform_residues(P.q, N, 34, lead=(2,))
        a = X.pfx_ct_create(ctx, len(qb), 1)
        o = X.pfx_ct_create(ctx, len(qb), 1)
        X.pfx_ct_import(ctx, words, 2.0 ** 45, a)
        want = O.rotate(P, O.Ct(words, 2.0 ** 45), 3, {g: O.galois_key(P, s, g, ka, ke)})
        for fuse in (128, 256):
            X.pfx_tuning_set(logn, ks_fuse=fuse)
            X.pfx_rotate(ctx, a, 3, [gk], o)
            assert np.array_equal(X.pfx_ct_export(ctx, o, N), want.c), fuse
        for h in (a, o):
            X.pfx_ct_destroy(h)
        X.pfx_swk_destroy(gk)
        X.pfx_sk_destroy(sk)
    finally:
        X.pfx_tuning_set(logn, **{f: getattr(saved, f) for f in X.TUNING_FIELDS})
        X.pfx_ctx_destroy(ctx)
