"""The no-allocation HMult + relinearisation (pfx_mul_relin_noalloc) against
pfx_mul_relin, word for word, through the C-ABI: two calls in a row on the
same GPU (the second at a lower level, so the shared scratch array holds the
first call's larger contents), the output aliasing an operand, and a product
whose scratch exceeds the array, refused with nothing written."""
import numpy as np
import pytest

from oracle import ckks as O
from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu

QB, PB, ALPHA, ML = [50] + [45] * 23, [50] * 4, 4, 17
DELTA = 2.0 ** 45


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def _setup(X, logn, seed):
    P = O.Params(logn, QB, PB, alpha=ALPHA, mod_log2=ML)
    ctx = X.pfx_ctx_create(X.make_params(logn, QB, PB, ALPHA, ML), 0)
    N = P.N
    s = I.ternary_secret(N, 192, seed)
    sk = X.pfx_sk_create(ctx, s)
    ext = P.ext_mods(P.L)
    kin = (I.uniform_residues(ext, N, seed + 1, lead=(P.beta,)), I.gaussian_error((P.beta, N), seed + 2))
    rlk = X.pfx_swk_create(ctx, sk, 0, *kin)
    return P, ctx, sk, rlk, (s, kin)


def _enc(X, P, ctx, sk, lv, seed):
    N = P.N
    m = O.encode(P, I.uniform_slots(N // 2, seed), DELTA, lv)
    pt = X.pfx_pt_import(ctx, m, DELTA)
    h = X.pfx_ct_create(ctx, P.L, 1)
    X.pfx_encrypt(ctx, sk, pt, I.uniform_residues(P.mods(lv), N, seed + 1), I.gaussian_error(N, seed + 2), h)
    X.pfx_ct_destroy(pt)
    return h


def test_noalloc_mul_relin_equals_mul_relin(X):
    assert X.pfx_noalloc_scratch_bytes() == 64 << 20
    P, ctx, sk, rlk, (s, kin) = _setup(X, 14, 601)
    st = X.pfx_stream_create(ctx)
    hs = []
    try:
        # two calls in a row, the second smaller (9 limbs after 24)
        for lv, sd in ((24, 610), (9, 620)):
            a, b = _enc(X, P, ctx, sk, lv, sd), _enc(X, P, ctx, sk, lv, sd + 5)
            want, got = X.pfx_ct_create(ctx, P.L, 1), X.pfx_ct_create(ctx, P.L, 1)
            hs += [a, b, want, got]
            X.pfx_mul_relin(ctx, a, b, rlk, want, st)
            X.pfx_mul_relin_noalloc(ctx, a, b, rlk, got, st)
            X.pfx_sync(ctx, st)
            w, g = X.pfx_ct_export(ctx, want, P.N, st), X.pfx_ct_export(ctx, got, P.N, st)
            assert w.shape == (2, lv, P.N) and np.array_equal(g, w), lv
            iw, ig = X.pfx_ct_info(want), X.pfx_ct_info(got)
            assert (ig.n_limbs, ig.degree, ig.scale) == (iw.n_limbs, iw.degree, iw.scale)
        # output aliasing an operand: the tensor product goes through the array too
        a, b = _enc(X, P, ctx, sk, 24, 630), _enc(X, P, ctx, sk, 24, 635)
        want = X.pfx_ct_create(ctx, P.L, 1)
        hs += [a, b, want]
        X.pfx_mul_relin(ctx, a, b, rlk, want, st)
        X.pfx_mul_relin_noalloc(ctx, a, b, rlk, a, st)
        X.pfx_sync(ctx, st)
        assert np.array_equal(X.pfx_ct_export(ctx, a, P.N, st), X.pfx_ct_export(ctx, want, P.N, st))
    finally:
        for h in hs:
            X.pfx_ct_destroy(h)
        X.pfx_swk_destroy(rlk)
        X.pfx_sk_destroy(sk)
        X.pfx_stream_destroy(ctx, st)
        X.pfx_ctx_destroy(ctx)


def test_noalloc_refuses_a_product_beyond_its_array(X):
    P, ctx, sk, rlk, _ = _setup(X, 16, 640)
    hs = []
    try:
        a, b = _enc(X, P, ctx, sk, 24, 650), _enc(X, P, ctx, sk, 24, 655)
        out = X.pfx_ct_create(ctx, P.L, 1)
        hs += [a, b, out]
        X.pfx_ct_import(ctx, np.zeros((2, 24, P.N), np.uint64), 1.0, out)
        with pytest.raises(X.PfxError) as e:
            X.pfx_mul_relin_noalloc(ctx, a, b, rlk, out)
        assert e.value.status == X.PFX_ENOMEM
        assert not X.pfx_ct_export(ctx, out, P.N).any()
        # the same level at N = 2^16 works through the allocating call
        X.pfx_mul_relin(ctx, a, b, rlk, out)
        X.pfx_sync(ctx)
        assert X.pfx_ct_info(out).n_limbs == 24
    finally:
        for h in hs:
            X.pfx_ct_destroy(h)
        X.pfx_swk_destroy(rlk)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)
