"""GPU: the BSGS plaintext-matrix linear transform (App. A.4) against the
oracle word for word, for two baby-step counts, at the top level and below;
and the decrypted slots against the FP64 matrix-vector product."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import linear as LT
from paper_2412_13269_amd import inputs as I
from tests.test_gpu_parity import CONFIGS, Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


@pytest.fixture(scope="module", params=["n12_3x50", "n13_9_limbs"])
def pair(request, X):
    cfg = CONFIGS[request.param]
    p = Pair(X, cfg["logn"], cfg["qb"], cfg["pb"], cfg["alpha"], cfg["ml"], cfg["h"], seed=29, scale=cfg["scale"])
    yield p
    p.close()


def _needed(P, steps, n1):
    half = P.N // 2
    st = [s % half for s in steps]
    return sorted({s % n1 for s in st} - {0}) + sorted({n1 * (s // n1) for s in st} - {0})


@pytest.mark.parametrize("n1", [4, 16])
def test_linear_transform_matches_oracle(pair, X, n1):
    P = pair.P
    half = P.N // 2
    steps = [0, 1, 2, 5, 7, 9, 13, 100, half - 1, half + 3]
    for k in _needed(P, steps, n1):
        pair.key(O.galois_element(P, k))
    for lv in (P.L, max(2, P.L - 2)):       # two limbs at least: the product's scale is scale^2
        co, cx, z = pair.enc(lv)
        ds = [(I.uniform_slots(half, 500 + k) + 1j * I.uniform_slots(half, 600 + k)) / len(steps)
              for k in range(len(steps))]
        words = [O.encode(P, d, pair.scale, lv) for d in ds]
        pts = []
        for w in words:
            pts.append(X.pfx_pt_import(pair.ctx, w, pair.scale))
            pair.handles.append(pts[-1])
        out = pair.ct(lv, deg=1)
        X.pfx_linear_transform(pair.ctx, cx, pts, steps, n1, list(pair.kx.values()), out)
        want = LT.linear_transform(P, co, words, pair.scale, steps, n1, pair.ko)
        pair.same(want, out)
        got = O.decode(P, O.decrypt(P, pair.s, O.Ct(pair.words(out), want.scale)), want.scale, half)
        ref = sum(d * np.roll(z, -(s % half)) for d, s in zip(ds, steps))
        assert np.max(np.abs(got - ref)) < 2 ** -15


def test_linear_transform_checks(pair, X):
    P = pair.P
    co, cx, z = pair.enc(P.L)
    w = O.encode(P, I.uniform_slots(P.N // 2, 700), pair.scale, P.L)
    pt = X.pfx_pt_import(pair.ctx, w, pair.scale)
    pair.handles.append(pt)
    out = pair.ct(P.L, deg=1)
    with pytest.raises(X.PfxError) as e:                        # no key for the step
        X.pfx_linear_transform(pair.ctx, cx, [pt], [P.N // 2 - 77], 1, [], out)
    assert e.value.status == X.PFX_ENOKEY
    with pytest.raises(X.PfxError) as e:                        # in place
        X.pfx_linear_transform(pair.ctx, cx, [pt], [0], 1, [], cx)
    assert e.value.status == X.PFX_EINVAL
    X.pfx_linear_transform(pair.ctx, cx, [pt], [0], 4, [], out)   # step 0 alone: a plaintext product
    want = O.ct_mul_plain(P, co, w, pair.scale)
    pair.same(want, out)


def test_dense_coeffs_to_slots_matches_oracle(X):
    # CoeffsToSlots (App. A.4) as one dense slot matrix at N = 2^12: 2048
    # diagonals, 63 hoisted baby steps and 31 giant steps (n1 = 64)
    from oracle import boot as B
    from tests.test_boot_oracle import transform_keys
    P = O.Params(12, [50, 45, 45, 45], [50, 50], alpha=2, mod_log2=17)
    n, delta, sd, n1 = P.N // 2, 2.0 ** 40, 2.0 ** 45, 64
    ctx = X.pfx_ctx_create(X.make_params(12, [50, 45, 45, 45], [50, 50], 2, 17), 0)
    s = I.ternary_secret(P.N, None, 401)
    sk = X.pfx_sk_create(ctx, s)
    ko = transform_keys(P, s, n1, 500)
    ext = P.ext_mods(P.L)
    kx, handles = [], []
    try:
        for i, g in enumerate(sorted(ko)):
            kx.append(X.pfx_swk_create(ctx, sk, g, I.uniform_residues(ext, P.N, 500 + 2 * i, lead=(P.beta,)),
                                       I.gaussian_error((P.beta, P.N), 501 + 2 * i)))
        z = I.uniform_slots(n, 402) + 1j * I.uniform_slots(n, 403)
        m = O.encode(P, z, delta, P.L)
        a, e = I.uniform_residues(P.mods(P.L), P.N, 404), I.gaussian_error(P.N, 405)
        xo = O.encrypt(P, s, m, a, e, delta)
        cx = X.pfx_ct_create(ctx, P.L, 1)
        handles.append(cx)
        pt = X.pfx_pt_import(ctx, m, delta)
        X.pfx_encrypt(ctx, sk, pt, a, e, cx)
        X.pfx_ct_destroy(pt)
        words = [O.encode(P, d, sd, P.L) for d in B.diagonals(B.c2s_matrix(P))]
        pts = []
        for w in words:
            pts.append(X.pfx_pt_import(ctx, w, sd))
            handles.append(pts[-1])
        out = X.pfx_ct_create(ctx, P.L, 1)
        handles.append(out)
        X.pfx_linear_transform(ctx, cx, pts, list(range(n)), n1, kx, out)
        want = LT.linear_transform(P, xo, words, sd, list(range(n)), n1, ko)
        assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c)
        mc = O.crt_centered(m, P.mods(P.L)).astype(float) / delta
        got = O.decode(P, O.decrypt(P, s, want), want.scale, n)
        assert np.max(np.abs(got - (mc[:n] + 1j * mc[n:]))) < 1e-6
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in kx:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)


@pytest.fixture(scope="module")
def pair_c1(X):
    cfg = CONFIGS["n12_3x50"]
    p = Pair(X, cfg["logn"], cfg["qb"], cfg["pb"], cfg["alpha"], cfg["ml"], cfg["h"], seed=37, scale=cfg["scale"])
    yield p
    p.close()


def test_linear_transform_group_beyond_one_launch(pair_c1, X):
    # 70 diagonals in one giant-step group (n1 = 128): the group sum takes two
    # multiply-accumulate launches of at most 64 terms, the second adding to
    # the first; a second group (steps 128 + i) rotated by 128 (N = 2^12)
    pair = pair_c1
    P = pair.P
    n1 = 128
    steps = list(range(70)) + [128 + i for i in (0, 3, 65)]
    for k in _needed(P, steps, n1):
        pair.key(O.galois_element(P, k))
    co, cx, z = pair.enc(P.L)
    half = P.N // 2
    ds = [(I.uniform_slots(half, 800 + k) + 1j * I.uniform_slots(half, 900 + k)) / len(steps)
          for k in range(len(steps))]
    words = [O.encode(P, d, pair.scale, P.L) for d in ds]
    pts = []
    for w in words:
        pts.append(X.pfx_pt_import(pair.ctx, w, pair.scale))
        pair.handles.append(pts[-1])
    out = pair.ct(P.L, deg=1)
    X.pfx_linear_transform(pair.ctx, cx, pts, steps, n1, list(pair.kx.values()), out)
    want = LT.linear_transform(P, co, words, pair.scale, steps, n1, pair.ko)
    pair.same(want, out)
