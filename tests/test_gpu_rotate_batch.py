"""Batched rotations with one key per entry (pfx_rotate_batch) against
pfx_rotate one at a time: 15 steps over ciphertexts at mixed levels at
N = 2^16, L = 24 (two and three batches), a step of zero, the argument
checks, and the oracle's words at N = 2^12."""
import numpy as np
import pytest

from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu

QB, PB, ALPHA, ML = [50] + [45] * 23, [50] * 4, 4, 17
STEPS = [1 << k for k in range(15)]


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def test_rotate_batch_equals_single_rotations(X):
    logn = 16
    N = 1 << logn
    ctx = X.pfx_ctx_create(X.make_params(logn, QB, PB, ALPHA, ML), 0)
    st = X.pfx_stream_create(ctx)
    seed = b"rotate-batch".ljust(32, b".")
    sk = X.pfx_keygen_secret(ctx, seed, 192)
    gks = X.pfx_keygen_galois(ctx, sk, STEPS + [-3], False, seed)
    q, _, _ = X.pfx_ctx_moduli(ctx, len(QB), len(PB))
    handles = []
    try:
        srcs = []
        for k, lv in enumerate((24, 24, 13, 5)):
            h = X.pfx_ct_create(ctx, len(QB), 1)
            X.pfx_ct_import(ctx, I.uniform_residues(q[:lv], N, 700 + k, lead=(2,)), 2.0 ** 45, h, st)
            srcs.append(h)
        handles += srcs
        # every step on the first ciphertext (two batches of the full level),
        # then mixed levels and steps, a negative step and a zero step
        cases = [(srcs[0], s) for s in STEPS] + [(srcs[1], 1), (srcs[2], 8), (srcs[3], 1 << 14),
                                                  (srcs[2], -3), (srcs[1], 0)]
        outs = [X.pfx_ct_create(ctx, len(QB), 1) for _ in cases]
        refs = [X.pfx_ct_create(ctx, len(QB), 1) for _ in cases]
        handles += outs + refs
        X.pfx_rotate_batch(ctx, [c for c, _ in cases], [s for _, s in cases], gks, outs, st)
        for (c, s), r in zip(cases, refs):
            X.pfx_rotate(ctx, c, s, gks, r, st)
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert np.array_equal(X.pfx_ct_export(ctx, o, N, st), X.pfx_ct_export(ctx, r, N, st)), cases[i][1]
            assert X.pfx_ct_info(o).n_limbs == X.pfx_ct_info(r).n_limbs
        # argument checks
        with pytest.raises(X.PfxError) as e:
            X.pfx_rotate_batch(ctx, [srcs[0]], [1], gks, [srcs[0]], st)
        assert e.value.status == X.PFX_EINVAL
        with pytest.raises(X.PfxError) as e:
            X.pfx_rotate_batch(ctx, [srcs[0], srcs[1]], [1, 2], gks, [outs[0], outs[0]], st)
        assert e.value.status == X.PFX_EINVAL
        with pytest.raises(X.PfxError) as e:
            X.pfx_rotate_batch(ctx, [srcs[0]], [7], gks, [outs[0]], st)
        assert e.value.status == X.PFX_ENOKEY
        X.pfx_sync(ctx, st)
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in gks:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_stream_destroy(ctx, st)
        X.pfx_ctx_destroy(ctx)


def test_rotate_batch_matches_oracle(X):
    from oracle import ckks as O
    logn, qb, pb, alpha = 12, [50] + [45] * 5, [50] * 2, 2
    N = 1 << logn
    P = O.Params(logn, qb, pb, alpha=alpha, mod_log2=ML)
    ctx = X.pfx_ctx_create(X.make_params(logn, qb, pb, alpha, ML), 0)
    try:
        s = I.ternary_secret(N, 64, 41)
        sk = X.pfx_sk_create(ctx, s)
        ext = P.ext_mods(P.L)
        steps = [1, 2, 7, -1]
        okeys, gks = {}, []
        for k, step in enumerate(steps):
            g = O.galois_element(P, step)
            ka, ke = I.uniform_residues(ext, N, 50 + 2 * k, lead=(P.beta,)), I.gaussian_error((P.beta, N), 51 + 2 * k)
            okeys[g] = O.galois_key(P, s, g, ka, ke)
            gks.append(X.pfx_swk_create(ctx, sk, g, ka, ke))
        words = [I.uniform_residues(P.q, N, 60 + k, lead=(2,)) for k in range(2)]
        a = [X.pfx_ct_create(ctx, len(qb), 1) for _ in words]
        for h, w in zip(a, words):
            X.pfx_ct_import(ctx, w, 2.0 ** 45, h)
        ins = [a[k % 2] for k in range(len(steps))]
        outs = [X.pfx_ct_create(ctx, len(qb), 1) for _ in steps]
        X.pfx_rotate_batch(ctx, ins, steps, gks, outs)
        for k, (step, o) in enumerate(zip(steps, outs)):
            want = O.rotate(P, O.Ct(words[k % 2], 2.0 ** 45), step, okeys)
            assert np.array_equal(X.pfx_ct_export(ctx, o, N), want.c), step
        for h in a + outs:
            X.pfx_ct_destroy(h)
        for k in gks:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
    finally:
        X.pfx_ctx_destroy(ctx)


def test_modup_sub_batches_give_the_same_words(X):
    # ks_modup_batch: the ModUp conversion, its row pass and the inner product
    # of a batch run a few entries at a time; batched rotations (a key each) and
    # batched HMult + relin (one key) give the words of the whole-batch launches
    logn = 16
    N = 1 << logn
    saved = X.pfx_tuning_get(logn)
    ctx = X.pfx_ctx_create(X.make_params(logn, QB, PB, ALPHA, ML), 0)
    st = X.pfx_stream_create(ctx)
    seed = b"modup sub-batches".ljust(32, b".")
    sk = X.pfx_keygen_secret(ctx, seed, 192)
    rlk = X.pfx_keygen_relin(ctx, sk, seed)
    gks = X.pfx_keygen_galois(ctx, sk, STEPS[:7], False, seed)
    q, _, _ = X.pfx_ctx_moduli(ctx, len(QB), len(PB))
    handles = []
    try:
        a = []
        for k in range(2):
            h = X.pfx_ct_create(ctx, len(QB), 1)
            X.pfx_ct_import(ctx, I.uniform_residues(q, N, 760 + k, lead=(2,)), 2.0 ** 45, h, st)
            a.append(h)
        outs = [X.pfx_ct_create(ctx, len(QB), 1) for _ in range(7)]
        handles += a + outs
        res = {}
        for sub in (0, 2, 3, 1):
            X.pfx_tuning_set(logn, ks_modup_batch=sub)
            X.pfx_rotate_batch(ctx, [a[k % 2] for k in range(7)], STEPS[:7], gks, outs, st)
            words = [X.pfx_ct_export(ctx, h, N, st) for h in outs]
            X.pfx_mul_relin_batch(ctx, [a[0], a[1], a[0], a[1], a[0]], [a[1], a[1], a[0], a[0], a[1]], rlk,
                                  outs[:5], st)
            res[sub] = words + [X.pfx_ct_export(ctx, h, N, st) for h in outs[:5]]
        for sub in (2, 3, 1):
            assert all(np.array_equal(x, y) for x, y in zip(res[sub], res[0])), sub
    finally:
        X.pfx_tuning_set(logn, **{f: getattr(saved, f) for f in X.TUNING_FIELDS})
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_stream_destroy(ctx, st)
        X.pfx_ctx_destroy(ctx)


def test_stream_join_orders_work_on_two_streams(X):
    # pfx_stream_wait_event: HMult + relin on a second stream forked from the
    # first, a rotation of its product on the first after the join; words equal
    # the same calls on one stream
    logn = 12
    N = 1 << logn
    ctx = X.pfx_ctx_create(X.make_params(logn, QB[:6], PB, ALPHA, ML), 0)
    st, st2 = X.pfx_stream_create(ctx), X.pfx_stream_create(ctx)
    fork, join = X.pfx_event_create(ctx), X.pfx_event_create(ctx)
    seed = b"stream join".ljust(32, b".")
    sk = X.pfx_keygen_secret(ctx, seed, 192)
    rlk = X.pfx_keygen_relin(ctx, sk, seed)
    gks = X.pfx_keygen_galois(ctx, sk, [3], False, seed)
    q, _, _ = X.pfx_ctx_moduli(ctx, 6, len(PB))
    hs = [X.pfx_ct_create(ctx, 6, 1) for _ in range(6)]
    a, b, p1, r1, p2, r2 = hs
    try:
        for k, h in enumerate((a, b)):
            X.pfx_ct_import(ctx, I.uniform_residues(q, N, 780 + k, lead=(2,)), 2.0 ** 45, h, st)
        X.pfx_mul_relin(ctx, a, b, rlk, p1, st)
        X.pfx_rotate(ctx, p1, 3, gks, r1, st)
        for _ in range(3):
            X.pfx_event_record(ctx, fork, st)
            X.pfx_stream_wait_event(ctx, st2, fork)
            X.pfx_mul_relin(ctx, a, b, rlk, p2, st2)
            X.pfx_event_record(ctx, join, st2)
            X.pfx_stream_wait_event(ctx, st, join)
            X.pfx_rotate(ctx, p2, 3, gks, r2, st)
            assert np.array_equal(X.pfx_ct_export(ctx, r2, N, st), X.pfx_ct_export(ctx, r1, N, st))
        with pytest.raises(X.PfxError):
            X.pfx_stream_wait_event(ctx, st, 0)
    finally:
        X.pfx_sync(ctx, st2)
        for h in hs:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_event_destroy(ctx, fork)
        X.pfx_event_destroy(ctx, join)
        X.pfx_stream_destroy(ctx, st2)
        X.pfx_stream_destroy(ctx, st)
        X.pfx_ctx_destroy(ctx)
