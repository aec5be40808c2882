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


@pytest.fixture(scope="module", params=["n12_3x50", "n13_9_limbs"])
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


def test_factorised_half_bootstrap_matches_oracle(X):
    # Half-BTS with the factorised CoeffsToSlots (3 sparse levels: 16, 31 and 15
    # diagonals at N = 2^12) over the 50 + 15 x 45-bit chain, word for word
    # against the oracle, eagerly and with the op list replayed from a graph
    from paper_2412_13269_amd import boot as HB
    from tests.test_boot_oracle import factorised_setup, run_factorised
    d = factorised_setup(12, 3, h=32, seed=910)
    P = d["P"]
    want = run_factorised(d)
    ctx = X.pfx_ctx_create(X.make_params(P.logn, [50] + [45] * 15, [50] * 4, 4, 17), 0)
    sk = X.pfx_sk_create(ctx, d["s"])
    gks = [X.pfx_swk_create(ctx, sk, g, a, e) for g, (a, e) in d["fkey_inputs"].items()]
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
        stages = []
        for steps, words, n1, scale in d["stages"]:
            pts = [X.pfx_pt_import(ctx, w, scale) for w in words]
            handles += pts
            stages.append((steps, pts, n1))
        # the library's own stage steps and baby-step counts are the oracle's
        for (s1, _), (s2, _, n1, _) in zip(HB.c2s_factor_stages(P.N, 3), d["stages"]):
            assert s1 == s2 and HB.bsgs_n1(s1) == n1
        regs = [X.pfx_ct_create(ctx, P.L, 1) for _ in range(plan.n_regs)]
        handles += regs
        out = HB.half_bootstrap_factorised(ctx, x, P.L, float(P.q[0]), stages, gks, rlk, plan, regs)
        assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c)
        assert X.pfx_ct_info(out).scale == want.scale
        stream = X.pfx_stream_create(ctx)
        try:
            for rep in range(2):
                out = HB.half_bootstrap_factorised(ctx, x, P.L, float(P.q[0]), stages, gks, rlk, plan, regs,
                                                   stream, X.RUN_GRAPH)
                X.pfx_sync(ctx, stream)
                assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c), rep
        finally:
            X.pfx_stream_destroy(ctx, stream)
        n = P.N // 2
        got = O.decode(P, O.decrypt(P, d["s"], want), want.scale, n)
        rev = B.bit_reverse(n)
        assert np.max(np.abs(got - (d["v"][:n] + 1j * d["v"][n:])[rev])) < 2 ** -10
        assert want.level == P.L - plan.depth - 2
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)


@pytest.mark.parametrize("log_r", [0, 3])
def test_factorised_half_bootstrap_at_full_size(X, log_r):
    # the paper's ring: N = 2^16, the 24 + 4 prime chain, a sparse secret of 32
    # non-zeros (the paper's bootstrapping secret), EvalMod on [-12, 12] (degree
    # 24, four double angles), CoeffsToSlots in 3 sparse levels (all 2^15
    # slots: 32, 63, 63 diagonals); the library's own diagonals, keys and
    # encoder.  Slot p of the result decrypts to the message's coefficients
    # rev(p) and rev(p) + N/2.  log_r = 3: sparse packing on n = 2^12 slots,
    # the trace-like map (3 automorphisms) after ModRaise, slot p and every
    # p + k n holding the coefficients 8 rev(p) and 8 (rev(p) + n).
    import math
    from numpy.polynomial import chebyshev as C
    from paper_2412_13269_amd import boot as HB
    from paper_2412_13269_amd import inputs as I
    logn, qb, pb = 16, [50] + [45] * 23, [50] * 4
    N, L = 1 << logn, len(qb)
    n = N >> (log_r + 1)
    delta, sd, K, r = 2.0 ** 40, 2.0 ** 40, 12.0, 4
    ctx = X.pfx_ctx_create(X.make_params(logn, qb, pb, 4, 17), 0)
    seed = b"half-bts at 2^16".ljust(32, b".")
    sk = X.pfx_keygen_secret(ctx, seed, 32)
    rlk = X.pfx_keygen_relin(ctx, sk, seed)
    fs = HB.c2s_factor_stages(N, 3, 0.5 / (1 << log_r), n)
    rots = set(HB.trace_rotations(N, log_r))
    for steps, _ in fs:
        rots |= HB.bsgs_rotations(N, steps, HB.bsgs_n1(steps))
    gks = X.pfx_keygen_galois(ctx, sk, sorted(rots), True, seed)
    q, _, _ = X.pfx_ctx_moduli(ctx, L, len(pb))
    q = [int(v) for v in q]
    coeffs = C.chebinterpolate(lambda t: np.cos(2 * math.pi * (K + 0.25) / 2 ** r * t), 24)
    plan = HB.HalfBootPlan(N, coeffs, r, K, q[0] / delta)
    handles = []
    try:
        v = I.uniform_slots(N, 920)
        words = (np.round(v * delta).astype(np.int64) % q[0]).astype(np.uint64)[None, :]
        x = X.pfx_ct_create(ctx, 1, 1)
        handles.append(x)
        pt = X.pfx_pt_import(ctx, words, delta)
        X.pfx_encrypt(ctx, sk, pt, I.uniform_residues(q[:1], N, 921), I.gaussian_error(N, 922), x)
        X.pfx_ct_destroy(pt)
        stages = []
        for i, (steps, diags) in enumerate(fs):
            assert all(st < n for st in steps) and all(len(dg) == n for dg in diags)
            scale = sd if i == 0 else float(q[L - 1 - i])
            pts = [X.pfx_encode(ctx, dg.real, dg.imag, L, scale) for dg in diags]
            handles += pts
            stages.append((steps, pts, HB.bsgs_n1(steps)))
        regs = [X.pfx_ct_create(ctx, L, 1) for _ in range(plan.n_regs)]
        handles += regs
        out = HB.half_bootstrap_factorised(ctx, x, L, float(q[0]), stages, gks, rlk, plan, regs, log_r=log_r)
        info = X.pfx_ct_info(out)
        assert info.n_limbs == L - plan.depth - 2
        m = X.pfx_decrypt(ctx, sk, out)
        got = X.pfx_decode(ctx, m, N // 2)
        X.pfx_ct_destroy(m)
        lg = n.bit_length() - 1
        rev = np.array([int(format(j, f"0{lg}b")[::-1], 2) for j in range(n)])
        sub = v[::1 << log_r]
        want = np.tile((sub[:n] + 1j * sub[n:])[rev], 1 << log_r)
        assert np.max(np.abs(got - want)) < 2 ** -10
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)


def test_sparse_half_bootstrap_matches_oracle(X):
    # sparse packing at N = 2^12 on n = 2^7 slots (r = 16): ModRaise, the
    # trace-like map (4 automorphisms), CoeffsToSlots in 2 levels (16 and 15
    # diagonals of length n), the conjugate split and EvalMod, word for word
    # against the oracle, eagerly and from a replayed graph
    from paper_2412_13269_amd import boot as HB
    from tests.test_boot_oracle import factorised_setup, run_factorised
    log_r, levels = 4, 2
    d = factorised_setup(12, levels, h=32, seed=930, log_r=log_r)
    P = d["P"]
    n = P.N >> (log_r + 1)
    want = run_factorised(d)
    ctx = X.pfx_ctx_create(X.make_params(P.logn, [50] + [45] * 15, [50] * 4, 4, 17), 0)
    sk = X.pfx_sk_create(ctx, d["s"])
    gks = [X.pfx_swk_create(ctx, sk, g, a, e) for g, (a, e) in d["fkey_inputs"].items()]
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
        stages = []
        for steps, words, n1, scale in d["stages"]:
            pts = [X.pfx_pt_import(ctx, w, scale) for w in words]
            handles += pts
            stages.append((steps, pts, n1))
        # the library's stage steps and baby-step counts, and its trace
        # rotations' Galois elements, are the oracle's
        for (s1, _), (s2, _, n1, _) in zip(HB.c2s_factor_stages(P.N, levels, 0.5 / (1 << log_r), n), d["stages"]):
            assert s1 == s2 and HB.bsgs_n1(s1) == n1
        assert [pow(5, k, 2 * P.N) for k in HB.trace_rotations(P.N, log_r)] == \
            [B.trace_galois(P, t) for t in range(log_r)]
        regs = [X.pfx_ct_create(ctx, P.L, 1) for _ in range(plan.n_regs)]
        handles += regs
        out = HB.half_bootstrap_factorised(ctx, x, P.L, float(P.q[0]), stages, gks, rlk, plan, regs, log_r=log_r)
        assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c)
        assert X.pfx_ct_info(out).scale == want.scale
        stream = X.pfx_stream_create(ctx)
        try:
            for rep in range(2):
                out = HB.half_bootstrap_factorised(ctx, x, P.L, float(P.q[0]), stages, gks, rlk, plan, regs,
                                                   stream, X.RUN_GRAPH, log_r=log_r)
                X.pfx_sync(ctx, stream)
                assert np.array_equal(X.pfx_ct_export(ctx, out, P.N), want.c), rep
        finally:
            X.pfx_stream_destroy(ctx, stream)
        got = O.decode(P, O.decrypt(P, d["s"], want), want.scale, P.N // 2)
        sub = d["v"][::1 << log_r]
        ref = np.tile((sub[:n] + 1j * sub[n:])[B.bit_reverse(n)], 1 << log_r)
        assert np.max(np.abs(got - ref)) < 2 ** -10
        assert want.level == P.L - plan.depth - (levels - 1)
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in gks + [rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_ctx_destroy(ctx)
