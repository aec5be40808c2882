"""The private query on the GPU (op list, eager and HIP-graph replay) against
the oracle circuit word for word, and at full size against FP64."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import query as Q
from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu

QB, PB, ALPHA, ML = [50] + [45] * 23, [50] * 4, 4, 17
DELTA = 2.0 ** 45


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def spread(x, w):
    s = x @ w
    t = float(np.median(s))
    c = np.zeros(8)
    c[1] = 1.0
    return c, t, 0.9 / float(np.max(np.abs(s - t)))


def gap_records(x, w, c, t, eta, gap, seed):
    """Keep records whose threshold input u satisfies gap <= |u| <= 0.95,
    drawing more from the same distribution until there are len(x) of them."""
    want, A = len(x), x.shape[1]
    keep, it = [], 0
    pool = x
    while sum(len(k) for k in keep) < want:
        s = pool @ w
        u = (sum(c[k] * s ** k for k in range(len(c))) - t) * eta
        keep.append(pool[(np.abs(u) >= gap) & (np.abs(u) <= 0.95)])
        it += 1
        pool = I.synthetic_database(4 * want, A, seed + 1000 + it)
    return np.concatenate(keep)[:want]


class Setup:
    """Library objects for one query; oracle twins built only when asked."""

    def __init__(self, X, logn, n_blocks, seed, gap=None, with_oracle=False, degree=7, **plan_kw):
        from paper_2412_13269_amd.query import QueryPlan
        self.X = X
        self.logn, self.N, self.n = logn, 1 << logn, 1 << (logn - 1)
        A, D = 8, degree
        self.D = D
        self.x = I.synthetic_database(self.n * n_blocks, A, seed)
        w, c, t, eta = I.query_parameters(A, D, seed + 1)
        if gap is not None:
            c, t, eta = spread(self.x, w)
            c = np.concatenate([c, np.zeros(max(0, D + 1 - len(c)))])[:D + 1]
            self.x = gap_records(self.x, w, c, t, eta, gap, seed)
        self.params = (w, c, t, eta)
        self.plan = QueryPlan(n_blocks, A, D, 3, logn - 1, **plan_kw)
        prm = X.make_params(logn, QB, PB, ALPHA, ML)
        self.ctx = X.pfx_ctx_create(prm, 0)
        q, p, _ = X.pfx_ctx_moduli(self.ctx, len(QB), len(PB))
        self.q = [int(v) for v in q]
        ext = self.q + [int(v) for v in p]
        beta = -(-len(QB) // ALPHA)
        N = self.N
        self.s = I.ternary_secret(N, 192, seed + 2)
        self.sk = X.pfx_sk_create(self.ctx, self.s)
        self.key_in = {0: (I.uniform_residues(ext, N, seed + 3, lead=(beta,)), I.gaussian_error((beta, N), seed + 4))}
        for k in range(logn - 1):
            g = pow(5, 1 << k, 2 * N)
            self.key_in[g] = (I.uniform_residues(ext, N, seed + 10 + 2 * k, lead=(beta,)),
                              I.gaussian_error((beta, N), seed + 11 + 2 * k))
        self.rlk = X.pfx_swk_create(self.ctx, self.sk, 0, *self.key_in[0])
        self.gks = [X.pfx_swk_create(self.ctx, self.sk, g, *v) for g, v in self.key_in.items() if g]
        # encrypted parameters (broadcast) and database plaintexts: oracle-encoded words
        self.P = O.Params(logn, QB, PB, alpha=ALPHA, mod_log2=ML) if with_oracle else None
        if with_oracle:       # words fed to both sides come from the oracle's encoder
            assert self.P.q == self.q
            encode = lambda z: O.encode(self.P, z, DELTA, len(QB))
        else:
            encode = lambda z: X.pfx_encode_words(prm, z, None, len(QB), DELTA)
        enc_words = [encode(np.full(self.n, v)) for v in list(w) + list(c) + [t, eta]]
        self.enc_in = []
        self.regs = [X.pfx_ct_create(self.ctx, len(QB), self.plan.reg_degree[i]) for i in range(self.plan.n_regs)]
        self.pts = []
        for i, m in enumerate(enc_words):
            a = I.uniform_residues(self.q, N, seed + 500 + 2 * i)
            e = I.gaussian_error(N, seed + 501 + 2 * i)
            self.enc_in.append((m, a, e))
            pt = X.pfx_pt_import(self.ctx, m, DELTA)
            X.pfx_encrypt(self.ctx, self.sk, pt, a, e, self.regs[i])
            X.pfx_ct_destroy(pt)
        self.db_words = []
        for b in range(n_blocks):
            for a in range(A):
                m = encode(self.x[b * self.n:(b + 1) * self.n, a])
                self.db_words.append(m)
                self.pts.append(X.pfx_pt_import(self.ctx, m, DELTA))
        self.stream = X.pfx_stream_create(self.ctx)

    def use_plan(self, plan):
        """Another op list over the same inputs: fresh work registers for it."""
        X = self.X
        assert plan.n_inputs == self.plan.n_inputs
        for h in self.regs[plan.n_inputs:]:
            X.pfx_ct_destroy(h)
        self.regs = self.regs[:plan.n_inputs] + [X.pfx_ct_create(self.ctx, len(QB), plan.reg_degree[i])
                                                 for i in range(plan.n_inputs, plan.n_regs)]
        self.plan = plan

    def run(self, graph=False, lanes=False):
        X = self.X
        mode = (X.RUN_GRAPH if graph else 0) | (X.RUN_LANES if lanes else 0)
        X.pfx_run_circuit(self.ctx, self.plan.ops, self.regs, self.plan.n_inputs, self.pts, self.rlk, self.gks,
                          mode, self.stream)
        X.pfx_sync(self.ctx, self.stream)
        return self.regs[self.plan.out]

    def count(self, ct):
        X = self.X
        m = X.pfx_decrypt(self.ctx, self.sk, ct)
        z = X.pfx_decode(self.ctx, m, self.n)
        X.pfx_ct_destroy(m)
        return z.real

    def oracle_out(self):
        P = self.P
        ct = lambda m, a, e: O.encrypt(P, self.s, m, a, e, DELTA)
        cts = [ct(*v) for v in self.enc_in]
        A, D = 8, self.D
        W, C, T, H = cts[:A], cts[A:A + D + 1], cts[A + D + 1], cts[A + D + 2]
        rlk = O.relin_key(P, self.s, *self.key_in[0])
        gks = {g: O.galois_key(P, self.s, g, *v) for g, v in self.key_in.items() if g}
        Xw = [[self.db_words[b * A + a] for a in range(A)] for b in range(len(self.db_words) // A)]
        return Q.query_circuit(P, Xw, DELTA, W, C, T, H, rlk, gks, sign_degree=self.plan.sign_degree,
                               sign_coeffs=self.plan.sign_coeffs)

    def close(self):
        X = self.X
        for h in self.regs + self.pts:
            X.pfx_ct_destroy(h)
        for k in self.gks + [self.rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(self.sk)
        X.pfx_stream_destroy(self.ctx, self.stream)
        X.pfx_ctx_destroy(self.ctx)


def test_query_words_match_oracle_eager_and_graph(X):
    S = Setup(X, 12, 2, 31, with_oracle=True)
    try:
        want = S.oracle_out()
        out = S.run(graph=False)
        got = X.pfx_ct_export(S.ctx, out, S.N)
        assert got.shape == want.c.shape
        assert np.array_equal(got, want.c)
        assert X.pfx_ct_info(out).scale == want.scale
        # graph: captured once, replayed; eager runs in between; every replay checked
        for rep in range(3):
            out = S.run(graph=True)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), rep
            out = S.run(graph=False)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), rep
        step, count = Q.fp64_query(S.x, *S.params)
        assert abs(S.count(out)[0] - count) < 0.25
    finally:
        S.close()


def test_query_on_lanes_matches_oracle(X):
    # parallel plan (one lane per record block, fork/join), eager and one
    # captured multi-stream graph, replays checked between eager runs
    S = Setup(X, 12, 3, 37, with_oracle=True, parallel=True)
    try:
        want = S.oracle_out()
        for graph, lanes in ((False, True), (True, True), (False, False), (True, True), (False, True), (True, True)):
            out = S.run(graph=graph, lanes=lanes)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), (graph, lanes)
            assert X.pfx_ct_info(out).scale == want.scale
    finally:
        S.close()


@pytest.mark.parametrize("plan_kw", [dict(interleave=True), dict(parallel=True, lanes=2, interleave=True)],
                         ids=["interleave", "lanes2-interleave"])
def test_interleaved_query_matches_oracle(X, plan_kw):
    # the blocks' products run as batched key switches (3 blocks: runs of 3,
    # or of 2 and 1 on two lanes), eagerly and from replayed graphs
    S = Setup(X, 12, 3, 47, with_oracle=True, **plan_kw)
    try:
        want = S.oracle_out()
        for graph, lanes in ((False, False), (True, False), (False, True), (True, True), (True, False),
                             (False, False), (True, True)):
            out = S.run(graph=graph, lanes=lanes)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), (graph, lanes)
            assert X.pfx_ct_info(out).scale == want.scale
    finally:
        S.close()


def test_lane_markers_with_cross_lane_dependency_are_rejected(X):
    S = Setup(X, 12, 1, 39)
    try:
        w0, t0, t1 = 0, S.plan.n_inputs, S.plan.n_inputs + 1
        bad = [(X.OP_LANE, 0, 0, -1, 0, 0.0), (X.OP_MUL_PLAIN, t0, w0, 0, 0, 0.0),
               (X.OP_LANE, 0, 0, -1, 1, 0.0), (X.OP_ADD, t1, t0, t0, 0, 0.0)]
        with pytest.raises(X.PfxError) as e:
            X.pfx_run_circuit(S.ctx, bad, S.regs, S.plan.n_inputs, S.pts, S.rlk, S.gks, X.RUN_LANES, S.stream)
        assert e.value.status == X.PFX_EINVAL
        good = bad[:2] + [(X.OP_LANE, 0, 0, -1, -1, 0.0)] + bad[3:]      # join first: fine
        X.pfx_run_circuit(S.ctx, good, S.regs, S.plan.n_inputs, S.pts, S.rlk, S.gks, X.RUN_LANES, S.stream)
        X.pfx_run_circuit(S.ctx, good, S.regs, S.plan.n_inputs, S.pts, S.rlk, S.gks, X.RUN_EAGER, S.stream)
        X.pfx_sync(S.ctx, S.stream)
    finally:
        S.close()


@pytest.mark.parametrize("degree", [3, 15])
def test_query_degrees_match_oracle(X, degree):
    S = Setup(X, 12, 1, 33 + degree, with_oracle=True, degree=degree)
    try:
        want = S.oracle_out()
        for graph in (False, True, True):
            out = S.run(graph=graph)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), graph
        assert X.pfx_ct_info(out).scale == want.scale
    finally:
        S.close()


def test_full_size_query_count(X):
    # 2^17 records x 8 attributes at N = 2^16 (4 blocks of 2^15 slots)
    S = Setup(X, 16, 4, 41, parallel=True)
    try:
        ref = X.pfx_ct_export(S.ctx, S.run(graph=False), S.N)
        out = S.run(graph=True, lanes=True)
        assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), ref)
        from paper_2412_13269_amd.query import QueryPlan
        for kw in (dict(interleave=True), dict(parallel=True, lanes=2, interleave=True)):
            S.use_plan(QueryPlan(4, 8, 7, 3, 15, **kw))
            for graph in (False, True):
                out = S.run(graph=graph, lanes=kw.get("parallel", False))
                assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), ref), (kw, graph)
        got = S.count(out)
        step, count = Q.fp64_query(S.x, *S.params)
        assert abs(got[0] - count) < 0.25
        assert np.max(np.abs(got - got[0])) < 1e-3
    finally:
        S.close()


def test_full_size_query_exact_count_on_gap_data(X):
    S = Setup(X, 16, 4, 43, gap=0.4)
    try:
        got = S.count(S.run(graph=False))
        step, count = Q.fp64_query(S.x, *S.params)
        exact = int(np.sum(step > 0.5))
        assert int(round(got[0])) == exact
    finally:
        S.close()


def test_elementwise_runs_match_single_calls(X):
    """Runs of independent elementwise ops (issued by the executor as collected
    launches) give the words of the same ops called one at a time."""
    logn, L = 12, 6
    prm = X.make_params(logn, QB[:L], PB, ALPHA, ML)
    ctx = X.pfx_ctx_create(prm, 0)
    N = 1 << logn
    q, _, _ = X.pfx_ctx_moduli(ctx, L, len(PB))
    q = [int(v) for v in q]
    handles = []
    try:
        ins = []
        for i in range(4):                       # two ciphertexts at L limbs, two at L - 1
            lv = L if i < 2 else L - 1
            h = X.pfx_ct_create(ctx, L, 1)
            X.pfx_ct_import(ctx, I.uniform_residues(q[:lv], N, 70 + i, lead=(2,)), DELTA, h)
            ins.append(h)
        pts = []
        for i in range(2):
            pts.append(X.pfx_pt_import(ctx, I.uniform_residues(q, N, 80 + i), DELTA))
        handles += ins + pts
        R = 4                                    # work registers 4..9 (degree 2 for 7..9)
        codes = [                                # in an order that keeps the scales compatible
            (X.OP_COPY, 0, 0.0), (X.OP_ADD, 1, 0.0), (X.OP_SUB, 1, 0.0), (X.OP_MUL_INT, -35, 0.0),
            (X.OP_MUL_INT_ACC, 21, 0.0), (X.OP_ADD_CONST, 0, 0.5), (X.OP_MUL_CONST, 0, 0.25),
            (X.OP_SCALE_MUL, 0, 2.0), (X.OP_MUL_PLAIN, 1, 0.0), (X.OP_MUL_PLAIN_ACC, 0, 0.0),
            (X.OP_ADD_PLAIN, 0, 0.0),
        ]
        ops = []
        for code, k, value in codes:             # one run of 3 per code, registers 4, 5, 6
            for j in range(3):
                b = (j + 1) % 2 if code in (X.OP_MUL_PLAIN, X.OP_ADD_PLAIN, X.OP_MUL_PLAIN_ACC) else (j + 1) % 4
                src = j if code in (X.OP_COPY,) else R + j
                if code in (X.OP_ADD, X.OP_SUB, X.OP_MUL_PLAIN, X.OP_ADD_PLAIN, X.OP_MUL_INT):
                    src = j % 4
                kk = k if code in (X.OP_MUL_INT, X.OP_MUL_INT_ACC) else 0
                if code in (X.OP_MUL_INT_ACC, X.OP_MUL_PLAIN_ACC):
                    ops.append((code, R + j, j + 1, b, kk, value))
                else:
                    ops.append((code, R + j, src, b, kk, value))
        for j in range(3):                       # tensor products and accumulation into 7..9
            ops.append((X.OP_MUL, 7 + j, j, (j + 1) % 4, 0, 0.0))
        for j in range(3):
            ops.append((X.OP_MUL_ACC, 7 + j, (j + 2) % 4, j, 0, 0.0))
        degs = [1] * 7 + [2] * 3
        regs = ins + [X.pfx_ct_create(ctx, L, degs[i]) for i in range(4, 10)]
        handles += regs[4:]
        X.pfx_run_circuit(ctx, ops, regs, 4, pts, None, [], X.RUN_EAGER, None)
        got = [X.pfx_ct_export(ctx, regs[i], N) for i in range(4, 10)]
        # the same ops one at a time
        ref = ins + [X.pfx_ct_create(ctx, L, degs[i]) for i in range(4, 10)]
        handles += ref[4:]
        for code, dst, a, b, k, value in ops:
            d, A = ref[dst], ref[a]
            if code == X.OP_COPY:
                X.pfx_ct_copy(ctx, A, d)
            elif code == X.OP_ADD:
                X.pfx_add(ctx, A, ref[b], d)
            elif code == X.OP_SUB:
                X.pfx_sub(ctx, A, ref[b], d)
            elif code == X.OP_MUL_PLAIN:
                X.pfx_mul_plain(ctx, A, pts[b], d)
            elif code == X.OP_ADD_PLAIN:
                X.pfx_add_plain(ctx, A, pts[b], d)
            elif code == X.OP_MUL_INT:
                X.pfx_mul_int(ctx, A, k, d)
            elif code == X.OP_MUL_INT_ACC:
                X.pfx_mul_int_acc(ctx, A, k, d)
            elif code == X.OP_MUL_PLAIN_ACC:
                X.pfx_mul_plain_acc(ctx, A, pts[b], d)
            elif code == X.OP_ADD_CONST:
                X.pfx_add_const(ctx, A, value, d)
            elif code == X.OP_MUL_CONST:
                X.pfx_mul_const(ctx, A, value, 0.0, d)
            elif code == X.OP_SCALE_MUL:
                sc = X.pfx_ct_info(A).scale * value
                X.pfx_ct_copy(ctx, A, d)
                X.pfx_ct_set_scale(d, sc)
            elif code == X.OP_MUL:
                X.pfx_mul(ctx, A, ref[b], d)
            elif code == X.OP_MUL_ACC:
                X.pfx_mul_acc(ctx, A, ref[b], d)
        for i in range(4, 10):
            assert np.array_equal(X.pfx_ct_export(ctx, ref[i], N), got[i - 4]), i
            assert X.pfx_ct_info(ref[i]).scale == X.pfx_ct_info(regs[i]).scale, i
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        X.pfx_ctx_destroy(ctx)


@pytest.mark.parametrize("degree", [7, 15])
def test_degree_15_sign_stages_match_oracle(X, degree):
    # the paper's first-threshold degrees (15, 15, 15): three stages of depth 5
    S = Setup(X, 12, 2, 61 + degree, with_oracle=True, degree=degree, sign_degree=15, interleave=True)
    try:
        want = S.oracle_out()
        for graph in (False, True, True):
            out = S.run(graph=graph)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), graph
        assert X.pfx_ct_info(out).scale == want.scale
        step, count = Q.fp64_query(S.x, *S.params, sign_degree=15)
        assert abs(S.count(out)[0] - count) < 0.25
    finally:
        S.close()


def _threshold1():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_minimax.json")))
    return g["threshold1"]["stages"]


@pytest.mark.parametrize("plan_kw", [dict(), dict(interleave=True)], ids=["plain", "interleave"])
def test_minimax_thresholds_match_oracle(X, plan_kw):
    # Tab. 2's first threshold (three minimax stages of degree 15): the
    # constants of every term at the sum's scale, one rescale per sum (MUL_CONST_LIKE)
    sc = _threshold1()
    S = Setup(X, 12, 2, 71, with_oracle=True, sign_coeffs=sc, **plan_kw)
    try:
        want = S.oracle_out()
        for graph in (False, True, False, True):
            out = S.run(graph=graph)
            assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), want.c), graph
            assert X.pfx_ct_info(out).scale == want.scale
        step, count = Q.fp64_query(S.x, *S.params, sign_coeffs=sc)
        assert abs(S.count(out)[0] - count) < 0.25
    finally:
        S.close()


def test_full_size_minimax_query_exact_count_at_a_small_margin(X):
    # 2^17 records at N = 2^16 whose threshold inputs keep |u| >= 2^-7: the
    # minimax thresholds count them exactly (three f7 stages do not at this margin)
    sc = _threshold1()
    S = Setup(X, 16, 4, 73, gap=2.0 ** -7, sign_coeffs=sc, parallel=True)
    try:
        ref = X.pfx_ct_export(S.ctx, S.run(graph=False), S.N)
        out = S.run(graph=True, lanes=True)
        assert np.array_equal(X.pfx_ct_export(S.ctx, out, S.N), ref)
        got = S.count(out)
        step, count = Q.fp64_query(S.x, *S.params, sign_coeffs=sc)
        exact = int(np.sum(step > 0.5))
        assert abs(got[0] - count) < 0.25
        assert int(round(got[0])) == exact
        assert np.max(np.abs(got - got[0])) < 1e-3
    finally:
        S.close()


def test_global_threshold_matches_oracle(X):
    # Threshold2 (Tab. 2, six minimax stages of degree 15 by our design, one
    # more than the paper's five) on a fresh 34-limb ciphertext of counts, as
    # after a bootstrapping: word for word, eagerly and from a replayed graph
    import json
    import os
    from paper_2412_13269_amd.query import GlobalThresholdPlan
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_minimax.json")))
    sc = g["threshold2"]["stages"]
    logn, qb = 12, [50] + [45] * 33
    N, n, t1, inv_p = 1 << logn, 1 << (logn - 1), 70000.5, 2.0 ** -17
    P = O.Params(logn, qb, PB, alpha=ALPHA, mod_log2=ML)
    ctx = X.pfx_ctx_create(X.make_params(logn, qb, PB, ALPHA, ML), 0)
    handles, keys, sks = [], [], []
    try:
        q, p, _ = X.pfx_ctx_moduli(ctx, len(qb), len(PB))
        assert [int(v) for v in q] == P.q
        s = I.ternary_secret(N, 192, 81)
        sk = X.pfx_sk_create(ctx, s)
        sks.append(sk)
        ext = P.ext_mods(P.L)
        k_a, k_e = I.uniform_residues(ext, N, 82, lead=(P.beta,)), I.gaussian_error((P.beta, N), 83)
        rlk = X.pfx_swk_create(ctx, sk, 0, k_a, k_e)
        keys.append(rlk)
        rng = np.random.default_rng(84)
        counts = np.concatenate([np.arange(69990, 70011), rng.integers(0, 1 << 17, n - 21)]).astype(np.float64)
        plan = GlobalThresholdPlan(sc, inv_p)
        regs = [X.pfx_ct_create(ctx, len(qb), 1) for _ in range(plan.n_regs)]
        handles += regs
        o_in = []
        for i, (z, sd) in enumerate(((counts, 85), (np.full(n, t1), 87))):
            m = O.encode(P, z, DELTA, P.L)
            a, e = I.uniform_residues(P.q, N, sd), I.gaussian_error(N, sd + 1)
            pt = X.pfx_pt_import(ctx, m, DELTA)
            X.pfx_encrypt(ctx, sk, pt, a, e, regs[i])
            X.pfx_ct_destroy(pt)
            o_in.append(O.encrypt(P, s, m, a, e, DELTA))
        want = Q.global_threshold(P, o_in[0], o_in[1], inv_p, sc, O.relin_key(P, s, k_a, k_e))
        st = X.pfx_stream_create(ctx)
        try:
            for graph in (False, True, False, True):
                X.pfx_run_circuit(ctx, plan.ops, regs, plan.n_inputs, [], rlk, [],
                                  X.RUN_GRAPH if graph else X.RUN_EAGER, st)
                X.pfx_sync(ctx, st)
                out = regs[plan.out]
                assert np.array_equal(X.pfx_ct_export(ctx, out, N), want.c), graph
                assert X.pfx_ct_info(out).scale == want.scale
        finally:
            X.pfx_stream_destroy(ctx, st)
        m = X.pfx_decrypt(ctx, sk, out)
        got = X.pfx_decode(ctx, m, n).real
        X.pfx_ct_destroy(m)
        far = np.abs(counts - t1) >= 2
        assert np.max(np.abs(got - (counts > t1))[far]) <= 2.0 ** -20
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in keys:
            X.pfx_swk_destroy(k)
        for k in sks:
            X.pfx_sk_destroy(k)
        X.pfx_ctx_destroy(ctx)
