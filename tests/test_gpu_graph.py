"""Replayed HIP graphs stay bound to the objects and scratch they were
captured with: a register destroyed and re-created (possibly at the freed
address, here with another capacity), a switching key re-made, or a stream's
scratch freed, makes the next graph-mode call capture again instead of
replaying stale device addresses; every graph-mode result equals the eager
run of the same op list, word for word, and the oracle."""
import numpy as np
import pytest

from oracle import ckks as O
from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu

LOGN, QB, PB, ALPHA, ML = 12, [50, 45, 45, 45], [50, 50], 2, 17
DELTA = 2.0 ** 45


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def test_graph_recaptured_when_objects_or_scratch_change(X):
    e0, _ = X.pfx_graph_cache_stats()
    P = O.Params(LOGN, QB, PB, alpha=ALPHA, mod_log2=ML)
    ctx = X.pfx_ctx_create(X.make_params(LOGN, QB, PB, ALPHA, ML), 0)
    N, L = P.N, P.L
    s = I.ternary_secret(N, 64, 71)
    sk = X.pfx_sk_create(ctx, s)
    ext = P.ext_mods(L)
    kin = (I.uniform_residues(ext, N, 72, lead=(P.beta,)), I.gaussian_error((P.beta, N), 73))
    rlk_o = O.relin_key(P, s, *kin)
    handles, keys = [], []
    st = X.pfx_stream_create(ctx)
    try:
        rlk = X.pfx_swk_create(ctx, sk, 0, *kin)
        keys.append(rlk)
        cts_o, ins = [], []
        for i in range(2):
            m = O.encode(P, I.uniform_slots(N // 2, 80 + i), DELTA, L)
            a, e = I.uniform_residues(P.mods(L), N, 90 + i), I.gaussian_error(N, 95 + i)
            cts_o.append(O.encrypt(P, s, m, a, e, DELTA))
            pt = X.pfx_pt_import(ctx, m, DELTA)
            h = X.pfx_ct_create(ctx, L, 1)
            X.pfx_encrypt(ctx, sk, pt, a, e, h)
            X.pfx_ct_destroy(pt)
            ins.append(h)
        handles += ins
        # r2 = r0 * r1 (relinearised), r3 = rescale(r2), r4 = r3 + r3
        ops = [(X.OP_MUL_RELIN, 2, 0, 1, 0, 0.0), (X.OP_RESCALE, 3, 2, 0, 0, 0.0), (X.OP_ADD, 4, 3, 3, 0, 0.0)]
        po = O.rescale(P, O.mul_relin(P, cts_o[0], cts_o[1], rlk_o))
        want = O.ct_add(P, po, po)

        def run(regs, key, mode):
            X.pfx_run_circuit(ctx, ops, regs, 2, [], key, [], mode, st)
            X.pfx_sync(ctx, st)
            return X.pfx_ct_export(ctx, regs[4], N, st)

        work = [X.pfx_ct_create(ctx, L, 1) for _ in range(3)]
        regs = ins + work
        assert np.array_equal(run(regs, rlk, X.RUN_EAGER), want.c)
        _, c0 = X.pfx_graph_cache_stats()
        for _ in range(3):                               # one capture, then replays
            assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 1

        # destroy a work register and make one of another capacity (degree 2:
        # its second polynomial sits elsewhere; the freed block is the likeliest
        # address for it): captured again, same words
        X.pfx_ct_destroy(work[0])
        work[0] = X.pfx_ct_create(ctx, L, 2)
        regs = ins + work
        assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 2
        work[0], old = X.pfx_ct_create(ctx, L, 1), work[0]
        X.pfx_ct_destroy(old)
        regs = ins + work
        assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 3

        # a re-made relinearisation key (same inputs, new object)
        X.pfx_swk_destroy(rlk)
        keys.remove(rlk)
        rlk = X.pfx_swk_create(ctx, sk, 0, *kin)
        keys.append(rlk)
        assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 4
        assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 4

        # another stream's scratch freed: every graph is captured again once
        other = X.pfx_stream_create(ctx)
        X.pfx_run_circuit(ctx, ops, regs, 2, [], rlk, [], X.RUN_EAGER, other)
        X.pfx_sync(ctx, other)
        X.pfx_stream_destroy(ctx, other)
        assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 5
        assert np.array_equal(run(regs, rlk, X.RUN_GRAPH), want.c)
        assert X.pfx_graph_cache_stats()[1] == c0 + 5

        # bounded: many distinct lists leave at most 64 entries
        for k in range(70):
            ops_k = ops + [(X.OP_MUL_INT, 4, 4, 0, k + 2, 0.0)]
            X.pfx_run_circuit(ctx, ops_k, regs, 2, [], rlk, [], X.RUN_GRAPH, st)
        X.pfx_sync(ctx, st)
        assert X.pfx_graph_cache_stats()[0] <= 64
        assert np.array_equal(X.pfx_ct_export(ctx, regs[4], N, st), O.ct_mul_int(P, want, 71).c)
        handles += work
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for k in keys:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(sk)
        X.pfx_stream_destroy(ctx, st)
        X.pfx_ctx_destroy(ctx)
    assert X.pfx_graph_cache_stats()[0] <= e0        # destroying the context dropped its graphs
