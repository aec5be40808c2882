"""Host-side checks of the query op lists (no GPU): every plan variant
computes the query's function, and the interleaved variants put the record
blocks' HMult + relin ops side by side as runs of independent ops.

The op lists run here through a slot-value interpreter: a register holds the
slot vector its ciphertext would decrypt to (rescale and relinearisation do
not change it), so a wrong register (a temporary reused while live, a wrong
operand) changes the result, which must equal the plain FP64 query."""
import numpy as np
import pytest

from oracle import query as Q
from paper_2412_13269_amd import inputs as I
from paper_2412_13269_amd import pfx as X
from paper_2412_13269_amd.query import QueryPlan

VARIANTS = [dict(), dict(parallel=True), dict(interleave=True), dict(parallel=True, lanes=2, interleave=True),
            dict(parallel=True, lanes=3, interleave=True), dict(interleave=2), dict(interleave=3)]


def interpret(plan, inputs, pts):
    reg = {i: np.asarray(v, dtype=np.float64) for i, v in enumerate(inputs)}
    for code, dst, a, b, k, value in plan.ops:
        if code == X.OP_LANE:
            continue
        A = reg[a]
        if code == X.OP_ADD:
            r = A + reg[b]
        elif code == X.OP_SUB:
            r = A - reg[b]
        elif code == X.OP_MUL_PLAIN:
            r = A * pts[b]
        elif code in (X.OP_MUL_RELIN, X.OP_MUL):
            r = A * reg[b]
        elif code == X.OP_MUL_ACC:
            r = reg[dst] + A * reg[b]
        elif code == X.OP_MUL_PLAIN_ACC:
            r = reg[dst] + A * pts[b]
        elif code == X.OP_MUL_INT_ACC:
            r = reg[dst] + A * k
        elif code == X.OP_DROP:
            r = A
        elif code == X.OP_RELIN:
            r = A
        elif code == X.OP_RESCALE:
            r = A
        elif code == X.OP_MUL_INT:
            r = A * k
        elif code == X.OP_ADD_CONST:
            r = A + value
        elif code == X.OP_MUL_CONST:
            r = A * value
        elif code in (X.OP_MUL_CONST_TO, X.OP_MUL_CONST_LIKE):
            assert b in reg                      # the register whose scale is the target
            r = A * value
        elif code == X.OP_SCALE_MUL:
            r = A / value
        elif code == X.OP_ROTATE_SUM:
            r = np.full_like(A, A.sum())
        else:
            raise AssertionError(f"op {code} not used by the query")
        assert dst >= plan.n_inputs
        if code in (X.OP_MUL, X.OP_MUL_ACC):     # a tensor product needs a degree-2 register
            assert plan.reg_degree[dst] == 2
        reg[dst] = np.broadcast_to(r, A.shape).copy() if np.ndim(r) else r
    return reg[plan.out]


@pytest.mark.parametrize("kw", VARIANTS, ids=lambda kw: "-".join(f"{k}{v}" for k, v in kw.items()) or "plain")
@pytest.mark.parametrize("degree", [3, 7, 15])
def test_plan_computes_the_query(kw, degree):
    n, A, blocks = 64, 8, 5
    x = I.synthetic_database(n * blocks, A, 11 + degree)
    w, c, t, eta = I.query_parameters(A, degree, 12 + degree)
    plan = QueryPlan(blocks, A, degree, 3, 6, **kw)
    inputs = [np.full(n, v) for v in list(w) + list(c) + [t, eta]]
    pts = [x[b * n:(b + 1) * n, a] for b in range(blocks) for a in range(A)]
    got = interpret(plan, inputs, pts)
    _, count = Q.fp64_query(x, w, c, t, eta)
    assert np.allclose(got, count, rtol=1e-9, atol=1e-9)


def _runs(ops):
    """Maximal runs of consecutive independent HMult + relin ops (the rule the
    library's executor applies before it batches them)."""
    runs, cur = [], []
    for o in ops:
        if o[0] == X.OP_MUL_RELIN:
            dst, a, b = o[1], o[2], o[3]
            ok = dst not in (a, b) and all(dst not in (p[1], p[2], p[3]) and p[1] not in (a, b) for p in cur)
            if ok and cur:
                cur.append(o)
                continue
            if cur:
                runs.append(len(cur))
            cur = [o] if dst not in (a, b) else []
            if not cur:
                runs.append(1)
        else:
            if cur:
                runs.append(len(cur))
            cur = []
    if cur:
        runs.append(len(cur))
    return runs


def test_interleaved_plan_batches_every_product_across_blocks():
    blocks = 4
    seq = QueryPlan(blocks, 8, 7, 3, 15)
    inter = QueryPlan(blocks, 8, 7, 3, 15, interleave=True)
    two = QueryPlan(blocks, 8, 7, 3, 15, parallel=True, lanes=2, interleave=True)
    n_mr = sum(1 for o in seq.ops if o[0] == X.OP_MUL_RELIN)
    assert sorted(o[0] for o in inter.ops) == sorted(o[0] for o in seq.ops)
    assert _runs(seq.ops) == [1] * n_mr
    assert _runs(inter.ops) == [blocks] * (n_mr // blocks)
    assert _runs(two.ops) == [2] * (n_mr // 2)
    assert inter.key_switches == seq.key_switches == two.key_switches


def test_grouped_interleave_bounds_the_registers():
    seq = QueryPlan(1, 8, 7, 3, 15)
    per_block = seq.n_regs - seq.n_inputs
    for blocks in (4, 9, 16):
        g = QueryPlan(blocks, 8, 7, 3, 15, interleave=4)
        n_mr = sum(1 for o in g.ops if o[0] == X.OP_MUL_RELIN)
        assert g.n_regs - g.n_inputs <= 4 * per_block + 1
        runs = _runs(g.ops)
        assert sum(runs) == n_mr and max(runs) == 4
        assert runs.count(4) == (blocks // 4) * (n_mr // blocks)


def test_one_relinearisation_for_the_score_polynomial():
    # the D products C_k Y_k are summed at degree 2: D tensor products, one RELIN per block
    for D in (3, 7, 15):
        plan = QueryPlan(2, 8, D, 3, 15)
        codes = [o[0] for o in plan.ops]
        assert codes.count(X.OP_MUL) == 2 and codes.count(X.OP_MUL_ACC) == 2 * (D - 1)
        assert codes.count(X.OP_RELIN) == 2
        assert codes.count(X.OP_MUL_PLAIN) == 2 and codes.count(X.OP_MUL_PLAIN_ACC) == 2 * 7
        assert sum(plan.reg_degree) == plan.n_regs + 1          # one degree-2 register


@pytest.mark.parametrize("kw", VARIANTS, ids=lambda kw: "-".join(f"{k}{v}" for k, v in kw.items()) or "plain")
def test_plan_with_degree_15_sign_stages(kw):
    n, A, blocks = 64, 8, 3
    x = I.synthetic_database(n * blocks, A, 41)
    w, c, t, eta = I.query_parameters(A, 7, 42)
    plan = QueryPlan(blocks, A, 7, 3, 6, sign_degree=15, **kw)
    inputs = [np.full(n, v) for v in list(w) + list(c) + [t, eta]]
    pts = [x[b * n:(b + 1) * n, a] for b in range(blocks) for a in range(A)]
    got = interpret(plan, inputs, pts)
    _, count = Q.fp64_query(x, w, c, t, eta, sign_degree=15)
    assert np.allclose(got, count, rtol=1e-9, atol=1e-9)


def _threshold1():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_minimax.json")))
    return g["threshold1"]["stages"]


@pytest.mark.parametrize("kw", VARIANTS, ids=lambda kw: "-".join(f"{k}{v}" for k, v in kw.items()) or "plain")
def test_plan_with_minimax_thresholds(kw):
    # Tab. 2's first threshold: three minimax stages of degree 15 (designed stage by stage)
    n, A, blocks = 64, 8, 3
    x = I.synthetic_database(n * blocks, A, 51)
    w, c, t, eta = I.query_parameters(A, 7, 52)
    sc = _threshold1()
    plan = QueryPlan(blocks, A, 7, 3, 6, sign_coeffs=sc, **kw)
    inputs = [np.full(n, v) for v in list(w) + list(c) + [t, eta]]
    pts = [x[b * n:(b + 1) * n, a] for b in range(blocks) for a in range(A)]
    got = interpret(plan, inputs, pts)
    _, count = Q.fp64_query(x, w, c, t, eta, sign_coeffs=sc)
    assert np.allclose(got, count, rtol=1e-9, atol=1e-9)
    # depth: 6 for the score and the threshold input, 5 per stage
    codes = [o[0] for o in plan.ops]
    assert codes.count(X.OP_MUL_CONST_LIKE) == blocks * 3 * 7
    assert codes.count(X.OP_MUL_RELIN) == blocks * (6 + 1 + 3 * 10)
    # one rescale per product and per sum (the attribute sum, the score sum
    # and one per minimax stage)
    assert codes.count(X.OP_RESCALE) == codes.count(X.OP_MUL_RELIN) + blocks * (2 + 3)


def test_minimax_stage_of_lower_degree_skips_unused_powers():
    # a degree-7 stage needs x^2, x^3, x^4, x^5, x^7 only (no x^8)
    n, A = 64, 8
    x = I.synthetic_database(n, A, 61)
    w, c, t, eta = I.query_parameters(A, 7, 62)
    sc = [[1.5, -0.5, 0.0, 0.0]]            # x (3 - x^2) / 2, degree 7 with zero tail terms
    plan = QueryPlan(1, A, 7, 3, 6, sign_coeffs=sc)
    inputs = [np.full(n, v) for v in list(w) + list(c) + [t, eta]]
    got = interpret(plan, inputs, [x[:, a] for a in range(A)])
    _, count = Q.fp64_query(x, w, c, t, eta, sign_coeffs=sc)
    assert np.allclose(got, count, rtol=1e-9, atol=1e-9)
    codes = [o[0] for o in plan.ops]
    assert codes.count(X.OP_MUL_RELIN) == 6 + 1 + 5


def test_global_threshold_plan_computes_the_step():
    import json
    import os
    from paper_2412_13269_amd.query import GlobalThresholdPlan
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_minimax.json")))
    sc = g["threshold2"]["stages"]
    counts = np.concatenate([np.arange(69990.0, 70011.0), np.linspace(0, 1 << 17, 43)])
    plan = GlobalThresholdPlan(sc, 2.0 ** -17)
    got = interpret(plan, [counts, np.full(len(counts), 70000.5)], [])
    want = Q.fp64_global_threshold(counts, 70000.5, 2.0 ** -17, sc)
    # terms summed in another order than Horner's: equal to rounding where the
    # stages are flat (|count - t1| >= 2); the two counts beside t1 lie below
    # the design's domain, where the stages amplify rounding
    far = np.abs(counts - 70000.5) >= 2
    assert np.allclose(got[far], want[far], rtol=0, atol=1e-10)
    assert np.allclose(got[~far], want[~far], rtol=1e-3, atol=1e-6)
    assert plan.depth == 31 and plan.n_inputs == 2
    codes = [o[0] for o in plan.ops]
    assert codes.count(X.OP_MUL_RELIN) == 6 * 10 and codes.count(X.OP_MUL_CONST_LIKE) == 6 * 7
