"""Host-side check of the EvalMod op list (no GPU): run through the slot-value
interpreter of the query plans, it computes the oracle's FP64 EvalMod steps,
and its depth is the documented one."""
import math

import numpy as np
import pytest

from oracle import evalmod as E
from paper_2412_13269_amd import pfx as X
from paper_2412_13269_amd.evalmod import EvalModPlan
from tests.test_evalmod_oracle import coeffs
from tests.test_query_plan import interpret


@pytest.mark.parametrize("deg,r", [(24, 3), (17, 2), (8, 0)])
def test_plan_computes_evalmod(deg, r):
    K = 8.0
    cs = coeffs(deg, K, r)
    plan = EvalModPlan(list(cs), r, K)
    t = np.random.default_rng(deg).uniform(-K, K, size=256)
    got = interpret(plan, [t], [])
    assert np.allclose(got, E.evalmod_fp64(t, cs, r, K), rtol=1e-12, atol=1e-12)
    assert plan.depth == 1 + math.ceil(math.log2(deg)) + 1 + r + 1


def test_plan_adds_terms_at_one_scale():
    # scale and level of every register over the 50 + 45-bit chain: each
    # ADD / SUB meets its operands at one scale (to rounding), the property
    # MUL_CONST_LIKE exists for; the output lands at the depth's level, with
    # one rescale per sum
    from oracle import ckks as O
    P = O.Params(7, [50] + [45] * 13, [50] * 3, alpha=4, mod_log2=17)
    plan = EvalModPlan(list(coeffs(24, 8.0, 3)), 3, 8.0)
    reg = {0: (2.0 ** 45, P.L)}
    worst = 0.0
    for code, dst, a, b, k, value in plan.ops:
        sa, la = reg[a]
        if code in (X.OP_ADD, X.OP_SUB):
            sb, lb = reg[b]
            worst = max(worst, abs(sa / sb - 1))
            reg[dst] = (sa, min(la, lb))
        elif code == X.OP_MUL_RELIN:
            sb, lb = reg[b]
            reg[dst] = (sa * sb, min(la, lb))
        elif code == X.OP_RESCALE:
            reg[dst] = (sa / P.q[la - 1], la - 1)
        elif code == X.OP_MUL_CONST:
            reg[dst] = (sa * P.q[la - 1], la)
        elif code == X.OP_MUL_CONST_TO:
            reg[dst] = (sa * (reg[b][0] * P.q[la - 1] / sa), la)
        elif code == X.OP_MUL_CONST_LIKE:
            reg[dst] = (sa * (reg[b][0] / sa), la)
        else:
            assert code in (X.OP_ADD_CONST, X.OP_MUL_INT)
            reg[dst] = (sa, la)
    assert worst < 1e-12
    assert reg[plan.out][1] == P.L - plan.depth
    assert [c for c, *_ in plan.ops].count(X.OP_RESCALE) == 1 + 23 + 1 + 3 + 1     # T_1, products, sum, r, out
