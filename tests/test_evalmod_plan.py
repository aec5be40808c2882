"""Host-side check of the EvalMod op list (no GPU): run through the slot-value
interpreter of the query plans, it computes the oracle's FP64 EvalMod steps,
and its depth is the documented one."""
import math

import numpy as np
import pytest

from oracle import evalmod as E
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
