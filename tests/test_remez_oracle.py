"""Pins of the oracle's composite minimax sign design (oracle/remez.py)
against the minimax theory and the paper's precision claims (Tab. 2): the
degree-1 closed form, equioscillation of the Remez solution, local
optimality under perturbation, the first threshold's 2^-12 on
[2^-8, 1] with degrees [15, 15, 15], stages bounded in [-1, 1], and the
stored coefficients (tests/golden/sign_minimax.json) reproduced."""
import json
import os

import numpy as np
import pytest

from oracle import remez as R

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_minimax.json")


@pytest.mark.parametrize("tau", [0.5, 0.25, 2.0 ** -8])
def test_degree_one_closed_form(tau):
    # best c x for 1 on [tau, 1]: equal error at both ends, c = 2 / (1 + tau)
    c, e, _ = R.remez_sign_stage(1, tau)
    assert c[0] == pytest.approx(2.0 / (1.0 + tau), rel=1e-12)
    assert e == pytest.approx((1.0 - tau) / (1.0 + tau), rel=1e-9)


@pytest.mark.parametrize("degree,tau", [(15, 2.0 ** -8), (7, 0.1), (15, 0.3)])
def test_equioscillation(degree, tau):
    c, e, ref = R.remez_sign_stage(degree, tau)
    n = (degree - 1) // 2
    assert len(ref) == n + 2
    err = 1.0 - R.eval_stage(c, ref)
    assert np.all(np.sign(err[1:]) == -np.sign(err[:-1]))          # alternating
    assert np.max(np.abs(np.abs(err) - e)) <= 1e-6 * e               # equal ripple = the max error
    assert ref[0] == pytest.approx(tau) and ref[-1] == pytest.approx(1.0)


def test_local_optimality():
    c, e, _ = R.remez_sign_stage(15, 2.0 ** -6)
    xs = np.linspace(2.0 ** -6, 1.0, 50001)
    rng = np.random.default_rng(3)
    for _ in range(40):
        d = c * (1.0 + 1e-4 * rng.standard_normal(c.shape))
        assert np.max(np.abs(1.0 - R.eval_stage(d, xs))) >= e * (1.0 - 1e-7)


def test_first_threshold_meets_the_papers_precision():
    cs, es, taus = R.composite_sign(8, degree=15, stages=3)
    xs = np.concatenate([np.linspace(2.0 ** -8, 1.0, 400001), np.geomspace(2.0 ** -8, 1.0, 20001)])
    f = R.eval_composite(cs, xs)
    assert np.max(np.abs(f - 1.0)) <= 2.0 ** -12                      # Tab. 2: alpha = 8, beta = 12
    assert np.allclose(R.eval_composite(cs, -xs), -f)                 # odd: the negative side alike
    assert es[-1] <= 2.0 ** -12 and taus[0] == 2.0 ** -8


def test_stages_stay_in_the_unit_interval():
    cs, es, taus = R.composite_sign(16, degree=15, stages=6)
    xs = np.linspace(0.0, 1.0, 200001)
    for c, e, t in zip(cs[:-1], es[:-1], taus[:-1]):
        v = R.eval_stage(c, xs)
        assert np.max(np.abs(v)) <= 1.0 + 1e-9
        on = R.eval_stage(c, np.linspace(t, 1.0, 20001))
        assert np.min(on) >= (1.0 - e) / (1.0 + e) - 1e-9
    full = R.eval_composite(cs, np.linspace(2.0 ** -16, 1.0, 200001))
    assert np.max(np.abs(full - 1.0)) <= 2.0 ** -20                   # six stages reach beta = 20


def test_stored_coefficients_are_the_oracle_design():
    g = json.load(open(GOLD))
    for key, alpha, stages in (("threshold1", 8, 3), ("threshold2", 16, 6)):
        cs, es, _ = R.composite_sign(alpha, degree=15, stages=stages)
        assert g[key]["alpha"] == alpha and len(g[key]["stages"]) == stages
        for want, got in zip(cs, g[key]["stages"]):
            assert np.array_equal(np.asarray(got), want)
