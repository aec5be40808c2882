"""Composite minimax sign polynomials (the thresholds of Sec. 5.3 / Alg. 2).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.

The paper compares encrypted values by composite minimax approximations of
sign(x) (its Tab. 2: degrees [15, 15, 15] with precision parameters alpha = 8,
beta = 12 for the first threshold, five stages of degree 15 with alpha = 16,
beta = 20 for the global one: |f(x) - sign(x)| <= 2^-beta for
2^-alpha <= |x| <= 1).  It prints no coefficients.  Reading (a design of our
own, written from the minimax theory, not from the cited work): the stages
are designed one after the other.  Stage k is the odd polynomial of degree d
that is the best uniform approximation of 1 on [tau_k, 1]; writing
p(x) = x Q(x^2), that is the weighted minimax problem

    min_Q max_{y in [tau^2, 1]} sqrt(y) |1 / sqrt(y) - Q(y)|

solved by the Remez exchange (equioscillation at deg Q + 2 points).  With
error e_k the stage maps [tau_k, 1] into [1 - e_k, 1 + e_k]; every stage but
the last is divided by 1 + e_k, so its image lies in [-1, 1] and the next
stage's domain starts at tau_(k+1) = (1 - e_k) / (1 + e_k).  tau_1 = 2^-alpha.
The composite error is the last stage's e.  Coefficients are returned in the
monomial basis of x (c_1, c_3, ..., c_d).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as C
from numpy.polynomial import polynomial as Pm


def remez_sign_stage(degree: int, tau: float, iters: int = 80, grid: int = 20000):
    """Odd minimax p of `degree` for 1 on [tau, 1] (sign on the symmetric set).

    Returns (c, e, ref): c[k] the coefficient of x^(2k+1), e = max |1 - p| on
    [tau, 1], and the final reference points (in x)."""
    assert degree % 2 == 1 and 0.0 < tau < 1.0
    n = (degree - 1) // 2                              # degree of Q in y = x^2
    a, b = tau * tau, 1.0

    def y_of(t):
        return (a + b) / 2 + (b - a) / 2 * t

    ts = np.unique(np.concatenate([np.cos(np.pi * np.arange(grid) / (grid - 1)), np.linspace(-1, 1, grid)]))
    ref = np.cos(np.pi * np.arange(n + 2)[::-1] / (n + 1))
    q = np.zeros(n + 1)
    for _ in range(iters):
        y = y_of(ref)
        w, f = np.sqrt(y), 1.0 / np.sqrt(y)
        A = np.empty((n + 2, n + 2))
        for k in range(n + 1):
            A[:, k] = w * C.chebval(ref, np.eye(n + 1)[k])
        A[:, n + 1] = (-1.0) ** np.arange(n + 2)
        sol = np.linalg.solve(A, w * f)
        q, level = sol[:n + 1], abs(sol[n + 1])
        err = 1.0 - np.sqrt(y_of(ts)) * C.chebval(ts, q)
        # one extremum per run of equal sign, then the n + 2 alternating largest
        s = np.sign(err)
        cut = np.flatnonzero(np.diff(s) != 0) + 1
        idx = np.array([seg[np.argmax(np.abs(err[seg]))] for seg in np.split(np.arange(len(ts)), cut)])
        while len(idx) > n + 2:
            idx = idx[1:] if abs(err[idx[0]]) < abs(err[idx[-1]]) else idx[:-1]
        if len(idx) < n + 2:
            break
        ref = ts[idx]
        if np.max(np.abs(err)) - level <= 1e-13 * max(1.0, level):
            break
    # monomial coefficients of Q in y, then p(x) = x Q(x^2)
    qy = C.Chebyshev(q, domain=[a, b]).convert(kind=Pm.Polynomial).coef
    qy = np.concatenate([qy, np.zeros(n + 1 - len(qy))])
    xs = np.linspace(tau, 1.0, 200001)
    e = float(np.max(np.abs(1.0 - xs * Pm.polyval(xs * xs, qy))))
    return qy, e, np.sqrt(y_of(ref))


def eval_stage(c, x):
    """p(x) = sum_k c[k] x^(2k+1)."""
    x = np.asarray(x, dtype=np.float64)
    return x * Pm.polyval(x * x, np.asarray(c, dtype=np.float64))


def composite_sign(alpha: int, degree: int = 15, stages: int | None = None, beta: int | None = None,
                   max_stages: int = 12):
    """Stages of the composite approximation of sign on [2^-alpha, 1].

    With `stages` given, exactly that many; otherwise as many as it takes for
    the error to reach 2^-beta.  Returns (coeffs per stage, error per stage,
    tau per stage)."""
    assert stages is not None or beta is not None
    tau, cs, es, taus = 2.0 ** -alpha, [], [], []
    while True:
        c, e, _ = remez_sign_stage(degree, tau)
        taus.append(tau)
        es.append(e)
        done = (stages is not None and len(cs) + 1 == stages) or \
               (stages is None and (e <= 2.0 ** -beta or len(cs) + 1 == max_stages))
        if done:
            cs.append(c)
            return cs, es, taus
        cs.append(c / (1.0 + e))               # image in [-1, 1]
        tau = (1.0 - e) / (1.0 + e)


def eval_composite(stages, x):
    for c in stages:
        x = eval_stage(c, x)
    return x
