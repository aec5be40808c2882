"""Seeded synthetic inputs for the RNS-CKKS path.

This module only draws random numbers.  It holds none of the scheme's
arithmetic, so both the HIP library and the CPU oracle can take its outputs
as their inputs: the secret key, the uniform polynomials `a` and the errors
`e` that encryption and key generation consume (Sec. 2.3 of the paper
samples them; here the caller draws them and passes them in), and the slot
values and database records that the evaluation works on.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def ternary_secret(n: int, h: int | None, seed: int) -> np.ndarray:
    """Secret in {-1, 0, 1}^n.

    h = None: every coefficient uniform over {-1, 0, 1}.
    h = k: exactly k non-zero coefficients at uniformly chosen positions,
    each +1 or -1 with probability 1/2 (the paper's Sets II/III use h = 192).
    """
    g = rng(seed)
    if h is None:
        return g.integers(-1, 2, size=n, dtype=np.int64).astype(np.int8)
    s = np.zeros(n, dtype=np.int8)
    pos = g.choice(n, size=h, replace=False)
    s[pos] = np.where(g.integers(0, 2, size=h) == 1, 1, -1).astype(np.int8)
    return s


def uniform_residues(moduli, n: int, seed: int, lead: tuple = ()) -> np.ndarray:
    """Array of shape lead + (len(moduli), n); row i uniform over [0, moduli[i])."""
    g = rng(seed)
    out = np.empty(tuple(lead) + (len(moduli), n), dtype=np.uint64)
    flat = out.reshape(-1, len(moduli), n)
    for b in range(flat.shape[0]):
        for i, q in enumerate(moduli):
            flat[b, i] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def gaussian_error(shape, seed: int, sigma: float = 3.2, bound: int = 19) -> np.ndarray:
    """Rounded Gaussian of standard deviation sigma, cut at |e| <= bound."""
    g = rng(seed)
    e = np.rint(g.normal(0.0, sigma, size=shape))
    return np.clip(e, -bound, bound).astype(np.int64)


def uniform_slots(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n real slot values uniform in [lo, hi)."""
    return rng(seed).uniform(lo, hi, size=n)


def synthetic_database(records: int, attributes: int, seed: int):
    """Patient-like table: attribute a ~ Normal(mu_a, sigma_a) with
    mu_a ~ U[0.5, 1.5], sigma_a ~ U[0.25, 1.0], clipped to [0, 2) as in the
    paper's experiment, then mapped to x - 1 in [-1, 1)."""
    g = rng(seed)
    mu = g.uniform(0.5, 1.5, size=attributes)
    sd = g.uniform(0.25, 1.0, size=attributes)
    x = g.normal(mu, sd, size=(records, attributes))
    x = np.clip(x, 0.0, np.nextafter(2.0, 0.0))
    return x - 1.0


def query_parameters(attributes: int, degree: int, seed: int):
    """Encrypted query parameters of the private query: weights w ~ U[-1,1]/A,
    score-polynomial coefficients c ~ U[-1,1] scaled to sum |c_k| = 1,
    threshold t ~ U[-0.5, 0.5], normalisation eta = 1/2."""
    g = rng(seed)
    w = g.uniform(-1.0, 1.0, size=attributes) / attributes
    c = g.uniform(-1.0, 1.0, size=degree + 1)
    c = c / np.abs(c).sum()
    t = float(g.uniform(-0.5, 0.5))
    return w, c, t, 0.5
