"""Writes sign_minimax.json: the composite minimax sign polynomials of the
paper's two thresholds (Tab. 2), designed by the oracle's Remez exchange
(oracle/remez.py).  These coefficients are input data of the query circuit,
shared by the oracle and the library's op list; nothing else writes them.

    python tests/golden/make_sign_minimax.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import remez as R  # noqa: E402


def design(alpha, beta, degree, stages):
    cs, es, taus = R.composite_sign(alpha, degree=degree, stages=stages)
    return {"alpha": alpha, "beta": beta, "degree": degree, "stages": [[float(v) for v in c] for c in cs],
            "stage_errors": [float(e) for e in es], "stage_domains": [float(t) for t in taus]}


def main():
    out = {
        "reading": "stage k: odd minimax of sign on [tau_k, 1] (Remez), stages but the last divided by 1 + e_k, "
                   "tau_(k+1) = (1 - e_k) / (1 + e_k), tau_1 = 2^-alpha; coefficients of x, x^3, ..., x^degree",
        # first threshold (Tab. 2): degrees [15, 15, 15], alpha = 8, beta = 12
        "threshold1": design(8, 12, 15, 3),
        # global threshold (Tab. 2: five stages of degree 15, alpha = 16, beta = 20); five stages of this
        # design reach 2^-9.5 only, six reach 2^-38
        "threshold2": design(16, 20, 15, 6),
    }
    with open(os.path.join(HERE, "sign_minimax.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
