"""Host-side check of the Half-BTS op list (no GPU): run through a slot-value
interpreter on complex slots (conjugation for the Galois element 2N - 1, X^k
for k a multiple of N/2 multiplies every slot by i^(2k/N)), it takes
CoeffsToSlots's output w/2 to EvalMod(Re w) + i EvalMod(Im w), the oracle's
FP64 EvalMod steps on each part; EvalMod's two lanes pair every HMult + relin
with its twin."""
import numpy as np
import pytest

from oracle import evalmod as E
from paper_2412_13269_amd import pfx as X
from paper_2412_13269_amd.boot import HalfBootPlan
from tests.test_evalmod_oracle import coeffs


def interpret(plan, N, z0):
    reg = {0: np.asarray(z0, dtype=np.complex128)}
    for code, dst, a, b, k, value in plan.ops:
        A = reg[a]
        if code == X.OP_ADD:
            r = A + reg[b]
        elif code == X.OP_SUB:
            r = A - reg[b]
        elif code == X.OP_MUL_RELIN:
            r = A * reg[b]
        elif code == X.OP_RESCALE:
            r = A
        elif code == X.OP_MUL_INT:
            r = A * k
        elif code == X.OP_ADD_CONST:
            r = A + value
        elif code in (X.OP_MUL_CONST, X.OP_MUL_CONST_TO, X.OP_MUL_CONST_LIKE):
            assert code == X.OP_MUL_CONST or b in reg
            r = A * value
        elif code == X.OP_GALOIS:
            assert k == 2 * N - 1
            r = np.conj(A)
        elif code == X.OP_MONO:
            assert k % (N // 2) == 0
            r = A * 1j ** (k // (N // 2))
        else:
            raise AssertionError(f"op {code} not used by Half-BTS")
        assert dst >= plan.n_inputs
        reg[dst] = r
    return reg[plan.out]


def test_plan_computes_evalmod_of_both_parts():
    N, K, r, f = 256, 8.0, 3, 1024.0
    cs = coeffs(24, K, r)
    plan = HalfBootPlan(N, cs, r, K, f)
    rng = np.random.default_rng(3)
    w = (rng.integers(-7, 8, size=N // 2) + rng.uniform(-0.01, 0.01, size=N // 2)
         + 1j * (rng.integers(-7, 8, size=N // 2) + rng.uniform(-0.01, 0.01, size=N // 2)))
    got = interpret(plan, N, w / 2)
    want = E.evalmod_fp64(w.real, cs, r, K, f) + 1j * E.evalmod_fp64(w.imag, cs, r, K, f)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-9)
    assert plan.depth == 1 + plan.evalmod.depth


def test_evalmod_lanes_pair_the_products():
    plan = HalfBootPlan(256, coeffs(24, 8.0, 3), 3, 8.0)
    ops = plan.ops
    mr = [i for i, o in enumerate(ops) if o[0] == X.OP_MUL_RELIN]
    assert len(mr) % 2 == 0
    for i, j in zip(mr[::2], mr[1::2]):          # twins: adjacent, independent
        assert j == i + 1
        a, b = ops[i], ops[j]
        assert a[1] not in (b[2], b[3]) and b[1] not in (a[2], a[3]) and a[1] != b[1]


def test_c2s_half_diagonals_are_half_the_oracle_matrix_diagonals():
    from oracle import boot as B
    from oracle import ckks as O
    from paper_2412_13269_amd.boot import c2s_half_diagonals
    P = O.Params(7, [50, 45], [50], alpha=1, mod_log2=17)
    got = c2s_half_diagonals(P.N)
    want = B.diagonals(B.c2s_matrix(P))
    assert len(got) == len(want) == P.N // 2
    assert max(np.max(np.abs(g - w / 2)) for g, w in zip(got, want)) < 1e-15


@pytest.mark.parametrize("logn", [5, 8, 12])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_factorised_c2s_stages_equal_the_oracle(logn, levels):
    # the library's stage diagonals (composed as diagonal vectors) against the
    # oracle's (products of sparse matrices): same steps, same values
    from oracle import boot as B
    from oracle import ckks as O
    from paper_2412_13269_amd import boot as HB
    P = O.Params(logn, [50, 45], [50], alpha=1, mod_log2=17)
    mine = HB.c2s_factor_stages(P.N, levels, 0.5)
    ref = [B.sparse_diagonals(M) for M in B.c2s_factor_matrices(P, levels, 0.5)]
    assert len(mine) == len(ref) <= levels
    for (s1, d1), (s2, d2) in zip(mine, ref):
        assert s1 == s2
        assert max(np.max(np.abs(x - y)) for x, y in zip(d1, d2)) < 1e-12


def test_bsgs_steps_cover_every_diagonal():
    from paper_2412_13269_amd import boot as HB
    N = 1 << 16
    for steps, _ in HB.c2s_factor_stages(N, 3):
        n1 = HB.bsgs_n1(steps)
        g = HB.bsgs_galois(N, steps, n1)
        for s in steps:
            for r in (s % n1, n1 * (s // n1)):
                assert r % (N // 2) == 0 or pow(5, r % (N // 2), 2 * N) in g
        assert len(g) <= 2 * int(np.sqrt(len(steps))) + 4
