"""Pins of the lookup-table evaluation and ring-repacking oracle (CPU only).

Each pin checks the oracle against something other than itself: the monomial
product against a schoolbook negacyclic product with X^k over Python
integers; the lookup identity (Sec. 3.4: the constant coefficient of
X^i * u_f is f(i)) after decryption; Lemma 1 (the repacked ciphertext decrypts
to sum_i m_i[0] X^i) on tiny rings, with N inputs and with fewer."""
import numpy as np
import pytest

from oracle import ckks as O
from oracle import repack as R
from paper_2412_13269_amd import inputs as I
from tests.test_oracle_pins import schoolbook_negacyclic

DELTA = 2.0 ** 30


def params(logn=5):
    return O.Params(logn, [50, 50], [50], alpha=1, mod_log2=logn + 1)


def keys(P, s, seed):
    ext = P.ext_mods(P.L)
    out = {}
    for i in range(P.logn):
        g = R.repack_galois(P, i)
        a = I.uniform_residues(ext, P.N, seed + 2 * i, lead=(P.beta,))
        e = I.gaussian_error((P.beta, P.N), seed + 2 * i + 1)
        out[g] = O.galois_key(P, s, g, a, e)
    return out


def enc_poly(P, s, coeffs, seed):
    m = O.from_ints(np.asarray(coeffs, dtype=np.int64), P.mods(P.L))
    return O.encrypt(P, s, m, I.uniform_residues(P.q, P.N, seed), I.gaussian_error(P.N, seed + 1), DELTA)


@pytest.mark.parametrize("k", [0, 1, 7, 31, 32, 33, 50, 63])
def test_monomial_is_the_negacyclic_product_with_x_to_the_k(k):
    P = params()
    a = I.uniform_residues(P.q, P.N, 3)
    got = R.monomial(a, k, P.q, P.N)
    for r, q in enumerate(P.q):
        xk = [0] * P.N
        kk = k % (2 * P.N)
        xk[kk % P.N] = (q - 1) if kk >= P.N else 1          # X^k = -X^(k-N) for N <= k < 2N
        assert [int(v) for v in got[r]] == schoolbook_negacyclic(a[r], xk, q), (k, r)


def test_lookup_constant_coefficient_is_f_of_the_point():
    P = params()
    s = I.ternary_secret(P.N, None, 11)
    f = I.uniform_slots(P.N, 12)
    U = enc_poly(P, s, R.lut_poly(f, DELTA), 13)
    for i, ct in zip(range(P.N), R.evaluate(P, U, range(P.N))):
        got = R.packed_values(P, s, ct, 1)[0]
        assert abs(got - f[i]) < 2 ** -20, i


@pytest.mark.parametrize("n", [32, 5])
def test_repack_decrypts_to_the_constant_coefficients(n):
    # Lemma 1: repack(c_0 .. c_{n-1}) encrypts sum_i m_i[0] X^i
    P = params()
    s = I.ternary_secret(P.N, None, 21)
    gks = keys(P, s, 300)
    rng = np.random.default_rng(22)
    ms = [rng.integers(-2 ** 29, 2 ** 29, size=P.N) for _ in range(n)]
    cts = [enc_poly(P, s, m, 400 + 2 * i) for i, m in enumerate(ms)]
    out = R.repack(P, cts, gks)
    got = R.packed_values(P, s, out, P.N)
    want = np.zeros(P.N)
    want[:n] = [m[0] / DELTA for m in ms]
    assert np.max(np.abs(got - want)) < 2 ** -16


def test_lookup_then_repack_gives_the_table_at_the_points():
    P = params(6)
    s = I.ternary_secret(P.N, None, 31)
    gks = keys(P, s, 500)
    f = I.uniform_slots(P.N, 32)
    U = enc_poly(P, s, R.lut_poly(f, DELTA), 33)
    points = np.random.default_rng(34).integers(0, P.N, size=P.N)
    out = R.repack(P, R.evaluate(P, U, points), gks)
    got = R.packed_values(P, s, out, P.N)
    assert np.max(np.abs(got - f[points])) < 2 ** -16


def test_score_constant_coefficient_is_the_sum_of_the_tables_at_the_points():
    # Sec. 4.2: record r = sum_l X^(k_rl) Enc(u_(f_l)) has f_0(k_r0) + ... in coefficient 0
    P = params()
    s = I.ternary_secret(P.N, None, 41)
    fs = [I.uniform_slots(P.N, 42 + l) for l in range(3)]
    Us = [enc_poly(P, s, R.lut_poly(f, DELTA), 50 + 2 * l) for l, f in enumerate(fs)]
    exps = np.random.default_rng(43).integers(0, P.N, size=(6, 3))
    for row, ct in zip(exps, R.score_records(P, Us, exps)):
        got = R.packed_values(P, s, ct, 1)[0]
        assert abs(got - sum(f[k] for f, k in zip(fs, row))) < 2 ** -18, row


def test_grouped_repack_packs_each_group():
    # two groups at N = 32: 40 records -> 32 + 8 (zero padded)
    P = params()
    s = I.ternary_secret(P.N, None, 61)
    gks = keys(P, s, 700)
    f = I.uniform_slots(P.N, 62)
    U = enc_poly(P, s, R.lut_poly(f, DELTA), 63)
    exps = np.random.default_rng(64).integers(0, P.N, size=(40, 1))
    outs = R.repack_groups(P, R.score_records(P, [U], exps), gks)
    assert len(outs) == 2
    got = np.concatenate([R.packed_values(P, s, o, P.N) for o in outs])
    want = np.zeros(2 * P.N)
    want[:40] = f[exps[:, 0]]
    assert np.max(np.abs(got - want)) < 2 ** -16


# ---- the library's op list (paper_2412_13269_amd/repack.py), run on plaintexts
def _run_plan_on_plaintexts(plan, inputs, q, N):
    """Registers hold integer polynomials mod q; the automorphism is the exact
    map X -> X^g, so Lemma 1 holds without noise."""
    from paper_2412_13269_amd import pfx as X
    reg = {i: np.asarray(v, dtype=np.uint64) for i, v in enumerate(inputs)}
    ninv = pow(N, -1, q)
    for code, dst, a, b, k, value in plan.ops:
        A = reg[a]
        if code == X.OP_INV_N:
            r = O.smul(A[None, :], [ninv], [q])[0]
        elif code == X.OP_MONO:
            r = R.monomial(A[None, :], int(k), [q], N)[0]
        elif code == X.OP_SUB:
            r = O.sub(A[None, :], reg[b][None, :], [q])[0]
        elif code == X.OP_ADD:
            r = O.add(A[None, :], reg[b][None, :], [q])[0]
        elif code == X.OP_GALOIS:
            r = O.automorphism(A[None, :], int(k), [q], int(np.log2(N)))[0]
        else:
            raise AssertionError(f"op {code} not in a repacking plan")
        assert dst >= plan.n_inputs
        reg[dst] = r
    return reg[plan.out]


@pytest.mark.parametrize("logn,n", [(5, 32), (5, 7), (6, 64), (6, 1), (6, 33)])
def test_repack_plan_packs_the_constant_coefficients(logn, n):
    from paper_2412_13269_amd.repack import RepackPlan, repack_keys_needed
    N, q = 1 << logn, params(logn).q[0]
    rng = np.random.default_rng(logn * 100 + n)
    ms = [rng.integers(0, q, size=N, dtype=np.uint64) for _ in range(n)]
    plan = RepackPlan(logn, n)
    assert {o[4] for o in plan.ops if o[0] == 22} <= set(repack_keys_needed(logn))
    got = _run_plan_on_plaintexts(plan, ms, q, N)
    want = np.zeros(N, dtype=np.uint64)
    want[:n] = [m[0] for m in ms]
    assert np.array_equal(got, want)


def test_lookup_plan_reads_the_table_at_the_points():
    from paper_2412_13269_amd.repack import RepackPlan
    logn = 6
    N, q = 1 << logn, params(logn).q[0]
    rng = np.random.default_rng(7)
    table = rng.integers(0, q, size=N)
    u = np.empty(N, dtype=np.uint64)                 # u_f = f(0) - sum_k f(N - k) X^k, mod q
    u[0] = table[0]
    u[1:] = (q - table[N - np.arange(1, N)]) % q
    points = rng.integers(0, N, size=N)
    plan = RepackPlan(logn, N, points=list(points))
    got = _run_plan_on_plaintexts(plan, [u], q, N)
    assert np.array_equal(got, table[points].astype(np.uint64))
