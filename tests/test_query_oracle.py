"""The query circuit on the oracle against its FP64 definition (CPU)."""
import numpy as np

from oracle import ckks as O
from oracle import query as Q
from paper_2412_13269_amd import inputs as I


def test_f7_closed_form():
    # odd, f7(+-1) = +-1, f7'(x) = (35/16)(1 - x^2)^3 (the defining integral)
    xs = np.linspace(-1, 1, 201)
    assert np.allclose(Q.f7(-xs), -Q.f7(xs))
    assert Q.f7(1.0) == 1.0 and Q.f7(-1.0) == -1.0
    h = 1e-6
    d = (Q.f7(xs + h) - Q.f7(xs - h)) / (2 * h)
    assert np.allclose(d, 35 / 16 * (1 - xs ** 2) ** 3, atol=1e-6)
    # three stages push |x| >= 0.4 to within 1e-6 of +-1 (the step's margin)
    u = np.linspace(0.4, 1.0, 61)
    assert np.all(np.abs(Q.f7(Q.f7(Q.f7(u))) - 1.0) < 1e-6)


def spread_parameters(x, w):
    """A query whose threshold input spreads over [-0.9, 0.9]: score polynomial
    p(s) = s, threshold at the median score, eta scaling the largest gap to 0.9."""
    s = x @ w
    t = float(np.median(s))
    c = np.zeros(8)
    c[1] = 1.0
    return c, t, 0.9 / float(np.max(np.abs(s - t)))


def gap_records(x, w, c, t, eta, gap, seed):
    """Keep records whose threshold input u satisfies gap <= |u| <= 0.95,
    drawing more from the same distribution until there are len(x) of them."""
    want, A = len(x), x.shape[1]
    keep, it = [], 0
    pool = x
    while sum(len(k) for k in keep) < want:
        s = pool @ w
        u = (sum(c[k] * s ** k for k in range(len(c))) - t) * eta
        keep.append(pool[(np.abs(u) >= gap) & (np.abs(u) <= 0.95)])
        it += 1
        pool = I.synthetic_database(4 * want, A, seed + 1000 + it)
    return np.concatenate(keep)[:want]


def build(logn, n_blocks, seed, gap=None, degree=7):
    P = O.Params(logn, [50] + [45] * 23, [50] * 4, alpha=4, mod_log2=17)
    N, n = P.N, P.N // 2
    A, D, delta = 8, degree, 2.0 ** 45
    x = I.synthetic_database(n * n_blocks, A, seed)
    w, c, t, eta = I.query_parameters(A, D, seed + 1)
    if gap is not None:
        c, t, eta = spread_parameters(x, w)
        c = np.concatenate([c, np.zeros(max(0, D + 1 - len(c)))])[:D + 1]
    if gap is not None:
        x = gap_records(x, w, c, t, eta, gap, seed)
    s_ = I.ternary_secret(N, 192, seed + 2)
    ext = P.ext_mods(P.L)
    ki = lambda sd: (I.uniform_residues(ext, N, sd, lead=(P.beta,)), I.gaussian_error((P.beta, N), sd + 1))
    rlk = O.relin_key(P, s_, *ki(seed + 3))
    gks = {}
    for k in range(logn - 1):
        g = O.galois_element(P, 1 << k)
        gks[g] = O.galois_key(P, s_, g, *ki(seed + 10 + 2 * k))
    enc_seed = [seed + 1000]

    def enc(v):
        enc_seed[0] += 3
        m = O.encode(P, np.full(n, v), delta, P.L)
        return O.encrypt(P, s_, m, I.uniform_residues(P.q, N, enc_seed[0]), I.gaussian_error(N, enc_seed[0] + 1), delta)
    W = [enc(v) for v in w]
    C = [enc(v) for v in c]
    T, H = enc(t), enc(eta)
    X = [[O.encode(P, x[b * n:(b + 1) * n, a], delta, P.L) for a in range(A)] for b in range(n_blocks)]
    return P, s_, x, (w, c, t, eta), X, delta, W, C, T, H, rlk, gks


def test_constant_add_and_product_are_slotwise():
    # App. A.1: a constant is the polynomial with only coefficient 0; adding it
    # adds the value to every slot, multiplying by round(v q) scales every slot
    P = O.Params(8, [50, 45, 45], [50], alpha=1, mod_log2=17)
    n, delta = P.N // 2, 2.0 ** 45
    s = I.ternary_secret(P.N, 32, 1)
    z = I.uniform_slots(n, 2)
    ct = O.encrypt(P, s, O.encode(P, z, delta, 3), I.uniform_residues(P.q, P.N, 3), I.gaussian_error(P.N, 4), delta)
    dec = lambda c: O.decode(P, O.decrypt(P, s, c), c.scale, n)
    got = dec(Q.add_const(P, ct, 0.75))
    assert np.max(np.abs(got - (z + 0.75))) < 2 ** -30
    got = dec(O.rescale(P, Q.mul_const_next(P, ct, 1 / 16)))
    assert np.max(np.abs(got - z / 16)) < 2 ** -30


def test_query_circuit_tracks_fp64():
    P, s_, x, (w, c, t, eta), X, delta, W, C, T, H, rlk, gks = build(10, 2, 7)
    out = Q.query_circuit(P, X, delta, W, C, T, H, rlk, gks, final_limbs=P.L)
    assert out.level == P.L - 18                             # the circuit's depth
    out = Q.query_circuit(P, X, delta, W, C, T, H, rlk, gks)
    assert out.level == Q.FINAL_LIMBS                        # InnerSum on the first limbs
    got = O.decode(P, O.decrypt(P, s_, out), out.scale, P.N // 2).real
    step, count = Q.fp64_query(x, w, c, t, eta)
    assert np.max(np.abs(got - count)) < 0.25
    assert np.max(np.abs(got - got[0])) < 1e-3      # every slot holds the total


def test_query_exact_count_on_gap_data():
    P, s_, x, (w, c, t, eta), X, delta, W, C, T, H, rlk, gks = build(10, 2, 11, gap=0.4)
    out = Q.query_circuit(P, X, delta, W, C, T, H, rlk, gks)
    got = O.decode(P, O.decrypt(P, s_, out), out.scale, P.N // 2).real
    step, count = Q.fp64_query(x, w, c, t, eta)
    exact = int(np.sum(step > 0.5))
    assert abs(count - exact) < 1e-3
    assert int(round(got[0])) == exact


def test_query_circuit_degrees_3_and_15():
    for D, depth in ((3, 17), (15, 19)):
        P, s_, x, (w, c, t, eta), X, delta, W, C, T, H, rlk, gks = build(9, 1, 13, degree=D)
        out = Q.query_circuit(P, X, delta, W, C, T, H, rlk, gks, final_limbs=P.L)
        assert out.level == P.L - depth
        got = O.decode(P, O.decrypt(P, s_, out), out.scale, P.N // 2).real
        step, count = Q.fp64_query(x, w, c, t, eta)
        assert abs(got[0] - count) < 0.25, D


def test_f15_closed_form():
    # the degree-15 member of the family: odd, f(+-1) = +-1, f'(x) = (6435/2048)(1 - x^2)^7
    xs = np.linspace(-1, 1, 201)
    f = lambda v: Q.f_sign(v, 15)
    assert np.allclose(f(-xs), -f(xs))
    assert f(1.0) == 1.0 and f(-1.0) == -1.0
    h = 1e-6
    d = (f(xs + h) - f(xs - h)) / (2 * h)
    assert np.allclose(d, 6435 / 2048 * (1 - xs ** 2) ** 7, atol=1e-5)
    u = np.linspace(0.2, 1.0, 81)                    # three stages: |x| >= 0.2 to within 1e-6 of +-1
    assert np.all(np.abs(f(f(f(u))) - 1.0) < 1e-6)


def test_query_circuit_with_degree_15_sign_stages():
    P, s_, x, (w, c, t, eta), X, delta, W, C, T, H, rlk, gks = build(9, 1, 17)
    out = Q.query_circuit(P, X, delta, W, C, T, H, rlk, gks, final_limbs=P.L, sign_degree=15)
    assert out.level == P.L - 21                             # three stages of depth 5
    got = O.decode(P, O.decrypt(P, s_, out), out.scale, P.N // 2).real
    step, count = Q.fp64_query(x, w, c, t, eta, sign_degree=15)
    assert abs(got[0] - count) < 0.25


def _threshold(name):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sign_minimax.json")))
    return g[name]["stages"]


def test_minimax_stage_decrypts_to_the_polynomial():
    # one homomorphic stage against the polynomial evaluated in FP64 on the
    # decrypted input (numpy's polyval, independent of the ciphertext arithmetic)
    from oracle import remez as R
    P = O.Params(9, [50] + [45] * 7, [50] * 2, alpha=2, mod_log2=17)
    n, delta = P.N // 2, 2.0 ** 45
    s = I.ternary_secret(P.N, 64, 5)
    z = np.concatenate([np.linspace(-1.0, 1.0, n // 2), I.uniform_slots(n // 2, 6).real])
    ct = O.encrypt(P, s, O.encode(P, z, delta, P.L), I.uniform_residues(P.q, P.N, 7), I.gaussian_error(P.N, 8), delta)
    ext = P.ext_mods(P.L)
    rlk = O.relin_key(P, s, I.uniform_residues(ext, P.N, 9, lead=(P.beta,)), I.gaussian_error((P.beta, P.N), 10))
    dec = lambda c: O.decode(P, O.decrypt(P, s, c), c.scale, n).real
    z0 = dec(ct)
    for c in _threshold("threshold1"):
        out = Q.minimax_stage(P, ct, c, rlk)
        assert out.level == ct.level - 5                    # x^2, x^3/x^4, x^5/x^7/x^8, x^9..x^15, c_15 x^15
        want = R.eval_stage(c, z0)
        got = dec(out)
        # each term c_k x^k carries x^k's error (about 2^-38 here) times |c_k|
        assert np.max(np.abs(got - want)) < 2.0 ** -34 * sum(abs(v) for v in c)
    # a degree-3 stage against its closed form x (3 - x^2) / 2
    out = Q.minimax_stage(P, ct, [1.5, -0.5], rlk)
    assert out.level == ct.level - 3
    assert np.max(np.abs(dec(out) - z0 * (3 - z0 ** 2) / 2)) < 2.0 ** -34 * 2


def test_query_circuit_with_the_first_threshold():
    # Tab. 2 thresholds: three minimax stages of degree 15 replace the f_d stages
    sc = _threshold("threshold1")
    P, s_, x, (w, c, t, eta), X, delta, W, C, T, H, rlk, gks = build(9, 1, 19)
    out = Q.query_circuit(P, X, delta, W, C, T, H, rlk, gks, final_limbs=P.L, sign_coeffs=sc)
    assert out.level == P.L - 21                             # 6 + three stages of depth 5
    got = O.decode(P, O.decrypt(P, s_, out), out.scale, P.N // 2).real
    step, count = Q.fp64_query(x, w, c, t, eta, sign_coeffs=sc)
    assert abs(got[0] - count) < 0.25
    # the thresholds separate: records with |u| >= 2^-8 land within 2^-11 of 0 or 1
    s = x @ w
    u = (sum(c[k] * s ** k for k in range(len(c))) - t) * eta
    far = (np.abs(u) >= 2.0 ** -8) & (np.abs(u) <= 1.0)
    assert np.all(np.abs(step[far] - (u[far] > 0)) <= 2.0 ** -11)


def test_global_threshold_decides_counts_two_away():
    # Threshold2 (Tab. 2: alpha = 16, beta = 20) on counts up to 2^17 with
    # p = 2^17: every count at least 2 from t1 (|u| >= 2^-16) is decided
    # within 2^-20; six stages of depth 5 after the p^-1 product
    sc = _threshold("threshold2")
    P = O.Params(9, [50] + [45] * 33, [50] * 4, alpha=4, mod_log2=17)
    n, delta, t1, inv_p = P.N // 2, 2.0 ** 45, 70000.5, 2.0 ** -17
    s = I.ternary_secret(P.N, 64, 25)
    rng = np.random.default_rng(26)
    counts = np.concatenate([np.arange(69990, 70011), rng.integers(0, 1 << 17, n - 21)]).astype(np.float64)
    enc = lambda z, sd: O.encrypt(P, s, O.encode(P, z, delta, P.L), I.uniform_residues(P.q, P.N, sd),
                                  I.gaussian_error(P.N, sd + 1), delta)
    ext = P.ext_mods(P.L)
    rlk = O.relin_key(P, s, I.uniform_residues(ext, P.N, 29, lead=(P.beta,)), I.gaussian_error((P.beta, P.N), 30))
    out = Q.global_threshold(P, enc(counts, 27), enc(np.full(n, t1), 31), inv_p, sc, rlk)
    assert out.level == P.L - 31
    got = O.decode(P, O.decrypt(P, s, out), out.scale, n).real
    far = np.abs(counts - t1) >= 2
    assert far.sum() >= n - 4
    assert np.max(np.abs(got - (counts > t1))[far]) <= 2.0 ** -20
    want = Q.fp64_global_threshold(counts, t1, inv_p, sc)
    assert np.max(np.abs(got - want)[far]) <= 2.0 ** -22
