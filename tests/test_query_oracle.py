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
