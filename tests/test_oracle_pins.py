"""Pins of the CPU oracle against what the mathematics fixes.

None of these re-types an oracle formula: each compares the oracle with an
independent definition (schoolbook products over Python integers, big-integer
CRT, a Lucas primality certificate, a direct evaluation of the slot
polynomial, a linear solve) or with an invariant the paper states.
"""
import cmath
import math

import numpy as np
import pytest

from oracle import ckks as O
from paper_2412_13269_amd import inputs as I


# ---------------------------------------------------------------- helpers
def schoolbook_negacyclic(a, b, q):
    """Product in Z_q[X]/(X^N + 1) over Python integers (Sec. 2.2)."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            v = int(a[i]) * int(b[j])
            if k < n:
                out[k] += v
            else:
                out[k - n] -= v
    return [x % q for x in out]


def poly_compose_power(a, g, q):
    """a(X^g) mod (X^N + 1, q) by expanding X^(i g) and folding X^N = -1 one
    power at a time (no closed-form exponent arithmetic)."""
    n = len(a)
    out = [0] * n
    for i, c in enumerate(a):
        e, sign = i * g, 1
        while e >= n:
            e -= n
            sign = -sign
        out[e] = (out[e] + sign * int(c)) % q
    return out


def factor_small(n):
    fs, d = [], 2
    while d * d <= n:
        while n % d == 0:
            fs.append(d)
            n //= d
        d += 1 if d == 2 else 2
    if n > 1:
        fs.append(n)
    return sorted(set(fs))


def lucas_certificate(q):
    """Lucas test: q is prime iff some a has order exactly q - 1 mod q.
    Needs the factorisation of q - 1 (2^m times a small cofactor)."""
    m = q - 1
    k = 0
    while m % 2 == 0:
        m //= 2
        k += 1
    primes = [2] + factor_small(m) if m > 1 else [2]
    for a in range(2, 200):
        if pow(a, q - 1, q) != 1:
            return False
        if all(pow(a, (q - 1) // r, q) != 1 for r in primes):
            return True
    return False


SMALL = O.Params(5, [50, 50, 50], [50], alpha=1, mod_log2=13)   # N = 32, three 50-bit primes and one special
SMALL4 = O.Params(4, [50, 45, 45, 45, 45], [50, 50], alpha=2, mod_log2=17)


# ---------------------------------------------------------------- primes
@pytest.mark.parametrize("P", [O.params_n12_three_50bit(), O.params_50_45_chain()], ids=["n12_3x50", "n16_l24"])
def test_primes_certified_and_ntt_friendly(P):
    allp = P.q + P.p
    assert len(set(allp)) == len(allp)
    for q in allp:
        assert q % (1 << P.mod_log2) == 1
        assert q < 2 ** 50
        assert lucas_certificate(q), q


def test_prime_rule_largest_below_and_nearest():
    P = O.params_50_45_chain()
    step = 1 << 17
    # q_0 is the largest prime below 2^50 on the 1 mod 2^17 lattice: every
    # lattice point above it is composite (a Fermat witness proves it).
    c = (1 << 50) + 1 - step
    while c > P.q[0]:
        assert pow(2, c - 1, c) != 1 or pow(3, c - 1, c) != 1
        c -= step
    # the 45-bit primes are the lattice points closest to 2^45
    far = max(abs(q - 2 ** 45) for q in P.q[1:])
    c = (1 << 45) + 1 - (far // step) * step
    while c <= (1 << 45) + 1 + far:
        if abs(c - 2 ** 45) < far and c not in P.q:
            assert pow(2, c - 1, c) != 1, c
        c += step


@pytest.mark.parametrize("P", [O.params_n12_three_50bit(), O.params_50_45_chain(), O.params_50_45_chain(logn=14)], ids=["n12_3x50", "n16_l24", "n14_l24"])
def test_psi_is_primitive_2n_root(P):
    for q, psi in zip(P.q + P.p, P.psi_q + P.psi_p):
        assert pow(psi, P.N, q) == q - 1          # order divides 2N but not N
        assert pow(psi, 2 * P.N, q) == 1


def test_five_generates_order_half_n():
    # Sec. 2.2: 5 has order N/2 mod 2N; with -1 it spans Z*_2N
    for logn in (4, 6, 12):
        n = 1 << logn
        orbit = {pow(5, j, 2 * n) for j in range(n // 2)}
        assert len(orbit) == n // 2
        assert orbit | {(-x) % (2 * n) for x in orbit} == set(range(1, 2 * n, 2))


# ---------------------------------------------------------------- NTT
@pytest.mark.parametrize("logn", [1, 2, 3, 5, 8])
def test_ntt_matches_definition(logn):
    q, psi = SMALL.q[0], O.find_psi(SMALL.q[0], 1 << logn)
    a = I.uniform_residues([q], 1 << logn, seed=logn)[0]
    fast = a.copy()
    O.lib().pfo_ntt(q, psi, logn, O._p(fast))
    slow = np.empty_like(a)
    O.lib().pfo_ntt_naive(q, psi, logn, O._p(a), O._p(slow))
    assert np.array_equal(fast, slow)
    back = fast.copy()
    O.lib().pfo_intt(q, psi, logn, O._p(back))
    assert np.array_equal(back, a)


def test_ntt_closed_forms():
    logn = 6
    n = 1 << logn
    q = SMALL.q[1]
    psi = O.find_psi(q, n)
    one = np.zeros(n, dtype=np.uint64)
    one[0] = 1
    O.lib().pfo_ntt(q, psi, logn, O._p(one))
    assert np.all(one == 1)                    # NTT(1) = 1 everywhere
    x = np.zeros(n, dtype=np.uint64)
    x[1] = 1
    O.lib().pfo_ntt(q, psi, logn, O._p(x))
    for j in range(n):                         # NTT(X)[j] = psi^(2 brv(j) + 1)
        assert int(x[j]) == pow(psi, 2 * O.bitrev(j, logn) + 1, q)


@pytest.mark.parametrize("logn", [3, 5, 7])
def test_ntt_product_is_negacyclic_convolution(logn):
    P = O.Params(logn, [50, 45], [50], alpha=1, mod_log2=17)
    a = I.uniform_residues(P.q, P.N, seed=1)
    b = I.uniform_residues(P.q, P.N, seed=2)
    got = O.polymul(a, b, P.q, P.psi_q, logn)
    for i, q in enumerate(P.q):
        assert [int(v) for v in got[i]] == schoolbook_negacyclic(a[i], b[i], q)
    naive = np.empty_like(a[0])
    O.lib().pfo_negacyclic_mul_naive(P.q[0], logn, O._p(np.ascontiguousarray(a[0])),
                                     O._p(np.ascontiguousarray(b[0])), O._p(naive))
    assert np.array_equal(naive, got[0])


# ---------------------------------------------------------------- encoding
def direct_slots(p_coeffs, n):
    """z_j = p(zeta_j), zeta_j = exp(i pi (5^j mod 4n) / 2n): Horner per slot."""
    out = []
    for j in range(n):
        zeta = cmath.exp(1j * math.pi * pow(5, j, 4 * n) / (2 * n))
        acc = 0j
        for c in reversed(list(p_coeffs)):
            acc = acc * zeta + c
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("n", [1, 2, 8, 16])
def test_encoding_inverts_the_slot_evaluation(n):
    N = 2 * n if n > 1 else 4
    z = I.uniform_slots(n, seed=3) + 1j * I.uniform_slots(n, seed=4)
    p = O.encode_real_coeffs(z, N)
    assert np.allclose(direct_slots(p, n), z, atol=1e-12)
    # linear-solve check: real p with p(zeta_j) = z_j and p(conj zeta_j) = conj z_j
    rows, rhs = [], []
    for j in range(n):
        zeta = cmath.exp(1j * math.pi * pow(5, j, 4 * n) / (2 * n))
        for root, val in ((zeta, z[j]), (zeta.conjugate(), np.conj(z[j]))):
            rows.append([root ** k for k in range(2 * n)])
            rhs.append(val)
    sol = np.linalg.solve(np.array(rows), np.array(rhs))
    assert np.allclose(sol.imag, 0, atol=1e-10)
    assert np.allclose(sol.real, p, atol=1e-10)


def test_encode_decode_roundtrip_and_constant():
    P = O.params_n12_three_50bit()
    z = I.uniform_slots(P.N // 2, seed=5)
    m = O.encode(P, z, 2.0 ** 40, 3)
    back = O.decode(P, m, 2.0 ** 40, P.N // 2)
    assert np.max(np.abs(back - z)) < 2 ** -30
    # a constant c sits in coefficient 0 only, as round(c Delta)
    c = 0.3125
    mc = O.encode(P, np.full(P.N // 2, c), 2.0 ** 40, 3)
    assert int(mc[0, 0]) == round(c * 2 ** 40)
    assert np.all(mc[:, 1:] == 0)


def test_slot_rotation_and_conjugation_are_automorphisms():
    # App. A.1: phi_(0,k) rotates the slots left by k, phi_(1,0) conjugates
    P = SMALL
    n = P.N // 2
    z = I.uniform_slots(n, seed=6) + 1j * I.uniform_slots(n, seed=7)
    m = O.encode(P, z, 2.0 ** 40, 2)
    for k in (1, 3):
        rot = O.automorphism(m, O.galois_element(P, k), P.mods(2), P.logn)
        assert np.allclose(O.decode(P, rot, 2.0 ** 40, n), np.roll(z, -k), atol=1e-9)
    cj = O.automorphism(m, 2 * P.N - 1, P.mods(2), P.logn)
    assert np.allclose(O.decode(P, cj, 2.0 ** 40, n), np.conj(z), atol=1e-9)


def test_slot_product_is_pointwise():
    # App. A.1: the ring product of two slot encodings multiplies the slots
    P = SMALL
    n = P.N // 2
    z1, z2 = I.uniform_slots(n, seed=8), I.uniform_slots(n, seed=9)
    m1, m2 = O.encode(P, z1, 2.0 ** 30, 3), O.encode(P, z2, 2.0 ** 30, 3)
    prod = O.polymul(m1, m2, P.mods(3), P.psis(3), P.logn)
    assert np.allclose(O.decode(P, prod, 2.0 ** 60, n), z1 * z2, atol=1e-7)


# ---------------------------------------------------------------- automorphisms
def test_automorphism_matches_substitution_and_composes():
    P = SMALL
    q = P.q[0]
    a = I.uniform_residues([q], P.N, seed=10)
    b = I.uniform_residues([q], P.N, seed=11)
    for g in (3, 5, 25, 2 * P.N - 1):
        got = O.automorphism(a, g, [q], P.logn)
        assert [int(v) for v in got[0]] == poly_compose_power(a[0], g, q)
    g1, g2 = 5, 2 * P.N - 1
    comp = O.automorphism(O.automorphism(a, g1, [q], P.logn), g2, [q], P.logn)
    assert np.array_equal(comp, O.automorphism(a, g1 * g2 % (2 * P.N), [q], P.logn))
    # Sec. 2.2: phi(a) phi(b) = phi(a b)
    ab = schoolbook_negacyclic(a[0], b[0], q)
    lhs = schoolbook_negacyclic(O.automorphism(a, 5, [q], P.logn)[0], O.automorphism(b, 5, [q], P.logn)[0], q)
    assert lhs == poly_compose_power(ab, 5, q)


# ---------------------------------------------------------------- RNS steps vs big integers
def test_bconv_is_the_fast_conversion():
    P = SMALL4
    src, dst = P.q[:3], P.q[3:] + P.p
    x = I.uniform_residues(src, P.N, seed=12)
    got = O.bconv(x, src, dst)
    Qp = math.prod(src)
    xs = O.crt_centered(x, src) % Qp
    for c in range(P.N):
        ys = [int(x[i, c]) * pow(Qp // qi, -1, qi) % qi for i, qi in enumerate(src)]
        big = sum(y * (Qp // qi) for y, qi in zip(ys, src))
        u, rem = divmod(big - int(xs[c]), Qp)
        assert rem == 0 and 0 <= u < len(src)
        assert [int(got[m, c]) for m in range(len(dst))] == [big % m for m in dst]


def test_rescale_is_rounded_division_by_last_prime():
    # Sec. 2.5: rescale returns round(c / q_last) with modulus Q / q_last
    P = SMALL4
    lv = 4
    c = I.uniform_residues(P.mods(lv), P.N, seed=13, lead=(2,))
    ct = O.Ct(c, 2.0 ** 45)
    out = O.rescale(P, ct)
    Q = math.prod(P.mods(lv))
    ql = P.q[lv - 1]
    Qd = Q // ql
    for k in range(2):
        big = O.crt_centered(c[k], P.mods(lv)) % Q          # the [0, Q) lift
        exp = [((int(v) + ql // 2) // ql) % Qd for v in big]
        got = O.crt_centered(out.c[k], P.mods(lv - 1)) % Qd
        assert [int(v) for v in got] == exp
    assert out.scale == 2.0 ** 45 / ql


def test_mod_down_rounds_up_to_the_fast_conversion_overflow():
    # Sec. 2.4.1: SwitchKey outputs round(P^-1 <d, swk>): the oracle's ModDown
    # equals round(x / P) - u exactly, u the integer overflow of the fast
    # conversion of [x + floor(P/2)]_P, 0 <= u < K.
    P = SMALL4
    lv = 3
    ext = P.ext_mods(lv)
    x = I.uniform_residues(ext, P.N, seed=14)
    got = O.mod_down(P, x, lv)
    Pb = math.prod(P.p)
    Qx = math.prod(ext)
    Ql = math.prod(P.mods(lv))
    xs = O.crt_centered(x, ext) % Qx
    gs = O.crt_centered(got, P.mods(lv)) % Ql
    for c in range(P.N):
        y = int(xs[c]) + Pb // 2
        yp = y % Pb
        conv = sum((yp % pk) * pow(Pb // pk, -1, pk) % pk * (Pb // pk) for pk in P.p)
        u = (conv - yp) // Pb
        assert 0 <= u < P.K
        assert (y // Pb - u) % Ql == int(gs[c])


# ---------------------------------------------------------------- encryption and keys
def _keys(P, seed, h=None):
    s = I.ternary_secret(P.N, h, seed)
    ext = P.ext_mods(P.L)
    a = I.uniform_residues(ext, P.N, seed + 1, lead=(P.beta,))
    e = I.gaussian_error((P.beta, P.N), seed + 2)
    return s, O.relin_key(P, s, a, e), e


def test_encryption_error_is_exact():
    # Sec. 2.3: c0 + c1 s = m + e with the sampled e, checked by schoolbook
    P = SMALL
    s = I.ternary_secret(P.N, None, 20)
    m = O.encode(P, I.uniform_slots(P.N // 2, 21), 2.0 ** 40, 3)
    a = I.uniform_residues(P.mods(3), P.N, 22)
    e = I.gaussian_error(P.N, 23)
    ct = O.encrypt(P, s, m, a, e, 2.0 ** 40)
    for i, q in enumerate(P.q):
        cs = schoolbook_negacyclic(ct.c[1][i], [int(v) % q for v in s], q)
        lhs = [(int(ct.c[0][i][k]) + cs[k] - int(m[i][k])) % q for k in range(P.N)]
        assert lhs == [int(v) % q for v in e]
    assert np.array_equal(O.decrypt(P, s, ct), O.add(m, O.from_ints(e, P.q), P.q))


def test_switching_key_decrypts_to_gadget_times_secret():
    # Sec. 2.4.1: swk_j = RLWE_s(0) + w_j P s_from over QP
    P = SMALL4
    s, rlk, e = _keys(P, 30, h=6)
    ext = P.ext_mods(P.L)
    Qb, Pb = math.prod(P.q), math.prod(P.p)
    s_int = [int(v) for v in s]
    s2 = [0] * P.N
    for i in range(P.N):
        for j in range(P.N):
            k = i + j
            if k < P.N:
                s2[k] += s_int[i] * s_int[j]
            else:
                s2[k - P.N] -= s_int[i] * s_int[j]
    for j, D in enumerate(P.digits(P.L)):
        Qj = math.prod(P.q[i] for i in D)
        w = (Qb // Qj) * pow(Qb // Qj, -1, Qj)
        for r, m in enumerate(ext):
            as_ = schoolbook_negacyclic(rlk.a[j][r], [v % m for v in s_int], m)
            got = [(int(rlk.b[j][r][k]) + as_[k] - Pb * w * s2[k]) % m for k in range(P.N)]
            assert got == [int(v) % m for v in e[j]]


def test_key_switch_noise_is_small():
    P = O.Params(6, [50, 45, 45, 45, 45], [50, 50], alpha=2, mod_log2=17)
    s, rlk, _ = _keys(P, 40, h=16)
    lv = 5
    d = I.uniform_residues(P.mods(lv), P.N, 41)
    k0, k1 = O.key_switch(P, d, rlk)
    mods = P.mods(lv)
    s_r = O.secret_rns(P, s, mods)
    s2 = O.polymul(s_r, s_r, mods, P.psis(lv), P.logn)
    want = O.polymul(d, s2, mods, P.psis(lv), P.logn)
    got = O.add(k0, O.polymul(k1, s_r, mods, P.psis(lv), P.logn), mods)
    diff = O.crt_centered(O.sub(got, want, mods), mods)
    assert max(abs(int(v)) for v in diff) < 2 ** 20


# ---------------------------------------------------------------- homomorphic identities (App. A.1)
def test_homomorphic_ops_track_fp64():
    P = O.Params(7, [50, 45, 45], [50, 50], alpha=1, mod_log2=17)
    n = P.N // 2
    delta = 2.0 ** 45
    s = I.ternary_secret(P.N, 16, 50)
    ext = P.ext_mods(P.L)
    mk = lambda seed: (I.uniform_residues(ext, P.N, seed, lead=(P.beta,)), I.gaussian_error((P.beta, P.N), seed + 1))
    rlk = O.relin_key(P, s, *mk(51))
    keys = {}
    for k in (1, 2, 4, 8, 16, 32):
        g = O.galois_element(P, k)
        keys[g] = O.galois_key(P, s, g, *mk(60 + k))
    keys[2 * P.N - 1] = O.galois_key(P, s, 2 * P.N - 1, *mk(90))
    z1, z2 = I.uniform_slots(n, 52), I.uniform_slots(n, 53)
    enc = lambda z, seed: O.encrypt(P, s, O.encode(P, z, delta, 3), I.uniform_residues(P.mods(3), P.N, seed),
                                    I.gaussian_error(P.N, seed + 1), delta)
    c1, c2 = enc(z1, 54), enc(z2, 56)
    dec = lambda ct: O.decode(P, O.decrypt(P, s, ct), ct.scale, n).real
    assert np.max(np.abs(dec(O.ct_add(P, c1, c2)) - (z1 + z2))) < 2 ** -20
    prod = O.mul_relin(P, c1, c2, rlk)
    assert np.max(np.abs(dec(prod) - z1 * z2)) < 2 ** -20
    rs = O.rescale(P, prod)
    assert rs.level == 2
    assert np.max(np.abs(dec(rs) - z1 * z2)) < 2 ** -20
    for k in (1, 8):
        assert np.max(np.abs(dec(O.rotate(P, c1, k, keys)) - np.roll(z1, -k))) < 2 ** -20
    zc = I.uniform_slots(n, 57) + 1j * I.uniform_slots(n, 58)
    cc = O.encrypt(P, s, O.encode(P, zc, delta, 3), I.uniform_residues(P.mods(3), P.N, 59), I.gaussian_error(P.N, 60), delta)
    got = O.decode(P, O.decrypt(P, s, O.conjugate(P, cc, keys)), delta, n)
    assert np.max(np.abs(got - np.conj(zc))) < 2 ** -20
    tot = O.rotate_sum(P, c1, 6, keys)
    assert np.max(np.abs(dec(tot) - z1.sum())) < 2 ** -16
    pm = O.encode(P, z2, delta, 3)
    mp = O.ct_mul_plain(P, c1, pm, delta)
    assert np.max(np.abs(dec(mp) - z1 * z2)) < 2 ** -20
    assert np.max(np.abs(dec(O.ct_mul_int(P, c1, -3)) - (-3 * z1))) < 2 ** -20


def test_prime_rule_reproduces_the_parameter_sets_of_tab1():
    """tests/golden/tab1_parameter_sets.json: Tab. 1 prints log(QP) and its split
    into prime sizes; the chain rule must give distinct NTT-friendly primes whose
    sizes add up to the printed total, and the secret generator the printed h."""
    import json
    import math
    import os
    from paper_2412_13269_amd import inputs as I
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tab1_parameter_sets.json")))
    for st in g["sets"]:
        n = 1 << st["log_n"]
        assert sum(st["q_bits"]) + sum(st["p_bits"]) == st["log_qp"], st["name"]
        q, p = O.gen_primes(st["log_n"] + 1, st["q_bits"], st["p_bits"])
        chain = q + p
        assert len(set(chain)) == len(chain)
        for c, b in zip(chain, st["q_bits"] + st["p_bits"]):
            assert O.is_prime(c) and (c - 1) % (2 * n) == 0
            assert abs(math.log2(c) - b) < 0.01, (st["name"], b, c)
        assert abs(sum(math.log2(c) for c in chain) - st["log_qp"]) < 0.5
        s = I.ternary_secret(n, None if st["h"] == "2N/3" else st["h"], 7)
        nz = int(np.count_nonzero(s))
        if st["h"] == "2N/3":
            assert abs(nz - 2 * n / 3) < 4 * math.sqrt(n)
        else:
            assert nz == st["h"]
