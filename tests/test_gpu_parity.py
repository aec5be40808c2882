"""GPU parity: every call of the C-ABI against the CPU oracle, word for word.

Both sides take the same seeded inputs (secret, uniform `a`, errors, encoded
plaintext words from the oracle) and must produce identical canonical
coefficient-domain words.  Decrypted values are also checked against FP64.
"""
import numpy as np
import pytest

from oracle import ckks as O
from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx   # fails loudly if libpfx.so is missing
    return pfx


class Pair:
    """Oracle and library contexts on one parameter set, with shared inputs."""

    def __init__(self, X, logn, qb, pb, alpha, ml=0, h=None, seed=1, scale=2.0 ** 45):
        self.X = X
        self.P = O.Params(logn, qb, pb, alpha=alpha, mod_log2=ml)
        self.prm = X.make_params(logn, qb, pb, alpha, ml)
        self.ctx = X.pfx_ctx_create(self.prm, 0)
        self.N = self.P.N
        self.scale = scale
        self.s = I.ternary_secret(self.N, h, seed)
        self.sk = X.pfx_sk_create(self.ctx, self.s)
        self.ko, self.kx = {}, {}
        self.seed = seed * 1000
        self.handles = []

    def _next(self):
        self.seed += 7
        return self.seed

    def key(self, g):
        if g not in self.ko:
            ext = self.P.ext_mods(self.P.L)
            a = I.uniform_residues(ext, self.N, self._next(), lead=(self.P.beta,))
            e = I.gaussian_error((self.P.beta, self.N), self._next())
            self.ko[g] = O.relin_key(self.P, self.s, a, e) if g == 0 else O.galois_key(self.P, self.s, g, a, e)
            self.kx[g] = self.X.pfx_swk_create(self.ctx, self.sk, g, a, e)
        return self.ko[g], self.kx[g]

    def ct(self, lv, cap=None, deg=2):
        h = self.X.pfx_ct_create(self.ctx, cap or self.P.L, deg)
        self.handles.append(h)
        return h

    def enc(self, lv, seed=None, z=None):
        z = I.uniform_slots(self.N // 2, seed or self._next()) if z is None else z
        m = O.encode(self.P, z, self.scale, lv)
        a = I.uniform_residues(self.P.mods(lv), self.N, self._next())
        e = I.gaussian_error(self.N, self._next())
        co = O.encrypt(self.P, self.s, m, a, e, self.scale)
        pt = self.X.pfx_pt_import(self.ctx, m, self.scale)
        self.handles.append(pt)
        cx = self.ct(lv)
        self.X.pfx_encrypt(self.ctx, self.sk, pt, a, e, cx)
        return co, cx, z

    def words(self, cx):
        return self.X.pfx_ct_export(self.ctx, cx, self.N)

    def same(self, co, cx):
        w = self.words(cx)
        assert w.shape == co.c.shape, (w.shape, co.c.shape)
        assert np.array_equal(w, co.c)
        info = self.X.pfx_ct_info(cx)
        assert info.scale == pytest.approx(co.scale, rel=1e-15)

    def close(self):
        for h in self.handles:
            self.X.pfx_ct_destroy(h)
        for k in self.kx.values():
            self.X.pfx_swk_destroy(k)
        self.X.pfx_sk_destroy(self.sk)
        self.X.pfx_ctx_destroy(self.ctx)


CONFIGS = {
    # N = 2^12, three 50-bit primes, one special prime, digits of one prime
    "n12_3x50": dict(logn=12, qb=[50, 50, 50], pb=[50], alpha=1, ml=0, h=None, scale=2.0 ** 40),
    # the 50 + 45-bit chain with 4 special primes at N = 2^13 and 9 limbs: a partial
    # last digit (9 = 4 + 4 + 1)
    "n13_9_limbs": dict(logn=13, qb=[50] + [45] * 8, pb=[50] * 4, alpha=4, ml=17, h=192, scale=2.0 ** 45),
}


@pytest.fixture(scope="module", params=list(CONFIGS))
def pair(request, X):
    cfg = CONFIGS[request.param]
    p = Pair(X, cfg["logn"], cfg["qb"], cfg["pb"], cfg["alpha"], cfg["ml"], cfg["h"], seed=11,
             scale=cfg["scale"])
    yield p
    p.close()


# ------------------------------------------------------------------ transforms and plumbing
def test_moduli_match(pair, X):
    q, p, psi = X.pfx_ctx_moduli(pair.ctx, pair.P.L, pair.P.K)
    assert [int(v) for v in q] == pair.P.q and [int(v) for v in p] == pair.P.p
    assert [int(v) for v in psi] == pair.P.psi_q + pair.P.psi_p


@pytest.mark.parametrize("inverse", [False, True])
def test_standalone_ntt(pair, X, inverse):
    P = pair.P
    nl = P.L + P.K
    batch = 2
    words = I.uniform_residues(P.q + P.p, P.N, 5, lead=(batch,))
    dev = X.pfx_dev_alloc(pair.ctx, words.nbytes)
    X.pfx_memcpy_htod(pair.ctx, dev, words)
    X.pfx_ntt(pair.ctx, dev, 0, nl, batch, inverse)
    got = np.empty_like(words)
    X.pfx_memcpy_dtoh(pair.ctx, got, dev)
    X.pfx_dev_free(pair.ctx, dev)
    fn = O.intt if inverse else O.ntt
    for b in range(batch):
        assert np.array_equal(got[b], fn(words[b], P.q + P.p, P.psi_q + P.psi_p, P.logn))


def test_import_export_roundtrip(pair, X):
    P = pair.P
    w = I.uniform_residues(P.mods(P.L), P.N, 6, lead=(3,))
    cx = pair.ct(P.L)
    X.pfx_ct_import(pair.ctx, w, 3.0, cx)
    assert np.array_equal(pair.words(cx), w)


def test_keygen_parity(pair, X):
    P = pair.P
    for g in (0, O.galois_element(P, 1), 2 * P.N - 1):
        ko, kx = pair.key(g)
        got = X.pfx_swk_export(pair.ctx, kx, P.beta, P.L + P.K, P.N)
        assert np.array_equal(got[:, 0], ko.b)
        assert np.array_equal(got[:, 1], ko.a)


def test_encrypt_decrypt_parity(pair, X):
    P = pair.P
    co, cx, z = pair.enc(P.L)
    pair.same(co, cx)
    mx = X.pfx_decrypt(pair.ctx, pair.sk, cx)
    pair.handles.append(mx)
    assert np.array_equal(pair.words(mx)[0], O.decrypt(P, pair.s, co))
    got = X.pfx_decode(pair.ctx, mx, P.N // 2)
    assert np.max(np.abs(got - z)) < 2.0 ** -20


# ------------------------------------------------------------------ arithmetic
def test_elementwise_ops(pair, X):
    P = pair.P
    lv = P.L
    c1o, c1x, z1 = pair.enc(lv)
    c2o, c2x, z2 = pair.enc(lv - 1)          # mixed levels: drops to lv - 1
    out = pair.ct(lv)
    X.pfx_add(pair.ctx, c1x, c2x, out)
    pair.same(O.ct_add(P, c1o, c2o), out)
    X.pfx_sub(pair.ctx, c1x, c2x, out)
    pair.same(O.ct_sub(P, c1o, c2o), out)
    X.pfx_neg(pair.ctx, c1x, out)
    pair.same(O.Ct(np.stack([O.neg(c, P.mods(lv)) for c in c1o.c]), c1o.scale), out)
    for k in (3, -5, 0, 1 << 40):
        X.pfx_mul_int(pair.ctx, c1x, k, out)
        pair.same(O.ct_mul_int(P, c1o, k), out)
    m = O.encode(P, I.uniform_slots(P.N // 2, 40), pair.scale, lv)
    pt = X.pfx_pt_import(pair.ctx, m, pair.scale)
    pair.handles.append(pt)
    X.pfx_mul_plain(pair.ctx, c1x, pt, out)
    pair.same(O.ct_mul_plain(P, c1o, m, pair.scale), out)
    X.pfx_add_plain(pair.ctx, c1x, pt, out)
    pair.same(O.ct_add_plain(P, c1o, m), out)
    # in place
    X.pfx_add(pair.ctx, c1x, c1x, c1x)
    pair.same(O.ct_add(P, c1o, c1o), c1x)


def test_accumulating_products(pair, X):
    """acc += a * b (tensor), acc += a * m (plaintext) and acc += a * k
    (integer): the oracle's product followed by its addition, word for word,
    including a level drop."""
    P = pair.P
    c1o, c1x, _ = pair.enc(P.L)
    c2o, c2x, _ = pair.enc(P.L)
    c3o, c3x, _ = pair.enc(P.L - 1)
    acc = pair.ct(P.L)
    X.pfx_mul(pair.ctx, c1x, c2x, acc)
    X.pfx_mul_acc(pair.ctx, c3x, c2x, acc)          # drops to L - 1 limbs
    want = O.ct_add(P, O.tensor(P, c1o, c2o), O.tensor(P, c3o, c2o))
    pair.same(want, acc)
    X.pfx_mul_acc(pair.ctx, c1x, c1x, acc)
    pair.same(O.ct_add(P, want, O.tensor(P, c1o, c1o)), acc)
    m1 = O.encode(P, I.uniform_slots(P.N // 2, 41), pair.scale, P.L)
    m2 = O.encode(P, I.uniform_slots(P.N // 2, 42), pair.scale, P.L)
    pt1, pt2 = X.pfx_pt_import(pair.ctx, m1, pair.scale), X.pfx_pt_import(pair.ctx, m2, pair.scale)
    pair.handles += [pt1, pt2]
    acc1 = pair.ct(P.L)
    X.pfx_mul_plain(pair.ctx, c1x, pt1, acc1)
    X.pfx_mul_plain_acc(pair.ctx, c2x, pt2, acc1)
    X.pfx_mul_plain_acc(pair.ctx, c3x, pt1, acc1)   # drops to L - 1 limbs
    want = O.ct_add(P, O.ct_add(P, O.ct_mul_plain(P, c1o, m1, pair.scale), O.ct_mul_plain(P, c2o, m2, pair.scale)),
                    O.ct_mul_plain(P, c3o, m1, pair.scale))
    pair.same(want, acc1)
    acc2 = pair.ct(P.L)
    X.pfx_mul_int(pair.ctx, c1x, -35, acc2)
    X.pfx_mul_int_acc(pair.ctx, c2x, 21, acc2)
    X.pfx_mul_int_acc(pair.ctx, c3x, -5, acc2)     # drops to L - 1 limbs
    want = O.ct_add(P, O.ct_add(P, O.ct_mul_int(P, c1o, -35), O.ct_mul_int(P, c2o, 21)), O.ct_mul_int(P, c3o, -5))
    pair.same(want, acc2)
    with pytest.raises(X.PfxError) as e:             # a degree-1 accumulator for a tensor product
        X.pfx_mul_acc(pair.ctx, c1x, c2x, acc1)
    assert e.value.status == X.PFX_EINVAL
    with pytest.raises(X.PfxError) as e:             # accumulator aliasing the operand
        X.pfx_mul_plain_acc(pair.ctx, acc1, pt1, acc1)
    assert e.value.status == X.PFX_EINVAL


def test_tensor_relinearize(pair, X):
    P = pair.P
    ko, kx = pair.key(0)
    c1o, c1x, z1 = pair.enc(P.L)
    c2o, c2x, z2 = pair.enc(P.L)
    t = pair.ct(P.L)
    X.pfx_mul(pair.ctx, c1x, c2x, t)
    to = O.tensor(P, c1o, c2o)
    pair.same(to, t)
    r = pair.ct(P.L)
    X.pfx_relinearize(pair.ctx, t, kx, r)
    ro = O.relinearize(P, to, ko)
    pair.same(ro, r)
    m = pair.ct(P.L)
    X.pfx_mul_relin(pair.ctx, c1x, c2x, kx, m)        # product formed inside the key switch
    pair.same(ro, m)
    dec = X.pfx_decrypt(pair.ctx, pair.sk, m)
    pair.handles.append(dec)
    assert np.max(np.abs(X.pfx_decode(pair.ctx, dec, P.N // 2) - z1 * z2)) < 2.0 ** -20
    c3o, c3x, _ = pair.enc(P.L - 1)                  # operands at different levels
    X.pfx_mul_relin(pair.ctx, c3x, c2x, kx, m)
    pair.same(O.mul_relin(P, c3o, c2o, ko), m)
    X.pfx_mul_relin(pair.ctx, c3x, c3x, kx, m)        # squaring
    pair.same(O.mul_relin(P, c3o, c3o, ko), m)
    X.pfx_mul_relin(pair.ctx, c1x, c2x, kx, c2x)     # output aliases the second input
    pair.same(ro, c2x)
    X.pfx_mul_relin(pair.ctx, c1x, c1x, kx, c1x)     # output aliases both
    pair.same(O.mul_relin(P, c1o, c1o, ko), c1x)


def test_mul_relin_batch(pair, X):
    """Batched HMult + relin: 11 pairs over three levels (more than one launch
    of 8 at the top level), word for word the per-pair results, and the first
    pairs against the oracle."""
    P = pair.P
    ko, kx = pair.key(0)
    levels = [P.L, P.L, P.L - 1, P.L, 2, P.L, P.L - 1, P.L, P.L, P.L, P.L]
    cts = [pair.enc(lv) for lv in levels]
    a = [cts[i][1] for i in range(11)]
    b = [cts[(i + 3) % 11][1] for i in range(11)]
    b[5] = a[5]                                       # a squaring inside the batch
    outs = [pair.ct(P.L) for _ in range(11)]
    X.pfx_mul_relin_batch(pair.ctx, a, b, kx, outs)
    one = pair.ct(P.L)
    for i in range(11):
        X.pfx_mul_relin(pair.ctx, a[i], b[i], kx, one)
        assert np.array_equal(pair.words(outs[i]), pair.words(one)), i
        assert X.pfx_ct_info(outs[i]).scale == X.pfx_ct_info(one).scale
        assert X.pfx_ct_info(outs[i]).n_limbs == min(levels[i], levels[(i + 3) % 11])
    for i in (0, 2, 4):
        pair.same(O.mul_relin(P, cts[i][0], cts[(i + 3) % 11][0], ko), outs[i])
    with pytest.raises(X.PfxError) as e:              # output aliases another pair's operand
        X.pfx_mul_relin_batch(pair.ctx, a[:2], b[:2], kx, [outs[0], a[1]])
    assert e.value.status == X.PFX_EINVAL
    with pytest.raises(X.PfxError) as e:              # two pairs write one output
        X.pfx_mul_relin_batch(pair.ctx, a[:2], b[:2], kx, [outs[0], outs[0]])
    assert e.value.status == X.PFX_EINVAL
    X.pfx_mul_relin_batch(pair.ctx, [], [], kx, [])   # empty batch


def test_rescale_batch(pair, X):
    """Batched rescale: ten ciphertexts over two levels and degrees 1 and 2,
    some in place, word for word the single rescales (themselves pinned to the
    oracle below)."""
    P = pair.P
    cts = [pair.enc(P.L if i % 3 else P.L - 1) for i in range(8)]
    src = [c[1] for c in cts]
    for i in (0, 1):                                 # two degree-2 tensor products
        t = pair.ct(P.L)
        X.pfx_mul(pair.ctx, cts[2 + i][1], cts[4 + i][1], t)
        src.append(t)
    want = []
    for h in src:
        o = pair.ct(P.L)
        X.pfx_rescale(pair.ctx, h, o)
        want.append((pair.words(o), X.pfx_ct_info(o)))
    copies = []
    for h in src:                                    # in-place entries work on copies
        c = pair.ct(P.L)
        X.pfx_ct_copy(pair.ctx, h, c)
        copies.append(c)
    ins = [copies[i] if i % 2 else src[i] for i in range(10)]
    outs = [copies[i] if i % 2 else pair.ct(P.L) for i in range(10)]
    X.pfx_rescale_batch(pair.ctx, ins, outs)
    for i in range(10):
        w, info = want[i]
        assert np.array_equal(pair.words(outs[i]), w), i
        got = X.pfx_ct_info(outs[i])
        assert (got.n_limbs, got.degree, got.scale) == (info.n_limbs, info.degree, info.scale), i
    pair.same(O.rescale(P, cts[0][0]), outs[0])
    with pytest.raises(X.PfxError) as e:             # writes another entry's input
        X.pfx_rescale_batch(pair.ctx, [src[0], src[2]], [outs[0], src[0]])
    assert e.value.status == X.PFX_EINVAL
    X.pfx_rescale_batch(pair.ctx, [], [])


def test_relinearize_batch(pair, X):
    """Batched relinearisation: five tensor products over two levels, two of
    them in place, word for word the single calls; the first against the
    oracle."""
    P = pair.P
    ko, kx = pair.key(0)
    cts = [pair.enc(P.L if i % 2 else P.L - 1) for i in range(6)]
    tens = []
    for i in range(5):
        t = pair.ct(P.L)
        X.pfx_mul(pair.ctx, cts[i][1], cts[i + 1][1], t)
        tens.append(t)
    want = []
    for t in tens:
        o = pair.ct(P.L)
        X.pfx_relinearize(pair.ctx, t, kx, o)
        want.append(pair.words(o))
    outs = [t if i in (1, 3) else pair.ct(P.L) for i, t in enumerate(tens)]
    X.pfx_relinearize_batch(pair.ctx, tens, kx, outs)
    for i in range(5):
        assert np.array_equal(pair.words(outs[i]), want[i]), i
        assert X.pfx_ct_info(outs[i]).degree == 1
    pair.same(O.relinearize(P, O.tensor(P, cts[0][0], cts[1][0]), ko), outs[0])
    with pytest.raises(X.PfxError) as e:             # degree-1 input
        X.pfx_relinearize_batch(pair.ctx, [outs[0]], kx, [pair.ct(P.L)])
    assert e.value.status == X.PFX_EINVAL


def test_rescale_every_level(pair, X):
    P = pair.P
    co, cx, z = pair.enc(P.L)
    for lv in range(P.L, 1, -1):
        X.pfx_rescale(pair.ctx, cx, cx)
        co = O.rescale(P, co)
        pair.same(co, cx)
    with pytest.raises(X.PfxError) as e:
        X.pfx_rescale(pair.ctx, cx, cx)
    assert e.value.status == X.PFX_ELEVEL


def test_key_switch_at_partial_levels(pair, X):
    P = pair.P
    ko, kx = pair.key(0)
    for lv in sorted({1, 2, 3, min(5, P.L), P.L}):
        d = I.uniform_residues(P.mods(lv), P.N, 100 + lv)
        dx = pair.ct(lv)
        X.pfx_ct_import(pair.ctx, d[None], 1.0, dx)
        out = pair.ct(lv)
        X.pfx_key_switch(pair.ctx, dx, kx, out)
        k0, k1 = O.key_switch(P, d, ko)
        w = pair.words(out)
        assert np.array_equal(w[0], k0) and np.array_equal(w[1], k1), lv


def test_rotations_and_conjugation(pair, X):
    P = pair.P
    co, cx, z = pair.enc(P.L)
    out = pair.ct(P.L)
    keys = []
    for step in (1, 7, -1):
        g = O.galois_element(P, step)
        ko, kx = pair.key(g)
        keys.append(kx)
        X.pfx_rotate(pair.ctx, cx, step, keys, out)
        ro = O.rotate(P, co, step, {g: ko})
        pair.same(ro, out)
    gc = 2 * P.N - 1
    ko, kx = pair.key(gc)
    X.pfx_conjugate(pair.ctx, cx, [kx], out)
    pair.same(O.conjugate(P, co, {gc: ko}), out)
    with pytest.raises(X.PfxError) as e:
        X.pfx_rotate(pair.ctx, cx, 3, keys, out)
    assert e.value.status == X.PFX_ENOKEY
    # in place (output aliases the input), and below the top level
    g = O.galois_element(P, 7)
    X.pfx_rotate(pair.ctx, cx, 7, keys, cx)
    pair.same(O.rotate(P, co, 7, {g: pair.key(g)[0]}), cx)
    lo_o, lo_x, _ = pair.enc(P.L - 1)
    X.pfx_rotate(pair.ctx, lo_x, -1, keys, out)
    g = O.galois_element(P, -1)
    pair.same(O.rotate(P, lo_o, -1, {g: pair.key(g)[0]}), out)


def test_rotate_sum(pair, X):
    P = pair.P
    co, cx, z = pair.enc(P.L)
    keys_o, keys_x = {}, []
    for k in range(3):
        g = O.galois_element(P, 1 << k)
        ko, kx = pair.key(g)
        keys_o[g] = ko
        keys_x.append(kx)
    out = pair.ct(P.L)
    X.pfx_rotate_sum(pair.ctx, cx, 3, keys_x, out)
    pair.same(O.rotate_sum(P, co, 3, keys_o), out)


def test_scale_mismatch_is_rejected(pair, X):
    P = pair.P
    c1o, c1x, _ = pair.enc(P.L)
    c2o, c2x, _ = pair.enc(P.L)
    X.pfx_ct_set_scale(c2x, pair.scale * 1.01)
    with pytest.raises(X.PfxError) as e:
        X.pfx_add(pair.ctx, c1x, c2x, c1x)
    assert e.value.status == X.PFX_ESCALE


# ------------------------------------------------------------------ full size (N = 2^16, L = 24)
@pytest.fixture(scope="module")
def full(X):
    p = Pair(X, 16, [50] + [45] * 23, [50] * 4, 4, 17, h=192, seed=201)
    yield p
    p.close()


def test_full_size_mul_relin_rescale_rotate(full, X):
    P = full.P
    ko, kx = full.key(0)
    g = O.galois_element(P, 1)
    go, gx = full.key(g)
    c1o, c1x, z1 = full.enc(24)
    c2o, c2x, z2 = full.enc(24)
    X.pfx_mul_relin(full.ctx, c1x, c2x, kx, c1x)
    c1o = O.mul_relin(P, c1o, c2o, ko)
    full.same(c1o, c1x)
    X.pfx_rescale(full.ctx, c1x, c1x)
    c1o = O.rescale(P, c1o)
    full.same(c1o, c1x)
    out = full.ct(24)
    X.pfx_rotate(full.ctx, c1x, 1, [gx], out)
    full.same(O.rotate(P, c1o, 1, {g: go}), out)
    dec = X.pfx_decrypt(full.ctx, full.sk, out)
    full.handles.append(dec)
    got = X.pfx_decode(full.ctx, dec, P.N // 2)
    assert np.max(np.abs(got - np.roll(z1 * z2, -1))) < 2.0 ** -20


def test_full_size_mul_relin_batch(full, X):
    """Four full-size pairs in one batched key switch equal four single calls."""
    P = full.P
    _, kx = full.key(0)
    cts = [full.enc(24)[1] for _ in range(5)]
    outs = [full.ct(24) for _ in range(4)]
    X.pfx_mul_relin_batch(full.ctx, cts[:4], cts[1:5], kx, outs)
    one = full.ct(24)
    for i in range(4):
        X.pfx_mul_relin(full.ctx, cts[i], cts[i + 1], kx, one)
        assert np.array_equal(full.words(outs[i]), full.words(one)), i


@pytest.mark.parametrize("inverse", [False, True])
def test_full_size_standalone_ntt_offset_primes(full, X, inverse):
    """N = 2^16: three blocks of 5 limbs on primes 3..7 (limb l of a block on
    prime 3 + l), against the oracle's transform."""
    P = full.P
    mods = (P.q + P.p)[3:8]
    psis = (P.psi_q + P.psi_p)[3:8]
    words = I.uniform_residues(mods, P.N, 17, lead=(3,))
    dev = X.pfx_dev_alloc(full.ctx, words.nbytes)
    X.pfx_memcpy_htod(full.ctx, dev, words)
    X.pfx_ntt(full.ctx, dev, 3, 5, 3, inverse)
    got = np.empty_like(words)
    X.pfx_memcpy_dtoh(full.ctx, got, dev)
    X.pfx_dev_free(full.ctx, dev)
    fn = O.intt if inverse else O.ntt
    for b in range(3):
        assert np.array_equal(got[b], fn(words[b], mods, psis, P.logn)), b


# ------------------------------------------------------------------ N = 2^15 on the 24-limb chain
# The middle ring degree of the batched workload: its column and row passes
# are 7 and 8 stages (the other tested rings have equal halves or fewer
# stages), with their own twiddle tables.
@pytest.fixture(scope="module")
def mid(X):
    p = Pair(X, 15, [50] + [45] * 23, [50] * 4, 4, 17, h=192, seed=215)
    yield p
    p.close()


@pytest.mark.parametrize("inverse", [False, True])
def test_n15_standalone_ntt_every_prime(mid, X, inverse):
    P = mid.P
    mods, psis = P.q + P.p, P.psi_q + P.psi_p
    words = I.uniform_residues(mods, P.N, 1517)
    dev = X.pfx_dev_alloc(mid.ctx, words.nbytes)
    X.pfx_memcpy_htod(mid.ctx, dev, words)
    X.pfx_ntt(mid.ctx, dev, 0, len(mods), 1, inverse)
    got = np.empty_like(words)
    X.pfx_memcpy_dtoh(mid.ctx, got, dev)
    X.pfx_dev_free(mid.ctx, dev)
    fn = O.intt if inverse else O.ntt
    assert np.array_equal(got, fn(words, mods, psis, P.logn))


def test_n15_key_switch_at_partial_levels(mid, X):
    """Whole digits (4, 24 limbs), a partial last digit (1, 2, 3, 5, 13) on the
    N = 2^15 ring, against the oracle's ModUp / inner product / ModDown."""
    P = mid.P
    ko, kx = mid.key(0)
    for lv in (1, 2, 3, 4, 5, 13, 24):
        d = I.uniform_residues(P.mods(lv), P.N, 1500 + lv)
        dx = mid.ct(lv)
        X.pfx_ct_import(mid.ctx, d[None], 1.0, dx)
        out = mid.ct(lv)
        X.pfx_key_switch(mid.ctx, dx, kx, out)
        k0, k1 = O.key_switch(P, d, ko)
        w = mid.words(out)
        assert np.array_equal(w[0], k0) and np.array_equal(w[1], k1), lv


def test_n15_mul_relin_rescale_rotate(mid, X):
    P = mid.P
    ko, kx = mid.key(0)
    c1o, c1x, z1 = mid.enc(24)
    c2o, c2x, z2 = mid.enc(24)
    out = mid.ct(24)
    X.pfx_mul_relin(mid.ctx, c1x, c2x, kx, out)
    po = O.mul_relin(P, c1o, c2o, ko)
    mid.same(po, out)
    X.pfx_rescale(mid.ctx, out, out)
    po = O.rescale(P, po)
    mid.same(po, out)
    keys = {}
    for step in (1, 1 << 13, -1):
        g = O.galois_element(P, step)
        keys[g] = mid.key(g)
    rot = mid.ct(24)
    for step in (1, 1 << 13, -1):
        X.pfx_rotate(mid.ctx, out, step, [k[1] for k in keys.values()], rot)
        mid.same(O.rotate(P, po, step, {g: k[0] for g, k in keys.items()}), rot)
    gc = 2 * P.N - 1
    kco, kcx = mid.key(gc)
    X.pfx_conjugate(mid.ctx, out, [kcx], rot)
    mid.same(O.conjugate(P, po, {gc: kco}), rot)
    dec = X.pfx_decrypt(mid.ctx, mid.sk, out)
    mid.handles.append(dec)
    got = X.pfx_decode(mid.ctx, dec, P.N // 2)
    assert np.max(np.abs(got - z1 * z2)) < 2.0 ** -20


def test_n15_rescale_down_the_chain(mid, X):
    """Rescale at every level from 24 to 2 (each dropped prime has its own
    constants), word for word."""
    P = mid.P
    co, cx, _ = mid.enc(24)
    for _ in range(23):
        X.pfx_rescale(mid.ctx, cx, cx)
        co = O.rescale(P, co)
        mid.same(co, cx)


def test_n15_mul_relin_batch_at_three_levels(mid, X):
    """Batched HMult + relin at N = 2^15 (entries at 24, 13 and 3 limbs) equals
    the oracle."""
    P = mid.P
    ko, kx = mid.key(0)
    cts = [mid.enc(lv) for lv in (24, 24, 13, 13, 3, 3)]
    outs = [mid.ct(24) for _ in range(3)]
    X.pfx_mul_relin_batch(mid.ctx, [cts[0][1], cts[2][1], cts[4][1]], [cts[1][1], cts[3][1], cts[5][1]], kx, outs)
    for k in range(3):
        mid.same(O.mul_relin(P, cts[2 * k][0], cts[2 * k + 1][0], ko), outs[k])
