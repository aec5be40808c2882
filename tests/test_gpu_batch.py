"""Batched HMult + relin + rescale over ciphertexts of uneven ring degree and
level: every mode (per-ciphertext launches, concurrent lanes, batched key
switches grouped by shape, HIP-graph replay, one persistent launch, one launch per
step) gives the same words, and sampled entries match the oracle."""
import numpy as np
import pytest

from oracle import ckks as O
from paper_2412_13269_amd import inputs as I

pytestmark = pytest.mark.gpu

QB, PB, ALPHA, ML = [50] + [45] * 23, [50] * 4, 4, 17


@pytest.fixture(scope="module")
def X():
    from paper_2412_13269_amd import pfx
    return pfx


def _modes_agree_and_match_oracle(X, lognums, shapes, in_place, oracle_levels):
    """Run the entries `shapes` ((log N, level) each) in every mode of the
    batched call; all modes must give the words of mode 0 (one ciphertext
    after the other), and for each ring degree the entries at the levels
    `oracle_levels` picks must equal the oracle."""
    ctxs, P, sks, rlks, keyin, secrets = {}, {}, {}, {}, {}, {}
    for ln in lognums:
        prm = X.make_params(ln, QB, PB, ALPHA, ML)
        ctxs[ln] = X.pfx_ctx_create(prm, 0)
        P[ln] = O.Params(ln, QB, PB, alpha=ALPHA, mod_log2=ML)
        N = 1 << ln
        secrets[ln] = I.ternary_secret(N, 192, ln)
        sks[ln] = X.pfx_sk_create(ctxs[ln], secrets[ln])
        ext = P[ln].ext_mods(P[ln].L)
        keyin[ln] = (I.uniform_residues(ext, N, 50 + ln, lead=(P[ln].beta,)),
                     I.gaussian_error((P[ln].beta, N), 60 + ln))
        rlks[ln] = X.pfx_swk_create(ctxs[ln], sks[ln], 0, *keyin[ln])
    c0 = ctxs[lognums[0]]
    stream = X.pfx_stream_create(c0)
    entries = []
    handles = []
    for i, (ln, lv) in enumerate(shapes):
        N = 1 << ln
        words = [I.uniform_residues(P[ln].mods(lv), N, 1000 + 10 * i + k, lead=(2,)) for k in range(2)]
        cts = []
        for w in words:
            h = X.pfx_ct_create(ctxs[ln], lv, 1)
            X.pfx_ct_import(ctxs[ln], w, 2.0 ** 45, h)
            cts.append(h)
        out = cts[0] if i in in_place else X.pfx_ct_create(ctxs[ln], lv, 1)
        handles += cts + ([] if out is cts[0] else [out])
        entries.append((ln, lv, words, cts, out))
    args = ([ctxs[e[0]] for e in entries], [e[3][0] for e in entries], [e[3][1] for e in entries],
            [rlks[e[0]] for e in entries], [e[4] for e in entries])
    def reset():
        for e in entries:            # clobber outputs, restore in-place inputs
            if e[4] is e[3][0]:
                X.pfx_ct_import(ctxs[e[0]], e[2][0], 2.0 ** 45, e[4])
            else:
                X.pfx_ct_import(ctxs[e[0]], np.zeros((2, e[1] - 1, 1 << e[0]), np.uint64), 1.0, e[4])

    try:
        X.pfx_batch_mul_relin_rescale(*args, 0, stream)
        X.pfx_sync(c0, stream)
        ref = [X.pfx_ct_export(ctxs[e[0]], e[4], 1 << e[0]) for e in entries]
        for mode in (1, 2, 3, 4, 5, 6, 2, 4, 3, 1, 4, 6, 5):
            reset()
            X.pfx_batch_mul_relin_rescale(*args, mode, stream)
            X.pfx_sync(c0, stream)
            for e, r in zip(entries, ref):
                assert np.array_equal(X.pfx_ct_export(ctxs[e[0]], e[4], 1 << e[0]), r), mode
        # oracle parity on the chosen entries of each ring degree
        for ln in lognums:
            Pl = P[ln]
            rlk_o = O.relin_key(Pl, secrets[ln], *keyin[ln])
            mine = [k for k, x in enumerate(entries) if x[0] == ln]
            for k in oracle_levels([entries[k][1] for k in mine]):
                e = entries[mine[k]]
                a, b = (O.Ct(w, 2.0 ** 45) for w in e[2])
                want = O.rescale(Pl, O.mul_relin(Pl, a, b, rlk_o))
                assert np.array_equal(ref[mine[k]], want.c), (ln, e[1])
    finally:
        for h in handles:
            X.pfx_ct_destroy(h)
        for ln in lognums:
            X.pfx_swk_destroy(rlks[ln])
            X.pfx_sk_destroy(sks[ln])
        X.pfx_stream_destroy(c0, stream)
        for ln in lognums:
            X.pfx_ctx_destroy(ctxs[ln])


def test_batch_modes_agree_and_match_oracle(X):
    # 24 entries of random shape, then 20 over few shapes (groups of up to 8 for
    # the batched modes, one of 10 split in two), two of them in place
    rng = np.random.default_rng(401)
    lognums = (12, 13, 14)
    shapes = [(int(rng.choice(lognums)), int(rng.integers(3, 25))) for _ in range(24)]
    shapes += [(13, 24)] * 10 + [(12, 7)] * 6 + [(14, 7)] * 4
    _modes_agree_and_match_oracle(X, lognums, shapes, (30, 41), lambda lvs: [0])


def test_batch_at_the_batched_workload_ring_degrees(X):
    """The batched workload's own shapes: ring degrees 2^14, 2^15, 2^16 and
    levels 3..24 drawn as the benchmark draws them, plus groups of one shape
    (a full group of 8 at 2^16 and 24 limbs, and one of 3 at 2^15 and 3
    limbs, one entry in place).  Every mode agrees with mode 0, and at each
    ring degree the entries at the lowest and the highest level drawn match
    the oracle."""
    rng = np.random.default_rng(401)
    lognums = (14, 15, 16)
    shapes = [(int(rng.choice(lognums)), int(rng.integers(3, 25))) for _ in range(18)]
    shapes += [(16, 24)] * 8 + [(15, 3)] * 3
    lo_hi = lambda lvs: sorted({int(np.argmin(lvs)), int(np.argmax(lvs))})
    _modes_agree_and_match_oracle(X, lognums, shapes, (20, 27), lo_hi)
