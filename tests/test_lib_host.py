"""Host-side checks of libpfx.so (no GPU): the library loads, exports every
symbol the header declares, and its host logic (prime chain, roots, slot
encoder) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import ckks as O
from paper_2412_13269_amd import inputs as I

X = pytest.importorskip("paper_2412_13269_amd.pfx", reason="libpfx.so not built")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "pfx.h")).read()
    names = set(re.findall(r"\b(pfx_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) > 40
    for n in sorted(names):
        assert hasattr(X._lib, n), n
    assert names == set(X.exported_symbols())


CHAINS = [
    (12, [50, 50, 50], [50], 1, 0),
    (16, [50] + [45] * 23, [50] * 4, 4, 17),
    (14, [50] + [45] * 23, [50] * 4, 4, 17),
    (15, [50] + [45] * 23, [50] * 4, 4, 17),
    (4, [50, 45, 45, 45, 45], [50, 50], 2, 17),
]


@pytest.mark.parametrize("logn,qb,pb,alpha,ml", CHAINS)
def test_prime_chain_matches_oracle(logn, qb, pb, alpha, ml):
    q, p, psi = X.pfx_params_primes(X.make_params(logn, qb, pb, alpha, ml))
    P = O.Params(logn, qb, pb, alpha=alpha, mod_log2=ml)
    assert [int(v) for v in q] == P.q
    assert [int(v) for v in p] == P.p
    assert [int(v) for v in psi] == P.psi_q + P.psi_p


def test_bad_params_are_rejected():
    with pytest.raises(X.PfxError) as e:
        X.pfx_params_primes(X.make_params(12, [55], [50], 1))
    assert e.value.status == X.PFX_EPARAM
    with pytest.raises(X.PfxError):
        X.pfx_params_primes(X.make_params(3, [50], [50], 1))
    with pytest.raises(X.PfxError):
        X.pfx_params_primes(X.make_params(12, [50], [50], 9))


@pytest.mark.parametrize("logn,n_slots,limbs,scale", [(12, 2048, 3, 2.0 ** 40), (16, 32768, 3, 2.0 ** 45),
                                                      (10, 128, 2, 2.0 ** 30)])
def test_encoder_matches_oracle_within_one(logn, n_slots, limbs, scale):
    qb = [50] * limbs
    prm = X.make_params(logn, qb, [50], 1, 17)
    P = O.Params(logn, qb, [50], alpha=1, mod_log2=17)
    z = I.uniform_slots(n_slots, 70) + 1j * I.uniform_slots(n_slots, 71)
    got = X.pfx_encode_words(prm, z.real, z.imag, limbs, scale)
    want = O.encode(P, z, scale, limbs)
    # parity unpinned at rounding ties: the two FFTs may round a tie apart
    d = (got.astype(object) - want.astype(object))
    for i, q in enumerate(P.q):
        dd = [(int(v) + 1) % q - 1 for v in d[i]]
        assert max(abs(v) for v in dd) <= 1
    back = X.pfx_decode_words(prm, want, scale, n_slots)
    assert np.max(np.abs(back - O.decode(P, want, scale, n_slots))) < 1e-9
    assert np.max(np.abs(back - z)) < 2.0 ** -25


def test_decoder_centres_negative_values():
    prm = X.make_params(10, [50, 50], [50], 1, 17)
    P = O.Params(10, [50, 50], [50], alpha=1, mod_log2=17)
    z = -0.75 * np.ones(512)
    w = O.encode(P, z, 2.0 ** 80, 2)       # a value beyond one prime: needs the full CRT
    assert np.allclose(X.pfx_decode_words(prm, w, 2.0 ** 80, 512).real, z, atol=1e-9)


def test_pass_tuning_table(tmp_path):
    """The pass-geometry table (host side): defaults, set/get, the file
    format the autotuner writes, and rejected values."""
    X.pfx_tuning_reset()
    t = X.pfx_tuning_get(16)
    assert [getattr(t, f) for f in X.TUNING_FIELDS] == [2048, 0, 1024, 16, 8, 256, 0, 8, 0]
    X.pfx_tuning_set(15, row_wg256=4096, min_col=32)
    t = X.pfx_tuning_get(15)
    assert (t.row_wg256, t.min_col, t.widen_wg) == (4096, 32, 1024)
    assert X.pfx_tuning_get(16).row_wg256 == 2048
    f = tmp_path / "tuning.txt"
    f.write_text("# comment\n14 0 0 512 8 4 128\n\n16 8192 4096 2048 16 8 512 256 4 2\n")
    X.pfx_tuning_load(str(f))      # a line of seven fields keeps the default ks_fuse
    assert [getattr(X.pfx_tuning_get(14), k) for k in X.TUNING_FIELDS] == [0, 0, 512, 8, 4, 128, 0, 8, 0]
    assert [getattr(X.pfx_tuning_get(16), k) for k in X.TUNING_FIELDS] == [8192, 4096, 2048, 16, 8, 512, 256, 4, 2]
    for bad in ({"min_col": 12}, {"widen_wg": 0}, {"ks_fuse": 64}, {"ks_batch": 9}, {"ks_batch": 0}, {"ks_modup_batch": 9}):
        with pytest.raises(X.PfxError):
            X.pfx_tuning_set(16, **bad)
    f.write_text("16 1 2 3\n")
    with pytest.raises(X.PfxError):
        X.pfx_tuning_load(str(f))
    X.pfx_tuning_reset()
    assert X.pfx_tuning_get(14).widen_wg == 1024
