"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch each one.  A pin that passes on a broken oracle would prove nothing."""
import math

import numpy as np
import pytest

from oracle import ckks as O
from tests import test_oracle_pins as T


def _expect_fail(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_mod_down_without_rounding_is_caught(monkeypatch):
    def floor_mod_down(P, x, level):
        Pb = math.prod(P.p)
        r = O.bconv(x[level:], P.p, P.mods(level))
        qs = P.mods(level)
        return O.smul(O.sub(x[:level], r, qs), [pow(Pb, -1, q) for q in qs], qs)
    monkeypatch.setattr(O, "mod_down", floor_mod_down)
    _expect_fail(T.test_mod_down_rounds_up_to_the_fast_conversion_overflow)


def test_rescale_truncating_is_caught(monkeypatch):
    orig = O.add_int
    monkeypatch.setattr(O, "add_int", lambda a, vals, mods: orig(a, [0] * len(vals), mods))
    _expect_fail(T.test_rescale_is_rounded_division_by_last_prime)


def test_wrong_slot_generator_is_caught(monkeypatch):
    monkeypatch.setattr(O, "_slot_exponents", lambda n: np.array([pow(3, j, 4 * n) for j in range(n)]))
    _expect_fail(T.test_encoding_inverts_the_slot_evaluation, 8)


def test_automorphism_without_sign_is_caught(monkeypatch):
    def unsigned_auto(a, g, mods, logn):
        n = 1 << logn
        out = np.empty_like(a)
        for i in range(n):
            out[:, (i * g) % n] = a[:, i]
        return out
    monkeypatch.setattr(O, "automorphism", unsigned_auto)
    _expect_fail(T.test_automorphism_matches_substitution_and_composes)


def test_gadget_without_p_is_caught(monkeypatch):
    def swk_gen_no_p(P, s, s_from_ext, a, e, galois):
        mods = P.ext_mods(P.L)
        s_ext = O.secret_rns(P, s, mods)
        Qb = math.prod(P.q)
        bs = []
        for j, D in enumerate(P.digits(P.L)):
            Qj = math.prod(P.q[i] for i in D)
            w_j = (Qb // Qj) * pow(Qb // Qj, -1, Qj)
            b = O.add(O.neg(O.polymul(a[j], s_ext, mods, P.ext_psis(P.L), P.logn), mods),
                      O.from_ints(e[j], mods), mods)
            bs.append(O.add(b, O.smul(s_from_ext, [w_j % m for m in mods], mods), mods))
        return O.SwitchKey(np.stack(bs), a, galois)
    monkeypatch.setattr(O, "swk_gen", swk_gen_no_p)
    _expect_fail(T.test_switching_key_decrypts_to_gadget_times_secret)


def test_cyclic_instead_of_negacyclic_is_caught(monkeypatch):
    # a root of order N (cyclic convolution) instead of 2N breaks the product pin
    def cyclic_root(q, n):
        g = 2
        while True:
            x = pow(g, (q - 1) // n, q)
            if pow(x, n // 2, q) == q - 1:
                return x
            g += 1
    monkeypatch.setattr(O, "find_psi", cyclic_root)
    _expect_fail(T.test_ntt_product_is_negacyclic_convolution, 3)


# ---- lookup-table evaluation and ring repacking (oracle/repack.py)
from oracle import repack as RP
from tests import test_repack_oracle as TR


def test_monomial_without_wrap_sign_is_caught(monkeypatch):
    def unsigned(a, k, mods, N):
        d = (np.arange(N) + k % (2 * N)) % N
        out = np.empty_like(a)
        out[:, d] = a
        return out
    monkeypatch.setattr(RP, "monomial", unsigned)
    _expect_fail(TR.test_lookup_constant_coefficient_is_f_of_the_point)


def test_repack_without_inverse_n_is_caught(monkeypatch):
    monkeypatch.setattr(RP, "ct_mul_inv_n", lambda P, x: x)
    _expect_fail(TR.test_repack_decrypts_to_the_constant_coefficients, 32)


def test_repack_with_shifted_galois_order_is_caught(monkeypatch):
    monkeypatch.setattr(RP, "repack_galois", lambda P, i: pow(5, 1 << i, 2 * P.N))
    _expect_fail(TR.test_repack_decrypts_to_the_constant_coefficients, 32)


def test_repack_with_wrong_sign_inside_the_automorphism_is_caught(monkeypatch):
    orig_sub = O.ct_sub
    monkeypatch.setattr(O, "ct_sub", lambda P, x, y: O.ct_add(P, x, y))
    try:
        _expect_fail(TR.test_repack_decrypts_to_the_constant_coefficients, 32)
    finally:
        monkeypatch.setattr(O, "ct_sub", orig_sub)


def test_score_with_reversed_exponent_is_caught(monkeypatch):
    orig = RP.ct_monomial
    monkeypatch.setattr(RP, "ct_monomial", lambda P, x, k: orig(P, x, -k))
    _expect_fail(TR.test_score_constant_coefficient_is_the_sum_of_the_tables_at_the_points)


def test_grouped_repack_dropping_the_tail_group_is_caught(monkeypatch):
    monkeypatch.setattr(RP, "repack_groups",
                        lambda P, cts, gks: [RP.repack(P, cts[g:g + P.N], gks) for g in range(0, len(cts) - P.N + 1, P.N)])
    _expect_fail(TR.test_grouped_repack_packs_each_group)


# ---- ring merging (oracle/merge.py)
from oracle import merge as MG
from tests import test_merge_oracle as TM


def test_embedding_by_zero_padding_is_caught(monkeypatch):
    def padded(a, r):
        out = np.zeros((a.shape[0], a.shape[1] * r), dtype=a.dtype)
        out[:, :a.shape[1]] = a
        return out
    monkeypatch.setattr(MG, "embed_poly", padded)
    _expect_fail(TM.test_embedding_is_a_ring_homomorphism)


def test_merge_without_the_input_shift_is_caught(monkeypatch):
    orig = RP.monomial
    monkeypatch.setattr(RP, "monomial", lambda a, k, mods, N: orig(a, 0, mods, N))
    _expect_fail(TM.test_merge_places_coefficient_j_of_input_i_at_j_r_plus_i, 4)


# ---- hoisted automorphisms (oracle/hoist.py)
from tests import test_hoist_oracle as THo


def test_hoisting_without_permuting_the_digits_is_caught(monkeypatch):
    from oracle import hoist as HO
    setup = THo.setup.__wrapped__()
    orig = O.automorphism

    def skip_digits(a, g, mods, logn):
        # the digit polynomials are the calls over the extended basis
        return a if len(mods) > setup[0].L else orig(a, g, mods, logn)
    monkeypatch.setattr(O, "automorphism", skip_digits)
    _expect_fail(THo.test_hoisted_rotations_decrypt_to_the_rotated_slots, setup)


# ---- BSGS linear transform (oracle/linear.py)
from tests import test_linear_oracle as TL


def test_transform_with_diagonals_rotated_forward_is_caught(monkeypatch):
    from oracle import linear as LTm
    monkeypatch.setattr(LTm, "giant_back", lambda P, n1, j: O.galois_element(P, n1 * j))
    _expect_fail(TL.test_transform_is_the_matrix_vector_product, TL.setup.__wrapped__(), 4)


# ---- ModRaise (oracle/boot.py)
from tests import test_boot_oracle as TB


def test_mod_raise_without_centring_is_caught(monkeypatch):
    from oracle import boot as BO
    monkeypatch.setattr(BO, "lift", lambda words, q0: words.astype(np.int64))
    _expect_fail(TB.test_raised_residues_are_the_centred_lift)


def test_trace_with_wrong_elements_is_caught(monkeypatch):
    from oracle import boot as BO
    orig = BO.trace_galois
    monkeypatch.setattr(BO, "trace_galois", lambda P, t: orig(P, t) - 2)
    _expect_fail(TB.test_trace_keeps_multiples_of_r_times_r_and_cancels_the_rest)


# ---- degree-15 sign stage (oracle/query.py)
from oracle import query as QO
from tests import test_query_oracle as TQ


def test_sign_coefficient_typo_is_caught(monkeypatch):
    c, den = QO.SIGN[15]
    bad = dict(QO.SIGN)
    bad[15] = (c[:3] + (c[3] + 10,) + c[4:], den)
    monkeypatch.setattr(QO, "SIGN", bad)
    _expect_fail(TQ.test_f15_closed_form)


# ---- EvalMod (oracle/evalmod.py)
from tests import test_evalmod_oracle as TE


def test_evalmod_with_a_wrong_chebyshev_split_is_caught(monkeypatch):
    from oracle import evalmod as EM
    monkeypatch.setattr(EM, "cheb_index_pair", lambda k: (k - 1, 1))
    _expect_fail(TE.test_fp64_steps_are_the_scaled_sine)


def test_evalmod_with_unmatched_scales_is_caught(monkeypatch):
    # constants taken at the next prime's scale whatever the target: the
    # terms of each sum meet at scales that differ by the primes' offsets
    from oracle import evalmod as EM
    monkeypatch.setattr(EM, "mul_const_like", lambda P, x, value, target: EM.mul_const_next(P, x, value))
    _expect_fail(TE.test_homomorphic_evalmod_decrypts_to_its_fp64_steps, TE.homomorphic_setup())


def test_evalmod_with_a_rescale_per_term_and_one_per_sum_mixed_is_caught(monkeypatch):
    # each term rescaled on its own before it joins a sum formed for one
    # rescale: the terms land a prime below the sum's scale
    from oracle import evalmod as EM
    orig = EM.mul_const_like
    monkeypatch.setattr(EM, "mul_const_like",
                        lambda P, x, value, target: EM.O.rescale(P, orig(P, x, value, target)))
    _expect_fail(TE.test_homomorphic_evalmod_decrypts_to_its_fp64_steps, TE.homomorphic_setup())


# ---- Half-BTS (oracle/boot.py)
def test_half_bootstrap_with_the_wrong_imaginary_unit_is_caught(monkeypatch):
    # X^(N/2) (+i) where the split of the imaginary part needs X^(3N/2) (-i)
    from oracle import repack as RP
    from tests import test_boot_oracle as TB
    orig = RP.ct_monomial
    monkeypatch.setattr(RP, "ct_monomial", lambda P, x, k: orig(P, x, P.N // 2 if k == 3 * P.N // 2 else k))
    _expect_fail(TB.test_half_bootstrap_puts_the_coefficients_in_the_slots)


# ---- the seeded sampler (oracle/sampler.py)
from oracle import sampler as SM
from tests import test_sampler_oracle as TS


def test_uniform_mask_one_bit_short_is_caught(monkeypatch):
    orig = SM.uniform_poly

    def short(seed, tag, index, limb, q, n):
        half = 1 << ((q - 1).bit_length() - 1)
        return orig(seed, tag, index, limb, max(2, half), n)     # masks one bit fewer, never reaches [half, q)
    monkeypatch.setattr(SM, "uniform_poly", short)
    _expect_fail(TS.test_uniform_is_uniform)


def test_gaussian_table_without_doubling_is_caught(monkeypatch):
    def one_sided(sigma=SM.SIGMA, bound=SM.BOUND):
        rho = [math.exp(-(k * k) / (2.0 * sigma * sigma)) for k in range(bound + 1)]
        total, acc, t = sum(rho), 0.0, []
        for k in range(bound):
            acc += rho[k] / total
            t.append(int(math.floor(acc * 2.0 ** 63)))
        return t + [1 << 63]
    monkeypatch.setattr(SM, "gaussian_table", one_sided)
    _expect_fail(TS.test_gaussian_table_and_moments)


def test_sparse_secret_without_signs_is_caught(monkeypatch):
    orig = SM.ternary_sparse
    monkeypatch.setattr(SM, "ternary_sparse", lambda seed, tag, index, n, h: np.abs(orig(seed, tag, index, n, h)))
    _expect_fail(TS.test_ternary_secrets)


# ---- the composite minimax sign design (oracle/remez.py)
from oracle import remez as RZ
from tests import test_remez_oracle as TRZ


def test_composite_without_normalisation_is_caught(monkeypatch):
    orig = RZ.remez_sign_stage

    def no_norm(alpha, degree=15, stages=None, beta=None, max_stages=12):
        tau, cs, es, taus = 2.0 ** -alpha, [], [], []
        for _ in range(stages):
            c, e, _ = orig(degree, tau)
            cs.append(c)                      # image left in [1 - e, 1 + e]: the next stage leaves its domain
            es.append(e)
            taus.append(tau)
            tau = 1.0 - e
        return cs, es, taus
    monkeypatch.setattr(RZ, "composite_sign", no_norm)
    _expect_fail(TRZ.test_stages_stay_in_the_unit_interval)


def test_remez_with_one_reference_point_short_is_caught(monkeypatch):
    def short(degree, tau, iters=80, grid=20000):
        c, e, ref = RZ.__dict__["_orig_remez"](degree - 2 if degree > 1 else degree, tau, iters, grid)
        return c, e, ref
    monkeypatch.setitem(RZ.__dict__, "_orig_remez", RZ.remez_sign_stage)
    monkeypatch.setattr(RZ, "remez_sign_stage", short)
    _expect_fail(TRZ.test_equioscillation, 15, 2.0 ** -8)


# ---- the minimax threshold stages of the query (oracle/query.py)


def test_minimax_stage_with_a_wrong_power_is_caught(monkeypatch):
    tree = dict(QO.ODD_TREE)
    tree[7] = (4, 2)                          # x^6 where x^7 belongs
    monkeypatch.setattr(QO, "ODD_TREE", tree)
    _expect_fail(TQ.test_minimax_stage_decrypts_to_the_polynomial)


def test_minimax_stage_with_terms_at_unmatched_scales_is_caught(monkeypatch):
    # every term taken at the next prime's scale instead of the sum's
    monkeypatch.setattr(QO, "mul_const_like", lambda P, x, value, target_scale: QO.mul_const_next(P, x, value))
    _expect_fail(TQ.test_minimax_stage_decrypts_to_the_polynomial)


def test_global_threshold_with_the_difference_reversed_is_caught(monkeypatch):
    orig = QO.O.ct_sub
    monkeypatch.setattr(QO.O, "ct_sub", lambda P, a, b: orig(P, b, a))
    _expect_fail(TQ.test_global_threshold_decides_counts_two_away)


# ---- the factorised CoeffsToSlots (oracle/boot.py)
from oracle import boot as BOOT


def test_factorised_c2s_with_stages_in_reverse_order_is_caught(monkeypatch):
    orig = BOOT.c2s_factor_matrices
    monkeypatch.setattr(BOOT, "c2s_factor_matrices",
                        lambda P, levels, factor=1.0, n=None: orig(P, levels, factor, n)[::-1])
    _expect_fail(TB.test_factorised_c2s_multiplies_out_to_the_dense_matrix, 6, 3)


def test_factorised_c2s_with_a_wrong_twiddle_is_caught(monkeypatch):
    from scipy import sparse
    import numpy as np

    def wrong(P, s, n=None):                # the root's exponent taken mod 2^(s+1) instead of 2^(s+2)
        n = n or P.N // 2
        ln, lh = 1 << s, 1 << (s - 1)
        rows, cols, vals = [], [], []
        for i in range(0, n, ln):
            for j in range(lh):
                w = np.exp(2j * np.pi * (pow(5, j, 2 * ln)) / (4 * ln))
                lo, hi = i + j, i + j + lh
                rows += [lo, lo, hi, hi]
                cols += [lo, hi, lo, hi]
                vals += [0.5, 0.5, 0.5 / w, -0.5 / w]
        return sparse.csr_matrix((vals, (rows, cols)), shape=(n, n), dtype=complex)
    monkeypatch.setattr(BOOT, "fft_stage_inverse", wrong)
    _expect_fail(TB.test_factorised_c2s_multiplies_out_to_the_dense_matrix, 6, 1)


def test_sparse_c2s_with_the_full_ring_roots_is_caught(monkeypatch):
    # the stages of n < N/2 slots built on the N/2 slot roots' twiddles
    orig = BOOT.fft_stage_inverse

    def wrong(P, s, n=None):
        full = orig(P, s + (P.N // 2).bit_length() - (n or P.N // 2).bit_length(), None)
        return full[:n, :n] if n else full
    monkeypatch.setattr(BOOT, "fft_stage_inverse", wrong)
    _expect_fail(TB.test_sparse_factorised_c2s_multiplies_out_to_the_dense_matrix, 6, 8, 1)


def test_sparse_half_bootstrap_without_the_trace_is_caught(monkeypatch):
    monkeypatch.setattr(BOOT, "subring_trace", lambda P, x, log_r, keys: x)
    _expect_fail(TB.test_sparse_half_bootstrap_puts_the_subring_coefficients_in_the_slots)


def test_sparse_half_bootstrap_with_a_short_trace_is_caught(monkeypatch):
    orig = BOOT.subring_trace
    monkeypatch.setattr(BOOT, "subring_trace", lambda P, x, log_r, keys: orig(P, x, log_r - 1, keys))
    _expect_fail(TB.test_sparse_half_bootstrap_puts_the_subring_coefficients_in_the_slots)
