"""The single-ciphertext key-switching workload, shared by bench.py and the
profiler runs.

N = 2^16, L = 24 ciphertext primes (one 50-bit, 23 near 2^45), K = 4 special
primes of 50 bits, digits of 4 primes (dnum = 6), scale 2^45, a secret with
192 non-zeros, 2^15 real slots uniform in [-1, 1].  One step runs every
operation of the path once on device-resident inputs: forward and inverse NTT
of all limbs of a ciphertext, HMult + relinearisation, rescale 24 -> 23, and
rotations by 2^k for k = 0..14 (15 distinct Galois keys): 16 key switches.

    python -m paper_2412_13269_amd.workload --steps 20 [--calibrate]

runs the step `--steps` times after one warm-up step, the command that
rocprofv3 wraps for kernel traces and counters.  `--query` runs instead the
private query on 2^17 records (4 blocks of 2^15, 8 attributes, degree-7 score,
(7,7,7) sign, InnerSum), blocks interleaved on one stream, eagerly, `--steps`
times after one warm-up run.  `--pfe` runs the private lookup-table
evaluation with ring repacking (PfeWorkload) `--steps` times after one
warm-up run.  `--half-bts [--graph]` runs Half-BTS at N = 2^12
(HalfBtsWorkload) likewise.  `--calibrate` first imports
one ciphertext five times: the library's plain word-to-double copy
(k_u64_to_f64) of one polynomial per launch, 24 limbs = 12 MiB read and 12 MiB
written, the reference against which HBM counters are scaled.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LOGN = 16
Q_BITS = [50] + [45] * 23
P_BITS = [50] * 4
ALPHA = 4
MOD_LOG2 = 17
SCALE = 2.0 ** 45
H = 192
ROT_STEPS = [1 << k for k in range(15)]
KS_PER_STEP = 1 + len(ROT_STEPS)


def key_inputs(moduli, n, beta, seed):
    from . import inputs as I
    return (I.uniform_residues(moduli, n, seed, lead=(beta,)),
            I.gaussian_error((beta, n), seed + 1))


class KsWorkload:
    """Context, keys and operands of the workload, all resident on the device."""

    def __init__(self, log=lambda *a: None):
        from . import inputs as I
        from . import pfx as X
        self.X = X
        prm = X.make_params(LOGN, Q_BITS, P_BITS, ALPHA, MOD_LOG2)
        self.ctx = ctx = X.pfx_ctx_create(prm, 0)
        self.N, self.L, self.K = N, L, K = 1 << LOGN, len(Q_BITS), len(P_BITS)
        self.beta = beta = -(-L // ALPHA)
        q, p, _ = X.pfx_ctx_moduli(ctx, L, K)
        self.q, self.p = q, p
        ext = [int(v) for v in q] + [int(v) for v in p]
        self.st = st = X.pfx_stream_create(ctx)
        log("keygen ...")
        self.s = I.ternary_secret(N, H, 2001)
        self.sk = X.pfx_sk_create(ctx, self.s)
        self.rlk = X.pfx_swk_create(ctx, self.sk, 0, *key_inputs(ext, N, beta, 2002))
        self.gks = []
        for k, step in enumerate(ROT_STEPS):
            g = pow(5, step, 2 * N)
            self.gks.append(X.pfx_swk_create(ctx, self.sk, g, *key_inputs(ext, N, beta, 3000 + 10 * k)))
        self.cts, self.pts = [], []
        for seed in (201, 202):
            pt = X.pfx_encode(ctx, I.uniform_slots(N // 2, seed), None, L, SCALE)
            ct = X.pfx_ct_create(ctx, L, 1)
            X.pfx_encrypt(ctx, self.sk, pt, I.uniform_residues(q, N, seed + 10), I.gaussian_error(N, seed + 20),
                          ct, st)
            self.cts.append(ct)
            self.pts.append(pt)
        self.prod = X.pfx_ct_create(ctx, L, 1)
        self.rot = X.pfx_ct_create(ctx, L, 1)
        self.rots = [X.pfx_ct_create(ctx, L, 1) for _ in ROT_STEPS]     # one output per rotation
        self.words = I.uniform_residues(q, N, 7, lead=(2,))          # one ciphertext: 2 x 24 limbs
        self.dbuf = X.pfx_dev_alloc(ctx, self.words.nbytes)
        X.pfx_memcpy_htod(ctx, self.dbuf, self.words, st)

    def step(self):
        """The 15 rotations (independent key switches, each with its own key
        and output) run as batched key switches (pfx_rotate_batch)."""
        X, ctx, st, L = self.X, self.ctx, self.st, self.L
        X.pfx_ntt(ctx, self.dbuf, 0, L, 2, False, st)
        X.pfx_ntt(ctx, self.dbuf, 0, L, 2, True, st)
        X.pfx_mul_relin(ctx, self.cts[0], self.cts[1], self.rlk, self.prod, st)
        X.pfx_rescale(ctx, self.prod, self.prod, st)
        self.rotations()

    def step_one_by_one(self):
        """The same step with every rotation its own key switch launch sequence."""
        X, ctx, st, L = self.X, self.ctx, self.st, self.L
        X.pfx_ntt(ctx, self.dbuf, 0, L, 2, False, st)
        X.pfx_ntt(ctx, self.dbuf, 0, L, 2, True, st)
        X.pfx_mul_relin(ctx, self.cts[0], self.cts[1], self.rlk, self.prod, st)
        X.pfx_rescale(ctx, self.prod, self.prod, st)
        for r, o in zip(ROT_STEPS, self.rots):
            X.pfx_rotate(ctx, self.cts[0], r, self.gks, o, st)

    def rotations(self):
        self.X.pfx_rotate_batch(self.ctx, [self.cts[0]] * len(ROT_STEPS), ROT_STEPS, self.gks, self.rots, self.st)

    def step_distinct_inputs(self):
        """The same step with every rotation reading a ciphertext of its own
        (copies of the input in separate buffers), so no rotation's input
        reads are served from a cache that a previous entry filled."""
        X, ctx, st, L = self.X, self.ctx, self.st, self.L
        if not hasattr(self, "srcs"):
            self.srcs = [X.pfx_ct_create(ctx, L, 1) for _ in ROT_STEPS]
            for c in self.srcs:
                X.pfx_ct_copy(ctx, self.cts[0], c, st)
        X.pfx_ntt(ctx, self.dbuf, 0, L, 2, False, st)
        X.pfx_ntt(ctx, self.dbuf, 0, L, 2, True, st)
        X.pfx_mul_relin(ctx, self.cts[0], self.cts[1], self.rlk, self.prod, st)
        X.pfx_rescale(ctx, self.prod, self.prod, st)
        X.pfx_rotate_batch(ctx, self.srcs, ROT_STEPS, self.gks, self.rots, st)

    def rotations_one_by_one(self):
        for r, o in zip(ROT_STEPS, self.rots):
            self.X.pfx_rotate(self.ctx, self.cts[0], r, self.gks, o, self.st)

    def calibrate_copy(self, reps=5):
        """Two k_u64_to_f64 launches per import, 24 limbs (12 MiB in, 12 MiB out) each."""
        X = self.X
        for _ in range(reps):
            X.pfx_ct_import(self.ctx, self.words, SCALE, self.rot, self.st)
        X.pfx_sync(self.ctx, self.st)

    def sync(self):
        self.X.pfx_sync(self.ctx, self.st)

    def close(self):
        X = self.X
        for h in self.cts + self.pts + [self.prod, self.rot] + self.rots:
            X.pfx_ct_destroy(h)
        for k in self.gks + [self.rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(self.sk)
        X.pfx_dev_free(self.ctx, self.dbuf)
        X.pfx_stream_destroy(self.ctx, self.st)
        X.pfx_ctx_destroy(self.ctx)


def query_runs(w, steps):
    """The interleaved 4-block query, eagerly, after one warm-up run."""
    import numpy as np
    from . import inputs as I
    from .query import QueryPlan
    X, ctx, st, N, L = w.X, w.ctx, w.st, w.N, w.L
    plan = QueryPlan(4, 8, 7, 3, LOGN - 1, interleave=True)
    x = I.synthetic_database(4 * (N // 2), 8, 301)
    wt, c, t, eta = I.query_parameters(8, 7, 302)
    regs = [X.pfx_ct_create(ctx, L, plan.reg_degree[i]) for i in range(plan.n_regs)]
    for i, v in enumerate(list(wt) + list(c) + [t, eta]):
        pt = X.pfx_encode(ctx, np.full(N // 2, v), None, L, SCALE)
        X.pfx_encrypt(ctx, w.sk, pt, I.uniform_residues(w.q, N, 400 + 2 * i), I.gaussian_error(N, 401 + 2 * i),
                      regs[i], st)
        X.pfx_ct_destroy(pt)
    db = [X.pfx_encode(ctx, x[b * (N // 2):(b + 1) * (N // 2), a], None, L, SCALE) for b in range(4) for a in range(8)]
    X.pfx_sync(ctx, st)
    import time
    time.sleep(0.5)      # an idle gap that marks the end of the setup in kernel traces
    for _ in range(steps + 1):
        X.pfx_run_circuit(ctx, plan.ops, regs, plan.n_inputs, db, w.rlk, w.gks, X.RUN_EAGER, st)
    X.pfx_sync(ctx, st)
    for h in regs + db:
        X.pfx_ct_destroy(h)
    return plan


# Phase one of the paper's exploration (Sec. 3.4, Sec. 4.2, Alg. 1): ring
# degree 2^12, one 50-bit ciphertext prime and one 50-bit special prime (the
# shape of the paper's Set I; primes 1 mod 2^17, so the first one is also the
# first prime of the N = 2^16 chain above and the outputs can be merged into
# that ring, Sec. 3.3), 16 encrypted lookup tables of 4096 entries (scale
# 2^40), 2^19 records of 16 attributes with uniform discretised values,
# repacked 4096 records per output ciphertext (128 groups).
PFE_LOGN = 12
PFE_TABLES = 16
PFE_RECORDS = 1 << 19
PFE_DELTA = 2.0 ** 40


class PfeWorkload:
    """Context, repacking keys, encrypted tables and the record matrix of the
    lookup-table phase, all resident on the device; run() is one pass over
    every record (pfx_pfe_repack)."""

    def __init__(self, records=PFE_RECORDS, tables=PFE_TABLES, log=lambda *a: None):
        import numpy as np
        from . import inputs as I
        from . import pfx as X
        from .repack import repack_keys_needed
        self.X = X
        prm = X.make_params(PFE_LOGN, [50], [50], 1, MOD_LOG2)
        self.ctx = ctx = X.pfx_ctx_create(prm, 0)
        self.N = N = 1 << PFE_LOGN
        self.records, self.m = records, tables
        self.groups = -(-records // N)
        q, p, _ = X.pfx_ctx_moduli(ctx, 1, 1)
        self.st = st = X.pfx_stream_create(ctx)
        self.s = s = I.ternary_secret(N, None, 801)
        self.sk = X.pfx_sk_create(ctx, s)
        log("pfe keygen ...")
        self.gks = []
        for i, g in enumerate(repack_keys_needed(PFE_LOGN)):
            a, e = key_inputs(list(q) + list(p), N, 1, 810 + 2 * i)
            self.gks.append(X.pfx_swk_create(ctx, self.sk, g, a, e))
        self.tables = []
        for l in range(tables):
            f = I.uniform_slots(N, 850 + l)
            u = np.empty(N)
            u[0] = f[0]
            u[1:] = -f[N - np.arange(1, N)]
            coef = np.rint(PFE_DELTA * u).astype(np.int64)          # u_f scaled and rounded
            words = np.stack([coef % np.int64(qi) for qi in q]).astype(np.uint64)
            pt = X.pfx_pt_import(ctx, words, PFE_DELTA)
            ct = X.pfx_ct_create(ctx, 1, 1)
            X.pfx_encrypt(ctx, self.sk, pt, I.uniform_residues(q, N, 900 + 2 * l), I.gaussian_error(N, 901 + 2 * l),
                          ct, st)
            X.pfx_ct_destroy(pt)
            self.tables.append(ct)
        exps = I.rng(950).integers(0, N, size=(records, tables)).astype(np.int64)
        self.d_exps = X.pfx_dev_alloc(ctx, exps.nbytes)
        X.pfx_memcpy_htod(ctx, self.d_exps, exps, st)
        self.outs = [X.pfx_ct_create(ctx, 1, 1) for _ in range(self.groups)]
        X.pfx_sync(ctx, st)

    @property
    def key_switches(self) -> int:
        return self.groups * (self.N - 1)

    def run(self):
        self.X.pfx_pfe_repack(self.ctx, self.tables, self.d_exps, self.records, self.gks, self.outs, self.st)

    def sync(self):
        self.X.pfx_sync(self.ctx, self.st)

    def close(self):
        X = self.X
        for h in self.tables + self.outs:
            X.pfx_ct_destroy(h)
        for k in self.gks:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(self.sk)
        X.pfx_dev_free(self.ctx, self.d_exps)
        X.pfx_stream_destroy(self.ctx, self.st)
        X.pfx_ctx_destroy(self.ctx)


class HalfBtsWorkload:
    """Half-BTS (Sec. 4.3, App. A.3-A.4) at N = 2^12 over the 50 + 13 x 45-bit
    chain with 4 special primes: a one-limb coefficient-encoded ciphertext,
    the 95 Galois keys of CoeffsToSlots (n1 = 64: 63 baby steps, 31 giant
    steps) and of the conjugation, the relinearisation key, the 2048
    diagonals of B/2 and the op list of the rest (degree-24 EvalMod, r = 3),
    all made by the library from seeded inputs."""

    def __init__(self, log=print):
        import numpy as np
        from numpy.polynomial import chebyshev as _cheb

        from . import boot as HB
        from . import inputs as I
        from . import pfx as X
        self.HB, self.X = HB, X
        logn, qb, pb, alpha, self.n1 = 12, [50] + [45] * 13, [50] * 4, 4, 64
        self.qb, self.pb = qb, pb
        self.ctx = X.pfx_ctx_create(X.make_params(logn, qb, pb, alpha, 17), 0)
        self.st = X.pfx_stream_create(self.ctx)
        N, L = 1 << logn, len(qb)
        self.N, self.L = N, L
        q, pr, _ = X.pfx_ctx_moduli(self.ctx, L, len(pb))
        self.q0 = float(q[0])
        ext = [int(v) for v in q] + [int(v) for v in pr]
        beta = -(-L // alpha)
        self.sk = X.pfx_sk_create(self.ctx, I.ternary_secret(N, 32, 801))
        n = N // 2
        steps = sorted({k % self.n1 for k in range(1, n)} - {0}) + \
            sorted({self.n1 * (k // self.n1) for k in range(n)} - {0})
        gs = sorted({pow(5, k, 2 * N) for k in steps}) + [2 * N - 1]
        log(f"half-BTS keygen ({len(gs)} Galois keys) ...")
        self.gks = [X.pfx_swk_create(self.ctx, self.sk, g, *key_inputs(ext, N, beta, 900 + 2 * i))
                    for i, g in enumerate(gs)]
        self.rlk = X.pfx_swk_create(self.ctx, self.sk, 0, *key_inputs(ext, N, beta, 802))
        delta, sd = 2.0 ** 40, 2.0 ** 40
        self.diags = [X.pfx_encode(self.ctx, d.real, d.imag, L, sd) for d in HB.c2s_half_diagonals(N)]
        a = (8.0 + 0.25) / 8
        self.plan = HB.HalfBootPlan(N, _cheb.chebinterpolate(lambda v: np.cos(2 * np.pi * a * v), 24), 3, 8.0,
                                    self.q0 / delta)
        # one register set per mode: a captured graph stays bound to its registers
        self.regs = {m: [X.pfx_ct_create(self.ctx, L, 1) for _ in range(self.plan.n_regs)]
                     for m in (X.RUN_EAGER, X.RUN_GRAPH)}
        self.x = X.pfx_ct_create(self.ctx, 1, 1)
        v = I.uniform_slots(N, 804)
        m = np.mod(np.round(v * delta).astype(np.int64), np.int64(q[0])).astype(np.uint64)[None, :]
        pt = X.pfx_pt_import(self.ctx, m, delta)
        X.pfx_encrypt(self.ctx, self.sk, pt, I.uniform_residues([int(q[0])], N, 805), I.gaussian_error(N, 806),
                      self.x)
        X.pfx_ct_destroy(pt)
        self.galois_keys = len(gs)

    def run(self, mode=0):
        """mode: RUN_EAGER (0) or RUN_GRAPH for the op-list part."""
        self.HB.half_bootstrap(self.ctx, self.x, self.L, self.q0, self.diags, self.n1, self.gks, self.rlk,
                               self.plan, self.regs[mode], self.st, mode)

    def run_circuit(self, mode=0):
        self.X.pfx_run_circuit(self.ctx, self.plan.ops, self.regs[mode], self.plan.n_inputs, [], self.rlk, self.gks,
                          mode, self.st)

    def result_words(self, mode):
        return self.X.pfx_ct_export(self.ctx, self.regs[mode][self.plan.out], self.N, self.st)

    def sync(self):
        self.X.pfx_sync(self.ctx, self.st)

    def describe(self):
        return {"N": self.N, "limbs": self.L, "special_primes": len(self.pb), "diagonals": self.N // 2,
                "n1": self.n1, "galois_keys": self.galois_keys, "evalmod_degree": 24, "double_angles": 3,
                "depth": self.plan.depth}

    def close(self):
        X = self.X
        for regs in self.regs.values():
            for h in regs:
                X.pfx_ct_destroy(h)
        for h in self.diags + [self.x]:
            X.pfx_ct_destroy(h)
        for k in self.gks + [self.rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(self.sk)
        X.pfx_stream_destroy(self.ctx, self.st)
        X.pfx_ctx_destroy(self.ctx)


class FactorisedHalfBtsWorkload:
    """Half-BTS at the paper's ring, N = 2^16, over the 24 + 4 prime chain:
    ModRaise, CoeffsToSlots in 3 sparse levels (factorised, slots left in
    bit-reversed order), the conjugate split and two EvalMod lanes (degree 24,
    K = 12, four double angles); a sparse secret of 32 non-zeros (the paper's
    bootstrapping secret), seeded keys (39 Galois keys and the
    relinearisation key), all made by the library.  log_r > 0: sparse
    packing on N / 2^(log_r + 1) slots, the trace-like map after ModRaise."""

    def __init__(self, log=print, levels=3, log_r=0):
        import math

        import numpy as np
        from numpy.polynomial import chebyshev as _cheb

        from . import boot as HB
        from . import inputs as I
        from . import pfx as X
        self.HB, self.X, self.np = HB, X, np
        logn, qb, pb = LOGN, Q_BITS, P_BITS
        self.ctx = X.pfx_ctx_create(X.make_params(logn, qb, pb, ALPHA, MOD_LOG2), 0)
        self.st = X.pfx_stream_create(self.ctx)
        N, L = 1 << logn, len(qb)
        self.N, self.L, self.levels, self.log_r = N, L, levels, log_r
        self.n = N >> (log_r + 1)
        q, _, _ = X.pfx_ctx_moduli(self.ctx, L, len(pb))
        q = [int(v) for v in q]
        self.q0 = float(q[0])
        seed = b"half-bts at 2^16".ljust(32, b".")
        self.sk = X.pfx_keygen_secret(self.ctx, seed, 32)
        self.rlk = X.pfx_keygen_relin(self.ctx, self.sk, seed)
        fs = HB.c2s_factor_stages(N, levels, 0.5 / (1 << log_r), self.n)
        rots = set(HB.trace_rotations(N, log_r))
        for steps, _ in fs:
            rots |= HB.bsgs_rotations(N, steps, HB.bsgs_n1(steps))
        log(f"half-BTS at N=2^16: keygen ({len(rots) + 1} Galois keys) ...")
        self.gks = X.pfx_keygen_galois(self.ctx, self.sk, sorted(rots), True, seed)
        self.delta, sd, K, r = 2.0 ** 40, 2.0 ** 40, 12.0, 4
        self.stages, self.pts = [], []
        for i, (steps, diags) in enumerate(fs):
            scale = sd if i == 0 else float(q[L - 1 - i])
            pts = [X.pfx_encode(self.ctx, d.real, d.imag, L, scale) for d in diags]
            self.pts += pts
            self.stages.append((steps, pts, HB.bsgs_n1(steps)))
        a = (K + 0.25) / 2 ** r
        self.plan = HB.HalfBootPlan(N, _cheb.chebinterpolate(lambda v: np.cos(2 * math.pi * a * v), 24), r, K,
                                    self.q0 / self.delta)
        self.regs = {m: [X.pfx_ct_create(self.ctx, L, 1) for _ in range(self.plan.n_regs)]
                     for m in (X.RUN_EAGER, X.RUN_GRAPH)}
        self.x = X.pfx_ct_create(self.ctx, 1, 1)
        self.v = I.uniform_slots(N, 920)
        m = np.mod(np.round(self.v * self.delta).astype(np.int64), np.int64(q[0])).astype(np.uint64)[None, :]
        pt = X.pfx_pt_import(self.ctx, m, self.delta)
        X.pfx_encrypt(self.ctx, self.sk, pt, I.uniform_residues(q[:1], N, 921), I.gaussian_error(N, 922), self.x)
        X.pfx_ct_destroy(pt)
        self.galois_keys = len(self.gks)
        self.diagonals = [len(s[0]) for s in fs]

    def run(self, mode=0):
        self.HB.half_bootstrap_factorised(self.ctx, self.x, self.L, self.q0, self.stages, self.gks, self.rlk,
                                          self.plan, self.regs[mode], self.st, mode, self.log_r)

    def run_circuit(self, mode=0):
        self.X.pfx_run_circuit(self.ctx, self.plan.ops, self.regs[mode], self.plan.n_inputs, [], self.rlk,
                               self.gks, mode, self.st)

    def result_words(self, mode):
        return self.X.pfx_ct_export(self.ctx, self.regs[mode][self.plan.out], self.N, self.st)

    def max_error(self, mode=0) -> float:
        """Largest slot error of the last result against the message's
        coefficients (those of the subring for sparse packing) in bit-reversed
        slot order, over all N/2 slots."""
        np, X = self.np, self.X
        n, r = self.n, 1 << self.log_r
        m = X.pfx_decrypt(self.ctx, self.sk, self.regs[mode][self.plan.out])
        got = X.pfx_decode(self.ctx, m, self.N // 2)
        X.pfx_ct_destroy(m)
        rev = np.array([int(format(j, f"0{n.bit_length() - 1}b")[::-1], 2) for j in range(n)])
        sub = self.v[::r]
        return float(np.max(np.abs(got - np.tile((sub[:n] + 1j * sub[n:])[rev], r))))

    def sync(self):
        self.X.pfx_sync(self.ctx, self.st)

    def describe(self):
        return {"N": self.N, "limbs": self.L, "special_primes": len(P_BITS), "c2s_levels": self.levels,
                "diagonals_per_level": self.diagonals, "galois_keys": self.galois_keys, "secret_weight": 32,
                "evalmod_degree": 24, "evalmod_K": 12, "double_angles": 4,
                "depth": self.plan.depth + self.levels - 1, "slot_order": "bit-reversed", "slots": self.n,
                "trace_automorphisms": self.log_r}

    def close(self):
        X = self.X
        for h in self.pts + [self.x] + [r for regs in self.regs.values() for r in regs]:
            X.pfx_ct_destroy(h)
        for k in self.gks + [self.rlk]:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(self.sk)
        X.pfx_stream_destroy(self.ctx, self.st)
        X.pfx_ctx_destroy(self.ctx)


def calibrate_copy_standalone(reps=5):
    """The copy of KsWorkload.calibrate_copy (k_u64_to_f64 over 24 limbs of
    N = 2^16: 12 MiB in, 12 MiB out per launch, two per import) on a context of
    the same parameters without keys, for runs of the other workloads."""
    from . import inputs as I
    from . import pfx as X
    ctx = X.pfx_ctx_create(X.make_params(LOGN, Q_BITS, P_BITS, ALPHA, MOD_LOG2), 0)
    q, _, _ = X.pfx_ctx_moduli(ctx, len(Q_BITS), len(P_BITS))
    words = I.uniform_residues(q, 1 << LOGN, 9, lead=(2,))
    ct = X.pfx_ct_create(ctx, len(Q_BITS), 1)
    for _ in range(reps):
        X.pfx_ct_import(ctx, words, SCALE, ct)
    X.pfx_sync(ctx)
    X.pfx_ct_destroy(ct)
    X.pfx_ctx_destroy(ctx)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--calibrate", action="store_true")
    ap.add_argument("--query", action="store_true")
    ap.add_argument("--pfe", action="store_true")
    ap.add_argument("--half-bts", action="store_true")
    ap.add_argument("--half-bts-n16", action="store_true", help="the factorised Half-BTS at N = 2^16")
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--rotations-only", action="store_true",
                    help="each step is the 15 rotations alone, one key switch launch sequence each "
                         "(after the copy calibration, if asked)")
    ap.add_argument("--one-by-one", action="store_true",
                    help="the step with its rotations one at a time instead of batched")
    args = ap.parse_args()
    if args.half_bts_n16:
        from . import pfx as X
        import time
        w = FactorisedHalfBtsWorkload(log=lambda *a: print(*a, flush=True))
        w.run(X.RUN_EAGER)
        w.sync()
        time.sleep(0.5)  # an idle gap that marks the end of the setup in kernel traces
        for _ in range(args.steps):
            w.run(X.RUN_EAGER)
        w.sync()
        print(f"{args.steps} Half-BTS runs done at N=2^16", flush=True)
        w.close()
        return
    if args.half_bts:
        from . import pfx as X
        mode = X.RUN_GRAPH if args.graph else X.RUN_EAGER
        import time
        if args.calibrate:
            calibrate_copy_standalone()
            print("copy calibration done", flush=True)
        w = HalfBtsWorkload(log=lambda *a: print(*a, flush=True))
        w.run(mode)
        w.sync()
        time.sleep(0.5)  # an idle gap that marks the end of the setup in kernel traces
        for _ in range(args.steps):
            w.run(mode)
        w.sync()
        print(f"{args.steps} Half-BTS runs done at N=2^12", flush=True)
        w.close()
        return
    if args.pfe:
        import time
        if args.calibrate:
            calibrate_copy_standalone()
            print("copy calibration done", flush=True)
        w = PfeWorkload(log=lambda *a: print(*a, flush=True))
        w.run()
        w.sync()
        time.sleep(0.5)  # an idle gap that marks the end of the setup in kernel traces
        for _ in range(args.steps):
            w.run()
        w.sync()
        print(f"{args.steps} lookup-table passes done ({w.records} records, {w.key_switches} key switches each)",
              flush=True)
        w.close()
        return
    w = KsWorkload(log=lambda *a: print(*a, flush=True))
    if args.query:
        plan = query_runs(w, args.steps)
        print(f"{args.steps} queries done ({plan.key_switches} key switches each)", flush=True)
        w.close()
        return
    if args.calibrate:
        w.calibrate_copy()
        print("copy calibration done", flush=True)
    step = w.rotations_one_by_one if args.rotations_only else (w.step_one_by_one if args.one_by_one else w.step)
    step()
    w.sync()
    for _ in range(args.steps):
        step()
    w.sync()
    if args.rotations_only:
        print(f"{args.steps + 1} steps of {len(ROT_STEPS)} rotations done "
              f"({(args.steps + 1) * len(ROT_STEPS)} rotations after the calibration)", flush=True)
    else:
        print(f"{args.steps} steps done ({KS_PER_STEP * args.steps} key switches)", flush=True)
    w.close()


if __name__ == "__main__":
    main()
