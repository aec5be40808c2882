"""Autotuner of the NTT pass geometry per ring degree (run on the GPU).

For each ring degree 2^12 .. 2^16 on the 24 + 4 prime chain (digits of four
primes) it times, at 24, 13 and 4 limbs, the operations whose launches the
geometry shapes: HMult + relin + rescale (the batched form's entry), a
rotation, and the forward and inverse transform of a ciphertext's limbs.  The
objective is the sum of their median device times (HIP events, 3 warm-up and
`reps` timed calls each).  The search is coordinate descent over the fields of
pfx_pass_tuning (two sweeps, each field over its candidate values with the
others fixed); the winner must beat the defaults by more than `min_gain` on a
re-measurement, else the defaults are kept.  The result goes to tuning.txt
next to libpfx.so, which the library loads on its first context.

    python -m paper_2412_13269_amd.autotune [--lognums 12 13 14 15 16] [--reps 10]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from paper_2412_13269_amd import inputs as I
from paper_2412_13269_amd import pfx as X

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "tuning.txt")
QB, PB, ALPHA, ML = [50] + [45] * 23, [50] * 4, 4, 17
LEVELS = (24, 13, 4)
DEFAULT = {"row_wg256": 2048, "col_wg256": 0, "widen_wg": 1024, "min_col": 16, "min_col_special": 8,
           "rs_widen_wg": 256, "ks_fuse": 0, "ks_batch": 8, "ks_modup_batch": 0}
CANDIDATES = {"row_wg256": [0, 512, 1024, 2048, 4096, 8192, 1 << 30],
              "col_wg256": [0, 2048, 4096, 1 << 30],
              "widen_wg": [256, 512, 1024, 2048],
              "min_col": [8, 16, 32],
              "min_col_special": [4, 8, 16],
              "rs_widen_wg": [128, 256, 512, 1024],
              "ks_fuse": [0, 128],
              "ks_batch": [2, 3, 4, 5, 8],
              "ks_modup_batch": [0, 2, 3, 4]}
BATCH_STEPS = list(range(1, 9))     # eight rotations, each with its own key


class Bench:
    """Keys, ciphertexts and device words of one ring degree."""

    def __init__(self, logn: int):
        self.logn, self.N = logn, 1 << logn
        self.ctx = X.pfx_ctx_create(X.make_params(logn, QB, PB, ALPHA, ML), 0)
        self.st = X.pfx_stream_create(self.ctx)
        seed = bytes([logn]) * 32
        self.sk = X.pfx_keygen_secret(self.ctx, seed, 192 if logn >= 13 else 64)
        self.rlk = X.pfx_keygen_relin(self.ctx, self.sk, seed)
        self.gks = X.pfx_keygen_galois(self.ctx, self.sk, BATCH_STEPS, False, seed)
        q, _, _ = X.pfx_ctx_moduli(self.ctx, len(QB), len(PB))
        self.cts, self.outs, self.routs = {}, {}, {}
        for lv in LEVELS:
            pair = []
            for k in range(2):
                h = X.pfx_ct_create(self.ctx, lv, 1)
                X.pfx_ct_import(self.ctx, I.uniform_residues(q[:lv], self.N, 7000 + 10 * lv + k, lead=(2,)),
                                2.0 ** 45, h)
                pair.append(h)
            self.cts[lv] = pair
            self.outs[lv] = X.pfx_ct_create(self.ctx, lv, 1)
            self.routs[lv] = [X.pfx_ct_create(self.ctx, lv, 1) for _ in BATCH_STEPS]
        self.words = X.pfx_dev_alloc(self.ctx, 2 * len(QB) * self.N * 8)
        X.pfx_memcpy_htod(self.ctx, self.words, I.uniform_residues(q, self.N, 7999, lead=(2,)))
        self.ev0, self.ev1 = X.pfx_event_create(self.ctx), X.pfx_event_create(self.ctx)

    def time(self, fn, reps: int) -> float:
        ts = []
        for r in range(3 + reps):
            X.pfx_event_record(self.ctx, self.ev0, self.st)
            fn()
            X.pfx_event_record(self.ctx, self.ev1, self.st)
            if r >= 3:
                ts.append(X.pfx_event_elapsed(self.ctx, self.ev0, self.ev1))
        return float(np.median(ts))

    def objective(self, reps: int) -> float:
        c, st, tot = self.ctx, self.st, 0.0
        for lv in LEVELS:
            a, b = self.cts[lv]
            o = self.outs[lv]

            def mrr():
                X.pfx_mul_relin(c, a, b, self.rlk, o, st)
                X.pfx_rescale(c, o, o, st)
            tot += self.time(mrr, reps)
            tot += self.time(lambda: X.pfx_rotate(c, a, 1, self.gks, o, st), reps)
            tot += self.time(lambda: X.pfx_rotate_batch(c, [a] * len(BATCH_STEPS), BATCH_STEPS, self.gks,
                                                        self.routs[lv], st), reps)
            tot += self.time(lambda: X.pfx_ntt(c, self.words, 0, lv, 2, False, st), reps)
            tot += self.time(lambda: X.pfx_ntt(c, self.words, 0, lv, 2, True, st), reps)
        return tot

    def close(self):
        for pair in self.cts.values():
            for h in pair:
                X.pfx_ct_destroy(h)
        for h in list(self.outs.values()) + [h for hs in self.routs.values() for h in hs]:
            X.pfx_ct_destroy(h)
        for k in [self.rlk] + self.gks:
            X.pfx_swk_destroy(k)
        X.pfx_sk_destroy(self.sk)
        X.pfx_dev_free(self.ctx, self.words)
        for e in (self.ev0, self.ev1):
            X.pfx_event_destroy(self.ctx, e)
        X.pfx_stream_destroy(self.ctx, self.st)
        X.pfx_ctx_destroy(self.ctx)


def tune(logn: int, reps: int, min_gain: float, log=print) -> dict:
    b = Bench(logn)
    try:
        def score(cfg):
            X.pfx_tuning_set(logn, **cfg)
            return b.objective(reps)
        best = dict(DEFAULT)
        base = score(best)
        best_s = base
        for sweep in range(2):
            for field, values in CANDIDATES.items():
                for v in values:
                    if v == best[field]:
                        continue
                    cfg = dict(best, **{field: v})
                    s = score(cfg)
                    if s < best_s:
                        best, best_s = cfg, s
            log(f"  log N = {logn}: sweep {sweep + 1}: {best_s:.1f} ms against {base:.1f} ms default")
        # confirm on a re-measurement (two more of each)
        d = score(dict(DEFAULT)) + score(dict(DEFAULT))
        t = score(best) + score(best)
        keep = best if t < d * (1.0 - min_gain) else dict(DEFAULT)
        log(f"  log N = {logn}: re-measured {t / 2:.2f} ms tuned, {d / 2:.2f} ms default -> "
            f"{'tuned' if keep is best else 'default'}")
        X.pfx_tuning_set(logn, **keep)
        return {"config": keep, "tuned_ms": t / 2, "default_ms": d / 2}
    finally:
        b.close()


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--lognums", type=int, nargs="*", default=[12, 13, 14, 15, 16])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--min-gain", type=float, default=0.01)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args(argv)
    X.pfx_tuning_reset()
    lines = ["# NTT pass geometry per ring degree, chosen by paper_2412_13269_amd/autotune.py on an MI355X",
             f"# command: python -m paper_2412_13269_amd.autotune --lognums {' '.join(map(str, args.lognums))} "
             f"--reps {args.reps}",
             "# objective: HMult + relin + rescale, a rotation, forward and inverse NTT of a ciphertext, at",
             "# 24, 13 and 4 limbs of the 24 + 4 prime chain (sum of median device times)",
             "# plus eight batched rotations (pfx_rotate_batch)",
             "# log_n row_wg256 col_wg256 widen_wg min_col min_col_special rs_widen_wg ks_fuse ks_batch"
             " ks_modup_batch   (tuned ms / default ms)"]
    t0 = time.time()
    for ln in args.lognums:
        r = tune(ln, args.reps, args.min_gain, log=lambda *a: print(*a, flush=True))
        c = r["config"]
        lines.append(f"{ln} " + " ".join(str(c[f]) for f in X.TUNING_FIELDS))
        lines.append(f"#   {r['tuned_ms']:.3f} / {r['default_ms']:.3f}")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out} in {time.time() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
