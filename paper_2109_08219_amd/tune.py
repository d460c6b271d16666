"""Autotuner: subrange size (Rule 4) and delegates per subrange (Rule 3), measured.

Batched form:
For every bucket (floor(log2 n), floor(log2 k)) that the batched kernel owns,
a batch of synthetic problems of that bucket (half uint32 uniform, half
float32 normal, lengths and k uniform inside the bucket) is timed with each
candidate (alpha, beta): Rule 4's alpha and its neighbours with one or two
delegates per subrange, as the kernel would actually run them (raised to
fit its delegate vector, lowered to keep more delegates than k), the
workgroup radix select without delegates (written as alpha 0), and no
entry (Rule 4 itself, beta 1); each is timed twice,
interleaved, keeping the faster run.  A bucket gets an entry only when an
alternative beats Rule 4.  The table is written to tuning.json,
which the binding loads when it opens the library.  Every alpha gives the
same results; only the time changes.

Single problems (--single): for n = 2^20 .. 2^30 and k = 2^0 .. 2^17 where
the planner takes the delegate method, its (alpha, beta) against alpha
within 2 of it and beta in {1, 2, 4}, on uint32 uniform and float32 normal
keys of n = 2^lg_n (the sum of both times; three interleaved rounds, the
fastest run counts); an entry is written only where a candidate beats the
planner by more than 3%.

    python -m paper_2109_08219_amd.tune [--out PATH] [--problems 512] [--reps 10] [--single | --keep-single | --keep-batched]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))


def _bucket_problems(torch, lg_n, lg_k, count, gen):
    lo, hi = max(2 ** lg_n, 4097), min(2 ** (lg_n + 1) - 1, 1 << 22)
    if lo > hi:
        return None
    ns = torch.randint(lo, hi + 1, (count,), generator=gen, device="cpu").tolist()
    out = []
    for i, n in enumerate(ns):
        k_lo, k_hi = 2 ** lg_k, min(2 ** (lg_k + 1) - 1, n, 2048)
        if k_lo > k_hi:
            return None
        k = int(torch.randint(k_lo, k_hi + 1, (1,), generator=gen, device="cpu"))
        if i % 2 == 0:
            t = torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda").view(torch.uint32)
        else:
            t = torch.randn(n, device="cuda")
        out.append((t, k))
    return out


def _time(torch, batch, reps):
    batch.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.run()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batched(drt, torch, problems, reps, log=print):
    entries = []
    gen = torch.Generator().manual_seed(20210908)
    torch.manual_seed(20210908)
    drt.tune_set([])
    for lg_n in range(12, 22):
        for lg_k in range(0, 12):
            probs = _bucket_problems(torch, lg_n, lg_k, problems, gen)
            if probs is None:
                continue
            # the alpha the kernel runs for a problem of this bucket under a table entry a
            rep_n, rep_k = probs[0][0].numel(), probs[0][1]
            base = drt.batched_plan(rep_n, rep_k)
            if base[0] != 2:
                continue
            cands = {}
            for b in (1, 2):
                for a in range(max(2, base[1] - 3), min(24, base[1] + 3) + 1):
                    drt.tune_set([(drt.FORM_BATCHED, lg_n, lg_k, a, b)])
                    r, eff, beff = drt.batched_plan(rep_n, rep_k)
                    if r == 2 and (eff, beff) != base[1:]:  # Rule 4's own plan is the "rule" candidate
                        cands.setdefault((eff, beff), (a, b))
            batch = drt.Batch(probs)
            # candidates: table entries ((alpha, beta) as requested; alpha 0 = radix select) and no
            # entry (Rule 4, beta 1), each timed twice, interleaved, keeping the faster run
            options = ([("rule", None)] + [(f"a{eff}b{beff}", ab) for (eff, beff), ab in sorted(cands.items())]
                       + [("radix", (0, 1))])
            times = {}
            for _ in range(2):
                for name, ab in options:
                    drt.tune_set([] if ab is None else [(drt.FORM_BATCHED, lg_n, lg_k, ab[0], ab[1])])
                    t = _time(torch, batch, reps)
                    times[name] = min(times.get(name, t), t)
            drt.tune_set([])
            best = min(times, key=times.get)
            ab_best = dict(options)[best]
            if ab_best is not None:  # no entry when Rule 4 is the fastest
                entries.append({"form": drt.FORM_BATCHED, "lg_n": lg_n, "lg_k": lg_k, "alpha": ab_best[0],
                                "beta": ab_best[1], "ms": round(times[best], 4), "rule_alpha": base[1],
                                "rule_ms": round(times["rule"], 4)})
            log(f"n~2^{lg_n} k~2^{lg_k}: rule alpha {base[1]} {times['rule']:.3f} ms, best {best} "
                f"{times[best]:.3f} ms  " + " ".join(f"{nm}:{t:.3f}" for nm, t in times.items()))
            del batch, probs
            torch.cuda.empty_cache()
    return entries


def tune_single(drt, torch, reps, log=print):
    entries = []
    torch.manual_seed(20210908)
    drt.tune_set([])
    full_u = torch.randint(-2 ** 31, 2 ** 31, (1 << 30,), dtype=torch.int32, device="cuda").view(torch.uint32)
    full_f = torch.randn(1 << 30, device="cuda")
    for lg_n in range(20, 31):
        n = 1 << lg_n
        keys = (full_u[:n], full_f[:n])
        for lg_k in range(0, 18):
            k = 1 << lg_k
            base = drt.plan(n, k)
            if base.mode != 1:
                continue
            vals = [torch.empty(k, dtype=t.dtype, device="cuda") for t in keys]
            idx = torch.empty(k, dtype=torch.int32, device="cuda")

            def time_opts(alpha, beta):
                tot = 0.0
                for t, v in zip(keys, vals):
                    run = (lambda: drt.topk_select(t, k, v, idx)) if alpha is None else \
                        (lambda: drt.topk_select(t, k, v, idx, alpha=alpha, beta=beta, mode=1))
                    for _ in range(2):
                        run()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        run()
                    e1.record()
                    e1.synchronize()
                    tot += e0.elapsed_time(e1) / reps
                return tot

            cands = [(a, b) for b in (1, 2, 4) for a in range(max(2, base.alpha - 2), min(24, base.alpha + 2) + 1)]
            times = {}
            for _ in range(3):  # three rounds, interleaved; the fastest run counts
                for name, (a, b) in [("plan", (None, None))] + [(f"a{a}b{b}", (a, b)) for a, b in cands]:
                    t = time_opts(a, b)
                    times[name] = min(times.get(name, t), t)
            best = min(times, key=times.get)
            line = f"single n=2^{lg_n} k=2^{lg_k}: plan a{base.alpha}b{base.beta} {times['plan']:.3f} ms, best {best} {times[best]:.3f} ms"
            if best != "plan" and times[best] < 0.97 * times["plan"]:
                a, b = dict((f"a{a}b{b}", (a, b)) for a, b in cands)[best]
                entries.append({"form": drt.FORM_SINGLE, "lg_n": lg_n, "lg_k": lg_k, "alpha": a, "beta": b,
                                "ms": round(times[best], 4), "rule_alpha": base.alpha, "rule_beta": base.beta,
                                "rule_ms": round(times["plan"], 4)})
                line += "  -> entry"
            log(line)
    del full_u, full_f
    torch.cuda.empty_cache()
    return entries


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--problems", type=int, default=512)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--single", action="store_true", help="also tune single problems (alpha, beta)")
    ap.add_argument("--keep-single", action="store_true",
                    help="re-tune the batched form only, keeping the single-problem entries of --out")
    ap.add_argument("--keep-batched", action="store_true",
                    help="re-tune single problems only, keeping the batched entries of --out")
    args = ap.parse_args(argv)
    if args.keep_single and args.keep_batched:
        sys.exit("--keep-single and --keep-batched exclude each other")
    kept = []
    if (args.keep_single or args.keep_batched) and os.path.exists(args.out):
        with open(args.out) as f:
            kept = [e for e in json.load(f)["entries"] if e["form"] == (1 if args.keep_batched else 0)]
    import torch
    import paper_2109_08219_amd as drt
    if not torch.cuda.is_available():
        sys.exit("the autotuner measures on the GPU; none is visible")
    t0 = time.time()
    if args.keep_batched:
        entries = kept + tune_single(drt, torch, max(3, args.reps // 2), log=lambda s: print(s, flush=True))
    else:
        entries = tune_batched(drt, torch, args.problems, args.reps, log=lambda s: print(s, flush=True))
        if args.single:
            entries += tune_single(drt, torch, max(3, args.reps // 2), log=lambda s: print(s, flush=True))
        else:
            entries += kept
    doc = {"device": torch.cuda.get_device_name(0), "problems_per_bucket": args.problems, "reps": args.reps,
           "seconds": round(time.time() - t0, 1), "entries": entries}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {len(entries)} entries to {args.out}", flush=True)


if __name__ == "__main__":
    main()
