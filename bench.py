#!/usr/bin/env python3
"""Benchmark of delegate-centric top-k on one MI355X.

Workload (one step): exact top-k of N = 2^30 keys resident in HBM, for both
input variants (uint32 i.i.d. uniform over [0, 2^32), and float32 standard
normal through the order-preserving uint32 encoding) and for each
k in {1, 1024, 131072}: six topk_select calls, sorted values + positions.

Reported: keys/s over the whole step (value), HBM GB/s of the mandatory read
(4 bytes per key), per-case timings, the roofline of the dominant kernel (the
delegate pass, timed live with HIP events on its own stream), and the CPU
oracle on a bounded sample of the same workload, and a probe kernel's read
bandwidth with the delegate pass's access pattern.  Beside the step, outside
its timed region:
  small    N = 2^20 uint32 uniform, k = 1024: latency;
  adversarial  N = 2^29, k = 16384: float32 N(0,1) sorted ascending with
           beta in {1, 2, 4, 8}, and uint32 uniform over [0, 16);
  batched  4096 independent instances (lengths log-uniform in [2^10, 2^20],
           uint32 uniform or float32 normal per instance, k uniform in
           [1, min(n, 2048)]) in one topk_select_batched call, queries/s,
           against a loop of topk_select over the same instances;
  serving  Poisson arrivals of requests over a device-resident pool of arrays
           (n log-uniform in [2^12, 2^26], uint32 uniform / float32 normal,
           k log-uniform in [1, 4096]): the continuous-batching server and the
           per-request loop at 0.8x and 1.5x the loop's saturation rate,
           queries/s and p50/p99 latency (arrival -> completion on the host).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-adversarial] [--no-batched] [--no-serving] [--no-smallest] [--no-by-k] [--no-host]
                       [--no-wide]
                       [--copy-calibration]
       python bench.py --delegate-vector A:B[,A:B...]
                       (profiling aid: only the delegate vector of the 2^30 uniform input for
                       each (alpha, beta), twice each, then exit; no JSON line)
       python bench.py --only adversarial|batched|serving|small
                       (profiling aid: that part alone, printed as {"section": ..., "result": ...};
                       not the benchmark line)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "top-k keys/s and HBM GB/s at N=2^30; batched queries/s + p99 latency"
HBM_PEAK_GBS = 8000.0
N = 1 << 30
KS = (1, 1024, 131072)
CPU_K = 1024
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "delegate_pass_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2109_08219_amd", "csrc", f) for f in ("kernels.h", "internal.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for_current_kernel():
    """HBM bytes per delegate-pass launch from the committed rocprofv3 counter
    runs (``key = value`` lines), if they were taken on the current kernel
    source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split("=", 1) for line in f if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _gpu_keys(torch, kind, n, gen):
    if kind == "uniform_u32":
        return torch.randint(-2 ** 31, 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=gen).view(torch.uint32)
    return torch.randn(n, device="cuda", generator=gen)


def bench_batched(drt, synth, torch, args):
    """4096 instances in one batched call vs a loop of topk_select over them."""
    print("[bench] batched: generating 4096 instances", file=sys.stderr, flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.DEFAULT_SEED)
    probs = [(_gpu_keys(torch, kind, n, gen), k) for kind, n, k, _ in synth.batched_workload(4096)]
    total = sum(t.numel() for t, _ in probs)
    b = drt.Batch(probs)
    for _ in range(max(1, args.warmup)):
        b.run()
    torch.cuda.synchronize()
    steps = max(5, args.steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    print("[bench] batched: per-query loop", file=sys.stderr, flush=True)
    outs = [(torch.empty(k, dtype=t.dtype, device="cuda"), torch.empty(k, dtype=torch.int32, device="cuda"))
            for t, k in probs]
    for (t, k), (v, ix) in zip(probs, outs):
        drt.topk_select(t, k, v, ix)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (t, k), (v, ix) in zip(probs, outs):
        drt.topk_select(t, k, v, ix)
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t0) * 1e3
    # the method's re-read per problem on the delegate route (route 2), not counted as useful
    # bytes: beta 1 re-reads exactly the k - 1 subranges whose delegate ranks above t; beta 2
    # at most (k - 1) / 2 subranges (those whose second delegate does), counted at that bound
    reread = 0
    routes = {1: 0, 2: 0, 3: 0}
    betas = {1: 0, 2: 0}
    for t, k in probs:
        r, a, beta = drt.batched_plan(t.numel(), k)
        routes[r] = routes.get(r, 0) + 1
        if r == 2:
            betas[beta] = betas.get(beta, 0) + 1
            reread += 4 * min(t.numel(), ((k - 1) // beta) << a)
    return {"instances": len(probs), "keys": total, "ms_per_batch": ms, "queries_per_s": len(probs) / ms * 1e3,
            "reread_bytes": reread, "routes": {str(r): c for r, c in routes.items()},
            "route2_beta": {str(b): c for b, c in betas.items()},
            "GBps": 4.0 * total / ms / 1e6, "loop_ms": ms_loop, "loop_queries_per_s": len(probs) / ms_loop * 1e3,
            "speedup_vs_loop": ms_loop / ms, "steps": steps}


def _median_ms(torch, fn, reps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return {"ms_median": ts[len(ts) // 2], "ms_min": ts[0], "ms_max": ts[-1], "ms_mean": sum(ts) / len(ts)}


def bench_small(drt, synth, torch, args):
    """N = 2^20 uint32 uniform, k = 1024: latency (4 MiB fits the caches; no roofline)."""
    x = synth.uniform_u32(1 << 20, synth.DEFAULT_SEED)
    t = torch.from_numpy(x).cuda()
    v = torch.empty(1024, dtype=t.dtype, device="cuda")
    ix = torch.empty(1024, dtype=torch.int32, device="cuda")
    r = _median_ms(torch, lambda: drt.topk_select(t, 1024, v, ix), max(20, args.steps), max(3, args.warmup))
    r.update(n=1 << 20, k=1024, keys_per_s=(1 << 20) / (r["ms_median"] / 1e3), mode=drt.plan(1 << 20, 1024).mode)
    return r


def bench_smallest_i32(drt, torch, t_u, t_f):
    """The k smallest and int32 keys at N = 2^30, on the step's own inputs: float32
    N(0,1) smallest first, and the uniform uint32 stream read as int32 (uniform over
    the signed range), largest and smallest first."""
    out = []
    for name, t, ks, largest in (("f32", t_f, KS, False), ("i32", t_u.view(torch.int32), (1024,), True),
                                 ("i32", t_u.view(torch.int32), (1024,), False)):
        for k in ks:
            v = torch.empty(k, dtype=t.dtype, device="cuda")
            ix = torch.empty(k, dtype=torch.int32, device="cuda")
            r = _median_ms(torch, lambda: drt.topk_select(t, k, v, ix, largest=largest), 10, 2)
            _, _, st = drt.topk_select(t, k, v, ix, largest=largest, stats=True)
            r.update(dtype=name, order="largest" if largest else "smallest", k=k, alpha=st.alpha, beta=st.beta,
                     keys_per_s=t.numel() / (r["ms_median"] / 1e3))
            out.append(r)
    return out


def bench_shard(drt, torch, t_u, t_f):
    """One GPU's share of an 8-way sharded N = 2^30 call, at its real shape: the first
    2^27 keys of each input, the step's k values (the local top-k each GPU would
    contribute before the all-gather)."""
    out = []
    for name, t in (("u32", t_u[: 1 << 27]), ("f32", t_f[: 1 << 27])):
        for k in KS:
            v = torch.empty(k, dtype=t.dtype, device="cuda")
            ix = torch.empty(k, dtype=torch.int32, device="cuda")
            r = _median_ms(torch, lambda: drt.topk_select(t, k, v, ix), 10, 3)
            r.update(dtype=name, k=k, keys_per_s=t.numel() / (r["ms_median"] / 1e3),
                     GBps=4 * t.numel() / (r["ms_median"] / 1e3) / 1e9)
            out.append(r)
    return out


def bench_host_stream(drt, synth, torch):
    """Keys in host memory (N = 2^30 uint32 uniform), streamed through the device in
    chunks of 2^26 keys by topk_select_host: pageable (numpy) and pinned (a torch
    tensor allocated with pin_memory=True) host buffers, k = 1024 and 131072.  The
    rate is bound by the host-to-device copy, not the kernels."""
    import numpy as np
    print("[bench] host stream: 2^30 keys in host memory", file=sys.stderr, flush=True)
    x = synth.uniform_u32(N, synth.DEFAULT_SEED)
    pinned = torch.empty(N, dtype=torch.int32, pin_memory=True)
    pinned.numpy().view(np.uint32)[:] = x
    out = []
    for name, arr in (("pageable", x), ("pinned", pinned.numpy().view(np.uint32))):
        for k in (1024, 131072):
            drt.topk_select_host(arr, k, chunk=1 << 26)  # warm-up
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                drt.topk_select_host(arr, k, chunk=1 << 26)
                ts.append(time.perf_counter() - t0)
            best = min(ts)
            out.append({"memory": name, "k": k, "ms_min": best * 1e3, "ms_median": sorted(ts)[1] * 1e3,
                        "keys_per_s": N / best, "GBps": 4 * N / best / 1e9})
    del x, pinned
    return out


def bench_delegates_vs_plain(drt, torch, t_u):
    """The paper's claim that delegates speed up the radix top-k they wrap: at
    N = 2^28 uint32 uniform, the delegate method (planner's alpha, beta) against
    the plain radix select over all keys (mode 2), k = 2^0 .. 2^20."""
    t = t_u[: 1 << 28]
    out = []
    for lg_k in (0, 4, 8, 10, 12, 14, 16, 18, 20):
        k = 1 << lg_k
        v = torch.empty(k, dtype=t.dtype, device="cuda")
        ix = torch.empty(k, dtype=torch.int32, device="cuda")
        row = {"k": k}
        for name, mode in (("delegates", 1), ("plain_radix", 2)):
            r = _median_ms(torch, lambda: drt.topk_select(t, k, v, ix, mode=mode), 5, 1)
            row[name + "_ms"] = r["ms_median"]
        row["speedup"] = row["plain_radix_ms"] / row["delegates_ms"]
        out.append(row)
    return out


def bench_wide(drt, torch):
    """64-bit keys at N = 2^28 (2 GiB, the same bytes as 2^29 4-byte keys): uint64
    uniform and float64 N(0,1), k in {1, 1024, 131072}; keys/s and GB/s of the
    mandatory 8-byte read.  Inputs drawn on the GPU."""
    print("[bench] 64-bit keys: 2^28", file=sys.stderr, flush=True)
    n = 1 << 28
    gen = torch.Generator(device="cuda")
    gen.manual_seed(20210919)
    out = []
    for name in ("u64", "f64"):
        if name == "u64":
            t = torch.randint(-2 ** 63, 2 ** 63 - 1, (n,), dtype=torch.int64, device="cuda",
                              generator=gen).view(torch.uint64)
        else:
            t = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
        for k in KS:
            v = torch.empty(k, dtype=t.dtype, device="cuda")
            ix = torch.empty(k, dtype=torch.int32, device="cuda")
            r = _median_ms(torch, lambda: drt.topk_select(t, k, v, ix), 10, 2)
            p = drt.plan(n, k, name)
            r.update(dtype=name, k=k, mode=p.mode, alpha=p.alpha, keys_per_s=n / (r["ms_median"] / 1e3),
                     GBps=8 * n / (r["ms_median"] / 1e3) / 1e9)
            out.append(r)
        del t
    torch.cuda.empty_cache()
    return out


def bench_inner_by_k(drt, torch, t_u):
    """The top-k algorithm the delegates assist, by k (the paper's choice of
    algorithm as k grows, Sections 5.1 and 6.1): N = 2^28 uint32 uniform, the
    planner's alpha and beta, with the fused one-kernel tail (variant 0, the
    default), MSD radix selects (1), the bitonic top-k (2, k <= 256) and
    bucket selects (3) for the first and second top-k; k = 2^0 .. 2^20."""
    t = t_u[: 1 << 28]
    names = {0: "fused", 1: "radix", 2: "bitonic", 3: "bucket"}
    out = []
    for lg_k in (0, 2, 4, 6, 8, 10, 12, 14, 16, 18, 20):
        k = 1 << lg_k
        v = torch.empty(k, dtype=t.dtype, device="cuda")
        ix = torch.empty(k, dtype=torch.int32, device="cuda")
        row = {"k": k}
        for variant, name in names.items():
            if variant == 2 and k > 256:
                continue
            r = _median_ms(torch, lambda: drt.topk_select(t, k, v, ix, mode=1, variant=variant), 5, 1)
            row[name + "_ms"] = r["ms_median"]
        row["best"] = min((row[n + "_ms"], n) for n in names.values() if n + "_ms" in row)[1]
        out.append(row)
    return out


def bench_adversarial(drt, torch, args):
    """N = 2^29, k = 16384: float32 N(0,1) sorted ascending (beta 1, 2, 4, 8) and uint32
    uniform over [0, 16) (planner's choice).  Inputs drawn on the GPU."""
    print("[bench] adversarial: 2^29 keys", file=sys.stderr, flush=True)
    n, k = 1 << 29, 16384
    gen = torch.Generator(device="cuda")
    gen.manual_seed(20210908)
    t = torch.randn(n, device="cuda", generator=gen)
    t = torch.sort(t).values
    v = torch.empty(k, dtype=t.dtype, device="cuda")
    ix = torch.empty(k, dtype=torch.int32, device="cuda")
    out = {"n": n, "k": k, "sorted_f32": {}}
    for beta in (1, 2, 4, 8):
        r = _median_ms(torch, lambda: drt.topk_select(t, k, v, ix, beta=beta), 10, 2)
        _, _, st = drt.topk_select(t, k, v, ix, beta=beta, stats=True)
        r.update(alpha=st.alpha, scanned=int(st.scanned), candidates=int(st.candidates),
                 keys_per_s=n / (r["ms_median"] / 1e3))
        out["sorted_f32"][f"beta{beta}"] = r
    del t
    h = torch.randint(0, 16, (n,), dtype=torch.int32, device="cuda", generator=gen).view(torch.uint32)
    vh = torch.empty(k, dtype=h.dtype, device="cuda")
    r = _median_ms(torch, lambda: drt.topk_select(h, k, vh, ix), 10, 2)
    _, _, st = drt.topk_select(h, k, vh, ix, stats=True)
    r.update(alpha=st.alpha, beta=st.beta, scanned=int(st.scanned), candidates=int(st.candidates),
             keys_per_s=n / (r["ms_median"] / 1e3))
    out["heavydup_u32"] = r
    del h
    torch.cuda.empty_cache()
    return out


def bench_serving(drt, synth, torch, np, pool_size=256, requests=10000):
    """Continuous-batching server vs the per-request loop under Poisson arrivals."""
    print("[bench] serving: building the array pool", file=sys.stderr, flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.DEFAULT_SEED + 1)
    pool = [_gpu_keys(torch, kind, n, gen) for kind, n, _ in synth.serving_workload(pool_size, 99)]
    pick = (synth.unit_uniform(requests, 5) * pool_size).astype(np.int64)
    ks = synth.log_uniform_int(requests, 0, 12, 6)
    reqs = [(pool[i], int(min(k, pool[i].numel()))) for i, k in zip(pick, ks)]
    b = drt.Batch(reqs)
    torch.cuda.synchronize()

    def run(plain, arrivals):
        with drt.Server(streams=1 if plain else 4, max_batch=1 if plain else 256, plain=plain) as srv:
            lat, el = srv.replay(b, arrivals)
            st = srv.stats()
        return {"queries_per_s": requests / el * 1e6, "p50_us": float(np.percentile(lat, 50)),
                "p99_us": float(np.percentile(lat, 99)), "mean_batch": st.launched_items / max(1, st.launches)}

    burst = np.zeros(requests)
    run(True, burst)  # warm both paths
    run(False, burst)
    mu_loop = run(True, burst)["queries_per_s"]
    res = {"requests": requests, "pool_arrays": pool_size,
           "pool_GiB": sum(t.numel() for t in pool) * 4 / 2 ** 30, "loop_saturation_qps": mu_loop,
           "server_saturation_qps": run(False, burst)["queries_per_s"], "rates": []}
    for f in (0.8, 1.5):
        print(f"[bench] serving: lambda = {f} x loop saturation", file=sys.stderr, flush=True)
        arr = synth.poisson_arrivals(requests, f * mu_loop, 3)
        res["rates"].append({"lambda_qps": f * mu_loop, "per_request_loop": run(True, arr),
                             "batched_server": run(False, arr)})
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-adversarial", action="store_true")
    ap.add_argument("--no-smallest", action="store_true", help="skip the k smallest / int32 cases")
    ap.add_argument("--no-host", action="store_true", help="skip top-k of keys in host memory")
    ap.add_argument("--no-wide", action="store_true", help="skip the 64-bit key cases")
    ap.add_argument("--no-by-k", action="store_true",
                    help="skip the by-k studies (delegates against the plain radix select, the inner "
                         "top-k algorithm) and the 2^27 shard cases")
    ap.add_argument("--delegate-vector", default=None, metavar="A:B,...",
                    help="only build the delegate vector for these (alpha, beta) pairs (for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy, whose HBM counters calibrate the traffic figure")
    ap.add_argument("--only", choices=("adversarial", "batched", "serving", "small"), default=None,
                    help="run one part alone (for profiler runs); prints that part's result, not the bench line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2109_08219_amd as drt
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        part = {"adversarial": lambda: bench_adversarial(drt, torch, args),
                "batched": lambda: bench_batched(drt, synth, torch, args),
                "serving": lambda: bench_serving(drt, synth, torch, np),
                "small": lambda: bench_small(drt, synth, torch, args)}[args.only]()
        print(json.dumps({"section": args.only, "result": part}), flush=True)
        return 0
    if args.delegate_vector:
        x_u = synth.uniform_u32(N, synth.DEFAULT_SEED)
        t_u = torch.from_numpy(x_u).to(dev)
        del x_u
        for pair in args.delegate_vector.split(","):
            a, b = (int(v) for v in pair.split(":"))
            for _ in range(2):
                drt.delegates(t_u, a, b)
            torch.cuda.synchronize()
            print(f"[bench] delegate vector alpha {a} beta {b} done", file=sys.stderr, flush=True)
        return 0
    print(f"[bench] generating 2 x 2^30 keys", file=sys.stderr, flush=True)
    x_u = synth.uniform_u32(N, synth.DEFAULT_SEED)  # kept: the CPU baseline reads the same host bytes
    t_u = torch.from_numpy(x_u).to(dev)
    x_f = synth.normal_f32(N, synth.DEFAULT_SEED)
    t_f = torch.from_numpy(x_f).to(dev)
    del x_f
    if args.copy_calibration:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale factor of the traffic measurement (1 GiB each way)
        src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cases = []
    for name, t in (("u32", t_u), ("f32", t_f)):
        for k in KS:
            cases.append(dict(dtype=name, k=k, keys=t,
                              vals=torch.empty(k, dtype=t.dtype, device=dev),
                              idx=torch.empty(k, dtype=torch.int32, device=dev)))
    stream = torch.cuda.current_stream()

    def call(c):
        drt.topk_select(c["keys"], c["k"], c["vals"], c["idx"], stream=stream)

    # plan / counters of each case (outside the timed region)
    for c in cases:
        _, _, st = drt.topk_select(c["keys"], c["k"], c["vals"], c["idx"], stats=True, stream=stream)
        c.update(alpha=st.alpha, beta=st.beta, scanned=int(st.scanned), candidates=int(st.candidates),
                 # the method's own traffic beyond the 4n-byte read (not counted as useful bytes):
                 # delegate vector written, qualifying subranges re-read, survivors written
                 overhead_bytes={"delegates": 8 * int(st.delegates), "reread": 4 * (int(st.scanned) << st.alpha),
                                 "survivors": 8 * int(st.candidates)})

    # per-case latency (events around single calls)
    reps = max(3, args.steps)
    for c in cases:
        for _ in range(args.warmup):
            call(c)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            e0.record(stream)
            call(c)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        c["ms_median"] = times[len(times) // 2]
        c["ms_min"] = times[0]
        c["ms_max"] = times[-1]
        c["ms_mean"] = sum(times) / len(times)

    # the timed region: K steps of all six calls
    for _ in range(args.warmup):
        for c in cases:
            call(c)
    torch.cuda.synchronize()
    drt.timing_read()  # drop anything recorded so far
    drt.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for c in cases:
            call(c)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    drt.timing_enable(False)
    del_ms, tail_ms, calls = drt.timing_read()

    # achievable read bandwidth of the delegate pass's access pattern (probe kernel)
    probe_out = torch.empty(1, dtype=torch.int32, device=dev)
    for _ in range(3):
        drt.read_probe(t_u, probe_out, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        drt.read_probe(t_u, probe_out, stream=stream)
    e1.record(stream)
    e1.synchronize()
    probe_GBps = 4.0 * N / (e0.elapsed_time(e1) / 20 / 1e3) / 1e9

    step_s = (t1 - t0) / args.steps
    keys_per_step = N * len(cases)
    value = keys_per_step / step_s
    del_avg_s = del_ms / calls / 1e3
    achieved = 4.0 * N / del_avg_s / 1e9
    traffic = traffic_for_current_kernel()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        print("[bench] CPU oracle on the 2^30 uint32 input, k = 1024", file=sys.stderr, flush=True)
        threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or (os.cpu_count() or 1)
        a = time.perf_counter()
        oracle.topk_threaded(x_u, CPU_K, "u32", threads=threads)
        t_thr = time.perf_counter() - a
        a = time.perf_counter()
        oracle.topk_reference(x_u, CPU_K, "u32")
        t_one = time.perf_counter() - a
        cpu = {"value": N / t_thr, "unit": "keys/s", "cores": threads, "kind": "oracle",
               "sample": f"the step's N = 2^30 uint32 input (the same host bytes the GPU reads), k = {CPU_K}: "
                         f"the oracle's selection split over {threads} threads then merged, {t_thr:.1f} s",
               "single_thread": {"value": N / t_one, "unit": "keys/s", "cores": 1,
                                 "sample": f"same input and k, the oracle's selection route on one thread, "
                                           f"{t_one:.1f} s"},
               "host_cpu_count": os.cpu_count()}
    del x_u

    case_rows = [{k: v for k, v in c.items() if k not in ("keys", "vals", "idx")} for c in cases]
    del cases
    smallest_i32 = None if args.no_smallest else bench_smallest_i32(drt, torch, t_u, t_f)
    by_k = None if args.no_by_k else bench_delegates_vs_plain(drt, torch, t_u)
    inner_by_k = None if args.no_by_k else bench_inner_by_k(drt, torch, t_u)
    shard = None if args.no_by_k else bench_shard(drt, torch, t_u, t_f)
    del t_u, t_f
    torch.cuda.empty_cache()
    small = bench_small(drt, synth, torch, args)
    wide = None if args.no_wide else bench_wide(drt, torch)
    adversarial = None if args.no_adversarial else bench_adversarial(drt, torch, args)
    batched = None if args.no_batched else bench_batched(drt, synth, torch, args)
    serving = None if args.no_serving else bench_serving(drt, synth, torch, np)
    host_stream = None if args.no_host else bench_host_stream(drt, synth, torch)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "exact top-k of N=2^30 keys resident in HBM: uint32 uniform and float32 "
                               "N(0,1), k in {1, 1024, 131072}, one call each per step",
                   "n": N, "k": list(KS), "inputs": ["uint32 uniform", "float32 normal"]},
        "hbm_GBps_mandatory_read": 4.0 * keys_per_step / step_s / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_delegate (delegate pass, 4 B/key read once)",
                     "avg_launch_us": del_avg_s * 1e6, "launches": calls,
                     "rest_of_path_avg_us": tail_ms / calls * 1e3,
                     "probe_read_GBps": probe_GBps, "frac_of_probe": achieved / probe_GBps},
        "cpu_baseline": cpu,
        "small_case": small,
        "smallest_and_i32": smallest_i32,
        "delegates_vs_plain_radix": by_k,
        "inner_by_k": inner_by_k,
        "wide_keys": wide,
        "shard_2p27": shard,
        "host_stream": host_stream,
        "adversarial": adversarial,
        "batched": batched,
        "serving": serving,
        "cases": [{k: c[k] for k in ("dtype", "k", "alpha", "beta", "scanned", "candidates", "ms_median", "ms_min",
                                     "ms_max", "ms_mean", "overhead_bytes")}
                  | {"keys_per_s": N / (c["ms_median"] / 1e3), "GBps": 4 * N / (c["ms_median"] / 1e3) / 1e9}
                  for c in case_rows],
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
