#!/usr/bin/env python
"""Throughput of linear elliptical slice sampling on one MI355X.

Workload (timed): the GP-classification-style truncation, d = 1000,
m = 2000 (1000 rows S L from the Cholesky factor of an RBF kernel with
lengthscale 0.2 on 1000 points in [0,1]^2, S a random +-1 diagonal, b = 0.1,
plus 1000 random halfspaces), 1024 chains, float32 storage and matrix-core
projections, float64 roots and interval ends, trim eps 1e-6, Philox seed 0.
One step = one transition of every chain (Algorithm 1 of arXiv 2407.10449):
draw, project, roots, sort + cumulative max, theta, move, safeguard check.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  `roofline` covers the dominant kernel (the projection
GEMM); its duration comes from HIP events around every launch of the same K
steps issued one by one on the library's stream (the headline value times a
replay of the captured K-step graph);
`cpu_baseline` is the float64 CPU oracle on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ESS chain-steps/s at d=1000,m=2000; batched+warm-start vs plain ESS/s, 1 GPU"
PEAK_FP32_MFMA_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "proj_gemm_split_gp_rbf_traffic.txt")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2407_10449_amd", "csrc", "gemm.hpp"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per projection launch from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("gemm_source_sha256_16") != kernel_source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(pr, seconds, n_chains=64, store=None, eps=1e-6):
    """The oracle (float64 numpy, BLAS threads as configured) on n_chains of the
    same problem, stepping until `seconds` of CPU work have passed."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import ess as ref
    store = np.float32 if store is None else store
    x = np.broadcast_to(pr.x0, (n_chains, pr.d)).copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        _, x, _ = ref.run(pr.A, pr.b, x, n_chains, 1, seed=0, eps=eps, store=store,
                          start_step=steps)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": n_chains * steps / dt, "unit": "chain-steps/s", "cores": int(threads),
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{pr.name} d={pr.d} m={pr.m}: {n_chains} chains x {steps} steps "
                      f"({dt:.1f} s, float64 numpy oracle)"}


def bench_trim_sweep(E, torch):
    """The paper leaves the trim width open (Section 3.3): safeguard
    rejections in float32 against eps on the Section 4.1 truncation N(0, 1)
    on [15, 16] (2000 chains x 1000 steps, the paper's 2e6 transitions, 8
    rejections reported at its own eps) and on gp_rbf (1024 chains x 200
    steps)."""
    import synth
    out = {}
    for name, pr, steps in (("univariate_15_16", synth.univariate(15.0, 16.0, n_chains=2000), 1000),
                            ("gp_rbf", synth.gp_rbf(), 200)):
        rows = []
        for eps in (0.0, 1e-7, 1e-6, 1e-5):
            s = E.Sampler(pr.A, pr.b, pr.x0, pr.n_chains, seed=0, precision=32, trim_eps=eps)
            _, nrej = s.run(steps, keep_trace=False)
            s.close()
            rows.append({"eps": eps, "rejections": int(nrej),
                         "rate": nrej / (pr.n_chains * steps)})
        out[name] = {"transitions": pr.n_chains * steps, "rows": rows}
    return out


def bench_config(E, torch, pr, precision, steps, cpu_seconds, cpu_chains):
    """One of the smaller workloads at its own chain count and step count:
    chain-steps/s of a graph replay, the per-kernel durations of the same steps
    launched one by one, and the oracle on the host."""
    C = pr.n_chains
    eps = 1e-6 if precision == 32 else 0.0
    s = E.Sampler(pr.A, pr.b, pr.x0, C, seed=0, precision=precision, trim_eps=eps)
    E.ess_run(s.ctx, steps, 1, None, False)          # capture and warm up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.ess_run(s.ctx, steps, 1, None, False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E.ess_profile(s.ctx, True)
    E.ess_run(s.ctx, steps, 1, None, False)
    kinds = {"project": E.ESS_KERNEL_PROJECT, "sample": E.ESS_KERNEL_SAMPLE,
             "other": E.ESS_KERNEL_OTHER}
    ker = {}
    for k, v in kinds.items():
        ms, n = E.ess_profile_read(s.ctx, v)
        ker[k] = ms / steps
    E.ess_profile(s.ctx, False)
    rej = int(s.rejections().sum())
    s.close()
    esz = 4 if precision == 32 else 8
    # algorithmic work per step: 4 m d flop per chain in the projections;
    # the per-chain kernel reads p, q of every row and b (shared, from cache)
    # and reads x, x', nu and writes x', nu (20 d bytes with float storage)
    proj_flops = 4.0 * pr.m * pr.d * C
    chain_bytes = C * (2 * pr.m * esz + 5 * pr.d * esz)
    peak_tflops = 157.3 if precision == 32 else 78.6
    dominant = max(("project", "sample"), key=lambda k: ker[k])
    out = {"workload": pr.name, "d": pr.d, "m": pr.m, "chains": C, "steps": steps,
           "precision": precision, "chain_steps_per_s": C * steps / dt,
           "ms_per_step": dt * 1e3 / steps, "rejections": rej,
           "kernels_ms_per_step": ker, "dominant_kernel": dominant,
           "projection": {"tflops": proj_flops / (ker["project"] * 1e-3) / 1e12,
                          "peak_tflops": peak_tflops,
                          "unit": "fp32 MFMA" if precision == 32 else "fp64 vector"},
           "per_chain_kernel": {"hbm_gbs": chain_bytes / (ker["sample"] * 1e-3) / 1e9,
                                "hbm_peak_gbs": 8000.0}}
    out["projection"]["frac"] = out["projection"]["tflops"] / peak_tflops
    out["per_chain_kernel"]["frac"] = out["per_chain_kernel"]["hbm_gbs"] / 8000.0
    out["cpu_baseline"] = cpu_baseline(pr, cpu_seconds, n_chains=cpu_chains,
                                       store=np.float32 if precision == 32 else np.float64,
                                       eps=eps)
    return out


def bench_batched(E, torch, steps=50, plain_steps=10):
    """256 uneven polytopes x 64 chains: one launch per step (tile shapes from
    the autotuner), against one context per problem run one after another."""
    import synth
    probs = synth.batched_uneven()
    spec = [dict(A=p.A, b=p.b, x0=p.x0, n_chains=p.n_chains, seed=i, trim_eps=1e-6)
            for i, p in enumerate(probs)]
    C = sum(p.n_chains for p in probs)
    s = E.BatchedSampler(spec)
    report = E.ess_autotune(s.ctx, 10)
    E.ess_run(s.ctx, steps, 1, None, False)          # capture the graph, warm up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.ess_run(s.ctx, steps, 1, None, False)          # timed: a graph replay
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E.ess_profile(s.ctx, True)                       # kernel durations: launched one by one
    E.ess_run(s.ctx, steps, 1, None, False)
    fused_ms, fused_n = E.ess_profile_read(s.ctx, E.ESS_KERNEL_BATCHED)
    tile_ms, tile_n = E.ess_profile_read(s.ctx, E.ESS_KERNEL_PROJECT)
    chain_ms, chain_n = E.ess_profile_read(s.ctx, E.ESS_KERNEL_SAMPLE)
    E.ess_profile(s.ctx, False)
    s.close()
    singles = [E.Sampler(p.A, p.b, p.x0, p.n_chains, seed=i, precision=32)
               for i, p in enumerate(probs)]
    for q in singles:
        E.ess_run(q.ctx, 2, 1, None, False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for q in singles:
        E.ess_run(q.ctx, plain_steps, 1, None, False)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t1
    for q in singles:
        q.close()
    flops = sum(4.0 * p.m * p.d * p.n_chains for p in probs)
    # durations per step, summed over the step's launches (one tile and one
    # chain launch per problem set; the sets' launches overlap on the device)
    kernels = ({"fused_step_ms": fused_ms / steps} if fused_n else
               {"tiles_ms": tile_ms / steps, "chains_ms": chain_ms / steps,
                "launches_per_step": round(tile_n / (steps + 1)),
                "projection_tflops": flops / (tile_ms / steps / 1e3) / 1e12 if tile_n else None})
    return {"workload": "batched_uneven: 256 polytopes, d log-uniform [16,512], m = d U{1..4}, 64 chains each",
            "chain_steps_per_s": C * steps / dt,
            "ms_per_step": dt * 1e3 / steps,
            "kernels_per_step": kernels,
            "per_problem_chain_steps_per_s": C * plain_steps / dt1,
            "speedup_vs_per_problem": (C * steps / dt) / (C * plain_steps / dt1),
            "autotune": report.strip().splitlines()[-1]}


def bench_warm_start(E, torch, log, steps=216000):
    """ESS/s at equal accuracy: batched + learned warm start against plain
    per-problem contexts (and against the batched context started plain)."""
    import numpy as np
    import synth
    from paper_2407_10449_amd import warmstart as W
    A, b0, draw = synth.warm_family()
    m, d = A.shape
    rng = np.random.default_rng(21)
    train_b, eval_b = draw(rng, 10000), draw(rng, 32)
    X, Y, t_gen = W.generate_pairs(E, A, train_b, chains_per_b=1, burn=500, n_keep=10, thin=10)
    net = E.Mlp((m, 512, 512, d), seed=0)
    hist, t_train = W.train(net, X, Y, epochs=10, batch=1024, lr=1e-3)
    cmp = W.compare(E, A, eval_b, net, steps=steps, log=log)
    net.close()
    cmp.update({"workload": f"warm_family d=256 m=768: 32 held-out b x 64 chains, {steps} steps each",
                "train_samples": int(X.shape[0]), "train_gen_s": t_gen, "train_s": t_train,
                "train_mse_before_after": [hist[0], hist[-1]]})
    return cmp


def bench_paper_timing(E, torch, dims=(100, 250, 500, 1000, 2000, 4000)):
    """Section 4.2's timing protocol on its own instances (A d x d N(0, 1),
    x0 N(0, I), b = A x0 + U[0, 1]^d, so m = d): wall time for 1000 samples
    as one chain x 1000 steps and as 10 chains x 100 steps, no burn-in or
    thinning, float32, after one untimed run of the same shape (graph
    capture)."""
    import numpy as np
    import synth
    out = []
    for d in dims:
        row = {"d": d, "m": d}
        pr = synth.paper_highdim(d=d)
        # Algorithm 3, and up to 4096 rows the quadratic comparators (Section
        # 2.2's likelihood testing at midpoints, Algorithm 2's sequential
        # intersection) on the same instance
        methods = ((("alg3", ""), ("midpoint", "_midpoint"), ("alg2", "_alg2")) if d <= 4096
                   else (("alg3", ""),))
        for method, tag in methods:
            for chains, steps in ((1, 1000), (10, 100)):
                s = E.Sampler(pr.A, pr.b, pr.x0, chains, seed=0, precision=32, method=method)
                s.run(steps, keep_trace=False, count_rejections=False)      # capture
                s.set_state(torch.as_tensor(np.broadcast_to(pr.x0, (chains, d)).copy()), 0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, nrej = s.run(steps, keep_trace=False)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                s.close()
                row[f"{chains}x{steps}{tag}_ms"] = dt * 1e3
                row[f"{chains}x{steps}{tag}_rejections"] = int(nrej)
        if "1x1000_midpoint_ms" in row:
            row["midpoint_over_alg3_1x1000"] = row["1x1000_midpoint_ms"] / row["1x1000_ms"]
            row["alg2_over_alg3_1x1000"] = row["1x1000_alg2_ms"] / row["1x1000_ms"]
        print(f"# paper timing d={d}: {row}", file=sys.stderr, flush=True)
        out.append(row)
    return {"workload": "Section 4.2 instances, float32, 1000 samples per run; *_midpoint: "
                        "likelihood testing at midpoints (O(m^2)) on the same instances; "
                        "*_alg2: Algorithm 2's sequential intersection",
            "rows": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and warm-start measurements")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched measurement and print its JSON (for profiling)")
    ap.add_argument("--warm-only", action="store_true",
                    help="run only the warm-start comparison and print its JSON")
    ap.add_argument("--warm-steps", type=int, default=216000,
                    help="steps per arm of the warm-start comparison")
    ap.add_argument("--trim-sweep-only", action="store_true",
                    help="only the trim-width sweep (rejections against eps)")
    ap.add_argument("--paper-timing-only", action="store_true",
                    help="run only Section 4.2's timing protocol and print its JSON")
    ap.add_argument("--paper-dims", default="100,250,500,1000,2000,4000,8000,16000",
                    help="comma-separated d values of the Section 4.2 timing protocol")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain elementwise copy of 256 MiB (reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    paper_dims = tuple(int(v) for v in args.paper_dims.split(",") if v)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: chains shard across GPUs with no per-step traffic, "
              "and this build runs and reports a single MI355X only (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_10449_amd as E
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    E.lib()
    if args.calibrate_copy:
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)     # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(E, torch, steps=args.steps)}), flush=True)
        return
    if args.trim_sweep_only:
        print(json.dumps({"trim_sweep": bench_trim_sweep(E, torch)}), flush=True)
        return
    if args.paper_timing_only:
        print(json.dumps({"paper_timing": bench_paper_timing(E, torch, paper_dims)}), flush=True)
        return
    if args.warm_only:
        log = lambda msg: print(msg, file=sys.stderr, flush=True)
        print(json.dumps({"warm_start": bench_warm_start(E, torch, log, args.warm_steps)}),
              flush=True)
        return
    pr = synth.gp_rbf()
    C, d, m = pr.n_chains, pr.d, pr.m
    s = E.Sampler(pr.A, pr.b, pr.x0, C, seed=0, precision=32, trim_eps=1e-6)
    E.ess_run(s.ctx, args.warmup, 1, None, False)
    torch.cuda.synchronize()

    # capture the K-step graph outside the timed region, then time a replay
    E.ess_run(s.ctx, args.steps, 1, None, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.ess_run(s.ctx, args.steps, 1, None, False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # kernel durations: the same K steps launched one by one, each launch
    # bracketed by HIP events on the stream it runs on
    E.ess_profile(s.ctx, True)
    E.ess_run(s.ctx, args.steps, 1, None, False)
    proj_ms, proj_n = E.ess_profile_read(s.ctx, E.ESS_KERNEL_PROJECT)
    samp_ms, samp_n = E.ess_profile_read(s.ctx, E.ESS_KERNEL_SAMPLE)
    other_ms, other_n = E.ess_profile_read(s.ctx, E.ESS_KERNEL_OTHER)
    E.ess_profile(s.ctx, False)
    rej = int(s.rejections().sum())
    s.close()

    value = C * args.steps / dt
    flops_per_launch = 4.0 * m * d * C           # A x' and A nu for every chain
    split_off = os.environ.get("ESS_PROJ") == "f32"
    proj_avg_s = proj_ms / max(proj_n, 1) / 1e3
    achieved = flops_per_launch / proj_avg_s / 1e12 if proj_n else None
    traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gp_rbf", "d": d, "m": m, "chains": C,
                   "storage": "f32",
                   "projections": ("f32 MFMA, f32 accumulate" if split_off else
                                   "f32 operands split exactly into three bf16 pieces, six "
                                   "bf16 MFMA products (dropped terms < 2^-24 |a x|), f32 "
                                   "accumulate; error vs f64 below the f32 MFMA kernel's"),
                   "roots": "f32 pretest drops b/r >= 1.01; z = b/r = b rsqrt(p^2 + q^2) in f64; "
                            "tau = f32 atan2(q, p); phi = acos z = 2 asin sqrt((1 - |z|)/2) "
                            "(mirrored for z < 0) in f32 from f64 1 - |z|",
                   "interval_ends_and_sampling": "f64", "trim_eps": 1e-6, "seed": 0},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_FP32_MFMA_TFLOPS) if achieved else None,
                     "traffic": traffic,
                     "kernel": ("proj_gemm_f32 (A x' and A nu, 4 m d C flop per launch)" if split_off
                                else "proj_gemm_split (A x' and A nu, 4 m d C algorithmic flop "
                                     "per launch; float32 contraction, so the float32 matrix "
                                     "peak is its roofline)")},
        "kernels_ms_per_step": {"project": proj_ms / max(proj_n, 1),
                                "sample": samp_ms / max(samp_n, 1),
                                "other": other_ms / args.steps,
                                "other_launches_per_run": other_n},
        "timing": "value: one K-step graph replay; kernel durations: the same K steps "
                  "launched one by one with HIP events around each launch",
        "rejections": rej,
    }
    if achieved and not split_off:
        # the bfloat16 matrix-core work actually issued: six products per
        # multiply-add of the float32 contraction
        out["roofline"]["executed_bf16"] = {"tflops": 6 * achieved, "peak": 2500.0,
                                            "frac": 6 * achieved / 2500.0}
    if not args.no_extras:
        log = lambda msg: print(msg, file=sys.stderr, flush=True)
        cpu_s = 0.0 if args.no_cpu_baseline else 5.0
        out["configs"] = [
            bench_config(E, torch, synth.small_fp64(), 64, 2000, cpu_s, 16),
            bench_config(E, torch, synth.box_halfspace(), 32, 1000, cpu_s, 64),
        ]
        log(f"configs: {out['configs']}")
        out["batched"] = bench_batched(E, torch)
        out["warm_start"] = bench_warm_start(E, torch, log, args.warm_steps)
        out["paper_timing"] = bench_paper_timing(E, torch, paper_dims)
        out["trim_sweep"] = bench_trim_sweep(E, torch)
        log(f"trim sweep: {out['trim_sweep']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
