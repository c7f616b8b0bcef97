#!/usr/bin/env python3
"""Benchmark of the regular-force path on one MI355X.

One step is one pass of the whole hot path over one block:
  1. nb6_load_particles  -- corrector update of the active particles' stored
                            state (device-resident inputs),
  2. nb6_predict_j       -- FP64 prediction of all N j-particles,
  3. nb6_regular_force   -- force, jerk and neighbour lists of the block
                            (force kernel + slice reduction/list gather).

Default workload: Plummer N = 131072 with IMF masses 0.1-100 and 10 %
primordial binaries, all particles active (1.7e10 pair interactions per
step), float-float coordinates, neighbour-list capacity 256.

Prints ONE JSON line on stdout.  ``value`` is Ginteractions/s of the whole
step, N_i (N - 1) / step time.  ``roofline`` rates the force kernel alone:
53 FP32 operations per interaction (the operation count of the paper's inner
loop, rsqrt counted once) over its measured launch time, against the
MI355X FP32 vector peak.  ``cpu_baseline`` is the FP64 oracle timed on the
host cores for a bounded sample of the same block; its output for that
sample also gives the ``accuracy`` report of the GPU result.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_INTERACTION = 53
FP32_PEAK_TFLOPS = 157.3          # 256 CU x 2.4 GHz x 256 FLOP/clk
MODES = {"ff": 1, "fp64": 2, "fp32": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cl, idx, gpu_out, cap, target_s):
    """Time the oracle on a sample of the block; compare the GPU rows."""
    import oracle
    from oracle.compare import compare

    xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
    rng = np.random.Generator(np.random.PCG64(12051222))
    order = rng.permutation(len(idx))
    nprobe = min(len(idx), 64)
    probe = np.sort(order[:nprobe])
    t0 = time.perf_counter()
    oracle.regular_force(cl.m, xp, vp, idx[probe], cl.h2[idx[probe]], cl.dtr[idx[probe]],
                         lcap=4096)
    tp = time.perf_counter() - t0
    ns = int(min(len(idx), max(nprobe, nprobe * target_s / max(tp, 1e-6))))
    samp = np.sort(order[:ns])
    si = idx[samp]
    t0 = time.perf_counter()
    ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
    dt = time.perf_counter() - t0
    pairs = ns * (cl.n - 1)
    acc, jerk, nnb, lst = gpu_out
    c = compare(acc[samp], jerk[samp], nnb[samp], lst[samp], cap, ref, cl.m, xp, vp, si,
                cl.h2[si], cl.dtr[si])
    base = {"value": pairs / dt / 1e9, "unit": "Ginteractions/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{ns} of the {len(idx)} active i against all {cl.n} j "
                      f"({pairs:.3g} pairs, {dt:.1f} s, FP64 C with OpenMP)"}
    return base, c.summary()


def serving_leg(args, nb6, torch):
    """Serving trace: 64 Plummer clusters (N log-uniform 4096..65536), blocks of
    2^k random active particles, open-loop Poisson arrivals at rho times the
    capacity of the plain form (one block per launch, FIFO on one stream).
    Both forms serve the same arrival sequence; latency = finish - arrival."""
    import threading

    from workloads import serving_trace

    t_gen = time.perf_counter()
    tr = serving_trace(n_requests=args.serve_requests)
    cls, reqs = tr["clusters"], tr["requests"]
    log(f"bench: serving trace: {len(cls)} clusters, {sum(tr['sizes'])} particles, "
        f"{len(reqs)} requests, inputs in {time.perf_counter() - t_gen:.1f} s")
    dev = torch.device("cuda:0")
    cap = args.serve_cap
    mode = MODES[args.mode]
    # block times: successive blocks of each cluster
    seen = [0] * len(cls)
    tbs = []
    for c, idx in reqs:
        tbs.append(cls[c].tb + seen[c] * 2.0 ** -12)
        seen[c] += 1
    # device-resident inputs of every request
    idx_all = np.concatenate([idx for _, idx in reqs]).astype(np.int32)
    h2_all = np.concatenate([cls[c].h2[idx] for c, idx in reqs])
    dtr_all = np.concatenate([cls[c].dtr[idx] for c, idx in reqs])
    off = np.concatenate([[0], np.cumsum([len(idx) for _, idx in reqs])])
    d_idx = torch.from_numpy(idx_all).to(dev)
    d_h2 = torch.from_numpy(h2_all).to(dev)
    d_dtr = torch.from_numpy(dtr_all).to(dev)
    work = np.array([len(idx) * (cls[c].n - 1) for c, idx in reqs], dtype=np.float64)

    def outputs(ni):
        return (torch.empty((ni, 3), dtype=torch.float64, device=dev),
                torch.empty((ni, 3), dtype=torch.float64, device=dev),
                torch.empty(ni, dtype=torch.int32, device=dev),
                torch.empty((ni, max(cap, 1)), dtype=torch.int32, device=dev))

    def load(ctx):
        for c, cl in enumerate(cls):
            nb6.check(ctx, nb6.nb6_load_particles(ctx, c, cl.n, cl.m, cl.x, cl.v, cl.a,
                                                  cl.jerk, cl.t))

    # ---- plain form: one block per launch, FIFO on one stream ----------------
    pctx = nb6.nb6_create(0)
    load(pctx)
    stream = torch.cuda.current_stream()
    outs = outputs(int(max(len(idx) for _, idx in reqs)))

    def plain_one(k):
        c, idx = reqs[k]
        ni = len(idx)
        a, j, nn, ls = outs
        nb6.check(pctx, nb6.nb6_predict_j(pctx, c, tbs[k], mode, stream))
        nb6.check(pctx, nb6.nb6_regular_force(
            pctx, c, ni, d_idx[off[k]:off[k + 1]], d_h2[off[k]:off[k + 1]],
            d_dtr[off[k]:off[k + 1]], mode, a[:ni], j[:ni], nn[:ni], ls[:ni], cap,
            nb6.NB6_MEM_DEVICE, stream))
        torch.cuda.synchronize()

    for k in range(min(20, len(reqs))):  # warm-up (allocations)
        plain_one(k)
    ncal = min(len(reqs), args.serve_calibrate)
    t0 = time.perf_counter()
    for k in range(ncal):
        plain_one(k)
    s_bar = (time.perf_counter() - t0) / ncal
    rhos = [float(x) for x in str(args.rho).split(",")]
    log(f"bench: plain service {s_bar * 1e3:.3f} ms/block")

    def wait_until(t_start, t_rel):
        while True:
            d = t_start + t_rel - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 2e-4) if d > 2e-4 else 0)

    def q(a, p):
        return round(float(np.quantile(a, p)) * 1e3, 4)

    total = work.sum()
    runs = []
    sctx = nb6.nb6_create(0, hbm_budget=args.serve_budget_mb << 20)
    load(sctx)
    # warm-up: start the queue and allocate every cluster's record stream
    warm = []
    for c, cl in enumerate(cls):
        o = outputs(16)
        wi = torch.arange(16, dtype=torch.int32, device=dev)
        rc, t = nb6.nb6_submit(sctx, c, cl.tb, mode, 16, wi, d_h2[:16], d_dtr[:16],
                               o[0], o[1], o[2], o[3], cap, nb6.NB6_MEM_DEVICE)
        nb6.check(sctx, rc)
        warm.append((t, o, wi))
    for t, _, _ in warm:
        nb6.nb6_poll(sctx, t, 1)
    del warm
    for rho in rhos:
        rate = rho / s_bar
        rng = np.random.Generator(np.random.PCG64(12051226))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))

        # plain form on the same arrival sequence
        lat_plain = np.empty(len(reqs))
        t_start = time.perf_counter()
        for k in range(len(reqs)):
            wait_until(t_start, arrivals[k])
            plain_one(k)
            lat_plain[k] = time.perf_counter() - t_start - arrivals[k]
        span_plain = time.perf_counter() - t_start

        # serving form: continuous batching through nb6_submit / nb6_poll
        tickets = [None] * len(reqs)
        infos = [None] * len(reqs)
        live = {}
        ready = threading.Semaphore(0)
        errors = []

        def poller():
            for k in range(len(reqs)):
                ready.acquire()
                rc, info = nb6.nb6_poll(sctx, tickets[k], 1)
                if rc not in (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW):
                    errors.append((k, rc))
                infos[k] = info
                live.pop(k, None)

        th = threading.Thread(target=poller)
        th.start()
        t_start = time.perf_counter()
        sub_wall = np.empty(len(reqs))
        for k in range(len(reqs)):
            c, idx = reqs[k]
            ni = len(idx)
            o = outputs(ni)
            live[k] = o
            wait_until(t_start, arrivals[k])
            sub_wall[k] = time.perf_counter() - t_start
            rc, t = nb6.nb6_submit(sctx, c, tbs[k], mode, ni, d_idx[off[k]:off[k + 1]],
                                   d_h2[off[k]:off[k + 1]], d_dtr[off[k]:off[k + 1]],
                                   o[0], o[1], o[2], o[3], cap, nb6.NB6_MEM_DEVICE)
            nb6.check(sctx, rc)
            tickets[k] = t
            ready.release()
        th.join()
        if errors:
            raise RuntimeError(f"served requests failed: {errors[:5]}")
        sub = np.array([i["submit_us"] for i in infos]) * 1e-6
        done = np.array([i["done_us"] for i in infos]) * 1e-6
        # latency from the arrival time (the submit call happens at the arrival)
        lat_serve = done - sub + np.maximum(sub_wall - arrivals, 0.0)
        span_serve = done.max() - sub.min() + max(0.0, sub_wall[0] - arrivals[0])
        batch = np.array([i["batch_size"] for i in infos])
        run = {"rho": rho, "arrival_rate_per_s": round(rate, 1),
               "served": {"p50_ms": q(lat_serve, 0.5), "p99_ms": q(lat_serve, 0.99),
                          "ginteractions_s": round(total / span_serve / 1e9, 3),
                          "mean_batch": round(float(batch.mean()), 2),
                          "max_batch": int(batch.max())},
               "plain": {"p50_ms": q(lat_plain, 0.5), "p99_ms": q(lat_plain, 0.99),
                         "ginteractions_s": round(total / span_plain / 1e9, 3)}}
        log(f"bench: rho={rho}: served p50/p99 = {run['served']['p50_ms']}/"
            f"{run['served']['p99_ms']} ms ({run['served']['ginteractions_s']} Gint/s, "
            f"mean batch {run['served']['mean_batch']}); plain p50/p99 = "
            f"{run['plain']['p50_ms']}/{run['plain']['p99_ms']} ms "
            f"({run['plain']['ginteractions_s']} Gint/s)")
        runs.append(run)
    nb6.nb6_destroy(sctx)
    nb6.nb6_destroy(pctx)
    head = runs[0]
    return {
        "workload": "64 Plummer clusters, N log-uniform 4096..65536; blocks of 2^k random "
                    "active particles, k uniform in 4..floor(log2 N); Poisson arrivals",
        "requests": len(reqs), "list_cap": cap, "hbm_budget_mb": args.serve_budget_mb,
        "plain_service_ms": round(s_bar * 1e3, 4),
        "p50_ms": head["served"]["p50_ms"], "p99_ms": head["served"]["p99_ms"],
        "rho": head["rho"], "runs": runs,
    }


def block_sweep(args, cfg, nb6, torch, T):
    """Force-call time for every block of the configuration (one JSON line each)."""
    cl = cfg["cluster"]
    n = cl.n
    stream = torch.cuda.current_stream()
    mode = MODES[args.mode]
    ctx = nb6.nb6_create(0, flags=nb6.NB6_OPT_TIMING, ipl_hint=args.ipl, slice_hint=args.slices)
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, cl.m, cl.x, cl.v, cl.a, cl.jerk, cl.t))
    nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, mode, stream))
    for name, idx in sorted(cfg["blocks"].items(), key=lambda kv: len(kv[1])):
        ni = len(idx)
        idx_d, h2_d, dtr_d = T(idx, torch.int32), T(cl.h2[idx]), T(cl.dtr[idx])
        acc = torch.empty((ni, 3), dtype=torch.float64, device="cuda:0")
        jerk = torch.empty_like(acc)
        nnb = torch.empty(ni, dtype=torch.int32, device="cuda:0")
        lst = torch.empty((ni, args.cap), dtype=torch.int32, device="cuda:0")
        reps = max(3, min(200, int(2e11 / max(ni * n, 1))))

        def call():
            nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, ni, idx_d, h2_d, dtr_d, mode, acc,
                                                 jerk, nnb, lst, args.cap, nb6.NB6_MEM_DEVICE,
                                                 stream))
        call()
        torch.cuda.synchronize()
        nb6.nb6_kernel_times(ctx)
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        ms, cnt = nb6.nb6_kernel_times(ctx)
        pairs = ni * (n - 1)
        print(json.dumps({"block": name, "N": n, "N_i": ni, "mode": args.mode,
                          "slices": nb6.nb6_last_slices(ctx), "reps": reps,
                          "call_us": round(wall * 1e6, 2),
                          "force_us": round(ms[1] / cnt[1] * 1e3, 2),
                          "finalize_us": round(ms[2] / cnt[2] * 1e3, 2),
                          "call_gint_s": round(pairs / wall / 1e9, 3),
                          "force_gint_s": round(pairs / (ms[1] / cnt[1] * 1e-3) / 1e9, 3)}),
              flush=True)
    nb6.nb6_destroy(ctx)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="ff", choices=sorted(MODES))
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 5])
    ap.add_argument("--block", default="all")
    ap.add_argument("--cap", type=int, default=256)
    ap.add_argument("--ipl", type=int, default=0, help="i-particles per lane (0: auto)")
    ap.add_argument("--slices", type=int, default=0, help="j-slices (0: auto)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--serve-calibrate", type=int, default=300)
    ap.add_argument("--serve-cap", type=int, default=128)
    ap.add_argument("--serve-budget-mb", type=int, default=1024)
    ap.add_argument("--block-sweep", action="store_true",
                    help="time every block of the configuration (per-size curve) and exit")
    ap.add_argument("--isa-rates", action="store_true",
                    help="only run the vector-instruction issue-rate probe and exit")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy of this size first: the known-size kernel that "
                         "calibrates the FETCH_SIZE/WRITE_SIZE counters")
    ap.add_argument("--rho", default="0.8,0.95,1.5",
                    help="offered load(s) as fractions of the plain form's capacity")
    args = ap.parse_args()

    if args.isa_rates:
        import subprocess
        probe = os.path.join(ROOT, "paper_1205_1222_amd", "isa_rates")
        if not os.path.exists(probe):
            sys.exit(f"{probe} is missing: run python -m paper_1205_1222_amd.build")
        sys.exit(subprocess.run([probe]).returncode)

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build measures one "
              "GPU only (the multi-GPU j-split is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1205_1222_amd import nb6
    from workloads import config

    if args.copy_mib > 0:
        n_el = (args.copy_mib << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_mib} MiB device to device (counter calibration)")
        del src, dst

    t_gen = time.perf_counter()
    cfg = config(args.config)
    cl = cfg["cluster"]
    idx_np = cfg["blocks"][args.block]
    n, ni = cl.n, len(idx_np)
    log(f"bench: config {args.config} ({cfg['description']}), block {args.block}: "
        f"N={n} N_i={ni}, inputs in {time.perf_counter() - t_gen:.1f} s")

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    T = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    if args.block_sweep:
        block_sweep(args, cfg, nb6, torch, T)
        return
    m_d, x_d, v_d, a_d, j_d, t_d = (T(q) for q in (cl.m, cl.x, cl.v, cl.a, cl.jerk, cl.t))
    idx_d = T(idx_np, torch.int32)
    # corrector output of the active particles (device-resident)
    um_d, ux_d, uv_d, ua_d, uj_d, ut_d = (
        T(q[idx_np]) for q in (cl.m, cl.x, cl.v, cl.a, cl.jerk, cl.t))
    h2_d = T(cl.h2[idx_np])
    dtr_d = T(cl.dtr[idx_np])
    acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    jerk = torch.empty_like(acc)
    nnb = torch.empty(ni, dtype=torch.int32, device=dev)
    lst = torch.empty((ni, max(args.cap, 1)), dtype=torch.int32, device=dev)
    mode = MODES[args.mode]

    ctx = nb6.nb6_create(0, flags=nb6.NB6_OPT_TIMING, ipl_hint=args.ipl,
                         slice_hint=args.slices)
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, m_d, x_d, v_d, a_d, j_d, t_d,
                                          mem_kind=nb6.NB6_MEM_DEVICE, stream=stream))

    def step():
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, ni, um_d, ux_d, uv_d, ua_d, uj_d, ut_d,
                                              idx_d, nb6.NB6_MEM_DEVICE, stream))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, mode, stream))
        nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, ni, idx_d, h2_d, dtr_d, mode, acc, jerk,
                                             nnb, lst, args.cap, nb6.NB6_MEM_DEVICE, stream))

    for w in range(args.warmup):
        step()
    torch.cuda.synchronize()
    nb6.check(ctx, nb6.nb6_sync_status(ctx, stream))
    nb6.nb6_kernel_times(ctx)  # drop the warm-up launches
    log(f"bench: warm-up done ({args.warmup} steps), slices={nb6.nb6_last_slices(ctx)}")

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_k, cnt_k = nb6.nb6_kernel_times(ctx)
    nb6.check(ctx, nb6.nb6_sync_status(ctx, stream))
    ev_ms = ev0.elapsed_time(ev1)
    log(f"bench: {args.steps} steps in {wall * 1e3:.2f} ms wall, {ev_ms:.2f} ms events; "
        f"kernel ms (predict, force, finalize) = {ms_k.round(4).tolist()}")

    pairs = ni * (n - 1)
    ms_step = wall * 1e3 / args.steps
    value = pairs / (ms_step * 1e-3) / 1e9
    regf_ms = ms_k[1] / max(cnt_k[1], 1)
    achieved = FLOP_PER_INTERACTION * pairs / (regf_ms * 1e-3) / 1e12
    out = {
        "metric": "Ginteractions/s regular force+jerk+nblist, %FP32 peak; p50/p99 block latency",
        "value": round(value, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": cfg["description"] + f"; block {args.block}",
            "N": n, "N_i": ni, "dx_mode": args.mode, "list_cap": args.cap,
            "seed": cfg["seed"], "slices": nb6.nb6_last_slices(ctx),
        },
        "pct_fp32_peak": round(100.0 * achieved / FP32_PEAK_TFLOPS, 2),
        "kernel_ginteractions_s": round(pairs / (regf_ms * 1e-3) / 1e9, 3),
        "kernel_ms": {"predict": ms_k[0] / max(cnt_k[0], 1), "force": regf_ms,
                      "finalize": ms_k[2] / max(cnt_k[2], 1)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None},
    }
    gpu_out = (acc.cpu().numpy(), jerk.cpu().numpy(), nnb.cpu().numpy(),
               lst[:, :args.cap].cpu().numpy())
    nb6.nb6_destroy(ctx)
    del acc, jerk, nnb, lst
    if not args.no_serving:
        out["serving"] = serving_leg(args, nb6, torch)
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a sample of the block ...")
        base, accuracy = cpu_baseline(cl, idx_np, gpu_out, args.cap, args.cpu_seconds)
        out["cpu_baseline"] = base
        out["accuracy"] = accuracy
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
