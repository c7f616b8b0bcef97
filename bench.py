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

Records beside the headline (each can be switched off): ``potential`` (the
same call with the potential output), ``irregular`` (the irregular force
over the lists the call returned, per block size), ``corrector`` (the
regular corrector per block size), ``modes`` (the other two coordinate
modes on the same block: rate, and accuracy on the same oracle rows),
``load`` (nb6_load_particles from host arrays: the whole cluster and a
block's subset update), ``serving`` (a trace of many clusters' blocks served
through nb6_submit / nb6_poll against one block per launch).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_INTERACTION = 53
FP32_PEAK_TFLOPS = 157.3          # 256 CU x 2.4 GHz x 256 FLOP/clk
MODES = {"ff": 1, "fp64": 2, "fp32": 4, "local": 8}


# Counter figures of the force kernel (HBM traffic, FP32 VALU instruction
# counts) come from rocprofv3 counter runs of this script, summarised by
# --counter-summary into COUNTER_FILE.  They are reported only while the
# kernel sources are the ones the counters were taken from.
KERNEL_SOURCES = ("paper_1205_1222_amd/csrc/nb6_kernels.hip",
                  "paper_1205_1222_amd/csrc/nb6_internal.h")
COUNTER_FILE = os.path.join("profiles", "regf_{mode}_plummer131072_all_counters.md")
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_SALU",
                 "SQ_INSTS_SMEM", "SQ_WAVES")


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counter_rows(path, counter):
    with open(path, newline="") as f:
        return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(f)
                if r["Counter_Name"] == counter]


def _is_force(name):
    return "regf_kernel" in name or "regf_lanes_kernel" in name


def _median(v):
    v = sorted(v)
    return v[len(v) // 2]


def counter_summary(fetch_csv, write_csv, valu_csv, copy_mib, config_line, pairs, mode="local"):
    """Markdown summary of the counter runs of the force kernel: per-launch HBM
    bytes (each counter scaled by what it reads for the device copy of copy_mib
    MiB made at the start of the same run) and FP32 VALU instruction counts."""
    copy_bytes = copy_mib << 20
    res = {}
    kernel = None
    for name, path, counter in (("read", fetch_csv, "FETCH_SIZE"),
                                ("write", write_csv, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        copies = [v for k, v in rows if "copyBuffer" in k]
        regf = [(k, v) for k, v in rows if _is_force(k)]
        if not copies or not regf:
            raise SystemExit(f"{path}: no copy or force-kernel dispatch with {counter}")
        kernel = regf[0][0]
        factor = copy_bytes / (max(copies) * 1024.0)
        med = _median([v for _, v in regf])
        res[name] = {"counter": counter, "kib_per_launch": med, "copy_kib": max(copies),
                     "factor": round(factor, 4), "bytes": int(round(med * 1024.0 * factor))}
    valu = {}
    if valu_csv:
        for c in VALU_COUNTERS:
            vals = [v for k, v in _counter_rows(valu_csv, c) if _is_force(k)]
            if vals:
                valu[c] = _median(vals)
    machine = {"kernel": kernel, "source_sha256": kernel_source_hash(), "config": config_line,
               "read_bytes": res["read"]["bytes"], "write_bytes": res["write"]["bytes"]}
    flops = None
    if all(c in valu for c in VALU_COUNTERS[1:5]):
        # wave instructions x 64 lanes; an FMA counts 2, add / mul / transcendental 1
        flops = 64.0 * (valu["SQ_INSTS_VALU_ADD_F32"] + valu["SQ_INSTS_VALU_MUL_F32"] +
                        2.0 * valu["SQ_INSTS_VALU_FMA_F32"] + valu["SQ_INSTS_VALU_TRANS_F32"])
        machine["fp32_flop"] = flops
    def out_dir(csv_path):  # the rocprofv3 output directory that held a CSV
        return os.path.relpath(os.path.dirname(os.path.abspath(csv_path)), ROOT)

    cmd = ("python3 bench.py --steps 2 --warmup 1 --no-serving --no-cpu-baseline --no-irregular "
           "--no-potential --no-corrector --no-load --no-modes --no-blocks --no-c5 --no-small "
           f"--mode {mode} --copy-mib {copy_mib}")
    lines = [
        f"# Counters of the force kernel, Plummer N = 131072, all 131072 active ({mode} coordinates)",
        "",
        "rocprofv3 counter runs of the benchmark (one counter group per run).  Each run "
        f"begins with a {copy_mib} MiB device-to-device copy whose known size calibrates "
        "the traffic counters (bytes = counter KiB x 1024 x factor).  Figures are the "
        "median over the run's force launches.",
        "",
        "Commands (repo root, on the MI355X; then this summary from the CSV files):",
        "",
        f"    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -f csv -d {out_dir(fetch_csv)} "
        f"-o fetch -- {cmd}",
        f"    timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -f csv -d {out_dir(write_csv)} "
        f"-o write -- {cmd}",
    ] + ([
        f"    timeout -s KILL 120 rocprofv3 --pmc {' '.join(VALU_COUNTERS)} -f csv "
        f"-d {out_dir(valu_csv)} -o valu -- {cmd}",
    ] if valu_csv else []) + [
        f"    python3 bench.py --counter-summary {fetch_csv} {write_csv} {valu_csv or '-'} "
        f"--copy-mib {copy_mib} --mode {mode}",
        "",
        f"Kernel: `{kernel}`; config: {config_line}; {pairs:.4g} pair interactions per launch.",
        "",
        "| Traffic counter | calibration copy (KiB) | factor | force kernel (KiB / launch) "
        "| bytes / launch |",
        "|:--|--:|--:|--:|--:|",
    ]
    for name in ("read", "write"):
        r = res[name]
        lines.append(f"| {r['counter']} | {r['copy_kib']:.0f} | {r['factor']} | "
                     f"{r['kib_per_launch']:.0f} | {r['bytes'] / 1e6:.1f} MB |")
    if valu:
        lines += ["", "| VALU counter | per launch | per interaction (x64 lanes / pairs) |",
                  "|:--|--:|--:|"]
        for c in VALU_COUNTERS:
            if c in valu:
                lines.append(f"| {c} | {valu[c]:.4g} | {64.0 * valu[c] / pairs:.3f} |")
        if flops is not None:
            lines += ["", f"FP32 VALU FLOP per launch (FMA = 2): {flops:.4g}, "
                          f"{flops / pairs:.2f} per interaction."]
    lines += ["", "counter-record: " + json.dumps(machine), ""]
    return "\n".join(lines)


def counters_from_profile(config_line):
    """The counter record of the configuration's coordinate mode (COUNTER_FILE)
    when it was taken from the current kernel sources and the same
    configuration, else None."""
    mode = re.search(r"\bmode (\w+)", config_line)
    path = os.path.join(ROOT, COUNTER_FILE.format(mode=mode.group(1) if mode else "local"))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        m = re.search(r"^counter-record: (\{.*\})$", f.read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("config") != config_line:
        return None
    return rec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cl, idx, gpu_outs, cap, target_s):
    """Time the oracle on a sample of the block; compare the GPU rows of each
    coordinate mode in gpu_outs (name -> outputs) with it."""
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
    summaries = {}
    for name, (acc, jerk, nnb, lst) in gpu_outs.items():
        summaries[name] = compare(acc[samp], jerk[samp], nnb[samp], lst[samp], cap, ref, cl.m,
                                  xp, vp, si, cl.h2[si], cl.dtr[si]).summary()
    cores = oracle.max_threads()
    # the same oracle on one core, on a smaller sample (then all cores again)
    n1 = max(1, min(len(idx), int(ns * 2.0 / max(dt * cores, 1e-6))))
    s1 = idx[np.sort(order[:n1])]
    t0 = time.perf_counter()
    oracle.regular_force(cl.m, xp, vp, s1, cl.h2[s1], cl.dtr[s1], lcap=4096, nthreads=1)
    dt1 = time.perf_counter() - t0
    oracle.regular_force(cl.m, xp, vp, s1[:1], cl.h2[s1[:1]], cl.dtr[s1[:1]], lcap=4096,
                         nthreads=cores)
    base = {"value": pairs / dt / 1e9, "unit": "Ginteractions/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{ns} of the {len(idx)} active i against all {cl.n} j "
                      f"({pairs:.3g} pairs, {dt:.1f} s, FP64 C with OpenMP)",
            "single_core_value": n1 * (cl.n - 1) / dt1 / 1e9,
            "single_core_sample": f"{n1} i ({dt1:.1f} s, one thread)"}
    return base, summaries


def served_accuracy(cls, reqs, tbs, kept, cap, rows=128):
    """Served results of the kept requests against the oracle: each request's
    cluster predicted to its block time by the oracle, and up to ``rows``
    sampled rows of the request compared with the usual bars."""
    import oracle
    from oracle.compare import compare

    rng = np.random.Generator(np.random.PCG64(12051232))
    worst = {"acc_rel_max": 0.0, "acc_scaled_max": 0.0, "jerk_rel_max": 0.0,
             "jerk_scaled_max": 0.0}
    tot = {"requests": 0, "rows": 0, "list_mismatch": 0, "nnb_mismatch": 0,
           "exempt_pairs": 0, "incomplete": 0}
    sizes = []
    for k in sorted(kept):
        c, idx = reqs[k]
        cl = cls[c]
        a_, j_, n_, l_ = (t.cpu().numpy() for t in kept[k])
        samp = np.sort(rng.choice(len(idx), min(rows, len(idx)), replace=False))
        si = idx[samp]
        xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, tbs[k])
        ref = oracle.regular_force(cl.m, xp, vp, si, cl.h2[si], cl.dtr[si], lcap=4096)
        summ = compare(a_[samp], j_[samp], n_[samp], l_[samp, :cap], cap, ref, cl.m, xp, vp, si,
                       cl.h2[si], cl.dtr[si]).summary()
        tot["requests"] += 1
        tot["rows"] += len(samp)
        for key in ("list_mismatch", "nnb_mismatch", "exempt_pairs", "incomplete"):
            tot[key] += summ[key]
        for key in worst:
            worst[key] = max(worst[key], summ.get(key, 0.0))
        sizes.append((cl.n, len(idx)))
    out = {**tot, **worst,
           "largest": sorted(sizes, key=lambda t: t[0] * t[1])[-3:],
           "cluster_sizes": [min(t[0] for t in sizes), max(t[0] for t in sizes)],
           "block_sizes": [min(t[1] for t in sizes), max(t[1] for t in sizes)]}
    log(f"bench: served results against the oracle: {out}")
    return out


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
    # requests whose results are kept and checked against the oracle (first
    # offered load): 16 blocks of >= 4096 particles of the >= 32768-body
    # clusters, 16 more blocks of >= 4096, and 32 of any size
    rng_s = np.random.Generator(np.random.PCG64(12051231))
    big_cl = [k for k, (c, idx) in enumerate(reqs) if cls[c].n >= 32768 and len(idx) >= 4096]
    big = [k for k, (c, idx) in enumerate(reqs) if len(idx) >= 4096]
    pick = set(rng_s.choice(big_cl, min(16, len(big_cl)), replace=False).tolist())
    rest = [k for k in big if k not in pick]
    pick |= set(rng_s.choice(rest, min(16, len(rest)), replace=False).tolist())
    rest = [k for k in range(len(reqs)) if k not in pick]
    pick |= set(rng_s.choice(rest, min(32, len(rest)), replace=False).tolist())
    check_reqs = sorted(pick)
    kept = {}
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
            if rho == rhos[0] and k in pick:
                kept[k] = o
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
        admit = np.array([i["admit_us"] for i in infos]) * 1e-6
        done = np.array([i["done_us"] for i in infos]) * 1e-6
        # latency from the arrival time (the submit call happens at the arrival)
        lat_serve = done - sub + np.maximum(sub_wall - arrivals, 0.0)
        span_serve = done.max() - sub.min() + max(0.0, sub_wall[0] - arrivals[0])
        batch = np.array([i["batch_size"] for i in infos])
        run = {"rho": rho, "arrival_rate_per_s": round(rate, 1),
               "served": {"p50_ms": q(lat_serve, 0.5), "p99_ms": q(lat_serve, 0.99),
                          "ginteractions_s": round(total / span_serve / 1e9, 3),
                          "mean_batch": round(float(batch.mean()), 2),
                          "max_batch": int(batch.max()),
                          # submit -> admission, and admission -> completion
                          "queue_p50_ms": q(admit - sub, 0.5),
                          "queue_p99_ms": q(admit - sub, 0.99),
                          "exec_p50_ms": q(done - admit, 0.5),
                          "exec_p99_ms": q(done - admit, 0.99)},
               "plain": {"p50_ms": q(lat_plain, 0.5), "p99_ms": q(lat_plain, 0.99),
                         "ginteractions_s": round(total / span_plain / 1e9, 3)}}
        log(f"bench: rho={rho}: served p50/p99 = {run['served']['p50_ms']}/"
            f"{run['served']['p99_ms']} ms ({run['served']['ginteractions_s']} Gint/s, "
            f"mean batch {run['served']['mean_batch']}, queue/exec p50 "
            f"{run['served']['queue_p50_ms']}/{run['served']['exec_p50_ms']} ms); plain p50/p99 = "
            f"{run['plain']['p50_ms']}/{run['plain']['p99_ms']} ms "
            f"({run['plain']['ginteractions_s']} Gint/s)")
        runs.append(run)
    nb6.nb6_destroy(sctx)
    nb6.nb6_destroy(pctx)
    accuracy = served_accuracy(cls, reqs, tbs, kept, cap) if args.serve_check else None
    head = runs[0]
    return {
        "workload": "64 Plummer clusters, N log-uniform 4096..65536; blocks of 2^k random "
                    "active particles, k uniform in 4..floor(log2 N); Poisson arrivals",
        "requests": len(reqs), "list_cap": cap, "hbm_budget_mb": args.serve_budget_mb,
        "plain_service_ms": round(s_bar * 1e3, 4),
        "p50_ms": head["served"]["p50_ms"], "p99_ms": head["served"]["p99_ms"],
        "rho": head["rho"], "runs": runs, "accuracy": accuracy,
    }


# Algorithmic bytes of the irregular force: per list entry the entry itself
# and the stored FP64 state of j (m, t, x, v, a, jerk: 112 B); per active
# particle its index, list count, stored state and the two output vectors.
IRR_BYTES_PER_PAIR = 4 + 112
IRR_BYTES_PER_I = 4 + 4 + 112 + 48
HBM_PEAK_GBS = 8000.0


def irregular_leg(args, nb6, torch, ctx, cl, idx_np, idx_d, nnb, lst):
    """Irregular force (section 3.3 step 4) over the lists the last regular
    call produced: nb6_set_lists for the block, then nb6_irregular_force of the
    whole block and of smaller random sub-blocks.  Kernel times from HIP
    events on the (timing) context ``ctx``; wall time per call, back to back,
    on a second context without event timing holding the same state."""
    stream = torch.cuda.current_stream()
    dev = idx_d.device
    ni = len(idx_np)
    cap = lst.shape[1]
    cnt = torch.clamp(nnb, max=cap).contiguous()
    nb6.nb6_kernel_times(ctx)
    t0 = time.perf_counter()
    nb6.check(ctx, nb6.nb6_set_lists(ctx, 0, ni, idx_d, cnt, lst, cap, nb6.NB6_MEM_DEVICE,
                                     stream))
    torch.cuda.synchronize()
    set_ms = (time.perf_counter() - t0) * 1e3
    wctx = nb6.nb6_create(0)
    nb6.check(wctx, nb6.nb6_load_particles(wctx, 0, cl.n, cl.m, cl.x, cl.v, cl.a, cl.jerk,
                                           cl.t))
    nb6.check(wctx, nb6.nb6_set_lists(wctx, 0, ni, idx_d, cnt, lst, cap, nb6.NB6_MEM_DEVICE,
                                      stream))
    pairs_all = int(cnt.sum().item())
    acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    jerk = torch.empty_like(acc)
    res = {"set_lists_ms": round(set_ms, 4), "list_cap": cap,
           "mean_list": round(pairs_all / ni, 2), "blocks": []}
    rng = np.random.Generator(np.random.PCG64(12051229))
    cnt_h = cnt.cpu().numpy()
    for size in sorted({1, 64, 1024, 16384, ni}):
        if size > ni:
            continue
        sel = np.arange(ni) if size == ni else np.sort(rng.choice(ni, size, replace=False))
        sub = torch.from_numpy(idx_np[sel].astype(np.int32)).to(dev)
        pairs = int(cnt_h[sel].sum())
        reps = max(5, min(200, int(3e7 / max(pairs, 1))))

        def call(c):
            nb6.check(c, nb6.nb6_irregular_force(c, 0, cl.tb, size, sub, acc[:size],
                                                 jerk[:size], nb6.NB6_MEM_DEVICE, stream))
        for c in (ctx, wctx):
            call(c)
        torch.cuda.synchronize()
        nb6.nb6_kernel_times(ctx)
        for _ in range(reps):
            call(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            call(wctx)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        ms, counts = nb6.nb6_kernel_times(ctx)
        k_ms = ms[3] / max(counts[3], 1)
        byts = pairs * IRR_BYTES_PER_PAIR + size * IRR_BYTES_PER_I
        res["blocks"].append({"N_i": size, "pairs": pairs, "call_us": round(wall * 1e6, 2),
                              "kernel_us": round(k_ms * 1e3, 2),
                              "gpairs_s": round(pairs / (k_ms * 1e-3) / 1e9, 3),
                              "algorithmic_gb_s": round(byts / (k_ms * 1e-3) / 1e9, 1)})
        log(f"bench: irregular N_i={size}: {pairs} pairs, kernel {k_ms * 1e3:.2f} us, "
            f"call {wall * 1e6:.2f} us")
    nb6.check(ctx, nb6.nb6_sync_status(ctx, stream))
    nb6.check(wctx, nb6.nb6_sync_status(wctx, stream))
    nb6.nb6_destroy(wctx)
    whole = res["blocks"][-1]
    # a gather rate: algorithmic bytes over kernel time; most of the state
    # records are served from the MALL, so this is not an HBM counter figure
    res["roofline"] = {"bound": "hbm", "achieved": whole["algorithmic_gb_s"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(whole["algorithmic_gb_s"] / HBM_PEAK_GBS, 4),
                       "traffic": None,
                       "basis": "algorithmic gather bytes (list entries and 112-B state "
                                "records) per kernel time; the records mostly hit the MALL"}
    return res


# Algorithmic bytes of the regular corrector per particle: t_old, eight
# [3]-vectors of force values, h_old, nnb, n_p in; four [3]-vectors, dt_new
# and h_new out.
CORR_BYTES_PER_I = 8 + 8 * 24 + 8 + 4 + 8 + 4 * 24 + 16


# Host bytes of one particle's stored state (m, t, x, v, a, jerk), the unit
# of a host-array nb6_load_particles; a subset update adds its 4-byte index.
LOAD_BYTES_PER_PARTICLE = 8 + 8 + 4 * 24


def load_leg(nb6, cl, reps=5):
    """nb6_load_particles from host arrays (copies and synchronisation
    included): the whole cluster, and a 4096-particle subset update (the
    corrector output of a block)."""
    ctx = nb6.nb6_create(0)
    n = cl.n
    arrays = [np.ascontiguousarray(a) for a in (cl.m, cl.x, cl.v, cl.a, cl.jerk, cl.t)]
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, *arrays))  # allocation
    t0 = time.perf_counter()
    for _ in range(reps):
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, *arrays))
    full = (time.perf_counter() - t0) / reps
    rng = np.random.Generator(np.random.PCG64(12051230))
    idx = np.sort(rng.choice(n, min(4096, n), replace=False)).astype(np.int32)
    sub = [np.ascontiguousarray(a[idx]) for a in arrays]
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, len(idx), *sub, idx))
    t0 = time.perf_counter()
    for _ in range(reps * 20):
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, len(idx), *sub, idx))
    part = (time.perf_counter() - t0) / (reps * 20)
    nb6.nb6_destroy(ctx)
    out = {"full_n": n, "full_ms": round(full * 1e3, 4),
           "full_gb_s": round(n * LOAD_BYTES_PER_PARTICLE / full / 1e9, 2),
           "subset_n": len(idx), "subset_us": round(part * 1e6, 2),
           "subset_gb_s": round(len(idx) * (LOAD_BYTES_PER_PARTICLE + 4) / part / 1e9, 2)}
    log(f"bench: load from host arrays: {out}")
    return out


def corrector_leg(args, nb6, torch, cl, nnb):
    """Regular corrector (section 3.3 step 7) of blocks of the configuration:
    device arrays, synthetic force values of the right magnitudes, the step
    of each particle its own regular step; back-to-back calls timed with
    events on the library's stream.  HBM-bound: roofline against 8 TB/s."""
    stream = torch.cuda.current_stream()
    dev = torch.device("cuda:0")
    n_all = len(nnb)
    rng = np.random.Generator(np.random.PCG64(12051230))
    t = 1.0
    vec = lambda scale: torch.from_numpy(rng.normal(0.0, scale, (n_all, 3))).to(dev)
    arrays = {"t_old": torch.from_numpy(t - cl.dtr[:n_all]).to(dev),
              "f_old": vec(1.0), "fd_old": vec(10.0), "f_new": vec(1.0), "fd_new": vec(10.0),
              "g_old": vec(0.1), "gd_old": vec(1.0), "g_new": vec(0.1), "gd_new": vec(1.0),
              "h_old": torch.from_numpy(np.sqrt(cl.h2[:n_all])).to(dev),
              "nnb": nnb.to(torch.int32).contiguous(),
              "n_p": torch.full((n_all,), 50.0, dtype=torch.float64, device=dev)}
    for k in ("df", "dfd", "f2", "f3"):
        arrays[k] = torch.empty((n_all, 3), dtype=torch.float64, device=dev)
    for k in ("dt_new", "h_new"):
        arrays[k] = torch.empty(n_all, dtype=torch.float64, device=dev)
    ctx = nb6.nb6_create(0)
    params = (0.02, 2.0 ** -20, 1.0, 0.5, 1.25)
    res = {"bytes_per_particle": CORR_BYTES_PER_I, "blocks": []}
    for size in sorted({1, 1024, 16384, n_all}):
        if size > n_all:
            continue
        sub = {k: v[:size] for k, v in arrays.items()}

        def call():
            nb6.check(ctx, nb6.nb6_regular_correct(ctx, size, t, sub, params,
                                                   nb6.NB6_MEM_DEVICE, stream))
        call()
        torch.cuda.synchronize()
        reps = max(20, min(2000, int(2e8 / (size * CORR_BYTES_PER_I))))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = size * CORR_BYTES_PER_I / (us * 1e-6) / 1e9
        res["blocks"].append({"N_i": size, "call_us": round(us, 2),
                              "algorithmic_gb_s": round(gbs, 1)})
        log(f"bench: corrector N_i={size}: {us:.2f} us per call, {gbs:.1f} GB/s algorithmic")
    nb6.check(ctx, nb6.nb6_sync_status(ctx, stream))
    nb6.nb6_destroy(ctx)
    whole = res["blocks"][-1]
    res["roofline"] = {"bound": "hbm", "achieved": whole["algorithmic_gb_s"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(whole["algorithmic_gb_s"] / HBM_PEAK_GBS, 4),
                       "traffic": None,
                       "basis": "algorithmic bytes per whole call on the stream (events "
                                "around back-to-back calls: includes the per-call launch "
                                "gap, about 11 us)"}
    return res


def potential_leg(args, nb6, torch, ctx, idx_d, h2_d, dtr_d, ni, mode, regf_ms, pairs):
    """The same force call with the optional potential output: force-kernel
    time against the call without it (one FP32 add per pair and a seventh
    partial component)."""
    stream = torch.cuda.current_stream()
    dev = idx_d.device
    acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    jerk = torch.empty_like(acc)
    pot = torch.empty(ni, dtype=torch.float64, device=dev)
    nnb = torch.empty(ni, dtype=torch.int32, device=dev)
    lst = torch.empty((ni, max(args.cap, 1)), dtype=torch.int32, device=dev)

    def call():
        nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, ni, idx_d, h2_d, dtr_d, mode, acc, jerk,
                                             nnb, lst, args.cap, nb6.NB6_MEM_DEVICE, stream,
                                             pot=pot))
    call()
    torch.cuda.synchronize()
    nb6.nb6_kernel_times(ctx)
    reps = max(3, min(20, int(args.steps)))
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    ms, cnt = nb6.nb6_kernel_times(ctx)
    k_ms = ms[1] / max(cnt[1], 1)
    log(f"bench: regular force with potential: kernel {k_ms:.4f} ms vs {regf_ms:.4f} ms")
    return {"kernel_ms": round(k_ms, 5), "kernel_ms_without": round(regf_ms, 5),
            "overhead_pct": round(100.0 * (k_ms / regf_ms - 1.0), 2),
            "kernel_ginteractions_s": round(pairs / (k_ms * 1e-3) / 1e9, 3),
            "finalize_ms": round(ms[2] / max(cnt[2], 1), 5)}


def block_sweep(args, cfg, nb6, torch, T, lanes=0, slices=None, max_ni=None, max_reps=200,
                host=True, emit=True):
    """Force-call time for every block of the configuration: wall time per call
    on a context without event timing (back-to-back calls on one stream, so
    host launch cost shows only where it exceeds the GPU time), per-kernel GPU
    times on a second context with event timing, and (with ``host``) the same
    call with host arrays.  Returns one record per block (and prints each as a
    JSON line with ``emit``)."""
    cl = cfg["cluster"]
    n = cl.n
    stream = torch.cuda.current_stream()
    mode = MODES[args.mode]
    slices = args.slices if slices is None else slices
    ctxs = []
    for flags in (0, nb6.NB6_OPT_TIMING):
        ctx = nb6.nb6_create(0, flags=flags, ipl_hint=args.ipl, slice_hint=slices,
                             jl_hint=lanes)
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, cl.m, cl.x, cl.v, cl.a, cl.jerk,
                                              cl.t))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, mode, stream))
        ctxs.append(ctx)
    records = []
    for name, idx in sorted(cfg["blocks"].items(), key=lambda kv: len(kv[1])):
        ni = len(idx)
        if max_ni is not None and ni > max_ni:
            continue
        idx_d, h2_d, dtr_d = T(idx, torch.int32), T(cl.h2[idx]), T(cl.dtr[idx])
        acc = torch.empty((ni, 3), dtype=torch.float64, device="cuda:0")
        jerk = torch.empty_like(acc)
        nnb = torch.empty(ni, dtype=torch.int32, device="cuda:0")
        lst = torch.empty((ni, args.cap), dtype=torch.int32, device="cuda:0")
        reps = max(3, min(max_reps, int(2e11 / max(ni * n, 1))))

        def call(ctx):
            nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, ni, idx_d, h2_d, dtr_d, mode, acc,
                                                 jerk, nnb, lst, args.cap, nb6.NB6_MEM_DEVICE,
                                                 stream))
        out = []
        for k, ctx in enumerate(ctxs):
            call(ctx)
            torch.cuda.synchronize()
            if k == 1:
                nb6.nb6_kernel_times(ctx)
            t0 = time.perf_counter()
            for _ in range(reps):
                call(ctx)
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t0) / reps)
        wall = out[0]
        ms, cnt = nb6.nb6_kernel_times(ctxs[1])
        pairs = ni * (n - 1)
        ipl, jl, ns, slen = nb6.nb6_last_plan(ctxs[1])
        force_ms = ms[1] / cnt[1]
        rec = {"block": name, "N": n, "N_i": ni, "mode": args.mode,
               "ipl": ipl, "lanes": jl, "slices": ns, "slice_len": slen,
               "forced": [lanes, slices], "reps": reps,
               "call_us": round(wall * 1e6, 2),
               "force_us": round(force_ms * 1e3, 2),
               "finalize_us": round(ms[2] / max(cnt[2], 1) * 1e3, 2),
               "call_gint_s": round(pairs / wall / 1e9, 3),
               "force_gint_s": round(pairs / (force_ms * 1e-3) / 1e9, 3),
               "force_frac": round(FLOP_PER_INTERACTION * pairs / (force_ms * 1e-3) / 1e12
                                   / FP32_PEAK_TFLOPS, 4)}
        if host:
            # the same call with host arrays in and out (copies and
            # synchronisation included), as a host program without device
            # buffers would make it
            h_idx, h_h2, h_dtr = idx.astype(np.int32), cl.h2[idx].copy(), cl.dtr[idx].copy()
            h_out = (np.empty((ni, 3)), np.empty((ni, 3)), np.empty(ni, np.int32),
                     np.empty((ni, args.cap), np.int32))
            host_reps = max(3, reps // 4)
            for k in range(host_reps + 1):
                if k == 1:
                    t0 = time.perf_counter()
                nb6.check(ctxs[0], nb6.nb6_regular_force(
                    ctxs[0], 0, ni, h_idx, h_h2, h_dtr, mode, *h_out, args.cap,
                    nb6.NB6_MEM_HOST), (nb6.NB6_OK, nb6.NB6_WARN_NB_OVERFLOW))
            rec["host_call_us"] = round((time.perf_counter() - t0) / host_reps * 1e6, 2)
        records.append(rec)
        if emit:
            print(json.dumps(rec), flush=True)
    for ctx in ctxs:
        nb6.nb6_destroy(ctx)
    return records


def small_config_leg(ci, block, args, nb6, torch, with_oracle):
    """A parity configuration as a measured line: C1 (1024 bodies, all
    active) or C2 (16384 bodies, a random block of 1024 on stored state
    predicted to the block time).  Every coordinate mode: wall time per call
    back to back (device arrays, a context without event timing), force and
    finalize kernel times (HIP events, a second context), rate; and its
    accuracy on the whole block against the oracle."""
    import oracle
    from oracle.compare import compare
    from workloads import config

    cfg = config(ci)
    cl = cfg["cluster"]
    idx = cfg["blocks"][block]
    n, ni = cl.n, len(idx)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    T = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    cap = args.cap
    res = {"workload": cfg["description"] + f"; block {block}", "N": n, "N_i": ni,
           "list_cap": cap, "modes": {}}
    # the wall clock on a context without event timing (its event records
    # would add host time to every call), the kernel times on one with it
    ctx = nb6.nb6_create(0)
    ctx_t = nb6.nb6_create(0, flags=nb6.NB6_OPT_TIMING)
    try:
        for c in (ctx, ctx_t):
            nb6.check(c, nb6.nb6_load_particles(c, 0, n, cl.m, cl.x, cl.v, cl.a, cl.jerk, cl.t))
            nb6.check(c, nb6.nb6_predict_j(c, 0, cl.tb, 0, stream))
        idx_d, h2_d, dtr_d = T(idx, torch.int32), T(cl.h2[idx]), T(cl.dtr[idx])
        acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty_like(acc)
        nnb = torch.empty(ni, dtype=torch.int32, device=dev)
        lst = torch.empty((ni, cap), dtype=torch.int32, device=dev)
        pairs = ni * (n - 1)
        if with_oracle:
            xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
            ref = oracle.regular_force(cl.m, xp, vp, idx, cl.h2[idx], cl.dtr[idx], lcap=4096)
        reps = 50
        for name in [args.mode] + [m for m in sorted(MODES) if m != args.mode]:
            def call(c):
                nb6.check(c, nb6.nb6_regular_force(c, 0, ni, idx_d, h2_d, dtr_d, MODES[name],
                                                   acc, jerk, nnb, lst, cap,
                                                   nb6.NB6_MEM_DEVICE, stream))
            call(ctx_t)
            call(ctx)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                call(ctx)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            nb6.nb6_kernel_times(ctx_t)
            for _ in range(reps):
                call(ctx_t)
            ms, cnt = nb6.nb6_kernel_times(ctx_t)
            call(ctx)  # the outputs the accuracy is taken from
            torch.cuda.synchronize()
            rec = {"call_us": round(wall * 1e6, 2),
                   "force_us": round(ms[1] / max(cnt[1], 1) * 1e3, 2),
                   "finalize_us": round(ms[2] / max(cnt[2], 1) * 1e3, 2),
                   "ginteractions_s": round(pairs / wall / 1e9, 3),
                   "plan": nb6.nb6_last_plan(ctx)}
            if with_oracle:
                summ = compare(acc.cpu().numpy(), jerk.cpu().numpy(), nnb.cpu().numpy(),
                               lst.cpu().numpy(), cap, ref, cl.m, xp, vp, idx, cl.h2[idx],
                               cl.dtr[idx]).summary()
                keys = ("n_i", "list_mismatch", "exempt_pairs", "nnb_mismatch", "acc_rel_max",
                        "acc_scaled_max", "jerk_rel_max", "jerk_scaled_max")
                rec["accuracy"] = {k: summ[k] for k in keys if k in summ}
            res["modes"][name] = rec
        for c in (ctx, ctx_t):
            nb6.check(c, nb6.nb6_sync_status(c, stream))
    finally:
        nb6.nb6_destroy(ctx)
        nb6.nb6_destroy(ctx_t)
    log(f"bench: C{ci} {block}: " + ", ".join(
        f"{k} {v['call_us']} us" for k, v in res["modes"].items()))
    return res


def c5_leg(args, nb6, torch, with_oracle, cpu_seconds):
    """C5: the 2^20-body Plummer sphere (equal masses, ~100 neighbours).  Every
    coordinate mode's force on all 2^20 active particles (force-kernel time
    from events, whole call from the wall clock), and each mode's accuracy on
    the configuration's 10^4 sampled active particles against the oracle (one
    oracle run, timed: the CPU rate at this size)."""
    import oracle
    from oracle.compare import compare
    from workloads import config

    t_gen = time.perf_counter()
    cfg = config(5)
    cl = cfg["cluster"]
    n = cl.n
    log(f"bench: C5 inputs in {time.perf_counter() - t_gen:.1f} s")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    T = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    ctx = nb6.nb6_create(0, flags=nb6.NB6_OPT_TIMING)
    cap = args.cap
    res = {"workload": cfg["description"], "N": n, "list_cap": cap, "modes": {}}
    try:
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, cl.m, cl.x, cl.v, cl.a, cl.jerk,
                                              cl.t))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, 0, stream))
        idx = cfg["blocks"]["all"]
        idx_d, h2_d, dtr_d = T(idx, torch.int32), T(cl.h2[idx]), T(cl.dtr[idx])
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty_like(acc)
        nnb = torch.empty(n, dtype=torch.int32, device=dev)
        lst = torch.empty((n, cap), dtype=torch.int32, device=dev)
        pairs = n * (n - 1)
        order = [args.mode] + [m for m in sorted(MODES) if m != args.mode]
        for name in order:
            def call():
                nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, n, idx_d, h2_d, dtr_d, MODES[name],
                                                     acc, jerk, nnb, lst, cap,
                                                     nb6.NB6_MEM_DEVICE, stream))
            call()
            torch.cuda.synchronize()
            nb6.nb6_kernel_times(ctx)
            t0 = time.perf_counter()
            for _ in range(2):
                call()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / 2
            ms, cnt = nb6.nb6_kernel_times(ctx)
            f_ms = ms[1] / cnt[1]
            res["modes"][name] = {
                "call_ms": round(wall * 1e3, 3), "kernel_ms": round(f_ms, 3),
                "ginteractions_s": round(pairs / wall / 1e9, 3),
                "kernel_ginteractions_s": round(pairs / (f_ms * 1e-3) / 1e9, 3),
                "pct_fp32_peak": round(100.0 * FLOP_PER_INTERACTION * pairs / (f_ms * 1e-3)
                                       / 1e12 / FP32_PEAK_TFLOPS, 2),
                "slices": nb6.nb6_last_slices(ctx)}
            log(f"bench: C5 all active, {name}: {res['modes'][name]}")
        nb6.check(ctx, nb6.nb6_sync_status(ctx, stream))
        del acc, jerk, nnb, lst
        if with_oracle:
            samp = cfg["blocks"]["sample10000"]
            outs = {}
            for name in order:
                a_, j_, n_, l_, _ = nb6.regular_force_host(ctx, 0, samp, cl.h2[samp],
                                                           cl.dtr[samp], MODES[name], cap)
                outs[name] = (a_, j_, n_, l_)
            xp, vp = oracle.predict(cl.x, cl.v, cl.a, cl.jerk, cl.t, cl.tb)
            t0 = time.perf_counter()
            ref = oracle.regular_force(cl.m, xp, vp, samp, cl.h2[samp], cl.dtr[samp], lcap=4096)
            dt = time.perf_counter() - t0
            res["oracle"] = {"sample": f"{len(samp)} sampled active i against all {n} j",
                             "seconds": round(dt, 2),
                             "ginteractions_s": round(len(samp) * (n - 1) / dt / 1e9, 4),
                             "cores": oracle.max_threads()}
            keys = ("n_i", "list_mismatch", "exempt_pairs", "nnb_mismatch", "acc_rel_p99",
                    "acc_rel_max", "acc_scaled_max", "jerk_rel_p99", "jerk_rel_max",
                    "jerk_scaled_max", "jerk_rel_floor1e-3_max")
            for name, (a_, j_, n_, l_) in outs.items():
                summ = compare(a_, j_, n_, l_, cap, ref, cl.m, xp, vp, samp, cl.h2[samp],
                               cl.dtr[samp]).summary()
                res["modes"][name]["accuracy"] = {k: summ[k] for k in keys if k in summ}
                log(f"bench: C5 accuracy {name}: {res['modes'][name]['accuracy']}")
    finally:
        nb6.nb6_destroy(ctx)
    return res


def traffic_config(args):
    """The configuration a traffic record belongs to."""
    return (f"config {args.config} block {args.block} mode {args.mode} cap {args.cap} "
            f"ipl {args.ipl} slices {args.slices} lanes {args.lanes}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="local", choices=sorted(MODES))
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 5])
    ap.add_argument("--block", default="all")
    ap.add_argument("--cap", type=int, default=256)
    ap.add_argument("--ipl", type=int, default=0, help="i-particles per lane (0: auto)")
    ap.add_argument("--slices", type=int, default=0, help="j-slices (0: auto)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-irregular", action="store_true")
    ap.add_argument("--no-potential", action="store_true")
    ap.add_argument("--no-corrector", action="store_true")
    ap.add_argument("--no-load", action="store_true",
                    help="skip the host-array load timing")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the other coordinate modes' rate and accuracy")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the 2^20-body configuration's rates and accuracy")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the C1 and C2 configurations' rates and accuracy")
    ap.add_argument("--no-blocks", action="store_true",
                    help="skip the per-size curve (every power-of-two block of C3)")
    ap.add_argument("--no-serve-check", dest="serve_check", action="store_false",
                    help="skip the oracle check of sampled served requests")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-calibrate", type=int, default=300)
    ap.add_argument("--serve-cap", type=int, default=128)
    ap.add_argument("--serve-budget-mb", type=int, default=256,
                    help="serving HBM budget: above the largest request's footprint "
                         "(~140 MB), below what the fused batches would hold unchecked")
    ap.add_argument("--block-sweep", action="store_true",
                    help="time every block of the configuration (per-size curve) and exit")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per i-particle (0: auto)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy of this size first: the known-size kernel that "
                         "calibrates the FETCH_SIZE/WRITE_SIZE counters")
    ap.add_argument("--counter-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "VALU_CSV"),
                    help="write the force kernel's counter summary from three rocprofv3 "
                         "counter CSV files (with --copy-mib; '-' for no VALU run) to its "
                         "profiles/ file and exit")
    ap.add_argument("--rho", default="0.5,0.8,0.95,1.5,2.5",
                    help="offered load(s) as fractions of the plain form's capacity")
    args = ap.parse_args()

    if args.counter_summary:
        if args.copy_mib <= 0:
            sys.exit("--counter-summary needs --copy-mib (the calibration copy's size)")
        from workloads import config
        cfg = config(args.config)
        pairs = len(cfg["blocks"][args.block]) * (cfg["cluster"].n - 1)
        f_csv, w_csv, v_csv = args.counter_summary
        text = counter_summary(f_csv, w_csv, None if v_csv == "-" else v_csv, args.copy_mib,
                               traffic_config(args), pairs, args.mode)
        with open(os.path.join(ROOT, COUNTER_FILE.format(mode=args.mode)), "w") as f:
            f.write(text)
        print(text)
        return

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the library runs on one GPU "
              "(the multi-GPU j-split is described in the design notes, not implemented).",
              file=sys.stderr)
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
        block_sweep(args, cfg, nb6, torch, T, lanes=args.lanes)
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
                         slice_hint=args.slices, jl_hint=args.lanes)
    nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, n, m_d, x_d, v_d, a_d, j_d, t_d,
                                          mem_kind=nb6.NB6_MEM_DEVICE, stream=stream))

    def step(md=mode):
        nb6.check(ctx, nb6.nb6_load_particles(ctx, 0, ni, um_d, ux_d, uv_d, ua_d, uj_d, ut_d,
                                              idx_d, nb6.NB6_MEM_DEVICE, stream))
        nb6.check(ctx, nb6.nb6_predict_j(ctx, 0, cl.tb, md, stream))
        nb6.check(ctx, nb6.nb6_regular_force(ctx, 0, ni, idx_d, h2_d, dtr_d, md, acc, jerk,
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
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None,
                     "flop_convention": f"{FLOP_PER_INTERACTION} FP32 operations per "
                                        "interaction (the operation count of the paper's "
                                        "inner loop, rsqrt counted once)",
                     "kernel_ms": round(regf_ms, 5), "pairs": pairs},
    }
    rec = counters_from_profile(traffic_config(args))
    if rec is not None:
        out["roofline"]["traffic"] = rec["read_bytes"] + rec["write_bytes"]
        out["roofline"]["traffic_read"] = rec["read_bytes"]
        out["roofline"]["traffic_write"] = rec["write_bytes"]
        out["roofline"]["traffic_unit"] = "bytes per force launch"
        if "fp32_flop" in rec:
            # the second reading of the peak fraction: counted FP32 VALU work
            # (FMA = 2) of the counter runs over this run's kernel time
            out["pct_fp32_peak_counted"] = round(
                100.0 * rec["fp32_flop"] / (regf_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 2)
            out["roofline"]["frac_counted"] = round(out["pct_fp32_peak_counted"] / 100.0, 4)
    gpu_out = (acc.cpu().numpy(), jerk.cpu().numpy(), nnb.cpu().numpy(),
               lst[:, :args.cap].cpu().numpy())
    out["lists"] = {"cap": args.cap, "mean": round(float(gpu_out[2].mean()), 2),
                    "max": int(gpu_out[2].max()),
                    "overflowed": int((gpu_out[2] > args.cap).sum())}
    if not args.no_potential:
        out["potential"] = potential_leg(args, nb6, torch, ctx, idx_d, h2_d, dtr_d, ni, mode,
                                         regf_ms, pairs)
    if not args.no_irregular:
        out["irregular"] = irregular_leg(args, nb6, torch, ctx, cl, idx_np, idx_d, nnb, lst)
    if not args.no_corrector:
        out["corrector"] = corrector_leg(args, nb6, torch, cl, nnb)
    if not args.no_load:
        out["load"] = load_leg(nb6, cl)
    # the other coordinate modes on the same workload (after the legs that
    # read the headline call's lists): rate, and (with the CPU baseline)
    # accuracy on the same oracle rows as the headline mode
    mode_outs = {}
    if not args.no_modes:
        out["modes"] = {}
        for name in sorted(MODES):
            if name == args.mode:
                continue
            step(MODES[name])
            torch.cuda.synchronize()
            nb6.nb6_kernel_times(ctx)
            ks = max(1, min(args.steps, 10))
            t0 = time.perf_counter()
            for k in range(ks):
                step(MODES[name])
            torch.cuda.synchronize()
            m_ms = (time.perf_counter() - t0) * 1e3 / ks
            mk, ck = nb6.nb6_kernel_times(ctx)
            nb6.check(ctx, nb6.nb6_sync_status(ctx, stream))
            f_ms = mk[1] / max(ck[1], 1)
            out["modes"][name] = {
                "value": round(pairs / (m_ms * 1e-3) / 1e9, 3), "ms_per_step": round(m_ms, 4),
                "kernel_ginteractions_s": round(pairs / (f_ms * 1e-3) / 1e9, 3),
                "pct_fp32_peak": round(100.0 * FLOP_PER_INTERACTION * pairs / (f_ms * 1e-3)
                                       / 1e12 / FP32_PEAK_TFLOPS, 2)}
            mode_outs[name] = (acc.cpu().numpy(), jerk.cpu().numpy(), nnb.cpu().numpy(),
                               lst[:, :args.cap].cpu().numpy())
            log(f"bench: mode {name}: {out['modes'][name]}")
    nb6.nb6_destroy(ctx)
    del acc, jerk, nnb, lst
    if not args.no_blocks and args.config == 3:
        out["blocks"] = block_sweep(args, cfg, nb6, torch, T, host=False, emit=False,
                                    max_reps=100)
        log("bench: per-size curve: " + ", ".join(
            f"{r['N_i']}: {r['call_us']} us" for r in out["blocks"]))
    if not args.no_serving:
        out["serving"] = serving_leg(args, nb6, torch)
    if not args.no_small:
        out["c1"] = small_config_leg(1, "all", args, nb6, torch, not args.no_cpu_baseline)
        out["c2"] = small_config_leg(2, "random1024", args, nb6, torch, not args.no_cpu_baseline)
    if not args.no_c5:
        out["c5"] = c5_leg(args, nb6, torch, not args.no_cpu_baseline, args.cpu_seconds)
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a sample of the block ...")
        base, accuracy = cpu_baseline(cl, idx_np, {args.mode: gpu_out, **mode_outs}, args.cap,
                                      args.cpu_seconds)
        out["cpu_baseline"] = base
        out["accuracy"] = accuracy.pop(args.mode)
        keys = ("n_i", "list_mismatch", "exempt_pairs", "acc_rel_max", "acc_scaled_max",
                "jerk_rel_max", "jerk_scaled_max")
        for name, summ in accuracy.items():
            out["modes"][name]["accuracy"] = {k: summ[k] for k in keys if k in summ}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
