"""Benchmark of the multislice Leiden path on one MI355X.

One step = one complete solve (mslm_leiden: every Leiden iteration, level, sweep,
refinement round, aggregation, split and the Q components) on a supra-graph that is
already resident in HBM.  Prints one JSON line (see the keys below).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3|cfg2|cfg1]
                    [--null-model multislice|global] [--no-cpu-baseline]
    python bench.py --workload cfg4 [--graphs 512]         # batched grid vs plain calls
    python bench.py --workload cfg5 [--requests 1000]      # served Poisson trace vs plain FIFO
    python bench.py --workload sweep                      # doubling N, edges, T (Table 1 SBMs)
    python bench.py --workload spectral [--spectral-graph cfg2|cfg3]   # Bethe-Hessian pathway
    python bench.py --workload long                       # windowed Patent/School-shaped runs
    python bench.py --workload variants                   # objective/input variants, config 2
    python bench.py --copy-calibration                     # 3 plain 1 GiB device copies

The default workload is config 3 (T=64 x N=1M DC-SBM, omega=1/2), the largest instance that
fits one GPU.  The timed steps run without instrumentation; the roofline comes from one extra
solve whose level-0 decision launches are bracketed by HIP events on the solve stream, and the
algorithmic bytes from one counting solve (the schedule is deterministic, so both do exactly the
work of every timed step).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time
from fractions import Fraction

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "Leiden supra-edge TEPS + %HBM peak; batched solves/s vs plain; p99 latency"

# algorithmic bytes of the level-0 decision kernels (see the design notes):
#   per unit decided: batch id 4 + row pointers 8 + own label 4 + degree 4 + decision 4
#   per adjacency entry scanned: column 4 + neighbour label 4 (+ weight 4 when weighted)
#   per candidate community: one Sigma(C, s) slot probe 8
BYTES_UNIT, BYTES_ENTRY, BYTES_WEIGHT, BYTES_CAND = 24, 8, 4, 8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, workers, cache=None):
    """The named workload's graph and solve parameters.  cache: a .npz path holding the graph
    drawn by an earlier run of the same workload (written there when absent), so that profiled
    runs can skip the multi-process generator."""
    from paper_2608_03695_amd import gen
    if cache:
        import numpy as np
        spec = {"cfg1": gen.CONFIG_SOLVE[1], "cfg2": gen.CONFIG_SOLVE[2],
                "cfg3": gen.CONFIG_SOLVE[3]}[name]
        if os.path.exists(cache):
            z = np.load(cache, allow_pickle=False)
            if str(z["name"]).startswith(name + "_"):
                w = z["weight"] if z["weight"].size else None
                tg = gen.TemporalGraph(int(z["n_nodes"]), int(z["n_slices"]), z["offsets"],
                                       z["src"], z["dst"], w, None, str(z["name"]))
                return tg, spec
        tg, _ = workload(name, workers)
        np.savez(cache, n_nodes=tg.n_nodes, n_slices=tg.n_slices, offsets=tg.offsets,
                 src=tg.src, dst=tg.dst,
                 weight=tg.weight if tg.weight is not None else np.zeros(0, np.int32),
                 name=tg.name)
        return tg, spec
    if name == "cfg1":
        return gen.config1(), gen.CONFIG_SOLVE[1]
    if name == "cfg2":
        return gen.config2(workers), gen.CONFIG_SOLVE[2]
    if name == "cfg3":
        return gen.config3(workers), gen.CONFIG_SOLVE[3]
    raise SystemExit(f"unknown workload {name}")


def host_cpu():
    """CPU model and the host threads this process may use (for the baseline's label)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


NULL_MODELS = {"multislice": 0, "global": 1}


def full_size_oracle(workload, null_model="multislice"):
    """The oracle's full-size solve time recorded with the committed expected result of this
    workload (taken once on a build host, not on the benchmark host), or None."""
    suffix = "_global" if null_model == "global" else ""
    path = os.path.join(ROOT, "tests", "golden",
                        f"{workload.split('_')[0]}{suffix}_expected.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return rec.get("oracle_timing")


def cpu_baseline(args):
    """The oracle, as it stands, on a bounded sample of the same workload: the workload's
    generator at a smaller size (same degree law, mixing, churn, weights, omega and gamma).
    Config 2 is small enough to run whole."""
    import oracle
    from paper_2608_03695_amd import gen
    if args.workload == "cfg3":
        tg = gen.dcsbm(250_000, 4, 10, 250, 0.4, 2.1, 0.02, weights_max=1, seed=3,
                       name="cfg3_law_N250k_T4")
        omega, gamma = Fraction(1, 2), 1
        what = ("config-3 generator law (exponent 2.1, mean degree 10, mu 0.4, churn 0.02, "
                "unit weights, omega 1/2) at N=250k x T=4, 250 communities")
    elif args.workload == "cfg2":
        tg = gen.config2(args.gen_workers)
        omega, gamma, what = 1, 1, "config 2 itself (N=100k x T=16), the whole workload"
    else:
        tg = gen.config1()
        omega, gamma, what = 1, 1, "config 1 itself, the whole workload"
    og = oracle.OracleGraph(tg, omega)
    rp, col, w, raw, twom = og.csr()
    m_supra = int(rp[-1]) // 2
    t0 = time.perf_counter()
    og.leiden(gamma, max_levels=32, max_iterations=2, seed=0,
              null_model=NULL_MODELS[args.null_model])
    dt = time.perf_counter() - t0
    model, avail = host_cpu()
    out = {"value": m_supra / dt, "unit": "supra-edges/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"{tg.name}: {what}; {m_supra} supra-edges, one full solve "
                     f"(2 iterations, {args.null_model} null model) in {dt:.1f} s",
           "host_cpu": model, "host_threads_available": avail}
    full = full_size_oracle(args.workload, args.null_model)
    if full is not None:
        out["full_size_oracle"] = full
    return out


def roofline(nbytes, ms, launches, kernel):
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
            "bytes_per_step": nbytes, "kernel_ms_per_step": ms, "launches_per_step": launches,
            "avg_launch_us": ms * 1e3 / max(launches, 1)}


def device_copy_gbs(torch):
    """Read+write bandwidth of a plain 1 GiB device-to-device copy, by HIP events."""
    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "device.hpp", "engine_solve.inc"):
        with open(os.path.join(ROOT, "paper_2608_03695_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, launches, null_model="multislice"):
    """HBM bytes per launch of the level-0 decision kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a 1 GiB copy), or None when the
    summary is for another workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "lm0_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("workload") != workload or rec.get("sources_sha256") != kernel_sources_sha():
        return None
    if null_model != "multislice":   # the record is of the multislice solve
        return None
    if rec.get("launches") != launches:
        return None
    return (rec["fetch_bytes"] + rec["write_bytes"]) / rec["launches"]


def _digest(memb, res):
    import hashlib
    h = hashlib.sha256(memb.astype("int32").tobytes())
    h.update(res["q_components"].astype("int64").tobytes())
    return h.hexdigest()


def bench_batched(args):
    """Config 4: the (graph x gamma x omega) grid of the batched workload as one batched call
    (mslm_batch_leiden, run in chunks of bounded size) against the same solves as one plain
    mslm_leiden call each, over the same resident graphs; every result must be identical."""
    from paper_2608_03695_amd import gen
    ng = args.graphs
    log(f"generating {ng} batched-workload graphs")
    tgs = gen.batch_graphs(range(ng), workers=args.gen_workers)
    import torch
    from paper_2608_03695_amd import mslm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    handles = [mslm.Graph(tg, 1) for tg in tgs]
    m_supra = sum(h.info()["nnz"] // 2 for h in handles)
    tuning = None
    if args.autotune:
        # tune on the batch's largest graph; a batch runs with the tuning of its first solve's graph
        big = max(range(ng), key=lambda i: handles[i].info()["nnz"])
        tu, ms0, ms1 = handles[big].autotune(1, 1, rounds=1)
        for h in handles:   # batched and plain calls alike
            h.set_tuning(**tu)
        tuning = {"chosen": tu, "tuned_on_graph": big, "ms_default": ms0, "ms_tuned": ms1}
        log(f"autotune on graph {big}: {tu} ({ms0:.1f} -> {ms1:.1f} ms)")
    solves = [(g, sp.gamma, sp.omega, sp.max_levels, sp.max_iterations, sp.seed)
              for g, sp in gen.batch_solves(ng)]
    log(f"{len(solves)} solves over {ng} graphs ({m_supra} supra-edges); warm-up")
    mslm.batch_leiden(handles, solves[: min(len(solves), 18)])
    torch.cuda.synchronize()
    # batched calls of 576 solves each (the library chunks further by size); a progress line
    # after each keeps long runs visibly alive
    dig_batch = []
    t_batch = 0.0
    step = 576
    for c0 in range(0, len(solves), step):
        t0 = time.perf_counter()
        got = mslm.batch_leiden(handles, solves[c0:c0 + step])
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
        dig_batch += [_digest(m, r) for m, r in got]
        del got
        log(f"batched {min(c0 + step, len(solves))}/{len(solves)}: {t_batch:.1f} s")
    # plain calls on every k-th solve of the grid (k = --plain-sample), same order
    picked = list(range(0, len(solves), max(1, args.plain_sample)))
    t0 = time.perf_counter()
    same = 0
    for n_done, i in enumerate(picked):
        gi, gam, om, lv, it, seed = solves[i]
        m, r = handles[gi].leiden(gam, om, max_levels=lv, max_iterations=it, seed=seed)
        same += _digest(m, r) == dig_batch[i]
        if n_done % 200 == 199:
            log(f"plain {n_done + 1}/{len(picked)}")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    return {
        "metric": "batched solves/s vs plain (config 4)",
        "value": len(solves) / t_batch, "unit": "solves/s",
        "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"cfg4_batched_{ng}_graphs_x_9_solves", "graphs": ng,
                   "solves": len(solves), "supra_edges_per_grid_point": m_supra},
        "batched_s": t_batch, "plain_sample": f"every {max(1, args.plain_sample)}th solve",
        "plain_s": t_plain, "plain_solves_per_s": len(picked) / t_plain,
        "speedup_vs_plain": (len(solves) / t_batch) / (len(picked) / t_plain),
        "identical_results": f"{same}/{len(picked)} sampled solves",
        "tuning": tuning,
    }


def bench_served(args):
    """Config 5: Poisson request stream through the continuous-batching server (admission by
    footprint, worker slots on their own streams) against a FIFO replay of the same trace
    through plain create + leiden + destroy, one request at a time."""
    import threading
    import numpy as np
    from paper_2608_03695_amd import gen
    ng = args.graphs
    log(f"generating {ng} batched-workload graphs and 8 config-2-sized graphs")
    small = gen.batch_graphs(range(ng), workers=args.gen_workers)
    large = [gen.large_serve_graph(i, workers=args.gen_workers) for i in range(8)]
    import torch
    from paper_2608_03695_amd import mslm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    free, total = torch.cuda.mem_get_info()
    budget = int(free * 0.6)

    def requests(rate):
        out = []
        for rq in gen.serve_trace(args.requests, rate, n_graphs=ng):
            tg = large[rq["graph"]] if rq["large"] else small[rq["graph"]]
            out.append((rq["t"], tg, rq["spec"]))
        return out

    def run_server(reqs, realtime):
        srv = mslm.Server(budget, max_slots=args.slots)
        tickets = [None] * len(reqs)
        done = {}

        def submit():
            t0 = time.perf_counter()
            for i, (t, tg, sp) in enumerate(reqs):
                if realtime:
                    dt = t - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                tickets[i] = srv.submit(tg, sp.gamma, sp.omega, sp.max_levels,
                                        sp.max_iterations, sp.seed)
        th = threading.Thread(target=submit)
        t0 = time.perf_counter()
        th.start()
        th.join()
        lat = []
        for i in range(len(reqs)):
            m, r, l = srv.wait(tickets[i])
            done[i] = _digest(m, r)
            lat.append(l)
            if i % 200 == 199:
                log(f"served {i + 1}/{len(reqs)}")
        t_all = time.perf_counter() - t0
        srv.close()
        return np.array(lat), t_all, done

    # capacity: every request submitted at once
    reqs0 = requests(1.0)
    log("capacity run")
    lat0, t0_all, _ = run_server([(0.0, tg, sp) for _, tg, sp in reqs0], False)
    capacity = len(reqs0) / t0_all
    rate = 0.7 * capacity
    reqs = requests(rate)
    log(f"capacity {capacity:.1f} solves/s; Poisson replay at {rate:.1f}/s")
    lat, t_all, dig_srv = run_server(reqs, True)
    # FIFO replay through plain calls on the same arrival times
    log("plain FIFO replay")
    lat_p = []
    dig_plain = {}
    t0 = time.perf_counter()
    for i, (t, tg, sp) in enumerate(reqs):
        now = time.perf_counter() - t0
        if now < t:
            time.sleep(t - now)
        g = mslm.Graph(tg, sp.omega)
        m, r = g.leiden(sp.gamma, sp.omega, max_levels=sp.max_levels,
                        max_iterations=sp.max_iterations, seed=sp.seed)
        g.close()
        lat_p.append(time.perf_counter() - t0 - t)
        dig_plain[i] = _digest(m, r)
        if i % 200 == 199:
            log(f"plain {i + 1}/{len(reqs)}")
    t_plain = time.perf_counter() - t0
    lat_p = np.array(lat_p)
    same = sum(dig_srv[i] == dig_plain[i] for i in range(len(reqs)))
    return {
        "metric": "served p50/p99 latency and solves/s vs plain FIFO (config 5)",
        "value": len(reqs) / t_all, "unit": "solves/s",
        "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "cfg5_poisson_mix", "requests": len(reqs), "graphs": ng,
                   "large_fraction": 0.05, "slots": args.slots, "budget_bytes": budget,
                   "rate_per_s": rate},
        "capacity_solves_per_s": capacity,
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "plain_p50_s": float(np.percentile(lat_p, 50)),
        "plain_p99_s": float(np.percentile(lat_p, 99)),
        "plain_solves_per_s": len(reqs) / t_plain,
        "identical_results": f"{same}/{len(reqs)}",
    }


def bench_sweep(args):
    """The doubling study of the paper's Fig. 2b on the SBM shapes of its Table 1: full solves
    (2 iterations) of the base graph and of the graphs with N, the edges and T doubled, under
    the multislice objective (Eq. 6) and the global null model (the objective the paper timed),
    with inputs resident; the ratio of each doubled shape's time to the base's."""
    from paper_2608_03695_amd import gen
    spec = gen.SWEEP_SOLVE
    graphs = {name: gen.sweep_graph(name, workers=min(args.gen_workers, 10))
              for name in gen.SWEEP_SHAPES}
    import torch
    from paper_2608_03695_amd import mslm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    stream = torch.cuda.current_stream()
    rows = {}
    for name, tg in graphs.items():
        g = mslm.Graph(tg, spec.omega, stream=stream)
        info = g.info()
        row = dict(N=tg.n_nodes, T=tg.n_slices, edges=int(tg.n_edges),
                   supra_edges=info["nnz"] // 2)
        for nm, key in ((0, "multislice"), (1, "global")):
            kw = dict(gamma=spec.gamma, max_levels=spec.max_levels,
                      max_iterations=spec.max_iterations, seed=spec.seed, null_model=nm)
            for _ in range(args.warmup):
                g.leiden(**kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, r = g.leiden(**kw)
            torch.cuda.synchronize()
            row[f"ms_{key}"] = (time.perf_counter() - t0) * 1000.0 / args.steps
            row[f"communities_{key}"] = r["n_communities"]
            row[f"q_{key}"] = r["q"]
        g.close()
        rows[name] = row
        log(f"{name}: {row}")
    base = rows["sbm"]
    for name, row in rows.items():
        for key in ("multislice", "global"):
            row[f"x_{key}"] = row[f"ms_{key}"] / base[f"ms_{key}"]
    return {"metric": "solve time of the SBM doubling study (Table 1 shapes)",
            "value": base["ms_multislice"], "unit": "ms per solve (base shape)",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "sweep_sbm_table1_doubling", "gamma": str(spec.gamma),
                       "omega": str(spec.omega), "iterations": spec.max_iterations},
            "shapes": rows}


def bench_spectral(args):
    """The Bethe-Hessian pathway (Section 3.1) on a config graph: H(r) with the default r, the
    k smallest eigenpairs by Lanczos, k-means of the embedding; inputs resident.  The roofline
    is that of the operator launches (HBM-bound): per launch the row pointers, columns, raw
    weights (weighted graphs), one 8-byte x read per entry, and d, x and y once per row."""
    tg, spec = workload(args.spectral_graph, args.gen_workers, args.graph_cache)
    import torch
    from paper_2608_03695_amd import mslm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    stream = torch.cuda.current_stream()
    g = mslm.Graph(tg, spec.omega, stream=stream)
    info = g.info()
    n, nnz = info["n_supra"], info["nnz"]
    k = args.spectral_k
    kw = dict(seed=1, embedding=False, lanczos_steps=args.spectral_steps)
    for _ in range(args.warmup):
        g.bethe_hessian(k, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        ev, _, lab, res = g.bethe_hessian(k, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    weighted = tg.weight is not None
    per_launch = 8 * (n + 1) + nnz * (4 + (4 if weighted else 0) + 8) + 24 * n
    launch_ms = res["spmv_ms"] / max(1, res["spmv_launches"])
    achieved = per_launch / (launch_ms * 1e-3) / 1e9
    g.close()
    return {"metric": "Bethe-Hessian pathway (Lanczos + k-means) per solve", "value": ms,
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"spectral_{tg.name}", "k": k, "omega": str(spec.omega),
                       "supra_nodes": n, "csr_entries": nnz},
            "eigenvalues": [float(x) for x in ev], "result": res,
            "roofline": {"bound": "hbm", "kernel": "k_bh_apply", "achieved": achieved,
                         "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                         "bytes_per_launch": per_launch, "kernel_ms_per_launch": launch_ms,
                         "traffic": None}}


def bench_long(args):
    """Windowed optimisation (Section 4, the School case) of the two long sequences shaped like
    Table 1's Patent (T = 891) and School (T = 7375), present-only coupling, windows of 64
    snapshots overlapping by 8, 2 iterations per window.  The windowed entry takes host edge
    lists, so each window's upload and supra-CSR build are inside the timed region."""
    import hashlib

    import numpy as np
    from paper_2608_03695_amd import gen
    spec = gen.LONG_SOLVE
    w, o = gen.LONG_WINDOW
    graphs = {name: gen.long_graph(name) for name in gen.LONG_SHAPES}
    import torch
    from paper_2608_03695_amd import mslm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    stream = torch.cuda.current_stream()
    kw = dict(gamma=spec.gamma, max_levels=spec.max_levels, max_iterations=spec.max_iterations,
              seed=spec.seed, present_only=True, stream=stream)
    rows = {}
    for name, tg in graphs.items():
        for _ in range(args.warmup):
            mslm.leiden_windowed(tg, spec.omega, w, o, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            memb, res = mslm.leiden_windowed(tg, spec.omega, w, o, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        sha = hashlib.sha256(np.ascontiguousarray(memb, dtype=np.int32).tobytes()).hexdigest()
        rows[name] = dict(N=tg.n_nodes, T=tg.n_slices, edges=int(tg.n_edges),
                          windows=res["windows"], ms=ms, ms_per_window=ms / res["windows"],
                          n_communities=res["n_communities"], sha256=sha)
        log(f"{name}: {rows[name]}")
    return {"metric": "windowed solve time of the long sequences (Table 1 shapes)",
            "value": rows["patent"]["ms"], "unit": "ms per solve (Patent shape)", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "long_sequences_patent_school_windowed",
                       "gamma": str(spec.gamma), "omega": str(spec.omega), "window": w,
                       "overlap": o, "present_only": True,
                       "iterations": spec.max_iterations},
            "shapes": rows}


def bench_variants(args):
    """The objective and input variants on config 2's graph (inputs resident, 1 warm-up and
    --steps timed solves each): per-slice resolutions, the multislice CPM, a warm start from
    the default solve's labels, categorical (all-to-all) coupling, and present-only coupling
    on the graph with 20 % of the node copies absent."""
    from paper_2608_03695_amd import gen
    tg, spec = workload("cfg2", args.gen_workers, args.graph_cache)
    tga = gen.with_absences(tg, 0.2, seed=1)
    T = tg.n_slices
    cat = [[0 if s == r else 1 for r in range(T)] for s in range(T)]
    import torch
    from paper_2608_03695_amd import mslm
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    stream = torch.cuda.current_stream()
    base = dict(gamma=spec.gamma, max_levels=spec.max_levels,
                max_iterations=spec.max_iterations, seed=spec.seed)
    g = mslm.Graph(tg, spec.omega, stream=stream)
    m0, _ = g.leiden(**base)
    cases = [
        ("multislice", g, base),
        ("per_slice_gamma", g, dict(base, gamma_slices=[Fraction(1, 2), Fraction(1), Fraction(2)]
                                    * (T // 3) + [Fraction(1)] * (T % 3))),
        ("cpm", g, dict(base, gamma=Fraction(1, 1000), null_model=mslm.MSLM_NULL_CPM)),
        ("warm_start", g, dict(base, initial=m0)),
    ]
    gc = mslm.Graph(tg, spec.omega, coupling=cat, stream=stream)
    cases.append(("categorical_coupling", gc, base))
    ga = mslm.Graph(tga, spec.omega, present_only=True, stream=stream)
    cases.append(("present_only_20pct_absent", ga, base))
    rows = {}
    for name, h, kw in cases:
        for _ in range(args.warmup):
            h.leiden(**kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, r = h.leiden(**kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        m_supra = h.info()["nnz"] // 2
        rows[name] = dict(ms=ms, supra_edges=m_supra, supra_edges_per_s=m_supra / (ms * 1e-3),
                          n_communities=r["n_communities"], sweeps=r["sweeps"],
                          levels=r["levels_run"])
        log(f"{name}: {rows[name]}")
    for h in (g, gc, ga):
        h.close()
    return {"metric": "supra-edge TEPS of the objective and input variants (config 2 graph)",
            "value": rows["multislice"]["supra_edges_per_s"], "unit": "supra-edges/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "variants_" + tg.name, "gamma": str(spec.gamma),
                       "omega": str(spec.omega)},
            "variants": rows}


def copy_calibration():
    """Three plain 1 GiB device-to-device copies (2^30 bytes read and 2^30 written each): the
    run that calibrates the FETCH_SIZE / WRITE_SIZE counters under rocprofv3 --pmc."""
    import torch
    n = 1 << 28                      # 2^28 int32 = 1 GiB
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied 3 x {b.numel() * 4} bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--null-model", choices=sorted(NULL_MODELS), default="multislice",
                    help="cfg1/cfg2/cfg3: the objective (multislice: Eq. 6; global: Eq. 5 over "
                         "the supra-graph, the objective of the paper's GPU path)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-count", action="store_true",
                    help="skip the profiled and the counting solve (keeps profiler traces to "
                         "the timed steps)")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes drawing the synthetic snapshots (1 under a profiler)")
    ap.add_argument("--graphs", type=int, default=512, help="cfg4/cfg5: batched-workload graphs")
    ap.add_argument("--requests", type=int, default=1000, help="cfg5: requests in the trace")
    ap.add_argument("--slots", type=int, default=4, help="cfg5: server worker slots")
    ap.add_argument("--plain-sample", type=int, default=8,
                    help="cfg4: time plain calls on every k-th solve of the grid")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner (one round) before the warm-up; the "
                         "timed steps use the tuning it picks (results are the same)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain 1 GiB device copies (counter calibration)")
    ap.add_argument("--graph-cache", default=None,
                    help=".npz file holding the drawn graph (read when present, else written)")
    ap.add_argument("--spectral-graph", default="cfg2",
                    help="spectral: the config graph the Bethe-Hessian pathway runs on")
    ap.add_argument("--spectral-k", type=int, default=8, help="spectral: eigenvectors/clusters")
    ap.add_argument("--spectral-steps", type=int, default=0,
                    help="spectral: Lanczos steps (0: the library's default)")
    ap.add_argument("--gen-only", action="store_true",
                    help="draw the workload's graph (into --graph-cache) and stop")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              f"multi-GPU path", file=sys.stderr)
        raise SystemExit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    if args.workload in ("cfg4", "cfg5", "sweep", "spectral", "long", "variants"):
        out = {"cfg4": bench_batched, "cfg5": bench_served, "sweep": bench_sweep,
               "spectral": bench_spectral, "long": bench_long,
               "variants": bench_variants}[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    # inputs are drawn before anything touches the GPU (the generator may use child processes)
    log(f"generating {args.workload}")
    tg, spec = workload(args.workload, args.gen_workers, args.graph_cache)
    if args.gen_only:
        log(f"drew {tg.name}: N={tg.n_nodes} T={tg.n_slices} E={tg.n_edges}")
        return
    import torch
    from paper_2608_03695_amd import mslm

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    log(f"N={tg.n_nodes} T={tg.n_slices} E={tg.n_edges}; uploading")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_c0 = time.perf_counter()
    g = mslm.Graph(tg, spec.omega, stream=stream)
    torch.cuda.synchronize()
    ms_create = (time.perf_counter() - t_c0) * 1000.0   # host upload + supra-CSR build
    info = g.info()
    m_supra = info["nnz"] // 2
    kw = dict(gamma=spec.gamma, max_levels=spec.max_levels, max_iterations=spec.max_iterations,
              seed=spec.seed, null_model=NULL_MODELS[args.null_model])
    tuning = None
    if args.autotune:
        # result-invariant execution choices picked by timing solves (not part of a step)
        tu, ms0, ms1 = g.autotune(rounds=1, **kw)
        tuning = {"chosen": tu, "ms_default": ms0, "ms_tuned": ms1}
        log(f"autotune: {tu} ({ms0:.1f} -> {ms1:.1f} ms)")
    for i in range(args.warmup):
        g.leiden(**kw)
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        _, r = g.leiden(**kw)   # synchronous: the membership is on the host when it returns
        step_ms.append((time.perf_counter() - ts) * 1000.0)
        results.append(r)
        log(f"step {i} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("timed steps done")
    ms_step = (t1 - t0) * 1000.0 / args.steps
    copy_gbs = device_copy_gbs(torch)
    # the schedule is deterministic: one profiled solve times the level-0 decision launches
    # (HIP events on the solve stream) and one counting solve gives the exact work of a step
    zero = {k: 0 for k in ("lm_units", "lm_entries", "lm_candidates", "lm0_units",
                           "lm0_entries", "lm0_candidates", "lm0_kernel_ms", "lm0_launches")}
    if args.no_count:
        rp = rc = zero
    else:
        _, rp = g.leiden(profile=True, **kw)
        log("profiled solve done")
        _, rc = g.leiden(count=True, **kw)
        log("counting solve done")
        if rp["q_components"].tolist() != results[-1]["q_components"].tolist() or \
                rc["q_components"].tolist() != results[-1]["q_components"].tolist():
            raise SystemExit("profiled or counting solve differs from the timed solves")
    weighted = tg.weight is not None

    def nbytes(pre):
        return (rc[pre + "_units"] * BYTES_UNIT
                + rc[pre + "_entries"] * (BYTES_ENTRY + (BYTES_WEIGHT if weighted else 0))
                + rc[pre + "_candidates"] * BYTES_CAND)
    qf = mslm.q_exact_global if args.null_model == "global" else mslm.q_exact
    q = qf(results[-1]["q_components"], tg.n_slices, tg.n_nodes, spec.gamma, spec.omega)
    out = {
        "tuning": tuning,
        "metric": METRIC,
        "value": m_supra / (ms_step * 1e-3),
        "unit": "supra-edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": tg.name, "n_nodes": tg.n_nodes, "n_slices": tg.n_slices,
                   "supra_nodes": info["n_supra"], "supra_edges": m_supra,
                   "gamma": str(spec.gamma), "omega": str(spec.omega),
                   "null_model": args.null_model,
                   "max_levels": spec.max_levels, "max_iterations": spec.max_iterations},
        # the HBM-bound loop: level-0 local-moving decisions (every sweep of every iteration)
        "roofline": roofline(nbytes("lm0"), rp["lm0_kernel_ms"], rp["lm0_launches"],
                             "level-0 decision launches: k_lm0_groups (units of at most 32 "
                             "entries, large colour batches), k_lm_multi<Policy0, ViewP> (to 1024 "
                             "entries; all bins of small batches), k_lm_block<Policy0, ViewP, 1024> "
                             "(to 4096) and the hub kernels"),
        # the work of the aggregated levels' decisions (not timed: their launches are short)
        "bytes_all_levels": nbytes("lm"),
        "ms_per_step_median": statistics.median(step_ms),
        "ms_per_step_std": statistics.pstdev(step_ms),
        # the graph's upload and supra-CSR build, paid once per graph (not in value)
        "ms_create": ms_create,
        "value_incl_create": m_supra / ((ms_step + ms_create) * 1e-3),
        "phases_ms": {k: results[-1][k] for k in ("ms_colour", "ms_local_move", "ms_refine",
                                                  "ms_aggregate", "ms_finish")},
        "solve": {"Q": float(q), "n_communities": results[-1]["n_communities"],
                  "sweeps": results[-1]["sweeps"], "levels": results[-1]["levels_run"],
                  "iterations": results[-1]["iterations_run"],
                  "exact_fallbacks": results[-1]["exact_fallbacks"]},
    }
    rl = out["roofline"]
    rl["copy_gbs"] = copy_gbs                 # a plain device copy on this GPU, same clock
    rl["frac_of_copy"] = rl["achieved"] / copy_gbs if copy_gbs else None
    rl["bytes_per_launch"] = rl["bytes_per_step"] / max(rl["launches_per_step"], 1)
    t = measured_traffic(tg.name, rl["launches_per_step"], args.null_model)
    if t is not None:
        rl["traffic"] = t
        rl["traffic_gbs"] = t * rl["launches_per_step"] / (rl["kernel_ms_per_step"] * 1e-3) / 1e9
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
