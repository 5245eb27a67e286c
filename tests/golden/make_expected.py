"""Write the oracle's expected results for the larger parity workloads.

Runs only the oracle (oracle/), never the HIP library: for each workload it records the
sha256 of the oracle's int32 membership, its Q components and schedule statistics.  The
GPU parity tests compare the HIP path's output against these files.

    python tests/golden/make_expected.py [cfg2] [cfg3] [cfg2_global] [cfg3_global] [cfg4]
                                         [sweep] [long]

Config 3 needs about 45 GB of host memory and tens of minutes on 8 threads.  cfg4 records the
oracle's digest (sha256 of the int32 membership and the int64 Q components) and statistics of
every solve of the batched workload's grid (gamma in {1/2, 1, 2} x omega in {1/10, 1, 10}) on
every 8th of its 512 graphs: 576 solves, run in parallel processes.  sweep records the same
digests for the four SBM shapes of the doubling study (Table 1) under the multislice and the
global null model.  long records the windowed solves of the two long sequences shaped like
Table 1's Patent and School (present-only coupling): the sha256 of the int32 labels.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import windows  # noqa: E402
from paper_2608_03695_amd import gen  # noqa: E402

WORKLOADS = {
    "cfg2": (lambda: gen.config2(8), gen.CONFIG_SOLVE[2]),
    "cfg3": (lambda: gen.config3(8), gen.CONFIG_SOLVE[3]),
}
# the same graphs and constants under the global null model (Eq. 5, the objective of the
# paper's GPU path): records cfg2_global_expected.json, cfg3_global_expected.json
GLOBAL = {"cfg2_global": "cfg2", "cfg3_global": "cfg3"}


CFG4_GRAPHS = range(0, 512, 8)


def _digest(memb, comps):
    h = hashlib.sha256(np.ascontiguousarray(memb, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(comps, dtype=np.int64).tobytes())
    return h.hexdigest()


def _cfg4_graph(g):
    """Every grid solve of batched-workload graph g (one process; oracle threads 1)."""
    tg = gen.batch_graph(g)
    out = []
    for gamma in gen.GAMMA_GRID:
        for omega in gen.OMEGA_GRID:
            memb, comps, st = oracle.OracleGraph(tg, omega).leiden(gamma, max_levels=32,
                                                                    max_iterations=2, seed=0)
            out.append(dict(graph=g, gamma=str(gamma), omega=str(omega),
                            digest=_digest(memb, comps),
                            stats={k: int(v) for k, v in st.items()}))
    return out


def make_cfg4():
    import concurrent.futures as cf
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    t0 = time.time()
    with cf.ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn")) as ex:
        per = list(ex.map(_cfg4_graph, CFG4_GRAPHS))
    solves = [s for grp in per for s in grp]
    out = dict(workload="cfg4 sample: every 8th of the 512 batched-workload graphs x the "
                        "3x3 (gamma, omega) grid", graphs=list(CFG4_GRAPHS),
               max_levels=32, max_iterations=2, seed=0, solves=solves,
               oracle_seconds=round(time.time() - t0, 1))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_expected.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("cfg4", len(solves), "solves", out["oracle_seconds"], "s")


def make_sweep():
    spec = gen.SWEEP_SOLVE
    out = dict(workload="SBM shapes of the doubling study", gamma=str(spec.gamma),
               omega=str(spec.omega), max_levels=spec.max_levels,
               max_iterations=spec.max_iterations, seed=spec.seed, solves=[])
    for name in gen.SWEEP_SHAPES:
        tg = gen.sweep_graph(name, workers=4)
        og = oracle.OracleGraph(tg, spec.omega)
        for nm in (0, 1):
            t0 = time.time()
            memb, comps, st = og.leiden(spec.gamma, max_levels=spec.max_levels,
                                        max_iterations=spec.max_iterations, seed=spec.seed,
                                        null_model=nm)
            out["solves"].append(dict(shape=name, graph=tg.name, n_edges=int(tg.n_edges),
                                      null_model=nm, digest=_digest(memb, comps),
                                      stats={k: int(v) for k, v in st.items()},
                                      oracle_s=round(time.time() - t0, 1)))
            print(name, nm, out["solves"][-1]["oracle_s"], "s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_expected.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def make_long():
    spec = gen.LONG_SOLVE
    w, o = gen.LONG_WINDOW
    out = dict(workload="long sequences shaped like Table 1's Patent and School",
               gamma=str(spec.gamma), omega=str(spec.omega), max_levels=spec.max_levels,
               max_iterations=spec.max_iterations, seed=spec.seed, window=w, overlap=o,
               present_only=True, solves=[])
    for name in gen.LONG_SHAPES:
        tg = gen.long_graph(name)
        t0 = time.time()
        memb, nw = windows.leiden_windowed(tg, spec.omega, w, o, gamma=spec.gamma,
                                           max_levels=spec.max_levels,
                                           max_iterations=spec.max_iterations, seed=spec.seed,
                                           present_only=True)
        sha = hashlib.sha256(np.ascontiguousarray(memb, dtype=np.int32).tobytes()).hexdigest()
        out["solves"].append(dict(shape=name, graph=tg.name, n_nodes=tg.n_nodes,
                                  n_slices=tg.n_slices, n_edges=int(tg.n_edges), windows=nw,
                                  n_communities=int(memb.max()) + 1, sha256=sha,
                                  oracle_s=round(time.time() - t0, 1)))
        print(name, out["solves"][-1]["oracle_s"], "s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_expected.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def main(names):
    for name in names:
        if name == "cfg4":
            make_cfg4()
            continue
        if name == "sweep":
            make_sweep()
            continue
        if name == "long":
            make_long()
            continue
        nm = 1 if name in GLOBAL else 0
        make, spec = WORKLOADS[GLOBAL.get(name, name)]
        t0 = time.time()
        tg = make()
        t1 = time.time()
        og = oracle.OracleGraph(tg, spec.omega)
        m_supra = int(oracle._load().orc_nnz(og._h)) // 2
        meta = dict(name=tg.name, n_nodes=tg.n_nodes, n_slices=tg.n_slices, n_edges=tg.n_edges)
        # the oracle holds its own copy of the graph: drop the edge lists before solving
        tg.src = tg.dst = tg.weight = None
        og._keep = None
        t2 = time.time()
        memb, comps, st = og.leiden(spec.gamma, max_levels=spec.max_levels,
                                    max_iterations=spec.max_iterations, seed=spec.seed,
                                    null_model=nm)
        t3 = time.time()
        qf = oracle.q_global_from_components if nm == 1 else oracle.q_from_components
        q = qf(comps, meta["n_nodes"], meta["n_slices"], spec.gamma, spec.omega)
        out = dict(workload=meta["name"], null_model=nm, n_nodes=meta["n_nodes"],
                   n_slices=meta["n_slices"],
                   n_edges=int(meta["n_edges"]), gamma=str(spec.gamma), omega=str(spec.omega),
                   max_levels=spec.max_levels, max_iterations=spec.max_iterations, seed=spec.seed,
                   membership_sha256=hashlib.sha256(memb.astype(np.int32).tobytes()).hexdigest(),
                   q_components=[int(x) for x in comps], q=f"{q.numerator}/{q.denominator}",
                   stats={k: int(v) for k, v in st.items()},
                   oracle_timing=dict(generate_s=round(t1 - t0, 1), create_s=round(t2 - t1, 1),
                                      solve_s=round(t3 - t2, 1), threads=oracle.num_threads(),
                                      supra_edges=m_supra,
                                      supra_edges_per_s=round(m_supra / (t3 - t2)),
                                      host="the build container, not the benchmark host"))
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_expected.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(name, out["membership_sha256"], out["q"][:40], out["stats"])


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS) + ["cfg4"])
