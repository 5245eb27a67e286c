"""Write the oracle's expected results for the larger parity workloads.

Runs only the oracle (oracle/), never the HIP library: for each workload it records the
sha256 of the oracle's int32 membership, its Q components and schedule statistics.  The
GPU parity tests compare the HIP path's output against these files.

    python tests/golden/make_expected.py [cfg2]
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
from paper_2608_03695_amd import gen  # noqa: E402

WORKLOADS = {
    "cfg2": (gen.config2, gen.CONFIG_SOLVE[2]),
}


def main(names):
    for name in names:
        make, spec = WORKLOADS[name]
        t0 = time.time()
        tg = make()
        og = oracle.OracleGraph(tg, spec.omega)
        memb, comps, st = og.leiden(spec.gamma, max_levels=spec.max_levels,
                                    max_iterations=spec.max_iterations, seed=spec.seed)
        q = oracle.q_from_components(comps, tg.n_nodes, tg.n_slices, spec.gamma, spec.omega)
        out = dict(workload=tg.name, n_nodes=tg.n_nodes, n_slices=tg.n_slices,
                   n_edges=int(tg.n_edges), gamma=str(spec.gamma), omega=str(spec.omega),
                   max_levels=spec.max_levels, max_iterations=spec.max_iterations, seed=spec.seed,
                   membership_sha256=hashlib.sha256(memb.astype(np.int32).tobytes()).hexdigest(),
                   q_components=[int(x) for x in comps], q=f"{q.numerator}/{q.denominator}",
                   stats={k: int(v) for k, v in st.items()},
                   oracle_seconds=round(time.time() - t0, 1),
                   oracle_threads=oracle.num_threads())
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_expected.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(name, out["membership_sha256"], out["q"][:40], out["stats"])


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
