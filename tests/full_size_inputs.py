"""Full-size inputs of the GPU parity tests, drawn once per GPU test session.

The config-3 graph (T=64 x N=1M) and the 64 sampled graphs of the batched workload take the
multi-process generator about a minute; ``prepare`` draws them at the start of a session that
selects GPU tests, before any test brings up the GPU in the test process (the generator's
workers are fresh interpreters), and stores them as .npz files in a temporary directory.
"""
import os
import tempfile

import numpy as np

from paper_2608_03695_amd import gen

DIR = os.path.join(tempfile.gettempdir(), "mslm_full_size_inputs")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CFG4_GRAPHS = list(range(0, 512, 8))


def _save(tg, path):
    np.savez(path, n_nodes=tg.n_nodes, n_slices=tg.n_slices, offsets=tg.offsets, src=tg.src,
             dst=tg.dst, weight=tg.weight if tg.weight is not None else np.zeros(0, np.int32),
             name=tg.name)


def load(path):
    z = np.load(path, allow_pickle=False)
    w = z["weight"] if z["weight"].size else None
    return gen.TemporalGraph(int(z["n_nodes"]), int(z["n_slices"]), z["offsets"], z["src"],
                             z["dst"], w, None, str(z["name"]))


def cfg3_path():
    return os.path.join(DIR, "cfg3.npz")


def cfg4_path(g):
    return os.path.join(DIR, f"cfg4_g{g}.npz")


def prepare(workers=16):
    os.makedirs(DIR, exist_ok=True)
    if os.path.exists(os.path.join(GOLDEN, "cfg3_expected.json")) and not os.path.exists(cfg3_path()):
        _save(gen.config3(workers), cfg3_path())
    if os.path.exists(os.path.join(GOLDEN, "cfg4_expected.json")):
        todo = [g for g in CFG4_GRAPHS if not os.path.exists(cfg4_path(g))]
        for g, tg in zip(todo, gen.batch_graphs(todo, workers=workers)):
            _save(tg, cfg4_path(g))
