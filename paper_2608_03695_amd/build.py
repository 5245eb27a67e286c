"""Build the HIP library libmslm.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmslm.so")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]
SOURCES = ["prims.hip", "engine.hip", "static_entry.hip", "spectral.hip", "host.cpp", "api.cpp",
           "server.cpp"]


def _needs(obj, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = False, verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC)
               if f.endswith((".hpp", ".inc"))] + [os.path.join(HERE, "..", "include", "mslm.h")]
    jobs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OUT_DIR, src + ".o")
        objs.append(obj)
        if force or _needs(obj, [path] + headers):
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            jobs.append(["hipcc", *FLAGS, *lang, "-c", path, "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = [ex.submit(subprocess.run, j, capture_output=True, text=True) for j in jobs]
        for j, f in zip(jobs, futs):
            r = f.result()
            if r.returncode != 0:
                sys.stderr.write(r.stderr)
                raise RuntimeError("hipcc failed: " + " ".join(j[-3:]))
            if verbose and r.stderr:
                sys.stderr.write(r.stderr)
    if force or jobs or not os.path.exists(LIB):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}",
                               *objs, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose=True))
