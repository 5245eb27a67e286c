import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side case")


def pytest_sessionstart(session):
    # The oracle is compiled here, at the start of the session and before any test touches
    # the GPU, when its library is missing or older than its source; the loader itself never
    # compiles (a process that drives the GPU must not start a compiler).
    import oracle
    if not oracle._is_current():
        oracle.build(force=True)
    # a session that selects GPU tests draws the full-size inputs first, before any test
    # brings up the GPU in this process
    markexpr = session.config.option.markexpr or ""
    if "gpu" in markexpr and "not gpu" not in markexpr:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import full_size_inputs
        full_size_inputs.prepare(workers=min(16, os.cpu_count() or 1))
