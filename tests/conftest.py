import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on cuda:0)")
    config.addinivalue_line("markers", "slow: full-size workloads")


def _ensure_built():
    from paper_1903_01665_amd import _build
    import oracle.build as ob
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        ob.build()
    if not os.path.exists(os.path.join(ROOT, "paper_1903_01665_amd", "gen", "libggen.so")):
        _build.build_gen()


_ensure_built()
