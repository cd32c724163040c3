import json
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU test")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


_SAFE = {"pi": math.pi, "sqrt": math.sqrt, "sin": math.sin, "cos": math.cos, "exp": math.exp}


def ev(expr):
    """Evaluate a hand-derived closed-form expression from a golden file."""
    if isinstance(expr, (int, float)):
        return float(expr)
    return float(eval(expr, {"__builtins__": {}}, _SAFE))


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    import oracle
    import workloads
    oracle.build()
    workloads.build()
    yield
