import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def to_oracle(inst):
    """Workload dict -> oracle problem (test-side glue only)."""
    from oracle.system import OracleProblem
    return OracleProblem(shape=tuple(inst["shape"]), step=tuple(inst["step"]), bc=tuple(inst["bc"]),
                         mset=tuple(inst["mset"]), coeff=np.asarray(inst["coeff"], np.float64),
                         rhs=np.asarray(inst["rhs"], np.float64),
                         bc_values=np.asarray(inst["bc_values"], np.float64))


@pytest.fixture
def oracle_problem():
    return to_oracle
