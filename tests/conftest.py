import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU statistics test")


@pytest.fixture(scope="session")
def cfgs():
    from gapsinputs import workloads
    return {
        "ee": workloads.config_dict(workloads.EE),
        "lo": workloads.config_dict(workloads.PP_LO),
        "nlo": workloads.config_dict(workloads.PP_NLO),
        "dy": workloads.config_dict(workloads.PP_DY),
        "muq": workloads.config_dict(workloads.PP_NLO_MUQ),
        "powheg": workloads.config_dict(workloads.PP_NLO_POWHEG),
        "dynlo": workloads.config_dict(workloads.PP_DY_NLO),
    }


@pytest.fixture(scope="session")
def oracles(cfgs):
    from oracle.pyoracle import Oracle
    return {k: Oracle(v) for k, v in cfgs.items()}
