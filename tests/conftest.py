import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_sessionstart(session):
    """Build the HIP library (host cross-compile) when no build is present."""
    if os.path.exists(os.path.join(ROOT, "paper_2010_16012_amd", "libpp.so")):
        return
    import importlib.util

    spec = importlib.util.spec_from_file_location("_pp_build", os.path.join(ROOT, "paper_2010_16012_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size workload (seconds to minutes)")


@pytest.fixture(scope="session")
def root_dir():
    return ROOT
