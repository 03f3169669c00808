import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU case")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


def pytest_sessionfinish(session, exitstatus):
    """Wait for the device and drop the cached workspaces and captured graphs
    before the interpreter exits, so no HIP memory is freed by exit-time
    teardown."""
    mod = sys.modules.get("paper_2408_10982_amd.binding")
    if mod is None or mod._lib is None:
        return
    import torch
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        torch.cuda.synchronize()
        mod.release()
        torch.cuda.empty_cache()
