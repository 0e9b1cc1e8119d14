import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP path")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import fastmm_oracle

    return fastmm_oracle


def pytest_runtest_logreport(report):
    # Print a failing test's report at once: a later crash of the process would otherwise
    # lose the summary that pytest prints at the end of the session.
    if report.failed and report.when in ("setup", "call"):
        text = getattr(report, "longreprtext", "") or ""
        print(f"\n---- {report.nodeid} failed ----\n{text[-2500:]}\n", flush=True)
