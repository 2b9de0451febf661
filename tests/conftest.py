import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.build()
    return oracle


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Report the per-entry gradient margins seen by helpers.grad_close: for
    each test, the smallest per-entry floor that would have passed (fraction
    of the largest reference gradient) and the normwise relative error."""
    from tests import helpers
    if not helpers.GRAD_STATS:
        return
    worst = max(helpers.GRAD_STATS.items(), key=lambda kv: kv[1][0])
    terminalreporter.write_sep("-", "gradient margins (needed per-entry floor, normwise error)")
    for k, (need, norm) in sorted(helpers.GRAD_STATS.items()):
        terminalreporter.write_line(f"{need:10.3e} {norm:10.3e}  {k}")
    terminalreporter.write_line(f"worst needed floor {worst[1][0]:.3e} ({worst[0]}); "
                                f"floor in use {helpers.GRAD_FLOOR:g}")
