import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: larger CPU case")


@pytest.fixture(scope="session")
def ora():
    from oracle import oracle as O
    O.build()
    return O


def pytest_terminal_summary(terminalreporter):
    """Totals of the oracle comparisons: entries compared and entries that
    passed only through the cancellation fallback."""
    parity = sys.modules.get("parity")
    rec = getattr(parity, "RECORD", None)
    if not rec:
        return
    n = sum(r[1] for r in rec)
    fb = sum(r[2] for r in rec)
    worst = max(rec, key=lambda r: r[2] / max(r[1], 1))
    terminalreporter.write_line(
        f"oracle parity: {len(rec)} comparisons, {n} entries, {fb} through the cancellation "
        f"fallback; highest share {worst[2]}/{worst[1]} ({worst[0]})")
