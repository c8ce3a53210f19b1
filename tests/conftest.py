import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer statistical test")


def pytest_terminal_summary(terminalreporter):
    """Totals of the replay comparisons of this session (GPU parity tests)."""
    mod = sys.modules.get("parity_util")
    if mod is None or mod.SESSION.compared == 0:
        return
    s = mod.SESSION
    terminalreporter.write_line(
        f"replay parity: {s.compared} records compared against the oracle, {s.finals} final chain states, "
        f"{s.exempt} decision-boundary cases; classes {s.classes}")
