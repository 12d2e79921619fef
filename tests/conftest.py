import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Per parity test: windows run, windows beyond tolerance (each verified frame
    by frame), frames with a flipped fragile decision, the worst window and the
    largest one-frame deviations."""
    helpers = sys.modules.get("_helpers")
    lines = getattr(helpers, "REPORT", None) if helpers else None
    if lines:
        terminalreporter.write_sep("-", "parity windows")
        for line in lines:
            terminalreporter.write_line(line)
