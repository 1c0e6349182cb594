import json
import os
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only checks (the FP32 rounding floor of the oracle)")


def pytest_runtest_logreport(report):
    """With CLAW_RECORD set, one JSONL record per test: outcome and duration."""
    path = os.environ.get("CLAW_RECORD")
    if not path or report.when != "call":
        return
    with open(path, "a") as fh:
        fh.write(json.dumps({"test": report.nodeid, "outcome": report.outcome, "seconds": report.duration,
                             "time_utc": time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime())}) + "\n")
