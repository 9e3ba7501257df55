import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: full-size parity cases")


def pytest_sessionfinish(session, exitstatus):
    """Record the strict-form violation counts of the parity checks (values
    outside 1e-12 |v*| + 1e-14 but inside the scale-aware tolerance)."""
    import json

    try:
        from helpers import STRICT_COUNTS
    except ImportError:
        return
    out = os.path.join(ROOT, "gpurun_out")
    if STRICT_COUNTS and os.path.isdir(out):
        tot = sum(v["strict_violations"] for v in STRICT_COUNTS.values())
        n = sum(v["compared"] for v in STRICT_COUNTS.values())
        with open(os.path.join(out, "parity_strict_counts.json"), "w") as fh:
            json.dump(dict(total_strict_violations=tot, total_compared=n, cases=STRICT_COUNTS), fh, indent=1)
