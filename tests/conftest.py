import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: full-size parity cases")


def _strict_totals():
    try:
        from helpers import STRICT_COUNTS
    except ImportError:
        return None
    if not STRICT_COUNTS:
        return None
    tot = sum(v["strict_violations"] for v in STRICT_COUNTS.values())
    n = sum(v["compared"] for v in STRICT_COUNTS.values())
    return tot, n, STRICT_COUNTS


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Print the strict-form violation counts of the parity checks (values
    outside 1e-12 |v*| + 1e-14 but inside the scale-aware tolerance)."""
    t = _strict_totals()
    if t:
        terminalreporter.write_line(f"parity strict form: {t[0]} of {t[1]} compared values outside "
                                    f"1e-12 |v*| + 1e-14, over {len(t[2])} cases")


def pytest_sessionfinish(session, exitstatus):
    """Also write those counts, per case, as JSON to the file that the
    environment variable OPF_PARITY_RECORD names (if set)."""
    import json

    path = os.environ.get("OPF_PARITY_RECORD")
    t = _strict_totals()
    if t and path:
        with open(path, "w") as fh:
            json.dump(dict(total_strict_violations=t[0], total_compared=t[1], cases=t[2]), fh, indent=1)
