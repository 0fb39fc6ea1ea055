import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long statistical run")


@pytest.fixture(scope="session")
def gpu():
    """Skips unless a GPU is visible; returns the loaded HIP binding."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1112_4533_amd import sun
    sun.load()
    return sun


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """The parity measurements of the GPU comparisons (how close each one
    ran to its bound), printed even under -q, and written as JSON to
    $SUN_PARITY_EVIDENCE when that is set."""
    import json
    try:
        from gpu_common import EVIDENCE
    except Exception:
        return
    if not EVIDENCE:
        return
    path = os.environ.get("SUN_PARITY_EVIDENCE")
    if path:
        with open(path, "w") as f:
            json.dump(EVIDENCE, f, indent=0)
    tr = terminalreporter
    tr.section("parity evidence")
    keys = ("max_dU_over_tol", "max_dU_over_ctol", "max_K", "median_K", "max_cond", "max_dU_over_spread",
            "spread_admitted", "max_dU_over_spread_admitted", "flips", "expected_flips", "drift", "mean", "err",
            "exact", "z")
    for r in EVIDENCE:
        vals = " ".join(f"{k}={r[k]:.3g}" if isinstance(r.get(k), float) else f"{k}={r.get(k)}"
                        for k in keys if k in r)
        extra = f" margins={['%.2g' % m for m in r['flip_margins'][:5]]}" if r.get("flip_margins") else ""
        tr.write_line(f"{r.get('test', '')} [{r.get('what', '')}] {r.get('dtype')}: {vals}{extra}")
