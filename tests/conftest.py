import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


def pytest_terminal_summary(terminalreporter):
    """The largest error of the GPU's FP64 conservation sums against the
    oracle's, per precision, over the parity steps that ran."""
    mod = sys.modules.get("_gpu_common")
    errs = getattr(mod, "SUMS_ERR", None) if mod else None
    if not errs:
        return
    for prec in ("fp64", "fp32"):
        e = [x[2] for x in errs if x[1] == prec]
        if e:
            terminalreporter.write_line("conservation sums vs oracle, %s: max relative error %.3e over %d steps"
                                        % (prec, max(e), len(e)))
