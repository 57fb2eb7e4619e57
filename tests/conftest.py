import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def rel_err(a, b):
    """max |a - b| / max |b| (the parity metric)."""
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    den = float(np.max(np.abs(b)))
    if den == 0.0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - b))) / den


def directional_fd(f, x, d, h=3e-5):
    """d/dt f(x + t d) at t = 0 by central differences with one Richardson step.

    D(h) = (f(x + h d) - f(x - h d)) / 2h has error c2 h^2 + c4 h^4; the
    combination (4 D(h/2) - D(h)) / 3 cancels the h^2 term.
    """
    def D(s):
        return (f(x + s * d) - f(x - s * d)) / (2.0 * s)
    return (4.0 * D(0.5 * h) - D(h)) / 3.0
