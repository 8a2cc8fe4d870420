import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def rand_dicts(rng, m1, m2, n1, n2):
    d1 = rng.standard_normal((m1, n1))
    d2 = rng.standard_normal((m2, n2))
    return d1 / np.linalg.norm(d1, axis=0), d2 / np.linalg.norm(d2, axis=0)


def planted(rng, N, d1, d2, s, noise=0.0):
    """Signals D1 X D2^T (+ noise) with s random atoms each; returns (Y, X dense)."""
    m1, n1 = d1.shape
    m2, n2 = d2.shape
    X = np.zeros((N, n1, n2))
    for k in range(N):
        a = rng.choice(n1 * n2, size=s, replace=False)
        X[k, a % n1, a // n1] = rng.standard_normal(s)
    Y = np.einsum("pi,kij,qj->kpq", d1, X, d2) + noise * rng.standard_normal((N, m1, m2))
    return Y, X


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
