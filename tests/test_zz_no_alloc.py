"""The allocation-free sparse coding entry point (its workspace in the library's static device
array) against sdl_sparse_code on the same inputs: identical supports, coefficients and residuals
(the same kernels run on the same data), on two calls in a row whose second is smaller, in FP32
and FP64; too-large requests are refused before any work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2007_03800_amd import _native, api
from tests.conftest import planted, rand_dicts

pytestmark = pytest.mark.gpu


def noalloc(problems, **opts):
    o = api._options(problems, None, **opts)
    arr = api._array(problems)
    return _native.lib().sdl_sparse_code_noalloc(arr, len(problems), ctypes.byref(o), api._stream(None))


def _pair(Y, d1, d2, s, dtype):
    return (api.Problem.from_math(Y, d1, d2, s, dtype=dtype), api.Problem.from_math(Y, d1, d2, s, dtype=dtype))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["fp32", "fp64"])
def test_noalloc_equals_sparse_code_two_calls(dtype, rng):
    for shape, N in (((8, 8, 16, 16, 8), 3001), ((8, 8, 16, 16, 8), 777), ((12, 12, 24, 24, 12), 500),
                     ((5, 9, 11, 6, 7), 129)):
        m1, m2, n1, n2, s = shape
        d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
        Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
        a, b = _pair(Y, d1, d2, s, dtype)
        api.sparse_code(a)
        b.supp.fill_(-7)
        b.coef.fill_(123.0)
        b.res2.fill_(-1.0)
        _native.check(noalloc([b]))
        torch.cuda.synchronize()
        assert torch.equal(a.supp, b.supp), shape
        assert torch.equal(a.coef, b.coef), shape
        assert torch.equal(a.res2, b.res2), shape


def test_noalloc_several_problems_and_stats(rng):
    probs_a, probs_b = [], []
    for m1, m2, n1, n2, s, N in ((8, 8, 16, 16, 6, 600), (12, 12, 20, 20, 10, 300), (16, 16, 32, 32, 16, 64)):
        d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
        Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
        Y[1] = 0.0
        a, b = _pair(Y, d1, d2, s, torch.float32)
        probs_a.append(a)
        probs_b.append(b)
    sa, sb = api.new_stats(), api.new_stats()
    api.sparse_code(probs_a, stats=sa)
    o = api._options(probs_b, sb)
    _native.check(_native.lib().sdl_sparse_code_noalloc(api._array(probs_b), 3, ctypes.byref(o), api._stream(None)))
    torch.cuda.synchronize()
    for a, b in zip(probs_a, probs_b):
        assert torch.equal(a.supp, b.supp) and torch.equal(a.coef, b.coef) and torch.equal(a.res2, b.res2)
    assert sa.early_stops == sb.early_stops >= 3


def test_noalloc_refuses_what_does_not_fit(rng):
    d1, d2 = rand_dicts(rng, 32, 32, 64, 64)
    probs = [api.Problem.from_math(np.zeros((2, 32, 32)), d1, d2, 4, dtype=torch.float64) for _ in range(8)]
    assert noalloc(probs) == -4
    assert "workspace" in _native.lib().sdl_last_error().decode()
    assert noalloc(probs[:1], timing=1) == -1
    # what fits still runs after a refusal: zero signals give empty codes
    _native.check(noalloc(probs[:1]))
    torch.cuda.synchronize()
    assert torch.all(probs[0].supp == -1) and torch.all(probs[0].res2 == 0)
