"""One-wave-per-signal register kernel (large shapes) against the FP64 oracle.

FP64 bars as for the generic kernel (supports identical except near-ties within 1e-9,
coefficients and residuals within 1e-10 relative); FP32 bars as for the other
register-resident kernels (>= 97% identical supports, the rest near-ties within 1e-4,
coefficients within 2e-4 relative)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api
from paper_2007_03800_amd._native import SdlError
from tests.conftest import planted, rand_dicts
from tests.gpu_helpers import compare_codes

pytestmark = pytest.mark.gpu

SHAPES = [(12, 12, 20, 20, 10, 150), (12, 12, 24, 24, 12, 150), (16, 16, 32, 32, 16, 100), (32, 24, 48, 36, 20, 70)]
ids = lambda s: "x".join(map(str, s))  # noqa: E731


def codes(Y, d1, d2, s, dtype):
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.sparse_code(pr, kernel=3)
    torch.cuda.synchronize()
    return pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()


@pytest.mark.parametrize("shape", SHAPES, ids=ids)
def test_wave_fp64_matches_oracle(shape, rng):
    m1, m2, n1, n2, s, N = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, d1, d2, s, noise=0.1)
    Y[3] = 0.0
    so, co, ro = oracle.omp(Y, d1, d2, s)
    sg, cg, rg = codes(Y, d1, d2, s, torch.float64)
    agree, ties, bad, err = compare_codes(Y, d1, d2, sg, cg, so, co, 1e-9, 1e-10)
    print(shape, "agree", agree, "ties", ties, "bad", bad, "err %.2e" % err)
    assert bad == 0 and ties <= 1 and err <= 1e-10
    ok = np.all(sg == so, axis=1)
    np.testing.assert_allclose(rg[ok], ro[ok], rtol=1e-10, atol=1e-13)
    assert np.all(sg[3] == -1) and np.all(cg[3] == 0) and rg[3] == 0


@pytest.mark.parametrize("shape", SHAPES, ids=ids)
def test_wave_fp32_matches_oracle(shape, rng):
    m1, m2, n1, n2, s, N = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 3 * N, d1, d2, s, noise=0.03)
    so, co, _ = oracle.omp(Y, d1, d2, s, p=8)
    sg, cg, _ = codes(Y, d1, d2, s, torch.float32)
    agree, ties, bad, err = compare_codes(Y, d1, d2, sg, cg, so, co, 1e-4, 1e-4)
    print(shape, "agree", agree, "ties", ties, "bad", bad, "err %.2e" % err)
    assert agree >= 0.97 * len(Y) and bad == 0 and err <= 1e-4


@pytest.mark.parametrize("shape", SHAPES, ids=ids)
def test_wave_fp32_edges(shape, rng):
    """One and five signals (fewer than a workgroup's waves), an exactly 1-sparse signal
    (one atom, then the stop rule on a zero residual) and an all-zero signal."""
    m1, m2, n1, n2, s, _ = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    a = (7 * n1 + 3) % (n1 * n2)
    for N in (1, 5):
        Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
        if N == 5:
            Y[1] = 2.5 * np.outer(d1[:, a % n1], d2[:, a // n1])
            Y[2] = 0.0
        so, co, _ = oracle.omp(Y, d1, d2, s)
        sg, cg, rg = codes(Y, d1, d2, s, torch.float32)
        agree, ties, bad, err = compare_codes(Y, d1, d2, sg, cg, so, co, 1e-4, 1e-4)
        print(shape, N, "agree", agree, "ties", ties, "bad", bad, "err %.2e" % err)
        assert bad == 0 and err <= 1e-4
        if N == 5:
            assert sg[1, 0] == a and np.all(sg[1, 1:] == -1) and np.all(so[1, 1:] == -1)
            assert abs(cg[1, 0] - 2.5) < 1e-5 and rg[1] < 1e-8
            assert np.all(sg[2] == -1) and np.all(cg[2] == 0) and rg[2] == 0


def test_wave_bf16_signals_match_fp32_of_rounded(rng):
    """BF16 signals are widened exactly on load: the codes equal, bit for bit, the FP32
    codes of the rounded signals."""
    m1, m2, n1, n2, s, N = 16, 16, 32, 32, 16, 64
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
    Yb = torch.as_tensor(Y).to(torch.bfloat16)
    sb, cb, rb = codes(Yb, d1, d2, s, torch.bfloat16)
    sf, cf, rf = codes(Yb.double().numpy(), d1, d2, s, torch.float32)
    assert np.array_equal(sb, sf) and np.array_equal(cb, cf) and np.array_equal(rb, rf)


def test_wave_learn_tracks_oracle(rng):
    m1, m2, n1, n2, s, N = 32, 24, 48, 36, 20, 60
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, t1, t2, s, noise=0.05)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    ref = oracle.learn(Y, d1, d2, s, 2, p=8)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.float64)
    tr = api.learn(pr, 2, kernel=3)[0]
    np.testing.assert_allclose(tr, ref["rmse"], rtol=1e-10)
    for g, o in ((pr.d1(), ref["D1"]), (pr.d2(), ref["D2"])):
        assert np.abs(g - o).max() <= 1e-10 * np.abs(o).max()


def test_standalone_sums_path_reports_signals_per_wave():
    """Kernel option 3 in FP32: 16 lanes and four signals per wave on matrix-core quadrants at
    12x12 signals with 20x20 or 24x24 atoms, one wave per signal at the larger shapes."""
    for shape, spw in (((12, 12, 24, 24, 12), 4), ((12, 12, 20, 20, 10), 4), ((16, 16, 32, 32, 16), 1),
                       ((32, 24, 48, 36, 20), 1)):
        kinds = [v for v in api.kernel_variants(*shape) if v[3] == 2]
        assert len(kinds) == 1 and kinds[0][2] == spw, (shape, kinds)


def test_wave_unsupported_shape_rejected(rng):
    d1, d2 = rand_dicts(rng, 8, 8, 12, 12)
    pr = api.Problem.from_math(rng.standard_normal((10, 8, 8)), d1, d2, 4)
    with pytest.raises(SdlError) as e:
        api.sparse_code(pr, kernel=3)
    assert e.value.status == -7
