"""Register-resident FP32 kernel variants: each one against the FP64 oracle, and the autotuner."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api
from tests.conftest import planted, rand_dicts
from tests.gpu_helpers import compare_codes

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 16, 16, 8), (8, 8, 16, 16, 6), (8, 8, 12, 12, 4), (12, 12, 20, 20, 10), (12, 12, 24, 24, 12),
          (16, 16, 32, 32, 16)]


def _cases():
    out = []
    for sh in SHAPES:
        for v in api.kernel_variants(*sh):
            out.append((sh, v))
    return out


@pytest.mark.parametrize("shape,variant", _cases(), ids=lambda x: "x".join(map(str, x)))
def test_variant_parity(shape, variant, rng):
    m1, m2, n1, n2, s = shape
    N = 777  # several groups per wave plus a ragged tail
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
    Y[5] = 0.0
    so, co, ro = oracle.omp(Y, d1, d2, s)
    api.set_kernel_variant(m1, m2, n1, n2, s, variant)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.float32)
    api.sparse_code(pr, kernel=3 if variant[3] == 2 else 2)  # kind 2: one wave per signal
    torch.cuda.synchronize()
    sg, cg, rg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
    agree, ties, bad, err = compare_codes(Y, d1, d2, sg, cg, so, co, 1e-4, 1e-4)
    print(shape, variant, "agree", agree, "ties", ties, "bad", bad, "err %.2e" % err)
    assert agree >= 0.97 * N and bad == 0 and err <= 1e-4
    assert np.all(sg[5] == -1) and rg[5] == 0
    ok = np.all(sg == so, axis=1)
    np.testing.assert_allclose(rg[ok], ro[ok], rtol=2e-3, atol=1e-6)


@pytest.mark.parametrize("shape", [(8, 8, 16, 16, 8), (16, 16, 32, 32, 16)], ids=lambda x: "x".join(map(str, x)))
def test_autotune_picks_a_variant(shape, rng):
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 20000, d1, d2, s, noise=0.03)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.float32)
    api.autotune(pr, reps=3)
    cfg = api.tuned_config(m1, m2, n1, n2, s)
    print(shape, "tuned", cfg)
    assert cfg is not None and cfg[:4] in api.kernel_variants(m1, m2, n1, n2, s) and cfg[4] > 0
    assert api.tuned_config(5, 5, 7, 7, 3) is None
    # whichever path won, learning with it follows the oracle
    e1, e2 = rand_dicts(rng, m1, m2, n1, n2)
    sub = Y[:2000]
    ref = oracle.learn(sub, e1, e2, s, 2, p=8)
    pr = api.Problem.from_math(sub, e1, e2, s, dtype=torch.float32)
    tr = api.learn(pr, 2)[0]
    np.testing.assert_allclose(tr, ref["rmse"], rtol=0.01)
