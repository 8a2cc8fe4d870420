"""The FP32 small-pivot path: a Cholesky row whose pivot falls below pivot_fp64 * G_aa is
recomputed in FP64.  With pivot_fp64 = 1 every row after the first takes that path, so each
FP32 kernel family runs it on every step; the codes must still meet the FP32 bars against
the FP64 oracle and the recomputations are counted."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api
from tests.conftest import planted, rand_dicts
from tests.gpu_helpers import compare_codes

pytestmark = pytest.mark.gpu

# (shape, forced variant or None, kernel option): the matrix-core and the vector-ALU
# four-lane kernels, the vector-ALU kernel at a larger shape, the generic kernel, and the
# standalone-sums kernels (quadrants at 12x12 signals, one wave per signal above)
CASES = [((8, 8, 16, 16, 8), (1, 4, 2, 1), 2), ((8, 8, 16, 16, 8), (1, 4, 2, 0), 2),
         ((12, 12, 20, 20, 10), (1, 4, 1, 0), 2), ((5, 9, 11, 6, 7), None, 1),
         ((12, 12, 24, 24, 12), None, 3), ((12, 12, 20, 20, 10), None, 3), ((16, 16, 32, 32, 16), None, 3),
         ((32, 24, 48, 36, 20), None, 3)]
ids = ["x".join(map(str, c[0])) + "-k%d" % c[2] + ("-" + "".join(map(str, c[1])) if c[1] else "") for c in CASES]


@pytest.mark.parametrize("shape,variant,kernel", CASES, ids=ids)
def test_fp64_pivot_path_matches_oracle(shape, variant, kernel, rng):
    m1, m2, n1, n2, s = shape
    N = 300 if m1 * m2 <= 144 else 80
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
    so, co, _ = oracle.omp(Y, d1, d2, s, p=8)
    if variant is not None:
        assert variant in api.kernel_variants(*shape)
        api.set_kernel_variant(*shape, variant)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.float32)
    st = api.new_stats()
    api.sparse_code(pr, kernel=kernel, pivot_fp64=1.0, stats=st)
    torch.cuda.synchronize()
    sg, cg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy()
    agree, ties, bad, err = compare_codes(Y, d1, d2, sg, cg, so, co, 1e-4, 1e-4)
    n_rows = int((sg >= 0).sum()) - N  # rows after each signal's first
    print(shape, variant, kernel, "agree", agree, "ties", ties, "bad", bad, "err %.2e" % err,
          "fp64 rows", st.fp64_pivots, "of", n_rows)
    assert agree >= 0.97 * N and bad == 0 and err <= 1e-4
    # a row whose |w|^2 is below FP32's resolution of G_aa keeps delta^2 == G_aa exactly and is
    # not below pivot_fp64 * G_aa: nearly every row, not every one, takes the FP64 path
    assert n_rows > 0 and st.fp64_pivots >= 0.95 * n_rows
