"""The dictionary-update sums (Algorithm 1 steps 1 and 3; Corollary 1 for D1, Result 1 for D2) as
every sparse-coding path produces them, element by element against the oracle's sums formed by
their definitions (dense T_k = X_k D2^T, Z_k = D1 X_k) from the GPU's own codes.

On the register-resident FP32 kernels the sums are accumulated in the sparse-coding launch's
epilogue; sdl_sparse_code_sums returns exactly the reduced [A | B | sum res2] that sdl_learn
solves.  Cases: every compiled register-resident variant (vector-ALU and matrix-core layouts, one
and two epilogue passes), FP32 and bfloat16 signals, a ragged last group of signals; the
standalone-sums kernel (one wave per signal, FP64 and FP32); and one learning iteration whose D1
and D2 are checked against the oracle's update from the same codes.

Bars: FP32 arithmetic -- |A - A_ref| <= 1e-4 max(|A_ref|, 1e-3 max|A_ref|) element-wise, the same
for B (sums of FP32 products over a workgroup's signals, FP64 across workgroups); FP64 arithmetic
-- 1e-10 relative to the largest entry.  The residual total equals the sum of the returned res2
(FP64 order of summation aside) and the explicit residual of the returned codes."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api
from tests.conftest import planted, rand_dicts

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 16, 16, 8), (8, 8, 16, 16, 6), (8, 8, 12, 12, 4), (12, 12, 20, 20, 10), (12, 12, 24, 24, 12),
          (16, 16, 32, 32, 16)]
N_RAGGED = 1237  # 77 groups of 16 signals and a last group of 5


def _cases():
    out = []
    for sh in SHAPES:
        for v in api.kernel_variants(*sh):
            out.append((sh, v))
    return out


def _rounded_bf16(Y):
    return torch.as_tensor(Y).to(torch.bfloat16).double().numpy()


def sums_error(g, o):
    """max element-wise |g - o| / max(|o|, 1e-3 max|o|)"""
    scale = np.maximum(np.abs(o), 1e-3 * np.abs(o).max()) + 1e-300
    return float((np.abs(g - o) / scale).max())


def explicit_res2(Y, d1, d2, supp, coef):
    X = oracle.densify(supp, coef, d1.shape[1], d2.shape[1])
    R = Y - np.einsum("pi,kij,qj->kpq", d1, X, d2)
    return np.sum(R ** 2, axis=(1, 2))


def check_sums(pr, Y, d1, d2, side, sums, fp64):
    A, B, r2 = api.split_sums(sums, side, pr)
    sg, cg, rg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
    Ao, Bo = oracle.tmod_sums(side, Y, d1, d2, sg, cg)
    if fp64:
        ea = np.abs(A - Ao).max() / np.abs(Ao).max()
        eb = np.abs(B - Bo).max() / np.abs(Bo).max()
        bar = 1e-10
    else:
        ea, eb = sums_error(A, Ao), sums_error(B, Bo)
        bar = 1e-4
    rx = explicit_res2(Y, d1, d2, sg, cg).sum()
    print("side %d: A err %.2e, B err %.2e, res2 total %.6e (sum of res2 %.6e, explicit %.6e)"
          % (side, ea, eb, r2, rg.sum(), rx))
    assert ea <= bar and eb <= bar, (ea, eb)
    assert abs(r2 - rg.sum()) <= 1e-9 * rg.sum()
    assert abs(r2 - rx) <= (1e-9 if fp64 else 1e-3) * rx


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["fp32", "bf16"])
@pytest.mark.parametrize("shape,variant", _cases(), ids=lambda x: "x".join(map(str, x)))
def test_kernel_sums_match_oracle(shape, variant, dtype, rng):
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N_RAGGED, d1, d2, s, noise=0.03)
    Y[3] = 0.0
    if dtype == torch.bfloat16:
        Y = _rounded_bf16(Y)
    else:
        Y = Y.astype(np.float32).astype(np.float64)  # exactly the values the kernel reads
    e1, e2 = rand_dicts(rng, m1, m2, n1, n2)  # code with dictionaries other than the generating ones
    api.set_kernel_variant(m1, m2, n1, n2, s, variant)
    kernel = 3 if variant[3] == 2 else 2  # kind 2: one wave per signal + the standalone sums kernel
    for side in (1, 2):
        pr = api.Problem.from_math(Y, e1, e2, s, dtype=dtype)
        sums = api.sparse_code_sums(pr, side, kernel=kernel)
        torch.cuda.synchronize()
        print(shape, variant, dtype)
        check_sums(pr, Y, e1, e2, side, sums, False)


@pytest.mark.parametrize("shape", [(8, 8, 12, 12, 4, 2000), (5, 9, 11, 6, 7, 129), (32, 24, 48, 36, 20, 40)],
                         ids=lambda x: "x".join(map(str, x)))
@pytest.mark.parametrize("kernel", [0, 1])
def test_fp64_sums_match_oracle(shape, kernel, rng):
    m1, m2, n1, n2, s, N = shape
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, t1, t2, s, noise=0.1)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    for side in (1, 2):
        pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.float64)
        sums = api.sparse_code_sums(pr, side, kernel=kernel)
        torch.cuda.synchronize()
        check_sums(pr, Y, d1, d2, side, sums, True)


def test_sums_empty_problem(rng):
    d1, d2 = rand_dicts(rng, 8, 8, 16, 16)
    pr = api.Problem.from_math(np.zeros((0, 8, 8)), d1, d2, 8, dtype=torch.float32)
    sums = api.sparse_code_sums(pr, 1)
    torch.cuda.synchronize()
    assert sums.shape[0] == 16 * 16 + 8 * 16 + 1 and torch.all(sums == 0)


@pytest.mark.parametrize("shape", [(8, 8, 16, 16, 8), (8, 8, 12, 12, 4), (12, 12, 24, 24, 12)],
                         ids=lambda x: "x".join(map(str, x)))
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["fp32", "bf16"])
def test_learn_iteration_updates_match_oracle(shape, dtype, rng):
    """One Algorithm 1 iteration as sdl_learn runs it (its sums in the sparse-coding epilogue where the
    shape has a register-resident kernel): D1 equals the oracle's Corollary 1 update from the codes
    of the first sweep, and D2 the oracle's Result 1 update from the codes of the second sweep
    (each sweep's codes taken by the same kernel through sdl_sparse_code_sums), 1e-4 relative."""
    m1, m2, n1, n2, s = shape
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 2001, t1, t2, s, noise=0.05)
    Y = _rounded_bf16(Y) if dtype == torch.bfloat16 else Y.astype(np.float32).astype(np.float64)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    # the kernel sdl_learn uses for this shape: the autotuner's choice on these signals
    api.autotune(api.Problem.from_math(Y, d1, d2, s, dtype=dtype), reps=1)
    pl = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.learn(pl, 1)
    g1, g2 = pl.d1(), pl.d2()
    p1 = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.sparse_code_sums(p1, 1)
    torch.cuda.synchronize()
    o1 = oracle.tmod_update(1, Y, d1, d2, p1.supp.cpu().numpy(), p1.coef.cpu().double().numpy())[0]
    p2 = api.Problem.from_math(Y, g1, d2, s, dtype=dtype)
    api.sparse_code_sums(p2, 2)
    torch.cuda.synchronize()
    o2 = oracle.tmod_update(2, Y, g1, d2, p2.supp.cpu().numpy(), p2.coef.cpu().double().numpy())[1]
    e1 = np.abs(g1 - o1).max() / np.abs(o1).max()
    e2 = np.abs(g2 - o2).max() / np.abs(o2).max()
    print(shape, dtype, "D1 err %.2e, D2 err %.2e" % (e1, e2))
    assert e1 <= 1e-4 and e2 <= 1e-4


@pytest.mark.parametrize("shape", [(12, 12, 24, 24, 12), (8, 8, 16, 16, 8), (12, 12, 20, 20, 10)],
                         ids=lambda x: "x".join(map(str, x)))
def test_mixed_bf16_sums_match_oracle(shape, rng):
    """SDL_MIXED_BF16: the sums on the BF16 matrix cores (each T_k entry formed in FP32 from the
    codes and rounded once to BF16; the signals are BF16 already; FP32 accumulation, FP64 across
    workgroups) against the oracle's FP64 sums from the same codes.  Bar: the rounding of T_k
    (relative 2^-9 per entry, independent across signals) enters every product of a sum once, so
    an entry's error grows like 2^-8 sqrt(n) |product| over its n terms while the diagonal entries
    grow like n |product|: relative to the largest entry the error is about 2^-8 / sqrt(n), which
    for the few hundred terms per entry here is a few 1e-4; the bar is 1e-3 of the largest entry
    (entries far below the largest carry the same absolute error, so element-wise ratios are
    reported, not bounded)."""
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N_RAGGED, d1, d2, s, noise=0.03)
    Y = _rounded_bf16(Y)
    e1, e2 = rand_dicts(rng, m1, m2, n1, n2)
    for side in (1, 2):
        pr = api.Problem.from_math(Y, e1, e2, s, dtype=torch.bfloat16)
        sums = api.sparse_code_sums(pr, side, mixed=True)
        torch.cuda.synchronize()
        A, B, r2 = api.split_sums(sums, side, pr)
        sg, cg, rg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
        Ao, Bo = oracle.tmod_sums(side, Y, e1, e2, sg, cg)
        ea, eb = sums_error(A, Ao), sums_error(B, Bo)
        na_ = np.abs(A - Ao).max() / np.abs(Ao).max()
        nb_ = np.abs(B - Bo).max() / np.abs(Bo).max()
        print(shape, "side %d: A err %.2e (normwise %.2e), B err %.2e (normwise %.2e)" % (side, ea, na_, eb, nb_))
        assert na_ <= 1e-3 and nb_ <= 1e-3
        assert abs(r2 - rg.sum()) <= 1e-9 * rg.sum()
