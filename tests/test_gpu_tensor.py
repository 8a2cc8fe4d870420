"""n-dimensional signals (Remark 3) on the GPU against the oracle's n-mode composition (tensor_omp,
tensor_update, tensor_learn), which is itself pinned against the two-dimensional oracle, hard
thresholding and stacked lstsq.

Bars as for two modes: FP64 supports identical except classified near-ties (1e-9), coefficients
1e-10 element-wise (relative to max(|x|, 0.02 max|x|)), dictionaries 1e-10 relative from identical
codes and 1e-9 over a learning run; FP32 supports identical except near-ties at 1e-4, coefficients
1e-4, dictionaries 1e-4 from identical codes.  Cases: two, three and four modes, non-square modes,
a ragged signal count, the error-driven stop, an atom no code uses, an empty problem, and the
mode sums with every partial row filled (20,000 signals of the benchmarked shape)."""
import numpy as np
import pytest
import torch

from oracle import tensor as ot
from paper_2007_03800_amd import api, synth
from tests.gpu_helpers import compare_codes, kron_all

pytestmark = pytest.mark.gpu

SHAPES = [((8, 8), (16, 16), 8), ((4, 3, 5), (6, 5, 7), 5), ((8, 8, 4), (12, 12, 6), 8),
          ((3, 3, 3, 2), (4, 4, 4, 3), 4)]


def unit_cols(rng, m, n):
    d = rng.standard_normal((m, n))
    return d / np.linalg.norm(d, axis=0)


def planted(rng, N, Ds, s, noise):
    K = kron_all(Ds)
    Y = np.zeros((N, K.shape[0]))
    for k in range(N):
        a = rng.choice(K.shape[1], s, replace=False)
        Y[k] = K[:, a] @ rng.standard_normal(s)
    Y += noise * rng.standard_normal(Y.shape)
    ms = [D.shape[0] for D in Ds]
    return Y.reshape((N,) + tuple(reversed(ms))).transpose((0,) + tuple(range(len(ms), 0, -1))).copy()


def _codes(pr):
    return pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()


@pytest.mark.parametrize("dtype,band,ctol", [(torch.float64, 1e-9, 1e-10), (torch.float32, 1e-4, 1e-4)],
                         ids=["fp64", "fp32"])
@pytest.mark.parametrize("ms,ns,s", SHAPES, ids=lambda x: "x".join(map(str, x)) if isinstance(x, tuple) else str(x))
def test_tensor_codes_match_oracle(ms, ns, s, dtype, band, ctol, rng):
    T = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    Y = planted(rng, 301, T, s, 0.05)
    Y[7] = 0.0
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    E = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    pr = api.TensorProblem.from_math(Y, E, s, dtype=dtype)
    api.tensor_sparse_code(pr)
    torch.cuda.synchronize()
    sg, cg, rg = _codes(pr)
    so, co, ro = ot.tensor_omp(Y, E, s)
    Ec = E if dtype == torch.float64 else [e.astype(np.float32).astype(np.float64) for e in E]
    agree, ties, bad, err = compare_codes(Y, None, None, sg, cg, so, co, band, K=kron_all(Ec))
    print(ms, ns, s, dtype, "agree %d, ties %d, bad %d, coef err %.2e" % (agree, ties, bad, err))
    assert bad == 0 and err <= ctol
    assert np.all(sg[7] == -1) and rg[7] == 0.0
    ok = np.all(sg == so, axis=1)
    np.testing.assert_allclose(rg[ok], ro[ok], rtol=1e-9 if dtype == torch.float64 else 1e-3,
                               atol=1e-12 if dtype == torch.float64 else 1e-6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_tensor_error_driven_stop(dtype, rng):
    ms, ns = (4, 4, 3), (6, 6, 4)
    T = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    Y = planted(rng, 400, T, 6, 0.05)
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    err2 = (1.15 * 0.05) ** 2 * 48
    pr = api.TensorProblem.from_math(Y, T, 24, dtype=dtype)
    api.tensor_sparse_code(pr, err2=err2)
    torch.cuda.synchronize()
    sg, cg, rg = _codes(pr)
    so, co, ro = ot.tensor_omp(Y, T, 24, err2=err2)
    ng, no = np.sum(sg >= 0, 1), np.sum(so >= 0, 1)
    print(dtype, "atoms %.2f mean, count mismatches %d" % (no.mean(), int((ng != no).sum())))
    assert len(set(no.tolist())) > 2
    same = ng == no
    for k in np.nonzero(~same)[0]:  # only where the energy sits at the threshold within rounding
        t = int(min(ng[k], no[k]))
        r_t = ot.tensor_omp(Y[k:k + 1], T, max(t, 1))[2][0] if t > 0 else float(np.sum(Y[k] ** 2))
        tol = 1e-9 * err2 if dtype == torch.float64 else 64 * 2.0 ** -24 * float(np.sum(Y[k] ** 2))
        assert abs(r_t - err2) <= tol
    band = 1e-9 if dtype == torch.float64 else 1e-4
    ks = np.nonzero(same)[0]
    agree, ties, bad, err = compare_codes(Y[ks], None, None, sg[ks], cg[ks], so[ks], co[ks], band, K=kron_all(T))
    assert bad == 0 and err <= (1e-10 if dtype == torch.float64 else 1e-4)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)], ids=["fp64", "fp32"])
@pytest.mark.parametrize("ms,ns,s", SHAPES[1:], ids=lambda x: "x".join(map(str, x)) if isinstance(x, tuple) else str(x))
def test_tensor_update_matches_oracle(ms, ns, s, dtype, tol, rng):
    """Every mode's update from the GPU's own codes against the oracle's update from the same codes."""
    T = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    Y = planted(rng, 777, T, s, 0.05)
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    E = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    for mode in range(1, len(ms) + 1):
        pr = api.TensorProblem.from_math(Y, E, s, dtype=dtype)
        api.tensor_sparse_code(pr)
        torch.cuda.synchronize()
        sg, cg, _ = _codes(pr)
        Dn, co, w = ot.tensor_update(mode, Y, E, sg, cg)
        api.tensor_update(pr, mode)
        torch.cuda.synchronize()
        got = pr.dicts()
        errs = [np.abs(g - o).max() / np.abs(o).max() for g, o in zip(got, Dn)]
        cerr = np.abs(pr.coef.cpu().double().numpy() - co).max() / np.abs(co).max()
        print(ms, mode, dtype, "D errs", ["%.1e" % e for e in errs], "coef %.1e" % cerr)
        assert max(errs) <= tol and cerr <= tol


def test_tensor_update_keeps_unused_atom(rng):
    ms, ns = (4, 3, 5), (6, 5, 7)
    T = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    Y = planted(rng, 200, T, 3, 0.05)
    pr = api.TensorProblem.from_math(Y, T, 3)
    # codes that never use mode-1 index 5
    supp = rng.integers(0, 6 * 5 * 7, (200, 3))
    supp[supp % 6 == 5] -= 1
    pr.supp.copy_(torch.as_tensor(supp.astype(np.int32)))
    pr.coef.copy_(torch.as_tensor(rng.standard_normal((200, 3))))
    before = pr.dicts()[0].copy()
    Dn, _, _ = ot.tensor_update(1, Y, T, supp.astype(np.int32), pr.coef.cpu().numpy())
    api.tensor_update(pr, 1)
    torch.cuda.synchronize()
    got = pr.dicts()[0]
    np.testing.assert_array_equal(got[:, 5], before[:, 5])
    assert np.abs(got - Dn[0]).max() <= 1e-10


@pytest.mark.parametrize("ms,ns,s", [((4, 3, 5), (6, 5, 7), 4), ((3, 3, 3, 2), (4, 4, 4, 3), 3)],
                         ids=["3modes", "4modes"])
def test_tensor_learn_matches_oracle(ms, ns, s, rng):
    T = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    Y = planted(rng, 257, T, s, 0.02)
    E = [unit_cols(rng, m, n) for m, n in zip(ms, ns)]
    ref = ot.tensor_learn(Y, E, s, 3)
    pr = api.TensorProblem.from_math(Y, E, s)
    trace = api.tensor_learn(pr, 3)
    errs = [np.abs(g - o).max() / np.abs(o).max() for g, o in zip(pr.dicts(), ref["Ds"])]
    same = np.mean(np.all(pr.supp.cpu().numpy() == ref["supp"], axis=1))
    print(ms, "D errs", ["%.1e" % e for e in errs], "trace", trace, ref["rmse"], "same supports %.4f" % same)
    assert max(errs) <= 1e-9
    np.testing.assert_allclose(trace, ref["rmse"], rtol=1e-9)
    assert same == 1.0


def test_tensor_empty_problem(rng):
    E = [unit_cols(rng, 4, 6), unit_cols(rng, 3, 5), unit_cols(rng, 2, 3)]
    pr = api.TensorProblem.from_math(np.zeros((0, 4, 3, 2)), E, 3)
    api.tensor_sparse_code(pr)
    trace = api.tensor_learn(pr, 2)
    torch.cuda.synchronize()
    assert np.all(trace == 0.0)
    for g, e in zip(pr.dicts(), E):
        np.testing.assert_array_equal(g, e)


def test_tensor_workload_full_size_sampled():
    """The benchmarked three-mode workload (100,000 signals 8 x 8 x 4, 12 x 12 x 6 atoms, s = 8,
    FP32, K = 10 from random starting dictionaries): sampled final codes against the oracle's codes
    at the GPU's final dictionaries, and the RMSE trace non-increasing after the first iteration."""
    w = synth.TENSOR_WORKLOADS["tensor_8x8x4_n12x12x6_s8"]
    Y = synth.tensor_signals(w)
    E = synth.tensor_dictionaries(w, initial=True)
    pr = api.TensorProblem.from_math(Y, E, w.s, dtype=torch.float32)
    trace = api.tensor_learn(pr, w.iters)
    Ds = pr.dicts()
    rs = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.arange(300), np.arange(w.N - 300, w.N), rs.choice(w.N, 600, replace=False)]))
    Ysub = Y[idx].astype(np.float32).astype(np.float64)
    so, co, ro = ot.tensor_omp(Ysub, Ds, w.s)
    sg, cg = pr.supp.cpu().numpy()[idx], pr.coef.cpu().double().numpy()[idx]
    Dc = [d.astype(np.float32).astype(np.float64) for d in Ds]
    agree, ties, bad, err = compare_codes(Ysub, None, None, sg, cg, so, co, 1e-4, K=kron_all(Dc))
    print("trace", trace, "sampled %d: agree %d, ties %d, bad %d, coef err %.2e" % (len(idx), agree, ties, bad, err))
    assert bad == 0 and err <= 1e-4
    assert trace[-1] < 0.5 * trace[0]


def test_tensor_update_many_rows():
    """The FP32 mode sums at a signal count that fills every partial row (20,000 signals of the
    benchmarked 8 x 8 x 4 shape, 12 x 12 x 6 atoms, s = 8: 8,192 rows of about 2.4 signals each),
    each mode's update from the GPU's own codes against the oracle's update from the same codes."""
    w = synth.TENSOR_WORKLOADS["tensor_8x8x4_n12x12x6_s8"]
    N = 20000
    Y = synth.tensor_signals(w, 0, N).astype(np.float32).astype(np.float64)
    E = synth.tensor_dictionaries(w, initial=True)
    for mode in (1, 2, 3):
        pr = api.TensorProblem.from_math(Y, E, w.s, dtype=torch.float32)
        api.tensor_sparse_code(pr)
        torch.cuda.synchronize()
        sg, cg, _ = _codes(pr)
        Dn, co, _ = ot.tensor_update(mode, Y, E, sg, cg)
        api.tensor_update(pr, mode)
        torch.cuda.synchronize()
        errs = [np.abs(g - o).max() / np.abs(o).max() for g, o in zip(pr.dicts(), Dn)]
        cerr = np.abs(pr.coef.cpu().double().numpy() - co).max() / np.abs(co).max()
        print("mode", mode, "D errs", ["%.1e" % e for e in errs], "coef %.1e" % cerr)
        assert max(errs) <= 1e-4 and cerr <= 1e-4
