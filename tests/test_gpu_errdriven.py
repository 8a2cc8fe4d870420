"""Error-driven 2D-OMP (the stopping rule of the paper's denoising runs, Sec. IV): each signal
takes atoms until its residual energy is at or below err2 = eps^2, eps = 1.15 sigma sqrt(m1 m2),
with s = m1 m2 / 2 as the cap.  The generic kernel against the FP64 oracle with the same rule.

Bars: supports and coefficients as in the other parity tests (FP64 1e-10 relative, FP32 1e-4,
agreement >= 97%, every support mismatch a classified near-tie); the number of atoms of a signal
may differ from the oracle's only where the decision is a near-tie with the threshold: the
oracle's residual energy at the smaller count lies within 1e-9 relative of err2 (FP64), or within
64 u ||Y_k||^2 of it in FP32 (u = 2^-24): the kernel tracks the energy by the OMP recurrence
||R||^2 -= corr^2 / delta^2 from ||Y_k||^2 down, whose FP32 rounding error is a small multiple of
u ||Y_k||^2, while the oracle takes it from the explicit residual."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api, synth
from tests.gpu_helpers import compare_codes

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.mark.parametrize("dtype,band,ctol", [(torch.float64, 1e-9, 1e-10), (torch.float32, 1e-4, 1e-4)])
@pytest.mark.parametrize("kernel", [0, 1])
def test_error_driven_matches_oracle(dtype, band, ctol, kernel):
    w = synth.WORKLOADS["fp32_8x8_n16_s8"]
    N = 1500
    Y = synth.signals(w, 0, N)
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)  # the values the kernel reads
    d1, d2 = synth.true_dictionaries(w)
    m = w.m1 * w.m2
    s = m // 2
    err2 = (1.15 * w.sigma() * np.sqrt(m)) ** 2
    so, co, ro = oracle.omp(Y, d1, d2, s, err2=err2, p=8)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=dtype, device=DEV)
    st = api.new_stats()
    api.sparse_code(pr, kernel=kernel, err2=err2, stats=st)
    torch.cuda.synchronize()
    sg, cg, rg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
    ng, no = np.sum(sg >= 0, axis=1), np.sum(so >= 0, axis=1)
    assert st.early_stops == int(np.sum(ng < s))  # every signal that stopped below the cap, once
    assert len(set(no.tolist())) > 3 and np.mean(no < s) > 0.9  # the stop decides, rarely the cap
    same = ng == no
    for k in np.nonzero(~same)[0]:
        t = int(min(ng[k], no[k]))
        r_t = oracle.omp(Y[k:k + 1], d1, d2, max(t, 1))[2][0] if t > 0 else float(np.sum(Y[k] ** 2))
        tol = 1e-9 * err2 if dtype == torch.float64 else 64 * 2.0 ** -24 * float(np.sum(Y[k] ** 2))
        assert abs(r_t - err2) <= tol, (k, int(ng[k]), int(no[k]), r_t / err2, tol / err2)
    ks = np.nonzero(same)[0]
    agree, ties, bad, err = compare_codes(Y[ks], d1, d2, sg[ks], cg[ks], so[ks], co[ks], band, ctol)
    print("%s kernel %d: nnz %d..%d (mean %.1f), count mismatches %d, agree %d/%d, ties %d, bad %d, err %.1e"
          % (dtype, kernel, no.min(), no.max(), no.mean(), int((~same).sum()), agree, len(ks), ties, bad, err))
    if dtype == torch.float64:
        assert (~same).sum() <= 2 and bad == 0 and err <= ctol
        ok = ks[np.all(sg[ks] == so[ks], axis=1)]
        np.testing.assert_allclose(rg[ok], ro[ok], rtol=1e-9)
    else:
        assert (~same).sum() <= 0.01 * N and agree >= 0.97 * len(ks) and bad == 0 and err <= ctol


def test_error_driven_off_matches_plain():
    """err2 = 0 leaves every kernel choice and result unchanged."""
    w = synth.WORKLOADS["fp32_8x8_n16_s8"]
    Y = synth.signals(w, 0, 512)
    d1, d2 = synth.true_dictionaries(w)
    a = api.Problem.from_math(Y, d1, d2, w.s, dtype=torch.float32, device=DEV)
    b = api.Problem.from_math(Y, d1, d2, w.s, dtype=torch.float32, device=DEV)
    api.sparse_code(a)
    api.sparse_code(b, err2=0.0)
    torch.cuda.synchronize()
    assert torch.equal(a.supp, b.supp) and torch.equal(a.coef, b.coef)


def _composed_learn(Y, d1, d2, s, K, err2):
    """Algorithm 1 (OMP, D1 update, OMP, D2 update per iteration) composed from the oracle's
    calls, with the error-driven stop in every OMP sweep."""
    e1, e2 = d1, d2
    for _ in range(K):
        for side in (1, 2):
            supp, coef, _ = oracle.omp(Y, e1, e2, s, err2=err2)
            e1, e2, coef, _ = oracle.tmod_update(side, Y, e1, e2, supp, coef)
    return e1, e2


def test_learn_with_error_driven_stop_fp64(rng):
    """sdl_learn with err2 > 0 (generic kernel, standalone sums) equals Algorithm 1 composed from
    the oracle's error-driven OMP and dictionary updates (FP64, 1e-9)."""
    from tests.conftest import planted, rand_dicts
    t1, t2 = rand_dicts(rng, 6, 7, 9, 11)
    Y, _ = planted(rng, 400, t1, t2, 5, noise=0.2)
    d1, d2 = rand_dicts(rng, 6, 7, 9, 11)
    s, K = 12, 2
    err2 = float(np.median(np.sum(Y ** 2, axis=(1, 2)))) * 0.1
    ref0 = oracle.learn(Y, d1, d2, s, K)  # the composition itself, without the stop, is Algorithm 1
    c1, c2 = _composed_learn(Y, d1, d2, s, K, 0.0)
    np.testing.assert_allclose(c1, ref0["D1"], rtol=1e-12, atol=1e-12)
    e1, e2 = _composed_learn(Y, d1, d2, s, K, err2)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.float64, device=DEV)
    api.learn(pr, K, err2=err2)
    torch.cuda.synchronize()
    nnz = np.sum(pr.supp.cpu().numpy() >= 0, axis=1)
    assert len(set(nnz.tolist())) > 2  # the stop varies per signal
    for g, o in ((pr.d1(), e1), (pr.d2(), e2)):
        assert np.abs(g - o).max() <= 1e-10 * np.abs(o).max()
