"""SDL_MIXED_BF16: 2D-OMP whose correlations D1^T R_k D2 are recomputed every step on the BF16
matrix cores (FP32 accumulation), with every candidate whose BF16 |correlation| lies within
tie_band (2^-6) of the largest re-scored in FP32, FP32 residual and Cholesky, FP64 solves.

Against the FP64 oracle run on the same bfloat16-rounded signals.  Bars: supports identical
except classified near-ties, where a near-tie is now one within tie_band (the precision of the
BF16 correlations that decide the candidate set); coefficients (FP32 solves on the exact FP32
correlation of each pick) within 1e-4 element-wise as for FP32; RMSE within 1% of the oracle's;
support agreement reported.  Planted near-ties (two atoms whose correlations differ by about a
third of the band) check that the FP32 re-score, not the BF16 order, decides the pick."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api, synth
from tests.conftest import planted, rand_dicts
from tests.gpu_helpers import code_stats, full_size_checks

pytestmark = pytest.mark.gpu

DEV = "cuda"
BAND = 2.0 ** -6
SHAPES = [(12, 12, 24, 24, 12), (8, 8, 16, 16, 8), (12, 12, 20, 20, 10)]


def rounded(Y):
    return torch.as_tensor(Y).to(torch.bfloat16).double().numpy()


def mixed_codes(Yr, d1, d2, s, **opts):
    pr = api.Problem.from_math(Yr, d1, d2, s, dtype=torch.bfloat16, device=DEV)
    st = api.new_stats()
    api.sparse_code(pr, mixed=True, stats=st, **opts)
    torch.cuda.synchronize()
    return pr, st


def test_mixed_supported_shapes():
    for sh in SHAPES:
        assert api.mixed_supported(*sh)
    assert not api.mixed_supported(5, 9, 11, 6, 7)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_mixed_sparse_code_matches_oracle(shape, rng):
    m1, m2, n1, n2, s = shape
    N = 1237  # 77 groups of 16 and a ragged group of 5
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, d1, d2, s, noise=0.03)
    Y[4] = 0.0
    Yr = rounded(Y)
    pr, st = mixed_codes(Yr, d1, d2, s)
    so, co, ro = oracle.omp(Yr, d1, d2, s, p=8)
    sg, cg, rg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
    r = code_stats(Yr, d1, d2, sg, cg, so, co, BAND)
    rm = np.sqrt(rg.mean()) / np.sqrt(ro.mean())
    print(shape, "agree %d/%d ties %d bad %d coef err %.2e, rmse ratio %.7f, stats %s"
          % (r["agree"], N, r["ties"], r["bad"], r["coef_err"], rm, st.as_dict()))
    assert r["bad"] == 0, r["gaps"][:5]
    assert r["agree"] >= 0.97 * N and r["coef_err"] <= 1e-4
    assert abs(rm - 1) <= 0.01
    assert np.all(sg[4] == -1) and rg[4] == 0
    ok = np.all(sg == so, axis=1)
    np.testing.assert_allclose(rg[ok], ro[ok], rtol=2e-3, atol=1e-6)


def test_planted_near_ties_are_rescored(rng):
    """Signals y = a d_p + b d_q + small noise with |a| and |b| about 0.5% apart: the first pick is a
    near-tie inside the band.  The mixed kernel must choose what FP32 (and the FP64 oracle) choose."""
    m1, m2, n1, n2, s = 12, 12, 24, 24, 12
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    K = np.kron(d2, d1)
    N = 2000
    Y = np.zeros((N, m1, m2))
    for k in range(N):
        p, q = rng.choice(n1 * n2, 2, replace=False)
        a = rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 1.5)
        b = np.sign(rng.standard_normal()) * abs(a) * (1.0 + rng.choice([-1, 1]) * rng.uniform(0.003, 0.006))
        y = a * K[:, p] + b * K[:, q] + 1e-3 * rng.standard_normal(m1 * m2)
        Y[k] = y.reshape(m2, m1).T
    Yr = rounded(Y)
    pr, st = mixed_codes(Yr, d1, d2, s)
    so, co, _ = oracle.omp(Yr, d1, d2, s, p=8)
    sg = pr.supp.cpu().numpy()[:, :2]
    # the two planted atoms: the oracle's first pick leads the runner-up by more than the BF16
    # error of the correlations but by less than the band
    first_same = float(np.mean(sg[:, 0] == so[:, 0]))
    z = np.zeros((N, 2))
    r = code_stats(Yr, d1, d2, sg, z, so[:, :2], z, 1e-4)
    print("first pick as the oracle's %.4f; agree %d ties(1e-4) %d bad %d; stats %s"
          % (first_same, r["agree"], r["ties"], r["bad"], st.as_dict()))
    assert st.near_tie_rescores > 0.5 * N
    assert r["bad"] == 0  # every mismatch is a near-tie at FP32 resolution, not at BF16's


def test_mixed_learn_tracks_oracle(rng):
    w = synth.WORKLOADS["mixed_12x12_n24_s12"]
    Y = rounded(synth.signals(w, 0, 3000))
    e1, e2 = synth.initial_dictionaries(w)
    K = 3
    ref = oracle.learn(Y, e1, e2, w.s, K, p=8)
    pr = api.Problem.from_math(Y, e1, e2, w.s, dtype=torch.bfloat16)
    tr = api.learn(pr, K, mixed=True)[0]
    print("rmse gpu", tr, "oracle", ref["rmse"])
    np.testing.assert_allclose(tr, ref["rmse"], rtol=0.01)


def test_mixed_graph_equals_eager_and_deterministic(rng):
    m1, m2, n1, n2, s, N = 12, 12, 24, 24, 12, 3000
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y = rounded(planted(rng, N, t1, t2, s, noise=0.05)[0])
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    outs = []
    for use_graph in (1, 0, 1):
        pr = api.Problem.from_math(Y, d1, d2, s, dtype=torch.bfloat16)
        tr = api.learn(pr, 5, use_graph=use_graph, mixed=True)
        outs.append((tr, pr.d1(), pr.d2(), pr.supp.cpu().numpy(), pr.coef.cpu().numpy()))
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            np.testing.assert_array_equal(u, v)


def test_mixed_workload_full_size():
    """The mixed-precision workload at its full size (1,000,000 BF16 signals, 12x12, 24x24 atoms,
    s = 12) as the benchmark runs it: sampled final codes against the oracle's 2D-OMP at the GPU's
    final dictionaries (near-ties at the band), RMSE and support agreement on the first 5,000, and
    one full-batch D1 update from identical codes against the oracle's FP64 update."""
    w = synth.WORKLOADS["mixed_12x12_n24_s12"]
    Yb = torch.from_numpy(synth.signals(w, 0, w.N, layout="colmajor")).to(torch.bfloat16)
    Ym = Yb.double().numpy().transpose(0, 2, 1)
    Y = Yb.to(DEV).contiguous()
    e1, e2 = synth.initial_dictionaries(w)

    def fresh():
        return api.Problem(Y, torch.from_numpy(e1.T.copy()).to(DEV), torch.from_numpy(e2.T.copy()).to(DEV), w.s)

    pr = fresh()
    api.learn(pr, 2, mixed=True)
    torch.cuda.synchronize()
    n, agree, ties, bad, err, dd = full_size_checks(Ym, pr, w.s, fresh, n_each=700, band=BAND, mixed=True)
    so, _, ro = oracle.omp(Ym[:5000], pr.d1(), pr.d2(), w.s, p=8)
    rg = pr.res2[:5000].double().cpu().numpy()
    rm = np.sqrt(rg.mean()) / np.sqrt(ro.mean())
    sa = float(np.mean(np.all(np.sort(pr.supp[:5000].cpu().numpy(), 1) == np.sort(so, 1), axis=1)))
    print("sampled support agreement %d/%d, near-ties %d, other %d, coef err %.2e; D1 update diff %.2e; "
          "rmse ratio %.7f, support agreement (5000) %.4f" % (agree, n, ties, bad, err, dd, rm, sa))
    assert agree >= 0.97 * n and bad == 0 and err <= 1e-4
    assert dd <= 1e-4 and abs(rm - 1) <= 0.01
