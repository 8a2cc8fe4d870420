"""Learned support proposal on the GPU against the FP64 numpy MLP oracle and the 2D-OMP oracle.

Weights are generated here (seeded numpy) and loaded into the library, so both sides
start from the same parameters; labels for the gradient checks are the oracle's OMP
supports.  Bars: FP32 check mode gradients/logits within 1e-4 (relative to the largest
entry), BF16 within 5e-2 (relative norm per parameter block).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from paper_2007_03800_amd import api, synth
from tests.conftest import planted, rand_dicts
from tests.gpu_helpers import compare_codes

pytestmark = pytest.mark.gpu

M1 = M2 = 8
N1 = N2 = 16
S = 8


def weights(rng, H, A=256, M=64, scale=1.0):
    off, n = mlp.layout(M, H, A)
    p = np.zeros(n)
    fans = [M, H, H]
    for l in range(3):
        a, b = off[2 * l], off[2 * l + 1]
        p[a:b] = rng.standard_normal(b - a) * np.sqrt(2.0 / fans[l]) * scale
        p[b:off[2 * l + 2]] = 0.1 * rng.standard_normal(off[2 * l + 2] - b)
    return p.astype(np.float32)


def data(rng, B):
    d1, d2 = rand_dicts(rng, M1, M2, N1, N2)
    Y, _ = planted(rng, B, d1, d2, S, noise=0.05)
    supp, _, _ = oracle.omp(Y, d1, d2, S)
    return Y, supp, d1, d2


def to_dev(Y, supp):
    Yc = torch.from_numpy(np.ascontiguousarray(Y.transpose(0, 2, 1))).float().cuda()
    return Yc, torch.from_numpy(supp).cuda()


@pytest.mark.parametrize("H", [128, 512])
def test_gradient_fp32_check_mode(H, rng):
    p = weights(rng, H)
    Y, supp, _, _ = data(rng, 128)
    net = api.Proposer(M1, M2, N1, N2, hidden=H, fp32_check=True)
    net.set_params(p)
    Yd, sd = to_dev(Y, supp)
    loss, g = net.gradient(Yd, sd, S)
    x = mlp.inputs(Y)
    lref, gref = mlp.loss_and_grad(p.astype(np.float64), x, mlp.labels(supp, 256), 64, H, 256)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    off, _ = mlp.layout(64, H, 256)
    for b in range(6):
        gb, rb = g[off[b]:off[b + 1]], gref[off[b]:off[b + 1]]
        assert np.max(np.abs(gb - rb)) <= 1e-4 * np.max(np.abs(rb)), b


def test_gradient_bf16(rng):
    H = 512
    p = weights(rng, H)
    Y, supp, _, _ = data(rng, 256)
    net = api.Proposer(M1, M2, N1, N2, hidden=H)
    net.set_params(p)
    loss, g = net.gradient(*to_dev(Y, supp), S)
    lref, gref = mlp.loss_and_grad(p.astype(np.float64), mlp.inputs(Y), mlp.labels(supp, 256), 64, H, 256)
    assert abs(loss - lref) <= 1e-2 * abs(lref)
    off, _ = mlp.layout(64, H, 256)
    for b in range(6):
        gb, rb = g[off[b]:off[b + 1]], gref[off[b]:off[b + 1]]
        assert np.linalg.norm(gb - rb) <= 5e-2 * np.linalg.norm(rb), b


def test_logits_and_proposal_fp32(rng):
    H = 128
    p = weights(rng, H)
    Y, supp, d1, d2 = data(rng, 300)
    net = api.Proposer(M1, M2, N1, N2, hidden=H, fp32_check=True)
    net.set_params(p)
    Yd, _ = to_dev(Y, supp)
    z = net.logits(Yd).cpu().numpy()
    zref, _ = mlp.forward(p.astype(np.float64), mlp.inputs(Y), 64, H, 256)
    assert np.max(np.abs(z - zref)) <= 1e-4 * np.max(np.abs(zref))
    # proposal with everything accepted: top-s of the logits, LS on them
    pr = api.Problem.from_math(Y, d1, d2, S, dtype=torch.float32)
    acc = torch.zeros(len(Y), dtype=torch.int32, device="cuda")
    api.learned_sparse_code(net, pr, tau=1e30, accept=acc)
    torch.cuda.synchronize()
    assert int(acc.sum()) == len(Y)
    sg = pr.supp.cpu().numpy()
    np.testing.assert_array_equal(sg, mlp.top_s(z, S))  # same logits -> same top-s (ties: smallest index)
    cref, rref = mlp.least_squares_on_support(Y, d1, d2, sg)
    cg = pr.coef.cpu().double().numpy()
    assert np.max(np.abs(cg - cref)) <= 1e-3 * np.max(np.abs(cref))
    np.testing.assert_allclose(pr.res2.cpu().double().numpy(), rref, rtol=1e-2, atol=1e-5)


def test_logits_bf16(rng):
    """BF16 forward (the 128x128 tile kernel; 320 rows, so the last tile is half full) against
    the FP64 oracle: BF16 operands with FP32 accumulation, bar 2e-2 of the largest logit."""
    H = 512
    p = weights(rng, H)
    Y, supp, _, _ = data(rng, 320)
    net = api.Proposer(M1, M2, N1, N2, hidden=H)
    net.set_params(p)
    Yd, _ = to_dev(Y, supp)
    z = net.logits(Yd).cpu().numpy()
    zref, _ = mlp.forward(p.astype(np.float64), mlp.inputs(Y), 64, H, 256)
    err = np.max(np.abs(z - zref)) / np.max(np.abs(zref))
    print("bf16 logits max rel err %.2e" % err)
    assert err <= 2e-2


def test_all_rejected_equals_plain_omp(rng):
    Y, _, d1, d2 = data(rng, 1000)
    net = api.Proposer(M1, M2, N1, N2, hidden=128)
    a = api.Problem.from_math(Y, d1, d2, S, dtype=torch.float32)
    api.learned_sparse_code(net, a, tau=0.0)
    b = api.Problem.from_math(Y, d1, d2, S, dtype=torch.float32)
    api.sparse_code(b, kernel=2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.supp.cpu().numpy(), b.supp.cpu().numpy())
    np.testing.assert_array_equal(a.coef.cpu().numpy(), b.coef.cpu().numpy())
    np.testing.assert_array_equal(a.res2.cpu().numpy(), b.res2.cpu().numpy())


def test_training_gain_and_matched_rmse():
    """Trained on 2D-OMP supports at the generating dictionaries, the network beats the label
    prior and an untrained network at predicting OMP's atoms; with the calibrated acceptance
    test the learned coding keeps the RMSE within 1% of the FP64 oracle's (the 2D-OMP fallback
    takes every signal whose proposal fails the test)."""
    w = synth.WORKLOADS["learned_8x8_n16_s8"]
    d1, d2 = synth.true_dictionaries(w)
    ntr, ncal, nev = 100000, 5000, 5000
    Ytr = torch.from_numpy(synth.signals(w, 0, ntr, layout="colmajor")).float().cuda()
    tr = api.Problem(Ytr, torch.from_numpy(d1.T.copy()).cuda(), torch.from_numpy(d2.T.copy()).cuda(), w.s)
    api.sparse_code(tr)
    cal_y = synth.signals(w, ntr, ntr + ncal)
    ev_y = synth.signals(w, ntr + ncal, ntr + ncal + nev)
    so_ev, _, r_o = oracle.omp(ev_y, d1, d2, w.s, p=8)

    def hit_rate(net):
        Yd = torch.from_numpy(np.ascontiguousarray(ev_y.transpose(0, 2, 1))).float().cuda()
        top = mlp.top_s(net.logits(Yd).cpu().numpy(), w.s)
        return float(np.mean([len(set(top[k]) & set(so_ev[k])) for k in range(nev)])) / w.s

    untrained = api.Proposer(M1, M2, N1, N2, hidden=512, seed=3)
    h0 = hit_rate(untrained)
    net = api.Proposer(M1, M2, N1, N2, hidden=512, seed=3)
    losses = net.train(Ytr, tr.supp, w.s, epochs=8, batch=256, lr=1e-3)
    p = w.s / 256.0
    prior = -(p * np.log(p) + (1 - p) * np.log(1 - p))  # BCE of predicting the label frequency
    assert losses[-1] < 0.8 * prior
    h1 = hit_rate(net)
    cal = api.Problem.from_math(cal_y, d1, d2, w.s)
    tau = net.calibrate(cal)
    ev = api.Problem.from_math(ev_y, d1, d2, w.s)
    st = api.new_stats()
    api.learned_sparse_code(net, ev, tau=tau, stats=st)
    print("top-s hit rate untrained %.3f trained %.3f; tau %.3g; fallback rate %.3f; losses %s"
          % (h0, h1, tau, st.fallbacks / nev, np.round(losses, 4)))
    assert h1 > h0 + 0.2
    r_g = ev.res2.cpu().double().numpy()
    assert abs(np.sqrt(r_g.mean()) / np.sqrt(r_o.mean()) - 1) <= 0.01


def test_learn_with_proposer_runs_and_tracks_plain(rng):
    w = synth.WORKLOADS["learned_8x8_n16_s8"]
    d1, d2 = synth.true_dictionaries(w)
    Y = synth.signals(w, 0, 20000)
    net = api.Proposer(M1, M2, N1, N2, hidden=128, seed=5)
    a = api.Problem.from_math(Y, d1, d2, w.s)
    ta = api.learn(a, 3, proposer=net, tau=0.0)[0]   # every signal falls back: equals plain
    b = api.Problem.from_math(Y, d1, d2, w.s)
    tb = api.learn(b, 3)[0]
    np.testing.assert_allclose(ta, tb, rtol=1e-4)


def test_proposer_save_load_roundtrip(rng, tmp_path):
    """sdl_proposer_save / sdl_proposer_load: same weights, same logits, same shape."""
    net = api.Proposer(M1, M2, N1, N2, hidden=128, seed=11)
    net.set_params(weights(rng, 128))
    path = tmp_path / "net.bin"
    net.save(path)
    back = api.Proposer.load(path)
    assert (back.m1, back.m2, back.n1, back.n2, back.hidden) == (M1, M2, N1, N2, 128)
    np.testing.assert_array_equal(back.params(), net.params())
    Y, _, _, _ = data(rng, 256)
    Yd = torch.from_numpy(np.ascontiguousarray(Y.transpose(0, 2, 1))).float().cuda()
    assert torch.equal(back.logits(Yd), net.logits(Yd))


def _oracle_learned_learn(Y, e1, e2, s, K, supp, tau=None):
    """Algorithm 1 composed from the oracle's calls where every sparse coding takes the proposal
    supp (the network sees only Y, so its proposal is the same in every sweep): least squares on
    it, kept where its residual is <= tau ||Y||^2 (tau None: always), else the oracle's 2D-OMP."""
    yy = np.sum(Y ** 2, axis=(1, 2))

    def code(d1, d2):
        c, r = mlp.least_squares_on_support(Y, d1, d2, supp)
        sp = supp.astype(np.int32).copy()
        if tau is not None:
            rej = ~(r <= tau * yy)
            if rej.any():
                so, co, ro = oracle.omp(Y[rej], d1, d2, s, p=8)
                sp[rej], c[rej], r[rej] = so, co, ro
        return sp, c, r

    trace = []
    for _ in range(K):
        sp, c, r = code(e1, e2)
        trace.append(np.sqrt(r.sum() / (len(Y) * Y.shape[1] * Y.shape[2])))
        e1 = oracle.tmod_update(1, Y, e1, e2, sp, c)[0]
        sp, c, r = code(e1, e2)
        e2 = oracle.tmod_update(2, Y, e1, e2, sp, c)[1]
    sp, c, r = code(e1, e2)
    trace.append(np.sqrt(r.sum() / (len(Y) * Y.shape[1] * Y.shape[2])))
    return e1, e2, np.array(trace), r


@pytest.mark.parametrize("share", ["all", "half"])
def test_learn_with_accepted_proposals_matches_oracle(share, rng):
    """sdl_learn with the learned proposal where proposals are accepted, against Algorithm 1
    composed from the oracle's calls with the same proposals (the GPU network's top-s supports:
    the network's input is Y alone, so one proposal per signal serves every sweep).
    "all": tau accepts every proposal, so every sweep is least squares on the proposal and the
    updates are the oracle's from those codes (bars: dictionaries and trace 1e-4, FP32 least
    squares).  "half": tau is the median residual ratio of the proposals at the starting
    dictionaries, so about half are accepted and the rest take 2D-OMP; the oracle takes each
    decision from its own FP64 residuals (a decision can flip only for a residual within rounding
    of the threshold), bars 1e-3."""
    d1, d2 = rand_dicts(rng, M1, M2, N1, N2)
    Y, _ = planted(rng, 4000, d1, d2, S, noise=0.05)
    Y = Y.astype(np.float32).astype(np.float64)
    e1, e2 = rand_dicts(rng, M1, M2, N1, N2)
    net = api.Proposer(M1, M2, N1, N2, hidden=128, seed=5)
    net.set_params(weights(rng, 128))
    p0 = api.Problem.from_math(Y, e1, e2, S, dtype=torch.float32)
    acc = torch.zeros(len(Y), dtype=torch.int32, device="cuda")
    api.learned_sparse_code(net, p0, tau=1e30, accept=acc)
    torch.cuda.synchronize()
    assert bool(torch.all(acc == 1))
    supp = p0.supp.cpu().numpy()
    yy = np.sum(Y ** 2, axis=(1, 2))
    tau = 1e30 if share == "all" else float(np.median(p0.res2.cpu().double().numpy() / yy))
    K = 2
    o1, o2, otrace, _ = _oracle_learned_learn(Y, e1, e2, S, K, supp, None if share == "all" else tau)
    pr = api.Problem.from_math(Y, e1, e2, S, dtype=torch.float32)
    st = api.new_stats()
    trace = api.learn(pr, K, proposer=net, tau=tau, stats=st)[0]
    n = st.proposals_accepted + st.fallbacks
    accepted = st.proposals_accepted / n
    err = max(np.abs(pr.d1() - o1).max() / np.abs(o1).max(), np.abs(pr.d2() - o2).max() / np.abs(o2).max())
    print(share, "tau %.3g accepted share %.3f over %d codings; D err %.2e; trace %s oracle %s"
          % (tau, accepted, n, err, np.round(trace, 6), np.round(otrace, 6)))
    assert n == len(Y) * (2 * K + 1)
    bar = 1e-4 if share == "all" else 1e-3
    if share == "all":
        assert st.fallbacks == 0
    else:
        assert 0.2 < accepted < 0.8
    assert err <= bar
    np.testing.assert_allclose(trace, otrace, rtol=bar)
