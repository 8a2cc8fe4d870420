"""Pins of the n-dimensional oracle (Remark 3) against what fixes it independently of itself:

* two modes: the separate two-dimensional oracle in C (itself pinned against 1D OMP, the Gram
  identities and lstsq) gives the same codes, the same mode-1 and mode-2 updates (Corollary 1,
  Result 1) and the same Algorithm 1 trajectory;
* the atom convention: column a of the Kronecker dictionary is the outer product of the chosen
  columns, built here with einsum;
* orthonormal dictionaries (Remark 1 in n modes): the codes are the s largest entries of the core
  tensor Y x_1 D_1^T ... x_n D_n^T (einsum), with residual energy ||Y||^2 minus their squares; the
  error-driven stop takes the smallest count whose tail energy is within err2;
* the mode-d update: numpy lstsq of the stacked system [Y_1(d) ... Y_N(d)] = D [W_1(d) ... W_N(d)]
  (W built here by einsum, not by the oracle's mode products), then unit-norm columns; the
  rescaled codes reproduce the unnormalised model; the objective does not increase;
* planted noiseless codes are recovered exactly.
"""
import numpy as np
import pytest

import oracle
from oracle import tensor as ot


def unit_cols(rng, m, n):
    d = rng.standard_normal((m, n))
    return d / np.linalg.norm(d, axis=0)


def orth(rng, m):
    q, r = np.linalg.qr(rng.standard_normal((m, m)))
    return q * np.sign(np.diag(r))


def planted3(rng, N, Ds, s, noise):
    ns = [D.shape[1] for D in Ds]
    A = int(np.prod(ns))
    X = np.zeros((N, A))
    supp = np.zeros((N, s), np.int64)
    for k in range(N):
        a = rng.choice(A, s, replace=False)
        supp[k] = a
        X[k, a] = rng.choice([-1.0, 1.0], s) * rng.uniform(0.5, 1.5, s)
    X = X.reshape((N,) + tuple(ns), order="F")
    Y = np.einsum("kabc,pa,qb,rc->kpqr", X, *Ds)
    return Y + noise * rng.standard_normal(Y.shape), supp, X


def test_two_modes_codes_match_the_two_dimensional_oracle(rng):
    d1, d2 = unit_cols(rng, 6, 9), unit_cols(rng, 5, 8)
    Y = rng.standard_normal((120, 6, 5))
    for err2 in (0.0, 4.0):
        so, co, ro = oracle.omp(Y, d1, d2, 6, err2=err2)
        st, ct, rt = ot.tensor_omp(Y, [d1, d2], 6, err2=err2)
        np.testing.assert_array_equal(st, so)
        np.testing.assert_allclose(ct, co, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(rt, ro, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("mode", [1, 2])
def test_two_modes_update_matches_the_two_dimensional_oracle(mode, rng):
    d1, d2 = unit_cols(rng, 6, 9), unit_cols(rng, 5, 8)
    Y = rng.standard_normal((200, 6, 5))
    supp, coef, _ = oracle.omp(Y, d1, d2, 5)
    e1, e2, co, wo = oracle.tmod_update(mode, Y, d1, d2, supp, coef)
    Ds, ct, wt = ot.tensor_update(mode, Y, [d1, d2], supp, coef)
    np.testing.assert_allclose(Ds[0], e1, atol=1e-10)
    np.testing.assert_allclose(Ds[1], e2, atol=1e-10)
    np.testing.assert_allclose(ct, co, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(wt, wo, rtol=1e-10)


def test_two_modes_learning_matches_algorithm_1(rng):
    t1, t2 = unit_cols(rng, 6, 8), unit_cols(rng, 6, 8)
    Y = np.einsum("pa,kab,qb->kpq", t1, rng.standard_normal((150, 8, 8)) * (rng.random((150, 8, 8)) < 0.06), t2)
    Y += 0.01 * rng.standard_normal(Y.shape)
    d1, d2 = unit_cols(rng, 6, 8), unit_cols(rng, 6, 8)
    ref = oracle.learn(Y, d1, d2, 4, 3)
    got = ot.tensor_learn(Y, [d1, d2], 4, 3)
    np.testing.assert_allclose(got["Ds"][0], ref["D1"], atol=1e-9)
    np.testing.assert_allclose(got["Ds"][1], ref["D2"], atol=1e-9)
    np.testing.assert_allclose(got["rmse"], ref["rmse"], rtol=1e-9)
    np.testing.assert_array_equal(got["supp"], ref["supp"])


def test_atom_convention_is_the_outer_product(rng):
    Ds = [unit_cols(rng, 3, 4), unit_cols(rng, 2, 3), unit_cols(rng, 4, 2)]
    K = ot.kron_dictionary(Ds)
    assert K.shape == (24, 24)
    for a in rng.choice(24, 10, replace=False):
        i1, i2, i3 = a % 4, (a // 4) % 3, a // 12
        outer = np.einsum("p,q,r->pqr", Ds[0][:, i1], Ds[1][:, i2], Ds[2][:, i3])
        np.testing.assert_array_equal(K[:, a], outer.flatten("F"))
        assert ot.atom_multi_index(int(a), [4, 3, 2]) == [i1, i2, i3]


@pytest.mark.parametrize("ms,s", [((4, 3, 5), 7), ((3, 3, 3, 2), 5)])
def test_orthonormal_is_hard_thresholding_of_the_core(ms, s, rng):
    Ds = [orth(rng, m) for m in ms]
    Y = rng.standard_normal((60,) + ms)
    sub = "pqrs"[:len(ms)]
    core = np.einsum("k" + sub + "," + ",".join(p + c for p, c in zip(sub, "abcd")) + "->k" + "abcd"[:len(ms)], Y, *Ds)
    C = core.reshape(60, -1, order="F")
    top = np.argsort(-np.abs(C), axis=1, kind="stable")[:, :s]
    supp, coef, res2 = ot.tensor_omp(Y, Ds, s)
    np.testing.assert_array_equal(supp, top)
    np.testing.assert_allclose(coef, np.take_along_axis(C, top, 1), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(res2, np.sum(Y.reshape(60, -1) ** 2, 1) - np.sum(coef ** 2, 1), rtol=1e-9,
                               atol=1e-12)
    # error-driven stop: the smallest count whose tail energy is <= err2
    err2 = 0.5 * float(np.median(np.sum(Y.reshape(60, -1) ** 2, 1)))
    se, ce, re = ot.tensor_omp(Y, Ds, C.shape[1], err2=err2)
    srt = -np.sort(-C ** 2, axis=1)
    tail = np.sum(C ** 2, 1)[:, None] - np.concatenate([np.zeros((60, 1)), np.cumsum(srt, 1)], 1)
    expect = np.argmax(tail <= err2, axis=1)
    np.testing.assert_array_equal(np.sum(se >= 0, 1), expect)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_update_is_stacked_lstsq(mode, rng):
    Ds = [unit_cols(rng, 4, 6), unit_cols(rng, 3, 5), unit_cols(rng, 5, 4)]
    Y, _, _ = planted3(rng, 150, Ds, 3, 0.1)
    E = [unit_cols(rng, 4, 6), unit_cols(rng, 3, 5), unit_cols(rng, 5, 4)]
    supp, coef, _ = ot.tensor_omp(Y, E, 3)
    X = ot.densify(supp, coef, [6, 5, 4])
    d = mode - 1
    # W = X with every other mode multiplied by its dictionary, by einsum
    ops = [E[e] if e != d else np.eye(E[e].shape[1]) for e in range(3)]
    W = np.einsum("kabc,pa,qb,rc->kpqr", X, *ops)
    Wd = np.concatenate([np.moveaxis(W[k], d, 0).reshape(W.shape[1 + d], -1) for k in range(len(W))], axis=1)
    Yd = np.concatenate([np.moveaxis(Y[k], d, 0).reshape(Y.shape[1 + d], -1) for k in range(len(Y))], axis=1)
    used = np.abs(Wd).sum(axis=1) > 0
    Dls = np.array(E[d], copy=True)
    Dls[:, used] = np.linalg.lstsq(Wd[used].T, Yd.T, rcond=None)[0].T
    nrm = np.linalg.norm(Dls[:, used], axis=0)
    Dn, cn, w = ot.tensor_update(mode, Y, E, supp, coef)
    expect = Dls.copy()
    expect[:, used] = Dls[:, used] / nrm
    np.testing.assert_allclose(Dn[d], expect, atol=1e-10)
    for e in range(3):
        if e != d:
            np.testing.assert_array_equal(Dn[e], E[e])
    # rescaled codes with the normalised dictionary reproduce the unnormalised least-squares model
    Dun = [E[e] if e != d else Dls for e in range(3)]
    np.testing.assert_allclose(ot.reconstruct(supp, cn, Dn), ot.reconstruct(supp, coef, Dun), atol=1e-10)
    # the update never increases the objective
    f0 = np.sum((Y - ot.reconstruct(supp, coef, E)) ** 2)
    f1 = np.sum((Y - ot.reconstruct(supp, cn, Dn)) ** 2)
    assert f1 <= f0 * (1 + 1e-12)


def test_update_keeps_unused_atoms_and_reports_singular(rng):
    Ds = [unit_cols(rng, 4, 5), unit_cols(rng, 3, 4), unit_cols(rng, 2, 3)]
    Y = rng.standard_normal((40, 4, 3, 2))
    supp = np.zeros((40, 2), np.int32)
    supp[:, 1] = 1 + 5 * rng.integers(0, 4, 40)      # mode-1 index 1, any mode-2 index
    coef = rng.standard_normal((40, 2))
    Dn, _, w = ot.tensor_update(1, Y, Ds, supp, coef)
    np.testing.assert_array_equal(Dn[0][:, 2:], Ds[0][:, 2:])   # atoms 2..4 unused: kept
    assert np.all(w[2:] == 1.0)
    # atoms (0,0,0) and (0,1,0) in every code with coefficients in a fixed ratio: the two mode-2
    # rows of every W_k(2) are proportional, so the mode-2 Gram sum has rank one
    supp2 = np.tile(np.array([0, 5], np.int32), (40, 1))
    x0 = rng.standard_normal(40)
    with pytest.raises(ot.TensorOracleError):
        ot.tensor_update(2, Y, Ds, supp2, np.stack([x0, 2.0 * x0], axis=1))


def test_planted_recovery_three_modes(rng):
    Ds = [unit_cols(rng, 6, 8), unit_cols(rng, 6, 8), unit_cols(rng, 4, 5)]
    Y, true_supp, X = planted3(rng, 80, Ds, 3, 0.0)
    supp, coef, res2 = ot.tensor_omp(Y, Ds, 3)
    ok = np.array([set(supp[k]) == set(true_supp[k]) for k in range(80)])
    assert ok.mean() >= 0.9
    Xr = ot.densify(supp, coef, [8, 8, 5])
    np.testing.assert_allclose(Xr[ok], X[ok], atol=1e-10)
    assert np.all(res2[ok] <= 1e-20 * np.sum(Y[ok] ** 2, axis=(1, 2, 3)) + 1e-24)


def test_learn_is_the_composed_calls(rng):
    Ds = [unit_cols(rng, 4, 5), unit_cols(rng, 4, 5), unit_cols(rng, 3, 4)]
    Y, _, _ = planted3(rng, 60, Ds, 3, 0.05)
    E = [unit_cols(rng, 4, 5), unit_cols(rng, 4, 5), unit_cols(rng, 3, 4)]
    got = ot.tensor_learn(Y, E, 3, 2)
    F = [e.copy() for e in E]
    for _ in range(2):
        for d in range(3):
            supp, coef, _ = ot.tensor_omp(Y, F, 3)
            F, _, _ = ot.tensor_update(d + 1, Y, F, supp, coef)
    for a, b in zip(got["Ds"], F):
        np.testing.assert_array_equal(a, b)
    assert len(got["rmse"]) == 3 and got["rmse"][-1] < got["rmse"][0]
