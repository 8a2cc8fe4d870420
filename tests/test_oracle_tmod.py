"""Pins of the oracle's TMOD updates and of Algorithm 1's schedule.

Independent routes: numpy least squares on the stacked system, the MOD closed
form for D2 = I, the paper's Gram shortcut, planted exact recovery, and the
monotonicity of the dictionary updates.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import planted, rand_dicts


def objective(Y, d1, d2, supp, coef):
    X = oracle.densify(supp, coef, d1.shape[1], d2.shape[1])
    return float(np.sum((Y - np.einsum("pi,kij,qj->kpq", d1, X, d2)) ** 2))


def setup(rng, m1=6, m2=5, n1=9, n2=7, s=4, N=300, noise=0.05):
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, N, d1, d2, s, noise=noise)
    i1, i2 = rand_dicts(rng, m1, m2, n1, n2)
    supp, coef, _ = oracle.omp(Y, i1, i2, s)
    return Y, i1, i2, supp, coef


def test_gram_shortcut_matches_dense_sums(rng):
    """Sum T_k T_k^T = sum X_k G2 X_k^T and sum Z_k^T Z_k = sum X_k^T G1 X_k (text after Algorithm 1)."""
    Y, d1, d2, supp, coef = setup(rng)
    X = oracle.densify(supp, coef, d1.shape[1], d2.shape[1])
    A1, B1 = oracle.tmod_sums(1, Y, d1, d2, supp, coef)
    A2, B2 = oracle.tmod_sums(2, Y, d1, d2, supp, coef)
    G1, G2 = d1.T @ d1, d2.T @ d2
    np.testing.assert_allclose(A1, np.einsum("kij,jl,kml->im", X, G2, X), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(A2, np.einsum("kij,il,klm->jm", X, G1, X), rtol=1e-12, atol=1e-12)
    # B sides: sum Y_k D2 X_k^T and sum Y_k^T D1 X_k
    np.testing.assert_allclose(B1, np.einsum("kpq,qj,kij->pi", Y, d2, X), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(B2, np.einsum("kpq,pi,kij->qj", Y, d1, X), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("side", [1, 2])
def test_update_equals_stacked_lstsq(rng, side):
    """Corollary 1 / Result 1: the update is the LS solution of the stacked system, normalised."""
    Y, d1, d2, supp, coef = setup(rng)
    X = oracle.densify(supp, coef, d1.shape[1], d2.shape[1])
    n1d, n2d, c, w = oracle.tmod_update(side, Y, d1, d2, supp, coef)
    if side == 1:
        # [Y_1 ... Y_N] = D1 [T_1 ... T_N],  T_k = X_k D2^T
        T = np.concatenate([X[k] @ d2.T for k in range(len(Y))], axis=1)
        Ycat = np.concatenate(list(Y), axis=1)
        Dstar = np.linalg.lstsq(T.T, Ycat.T, rcond=None)[0].T
        got = n1d
        np.testing.assert_array_equal(n2d, d2)
    else:
        # [Y_1^T ... Y_N^T] = D2 [Z_1^T ... Z_N^T],  Z_k = D1 X_k
        Zt = np.concatenate([(d1 @ X[k]).T for k in range(len(Y))], axis=1)
        Ycat = np.concatenate([Y[k].T for k in range(len(Y))], axis=1)
        Dstar = np.linalg.lstsq(Zt.T, Ycat.T, rcond=None)[0].T
        got = n2d
        np.testing.assert_array_equal(n1d, d1)
    norms = np.linalg.norm(Dstar, axis=0)
    np.testing.assert_allclose(got, Dstar / norms, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(w, norms, rtol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(got, axis=0), 1.0, rtol=1e-14)


@pytest.mark.parametrize("side", [1, 2])
def test_normal_equations_and_invariant_product(rng, side):
    """After the update the gradient of eq. (1) w.r.t. the updated dictionary vanishes, and the
    rescaled codes leave every product D1 X_k D2^T equal to the unnormalised LS solution's."""
    Y, d1, d2, supp, coef = setup(rng)
    n1d, n2d, c, w = oracle.tmod_update(side, Y, d1, d2, supp, coef)
    Xn = oracle.densify(supp, c, d1.shape[1], d2.shape[1])
    R = Y - np.einsum("pi,kij,qj->kpq", n1d, Xn, n2d)
    if side == 1:
        grad = np.einsum("kpq,kij,qj->pi", R, Xn, n2d)
        scale = np.abs(np.einsum("kpq,kij,qj->pi", Y, Xn, n2d)).max()
    else:
        grad = np.einsum("kpq,kij,pi->qj", R, Xn, n1d)
        scale = np.abs(np.einsum("kpq,kij,pi->qj", Y, Xn, n1d)).max()
    assert np.abs(grad).max() <= 1e-11 * scale
    # objective never increases across a dictionary update (Sec. III)
    assert objective(Y, n1d, n2d, supp, c) <= objective(Y, d1, d2, supp, coef) * (1 + 1e-12)


def test_mod_special_case(rng):
    """With D2 = I the D1 update is MOD: D1 = Y X^T (X X^T)^{-1} on the concatenated data."""
    m1, m2, n1 = 6, 4, 10
    d1 = rand_dicts(rng, m1, m2, n1, m2)[0]
    d2 = np.eye(m2)
    Y, _ = planted(rng, 200, d1, d2, 3, noise=0.1)
    supp, coef, _ = oracle.omp(Y, rand_dicts(rng, m1, m2, n1, m2)[0], d2, 3)
    X = oracle.densify(supp, coef, n1, m2)
    Xc, Yc = np.concatenate(list(X), axis=1), np.concatenate(list(Y), axis=1)
    mod = Yc @ Xc.T @ np.linalg.inv(Xc @ Xc.T)
    new_d1 = oracle.tmod_update(1, Y, d1, d2, supp, coef)[0]
    np.testing.assert_allclose(new_d1, mod / np.linalg.norm(mod, axis=0), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("side", [1, 2])
def test_planted_exact_recovery(rng, side):
    m1, m2, n1, n2, s = 6, 6, 8, 8, 3
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, X = planted(rng, 400, t1, t2, s, noise=0.0)
    supp = np.full((len(Y), s), -1, np.int32)
    coef = np.zeros((len(Y), s))
    for k in range(len(Y)):
        i, j = np.nonzero(X[k])
        supp[k, :len(i)] = i + n1 * j
        coef[k, :len(i)] = X[k][i, j]
    r1, r2 = rand_dicts(rng, m1, m2, n1, n2)
    if side == 1:
        d1, d2, c, _ = oracle.tmod_update(1, Y, r1, t2, supp, coef)
        np.testing.assert_allclose(d1, t1, atol=1e-10)
    else:
        d1, d2, c, _ = oracle.tmod_update(2, Y, t1, r2, supp, coef)
        np.testing.assert_allclose(d2, t2, atol=1e-10)
    np.testing.assert_allclose(c, coef, atol=1e-10)


def test_unused_atom_is_kept(rng):
    Y, d1, d2, supp, coef = setup(rng, n1=9)
    used_row = supp % 9
    drop = (used_row == 4)
    supp = np.where(drop, -1, supp).astype(np.int32)
    coef = np.where(drop, 0.0, coef)
    new_d1, _, c, w = oracle.tmod_update(1, Y, d1, d2, supp, coef)
    np.testing.assert_array_equal(new_d1[:, 4], d1[:, 4])
    assert w[4] == 1.0
    # the other atoms solve the reduced LS problem
    keep = [i for i in range(9) if i != 4]
    X = oracle.densify(supp, coef, 9, d2.shape[1])
    T = np.concatenate([X[k][keep] @ d2.T for k in range(len(Y))], axis=1)
    Ycat = np.concatenate(list(Y), axis=1)
    Dstar = np.linalg.lstsq(T.T, Ycat.T, rcond=None)[0].T
    np.testing.assert_allclose(new_d1[:, keep], Dstar / np.linalg.norm(Dstar, axis=0), rtol=1e-9, atol=1e-11)


def test_singular_system_leaves_dictionary_unchanged(rng):
    """Rows 0 and 1 of every X_k equal -> sum T T^T singular with a positive diagonal."""
    m1, m2, n1, n2 = 5, 5, 4, 4
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    N = 50
    supp = np.zeros((N, 2), np.int32)
    coef = np.zeros((N, 2))
    j = rng.integers(0, n2, N)
    supp[:, 0] = 0 + n1 * j
    supp[:, 1] = 1 + n1 * j
    coef[:, 0] = coef[:, 1] = rng.standard_normal(N)
    Y = rng.standard_normal((N, m1, m2))
    with pytest.raises(oracle.OracleError) as e:
        oracle.tmod_update(1, Y, d1, d2, supp, coef)
    assert e.value.status == -5


def test_shards_sum_to_same_result(rng):
    """Algorithm 1's partial sums are additive: p shards give the p = 1 result to rounding."""
    Y, d1, d2, supp, coef = setup(rng, N=333)
    for side in (1, 2):
        A1, B1 = oracle.tmod_sums(side, Y, d1, d2, supp, coef, p=1)
        for p in (2, 7):
            A, B = oracle.tmod_sums(side, Y, d1, d2, supp, coef, p=p)
            np.testing.assert_allclose(A, A1, rtol=1e-13, atol=1e-13 * np.abs(A1).max())
            np.testing.assert_allclose(B, B1, rtol=1e-13, atol=1e-13 * np.abs(B1).max())


def test_learn_equals_composed_steps_and_is_monotone(rng):
    """Algorithm 1: OMP, D1, OMP, D2 per iteration; each dictionary update lowers eq. (1)."""
    m1, m2, n1, n2, s, K = 8, 8, 12, 12, 4, 3
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 300, t1, t2, s, noise=0.1)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    out = oracle.learn(Y, d1, d2, s, K)
    rm = []
    for _ in range(K):
        supp, coef, res2 = oracle.omp(Y, d1, d2, s)
        rm.append(np.sqrt(res2.sum() / (len(Y) * m1 * m2)))
        before = objective(Y, d1, d2, supp, coef)
        d1, d2, coef, _ = oracle.tmod_update(1, Y, d1, d2, supp, coef)
        assert objective(Y, d1, d2, supp, coef) <= before * (1 + 1e-12)
        supp, coef, _ = oracle.omp(Y, d1, d2, s)
        before = objective(Y, d1, d2, supp, coef)
        d1, d2, coef, _ = oracle.tmod_update(2, Y, d1, d2, supp, coef)
        assert objective(Y, d1, d2, supp, coef) <= before * (1 + 1e-12)
    supp, coef, res2 = oracle.omp(Y, d1, d2, s)
    rm.append(np.sqrt(res2.sum() / (len(Y) * m1 * m2)))
    np.testing.assert_array_equal(out["D1"], d1)
    np.testing.assert_array_equal(out["D2"], d2)
    np.testing.assert_array_equal(out["supp"], supp)
    np.testing.assert_allclose(out["rmse"], np.array(rm), rtol=1e-14)
    assert out["rmse"][-1] < out["rmse"][0]


def test_learn_other_schedule_and_shards(rng):
    m1, m2, n1, n2, s, K = 6, 6, 9, 9, 3, 4
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 250, t1, t2, s, noise=0.05)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    a = oracle.learn(Y, d1, d2, s, K, schedule=1)
    # schedule 1: OMP, then D2, then D1 with the same (rescaled) codes
    e1, e2 = d1, d2
    for _ in range(K):
        supp, coef, _ = oracle.omp(Y, e1, e2, s)
        e1, e2, coef, _ = oracle.tmod_update(2, Y, e1, e2, supp, coef)
        e1, e2, coef, _ = oracle.tmod_update(1, Y, e1, e2, supp, coef)
    np.testing.assert_array_equal(a["D1"], e1)
    np.testing.assert_array_equal(a["D2"], e2)
    b = oracle.learn(Y, d1, d2, s, K, schedule=0, p=1)
    c = oracle.learn(Y, d1, d2, s, K, schedule=0, p=5)
    np.testing.assert_allclose(c["rmse"], b["rmse"], rtol=1e-12)
    np.testing.assert_allclose(c["D1"], b["D1"], atol=1e-12)
