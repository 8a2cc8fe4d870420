"""Pins of the oracle's orthonormal variant (Remark 1): hard-thresholded codes and the
orthogonal Procrustes dictionary updates, against what the mathematics fixes.

* Codes: the s largest-magnitude entries of D1^T Y D2 computed by numpy (stable order, ties to
  the smaller atom); for orthonormal dictionaries 2D-OMP selects exactly these (Remark 1), so
  the oracle's own 2D-OMP must agree; residual energy = ||Y||^2 - sum of the kept C^2.
* Update: the polar factor U V^T of the B sum computed here by numpy (dense products and
  numpy's SVD); the result is orthonormal; it minimises the objective among orthonormal
  dictionaries (no random orthogonal matrix, and not the old dictionary, does better); the
  formula as printed in Remark 1 (the B sum multiplied by sum X X^T before the SVD) is a
  different matrix on these instances and does worse.
* Learning: each half-step is an exact minimiser, so the RMSE trace never increases; the call
  equals the composition of the oracle's code and update calls.
"""
import numpy as np
import pytest

import oracle


def orth(rng, m):
    q, r = np.linalg.qr(rng.standard_normal((m, m)))
    return q * np.sign(np.diag(r))


def planted_ortho(rng, N, m1, m2, s, noise):
    D1, D2 = orth(rng, m1), orth(rng, m2)
    Y = np.zeros((N, m1, m2))
    for k in range(N):
        X = np.zeros((m1, m2))
        a = rng.choice(m1 * m2, s, replace=False)
        X[a % m1, a // m1] = rng.standard_normal(s)
        Y[k] = D1 @ X @ D2.T + noise * rng.standard_normal((m1, m2))
    return Y, D1, D2


def objective(Y, D1, D2, supp, coef):
    X = oracle.densify(supp, coef, D1.shape[1], D2.shape[1])
    return float(np.sum((Y - np.einsum("pi,kij,qj->kpq", D1, X, D2)) ** 2))


@pytest.mark.parametrize("m1,m2,s", [(8, 8, 8), (6, 5, 4), (4, 4, 16)])
def test_ortho_code_is_hard_thresholding(m1, m2, s, rng):
    Y = rng.standard_normal((300, m1, m2))
    D1, D2 = orth(rng, m1), orth(rng, m2)
    supp, coef, res2 = oracle.ortho_code(Y, D1, D2, s, p=3)
    C = np.stack([(D1.T @ y @ D2).flatten("F") for y in Y])
    top = np.argsort(-np.abs(C), axis=1, kind="stable")[:, :s]
    np.testing.assert_array_equal(supp, top)
    np.testing.assert_allclose(coef, np.take_along_axis(C, top, 1), rtol=1e-13, atol=1e-14)
    closed = np.sum(Y ** 2, axis=(1, 2)) - np.sum(coef ** 2, axis=1)
    np.testing.assert_allclose(res2, closed, rtol=1e-10, atol=1e-12)
    so, co, _ = oracle.omp(Y, D1, D2, s)
    np.testing.assert_array_equal(supp, so)
    np.testing.assert_allclose(coef, co, rtol=1e-10, atol=1e-12)


def test_ortho_code_ties_to_smaller_atom():
    D1, D2 = np.eye(3), np.eye(3)
    Y = np.array([[[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, 1.0]]])  # three equal magnitudes
    supp, coef, _ = oracle.ortho_code(Y, D1, D2, 2)
    np.testing.assert_array_equal(supp[0], [0, 4])  # atoms i + 3 j of (0,0), (1,1)
    np.testing.assert_array_equal(coef[0], [1.0, -1.0])


def _polar(B):
    u, _, vt = np.linalg.svd(B)
    return u @ vt


@pytest.mark.parametrize("side", [1, 2])
@pytest.mark.parametrize("m1,m2", [(8, 8), (6, 4)])
def test_procrustes_update_is_polar_factor_and_optimal(side, m1, m2, rng):
    s, N = 5, 400
    Y, T1, T2 = planted_ortho(rng, N, m1, m2, s, 0.1)
    D1, D2 = orth(rng, m1), orth(rng, m2)
    supp, coef, _ = oracle.ortho_code(Y, D1, D2, s)
    X = oracle.densify(supp, coef, m1, m2)
    if side == 1:
        B = np.einsum("kpq,qj,kij->pi", Y, D2, X)   # sum_k Y_k D2 X_k^T
        G = np.einsum("kij,klj->il", X, X)          # sum_k X_k X_k^T
    else:
        B = np.einsum("kpq,pi,kij->qj", Y, D1, X)   # sum_k Y_k^T D1 X_k
        G = np.einsum("kij,kil->jl", X, X)          # sum_k X_k^T X_k
    e1, e2 = oracle.procrustes_update(side, Y, D1, D2, supp, coef)
    new, old = (e1, D1) if side == 1 else (e2, D2)
    np.testing.assert_array_equal(e2 if side == 1 else e1, D2 if side == 1 else D1)
    np.testing.assert_allclose(new, _polar(B), atol=1e-10)
    np.testing.assert_allclose(new.T @ new, np.eye(new.shape[0]), atol=1e-12)
    f_new = objective(Y, e1, e2, supp, coef)
    f_old = objective(Y, D1, D2, supp, coef)
    assert f_new <= f_old * (1 + 1e-12)
    for _ in range(20):
        q = orth(rng, new.shape[0])
        a1, a2 = (q, D2) if side == 1 else (D1, q)
        assert f_new <= objective(Y, a1, a2, supp, coef) * (1 + 1e-12)
    # the update as printed (SVD of the B sum times the X Gram sum) is another matrix, and worse
    printed = _polar(B @ G)
    assert np.abs(printed - new).max() > 1e-3
    a1, a2 = (printed, D2) if side == 1 else (D1, printed)
    assert objective(Y, a1, a2, supp, coef) > f_new * (1 + 1e-9)


def test_procrustes_recovers_planted_dictionary_noiseless(rng):
    Y, T1, T2 = planted_ortho(rng, 500, 8, 8, 6, 0.0)
    supp, coef, _ = oracle.ortho_code(Y, T1, T2, 6)
    e1, _ = oracle.procrustes_update(1, Y, orth(rng, 8), T2, supp, coef)
    np.testing.assert_allclose(e1, T1, atol=1e-10)


def test_procrustes_rank_deficient_keeps_dictionary(rng):
    D1, D2 = orth(rng, 4), orth(rng, 4)
    Y = rng.standard_normal((50, 4, 4))
    supp = np.zeros((50, 1), np.int32)          # every code uses atom (0, 0) only: B has rank 1
    coef = rng.standard_normal((50, 1))
    with pytest.raises(oracle.OracleError) as e:
        oracle.procrustes_update(1, Y, D1, D2, supp, coef)
    assert e.value.status == -5


def test_learn_ortho_monotone_and_composed(rng):
    Y, T1, T2 = planted_ortho(rng, 600, 8, 8, 8, 0.05)
    D1, D2 = orth(rng, 8), orth(rng, 8)
    K = 6
    ref = oracle.learn_ortho(Y, D1, D2, 8, K, p=4)
    assert np.all(np.diff(ref["rmse"]) <= 1e-12)
    assert ref["rmse"][-1] < 0.8 * ref["rmse"][0]
    e1, e2 = D1, D2
    for _ in range(K):
        for side in (1, 2):
            supp, coef, _ = oracle.ortho_code(Y, e1, e2, 8)
            e1, e2 = oracle.procrustes_update(side, Y, e1, e2, supp, coef)
    np.testing.assert_allclose(ref["D1"], e1, atol=1e-12)
    np.testing.assert_allclose(ref["D2"], e2, atol=1e-12)
