"""Pins of the oracle's 2D-OMP against what the paper and the mathematics fix.

None of these re-types the oracle's own code: each check uses an independent
route (explicit Kronecker dictionary with numpy least squares, closed forms for
orthonormal dictionaries, exhaustive subset search, invariants).
"""
import itertools

import numpy as np
import pytest

import oracle
from tests.conftest import planted, rand_dicts


def kron_dict(d1, d2):
    # column a = i + n1*j of D2 (x) D1 is vec(d1_i d2_j^T) under column-major vec (Sec. I)
    return np.kron(d2, d1)


def vec(M):
    return M.reshape(M.shape[:-2] + (-1,), order="F") if M.ndim == 2 else np.stack([m.flatten("F") for m in M])


def omp_1d_lstsq(D, y, s):
    """Textbook OMP on an explicit dictionary, numpy lstsq re-fit at every step."""
    S, r = [], y.copy()
    x = np.zeros(0)
    for _ in range(s):
        corr = np.abs(D.T @ r)
        corr[S] = -1.0
        a = int(np.argmax(corr))  # first maximum = smallest index on ties
        if corr[a] <= oracle.STOP_REL * np.linalg.norm(y):
            break
        S.append(a)
        x = np.linalg.lstsq(D[:, S], y, rcond=None)[0]
        r = y - D[:, S] @ x
    return S, x, float(r @ r)


def residual_via_kron(Y, supp, coef, d1, d2):
    X = oracle.densify(supp, coef, d1.shape[1], d2.shape[1])
    K = kron_dict(d1, d2)
    return np.array([np.sum((vec(Y[k]) - K @ vec(X[k])) ** 2) for k in range(len(Y))])


@pytest.mark.parametrize("shape", [(8, 8, 12, 12, 4), (4, 6, 5, 7, 3), (6, 4, 9, 5, 5), (3, 3, 4, 4, 2)])
def test_kronecker_identity_and_res2(rng, shape):
    """||Y - D1 X D2^T||_F == ||vec Y - (D2 (x) D1) vec X||_2 (Sec. I), on the oracle's output."""
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 20, d1, d2, s, noise=0.1)
    supp, coef, res2 = oracle.omp(Y, d1, d2, s)
    X = oracle.densify(supp, coef, n1, n2)
    two_d = np.array([np.sum((Y[k] - d1 @ X[k] @ d2.T) ** 2) for k in range(len(Y))])
    np.testing.assert_allclose(residual_via_kron(Y, supp, coef, d1, d2), two_d, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(res2, two_d, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("mode", ["separable", "kronecker"])
@pytest.mark.parametrize("shape", [(8, 8, 12, 12, 4), (4, 6, 5, 7, 3), (5, 5, 10, 8, 6)])
def test_2d_omp_equals_1d_omp(rng, mode, shape):
    """2D-OMP equals 1D OMP on D2 (x) D1 (Sec. II): identical supports, coefficients to 1e-10."""
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 40, d1, d2, s, noise=0.05)
    supp, coef, res2 = oracle.omp(Y, d1, d2, s, mode=mode)
    K = kron_dict(d1, d2)
    for k in range(len(Y)):
        S, x, r2 = omp_1d_lstsq(K, vec(Y[k]), s)
        assert list(supp[k, :len(S)]) == S
        assert np.all(supp[k, len(S):] == -1)
        np.testing.assert_allclose(coef[k, :len(S)], x, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(res2[k], r2, rtol=1e-9, atol=1e-13)


def test_modes_agree_exactly_on_supports(rng):
    d1, d2 = rand_dicts(rng, 6, 7, 9, 11)
    Y, _ = planted(rng, 60, d1, d2, 5, noise=0.1)
    a = oracle.omp(Y, d1, d2, 5, mode="separable")
    b = oracle.omp(Y, d1, d2, 5, mode="kronecker")
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10, atol=1e-12)


def test_residual_orthogonal_to_chosen_atoms(rng):
    """Least-squares optimality on the support: D_S^T r = 0."""
    d1, d2 = rand_dicts(rng, 8, 8, 16, 16)
    Y, _ = planted(rng, 50, d1, d2, 8, noise=0.1)
    supp, coef, _ = oracle.omp(Y, d1, d2, 8)
    X = oracle.densify(supp, coef, 16, 16)
    for k in range(len(Y)):
        R = Y[k] - d1 @ X[k] @ d2.T
        corr = d1.T @ R @ d2
        a = supp[k][supp[k] >= 0]
        assert np.max(np.abs(corr[a % 16, a // 16])) <= 1e-12 * np.linalg.norm(Y[k])


def test_residual_never_increases_and_supports_nest(rng):
    d1, d2 = rand_dicts(rng, 8, 8, 16, 16)
    Y, _ = planted(rng, 30, d1, d2, 8, noise=0.2)
    prev = np.sum(Y ** 2, axis=(1, 2))
    prev_supp = None
    for s in range(1, 9):
        supp, _, res2 = oracle.omp(Y, d1, d2, s)
        assert np.all(res2 <= prev * (1 + 1e-12))
        if prev_supp is not None:
            np.testing.assert_array_equal(supp[:, :s - 1], prev_supp)
        prev, prev_supp = res2, supp


def test_orthonormal_case_is_hard_thresholding(rng):
    """Remark 1: with orthogonal D1, D2 the s-sparse code is T_s(D1^T Y D2)."""
    m, s = 8, 6
    d1 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    d2 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    Y = rng.standard_normal((25, m, m))
    supp, coef, res2 = oracle.omp(Y, d1, d2, s)
    for k in range(len(Y)):
        C = (d1.T @ Y[k] @ d2).flatten("F")  # index a = i + n1*j
        top = np.argsort(-np.abs(C), kind="stable")[:s]
        assert list(supp[k]) == list(top)
        np.testing.assert_allclose(coef[k], C[top], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(res2[k], np.sum(Y[k] ** 2) - np.sum(C[top] ** 2), rtol=1e-10)


def test_exhaustive_best_subset_bound(rng):
    """OMP's residual is never below the best s-subset residual (brute force over C(A, s))."""
    m1, m2, n1, n2, s = 2, 3, 3, 3, 2
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    K = kron_dict(d1, d2)
    Y = rng.standard_normal((15, m1, m2))
    _, _, res2 = oracle.omp(Y, d1, d2, s)
    for k in range(len(Y)):
        y = vec(Y[k])
        best = min(np.sum((y - K[:, list(S)] @ np.linalg.lstsq(K[:, list(S)], y, rcond=None)[0]) ** 2)
                   for S in itertools.combinations(range(n1 * n2), s))
        assert res2[k] >= best * (1 - 1e-12) - 1e-15


def test_exhaustive_best_subset_equality_orthonormal_planted(rng):
    m, s = 3, 2
    d1 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    d2 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    K = kron_dict(d1, d2)
    Y, _ = planted(rng, 10, d1, d2, s, noise=0.0)
    supp, _, res2 = oracle.omp(Y, d1, d2, s)
    for k in range(len(Y)):
        y = vec(Y[k])
        best = min(np.sum((y - K[:, list(S)] @ np.linalg.lstsq(K[:, list(S)], y, rcond=None)[0]) ** 2)
                   for S in itertools.combinations(range(m * m), s))
        assert abs(res2[k] - best) <= 1e-20 + 1e-12 * np.sum(y ** 2)


def test_scale_and_sign_invariance(rng):
    d1, d2 = rand_dicts(rng, 8, 8, 16, 16)
    Y, _ = planted(rng, 20, d1, d2, 8, noise=0.1)
    a = oracle.omp(Y, d1, d2, 8)
    for c in (-3.0, 0.25):
        b = oracle.omp(c * Y, d1, d2, 8)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_allclose(b[1], c * a[1], rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(b[2], c * c * a[2], rtol=1e-10)


def test_zero_signal_gives_empty_code(rng):
    d1, d2 = rand_dicts(rng, 8, 8, 12, 12)
    Y = np.zeros((3, 8, 8))
    supp, coef, res2 = oracle.omp(Y, d1, d2, 4)
    assert np.all(supp == -1) and np.all(coef == 0) and np.all(res2 == 0)


def test_exactly_sparse_stops_early(rng):
    """A noiseless signal built from 2 atoms of an orthonormal pair needs only 2 steps."""
    m = 6
    d1 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    d2 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    Y, X = planted(rng, 5, d1, d2, 2, noise=0.0)
    supp, coef, res2 = oracle.omp(Y, d1, d2, 5)
    assert np.all(supp[:, 2:] == -1)
    assert np.all(supp[:, :2] >= 0)
    assert np.all(res2 <= 1e-26 * np.sum(Y ** 2, axis=(1, 2)) + 1e-30)


def test_duplicate_atoms_stop_on_dependence(rng):
    """Exact duplicate atoms: the Gram pivot of the duplicate is 0, so OMP stops (dep_eps rule)."""
    d1, d2 = rand_dicts(rng, 5, 5, 4, 4)
    d1[:, 1] = d1[:, 0]
    Y = 2.0 * np.outer(d1[:, 0], d2[:, 0])[None]
    supp, _, _ = oracle.omp(Y, d1, d2, 3, stop_rel=0.0)
    # atom 0 first; its duplicate (index 1) has the next largest |corr| only at rounding level,
    # and whichever atom comes next, a duplicate of a chosen atom is never accepted
    assert supp[0, 0] == 0
    chosen = [a for a in supp[0] if a >= 0]
    assert 1 not in chosen


def test_shards_do_not_change_codes(rng):
    d1, d2 = rand_dicts(rng, 8, 8, 12, 12)
    Y, _ = planted(rng, 101, d1, d2, 4, noise=0.1)
    a = oracle.omp(Y, d1, d2, 4, p=1)
    b = oracle.omp(Y, d1, d2, 4, p=7)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


# ---------------------------------------------------------------- error-driven stop (Sec. IV)

def test_error_driven_orthonormal_closed_form(rng):
    """Orthogonal D1, D2 (Remark 1): the greedy order is decreasing |D1^T Y D2|, so the
    error-driven code has the smallest t whose tail energy sum_{u>t} C_(u)^2 is <= eps^2
    (capped at s), on the first t entries of that order."""
    m, s = 8, 32  # cap m^2 / 2, as in the denoising runs
    d1 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    d2 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    Y = rng.standard_normal((40, m, m)) * rng.uniform(0.2, 2.0, (40, 1, 1))
    sigma = 0.5
    err2 = (1.15 * sigma * m) ** 2  # eps = 1.15 sigma sqrt(m1 m2)
    supp, coef, res2 = oracle.omp(Y, d1, d2, s, err2=err2)
    nnz_seen = set()
    for k in range(len(Y)):
        C = (d1.T @ Y[k] @ d2).flatten("F")
        order = np.argsort(-np.abs(C), kind="stable")
        tail = np.sum(Y[k] ** 2) - np.concatenate([[0.0], np.cumsum(C[order] ** 2)])  # energy after t atoms
        t = min(int(np.argmax(tail <= err2)) if np.any(tail <= err2) else s, s)
        nnz = int(np.sum(supp[k] >= 0))
        nnz_seen.add(nnz)
        assert nnz == t, (k, nnz, t)
        assert list(supp[k, :t]) == list(order[:t])
        np.testing.assert_allclose(coef[k, :t], C[order[:t]], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(res2[k], tail[t], rtol=1e-9, atol=1e-12)
    assert len(nnz_seen) > 3  # the stop really varies per signal


def test_error_driven_equals_kronecker_omp_and_is_minimal(rng):
    """General dictionaries: the separable error-driven 2D-OMP equals textbook 1D OMP with the
    same stop on the explicit Kronecker dictionary; a signal that stopped before the cap is
    within eps^2, and the same greedy run one atom shorter is not."""
    d1, d2 = rand_dicts(rng, 6, 7, 9, 11)
    Y, _ = planted(rng, 80, d1, d2, 8, noise=0.3)
    s = 21
    err2 = float(np.median(np.sum(Y ** 2, axis=(1, 2)))) * 0.05
    a = oracle.omp(Y, d1, d2, s, err2=err2)
    b = oracle.omp(Y, d1, d2, s, mode="kronecker", err2=err2)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_allclose(a[1], b[1], rtol=1e-9, atol=1e-11)
    nnz = np.sum(a[0] >= 0, axis=1)
    assert len(set(nnz.tolist())) > 2
    for t in sorted(set(nnz.tolist())):
        ks = np.nonzero(nnz == t)[0]
        if t < s:
            assert np.all(a[2][ks] <= err2)
        if t > 0:
            shorter = oracle.omp(Y[ks], d1, d2, t - 1)
            assert np.all(shorter[2] > err2)
            np.testing.assert_array_equal(shorter[0][:, :t - 1], a[0][ks, :t - 1])


def test_error_driven_off_is_plain_omp(rng):
    d1, d2 = rand_dicts(rng, 5, 6, 8, 9)
    Y, _ = planted(rng, 30, d1, d2, 4, noise=0.2)
    a = oracle.omp(Y, d1, d2, 6)
    b = oracle.omp(Y, d1, d2, 6, err2=0.0)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
