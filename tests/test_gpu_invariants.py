"""Invariants of the GPU outputs (no oracle needed) and robustness cases.

* codes: supports distinct and inside the atom range, -1 only in trailing slots with a
  zero coefficient; the reported res2 equals the explicit residual of the returned codes
  (FP64 on the host); the residual is orthogonal to the chosen atoms (least squares);
* dictionary updates leave unit-norm atoms;
* planted exact ties (two atoms with equal coefficients, so their first correlations are
  equal in exact arithmetic): every kernel picks that pair and reaches a zero residual;
* resuming: K = 10 iterations equal K = 5 followed by 5 more, bit for bit in the
  dictionaries and codes.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_03800_amd import api
from tests.conftest import planted, rand_dicts

pytestmark = pytest.mark.gpu

# (shape, dtype, kernel option): the matrix-core kernel (auto at this shape), a VALU
# multi-signal shape, the standalone-sums kernels (FP32 one-wave on matrix-core tiles:
# exact and padded in one dimension; FP32 quadrants: padded and exact; FP64 one-wave on
# the vector ALUs), the generic kernel in both precisions
KERNELS = [((8, 8, 16, 16, 8), torch.float32, 0), ((12, 12, 20, 20, 10), torch.float32, 2),
           ((16, 16, 32, 32, 16), torch.float32, 3), ((12, 12, 20, 20, 10), torch.float32, 3),
           ((12, 12, 24, 24, 12), torch.float32, 3),
           ((32, 24, 48, 36, 20), torch.float32, 3), ((5, 9, 11, 6, 7), torch.float32, 1),
           ((8, 8, 12, 12, 4), torch.float64, 1), ((32, 24, 48, 36, 20), torch.float64, 3)]
ids = ["x".join(map(str, k[0])) + "-" + ("f32" if k[1] == torch.float32 else "f64") + "-k%d" % k[2] for k in KERNELS]


def explicit(Y, d1, d2, supp, coef):
    """Residuals of the returned codes, in FP64."""
    n1 = d1.shape[1]
    R = Y.astype(np.float64).copy()
    for k in range(len(Y)):
        for a, x in zip(supp[k], coef[k]):
            if a >= 0:
                R[k] -= x * np.outer(d1[:, a % n1], d2[:, a // n1])
    return R


@pytest.mark.parametrize("shape,dtype,kernel", KERNELS, ids=ids)
def test_code_invariants(shape, dtype, kernel, rng):
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 300, d1, d2, s, noise=0.05)
    Y[7] = 0.0
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.sparse_code(pr, kernel=kernel)
    torch.cuda.synchronize()
    supp, coef, res2 = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
    for k in range(len(Y)):
        used = supp[k] >= 0
        nu = int(used.sum())
        assert np.all(used[:nu]) and not np.any(used[nu:]), supp[k]
        assert np.all(coef[k][~used] == 0)
        a = supp[k][used]
        assert len(set(a.tolist())) == nu and np.all(a < n1 * n2)
    R = explicit(Y, d1, d2, supp, coef)
    r2 = np.einsum("kij,kij->k", R, R)
    ynorm2 = np.einsum("kij,kij->k", Y, Y)
    tol = 1e-9 if dtype == torch.float64 else 1e-4
    assert np.all(np.abs(res2 - r2) <= tol * ynorm2 + 1e-30)
    # least squares: the residual is orthogonal to every chosen atom
    worst = 0.0
    for k in range(len(Y)):
        for a in supp[k][supp[k] >= 0]:
            g = d1[:, a % n1] @ R[k] @ d2[:, a // n1]
            worst = max(worst, abs(g) / max(np.sqrt(ynorm2[k]), 1e-300))
    assert worst <= (1e-10 if dtype == torch.float64 else 2e-4), worst
    assert np.all(supp[7] == -1) and res2[7] == 0


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_learned_atoms_unit_norm(dtype, rng):
    m1, m2, n1, n2, s = 8, 8, 16, 16, 6
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 3000, t1, t2, s, noise=0.05)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.learn(pr, 3)
    np.testing.assert_allclose(np.linalg.norm(pr.d1(), axis=0), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(pr.d2(), axis=0), 1.0, atol=1e-12)


@pytest.mark.parametrize("shape,dtype,kernel", KERNELS, ids=ids)
def test_planted_exact_ties(shape, dtype, kernel, rng):
    """Y = atom_a + atom_b: the two correlations are equal in exact arithmetic.  Kept are the
    pairs the FP64 oracle codes with exactly {a, b} and for which either first choice leads to
    the other atom (so the tie-break cannot change the path); every kernel must choose the same
    pair, in either order, and stop on a zero residual."""
    m1, m2, n1, n2, s = shape
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    A = n1 * n2
    cand = 400
    Y = np.zeros((cand, m1, m2))
    pairs = []
    for k in range(cand):
        a, b = rng.choice(A, 2, replace=False)
        pairs.append({int(a), int(b)})
        Y[k] = np.outer(d1[:, a % n1], d2[:, a // n1]) + np.outer(d1[:, b % n1], d2[:, b // n1])
    so, _, _ = oracle.omp(Y, d1, d2, s)

    def next_is_other(k, first, other):
        # after coding Y with `first` alone (unit-norm atoms), `other` must be the clear next pick
        atom = np.outer(d1[:, first % n1], d2[:, first // n1])
        r = Y[k] - np.sum(atom * Y[k]) * atom
        c = np.abs(d1.T @ r @ d2).flatten(order="F")
        c[first] = -1.0
        top = np.argsort(c)[::-1]
        return top[0] == other and c[top[0]] > 1.01 * c[top[1]]

    keep = [k for k in range(cand) if set(so[k][:2].tolist()) == pairs[k] and np.all(so[k][2:] == -1)
            and next_is_other(k, *sorted(pairs[k])) and next_is_other(k, *sorted(pairs[k])[::-1])]
    assert len(keep) >= 20
    Y = Y[keep]
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.sparse_code(pr, kernel=kernel)
    torch.cuda.synchronize()
    supp, res2 = pr.supp.cpu().numpy(), pr.res2.cpu().double().numpy()
    ynorm2 = np.einsum("kij,kij->k", Y, Y)
    tol = 1e-20 if dtype == torch.float64 else 1e-9
    for i, k in enumerate(keep):
        assert set(supp[i][:2].tolist()) == pairs[k], (k, supp[i], pairs[k])
        assert np.all(supp[i][2:] == -1) and res2[i] <= tol * ynorm2[i] + 1e-30


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_resume_equals_one_run(dtype, rng):
    m1, m2, n1, n2, s = 8, 8, 16, 16, 8
    t1, t2 = rand_dicts(rng, m1, m2, n1, n2)
    Y, _ = planted(rng, 4000, t1, t2, s, noise=0.05)
    d1, d2 = rand_dicts(rng, m1, m2, n1, n2)
    one = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    tr = api.learn(one, 10)[0]
    two = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    ta = api.learn(two, 5)[0]
    tb = api.learn(two, 5)[0]
    np.testing.assert_array_equal(one.d1(), two.d1())
    np.testing.assert_array_equal(one.d2(), two.d2())
    assert torch.equal(one.supp, two.supp) and torch.equal(one.coef, two.coef)
    np.testing.assert_allclose(np.concatenate([ta, tb[1:]]), tr, rtol=1e-12)
