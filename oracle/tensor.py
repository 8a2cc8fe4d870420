"""FP64 CPU oracle of the n-dimensional generalisation (Remark 3) of the method: signals are
tensors Y_k of size m_1 x ... x m_n, the dictionary is separable over the modes,
Y_k = X_k x_1 D_1 x_2 D_2 ... x_n D_n with D_d of size m_d x n_d, and each dictionary is updated by
the mode-d least squares of Remark 3: Y_(d) = D_d X_(d) T^T with T the Kronecker product of the
other modes' dictionaries, which is Corollary 1 with T fixed.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark may call it; the GPU
library never does.  Plain numpy, by the definitions, no blocking or reordering:

* Atom index a = i_1 + n_1 (i_2 + n_2 (i_3 + ...)) (first mode fastest), the column of the explicit
  Kronecker dictionary K = D_n (x) ... (x) D_1 acting on vec(Y_k) taken first index fastest.
* tensor_omp: OMP on K (Sec. II: 2D-OMP is OMP on the Kronecker dictionary; the same holds per
  mode here): every step takes the correlations K^T r of the explicit residual, masks chosen
  atoms, picks the largest |corr| (ties: smaller atom), checks the new Gram pivot, refactors the
  support's Gram matrix K_S^T K_S from scratch (plain Cholesky) and solves the normal equations.
  Stops as the two-dimensional oracle does: max |corr| <= stop_rel ||Y_k||, pivot <= dep_eps G_aa,
  or (err2 > 0) residual energy <= err2 before a step.
* tensor_sums / tensor_update: for mode d, with W_k = X_k x_e D_e over every other mode e,
  A = sum_k W_k(d) W_k(d)^T and B = sum_k Y_k(d) W_k(d)^T; the new D_d solves D_d A = B on the
  atoms some code uses (Cholesky; a pivot <= 1e-12 of its diagonal entry is singular and leaves
  the dictionary unchanged), its columns are normalised (w_i = the norm) and every coefficient of
  an atom with mode-d index i is multiplied by w_i, as in Corollary 1 / Result 1.
* tensor_learn: Algorithm 1 with one sweep per mode: for d = 1..n, sparse coding then the mode-d
  update; the RMSE of each iteration's first sweep, and of a final sweep, is recorded.

Pinned by tests/test_oracle_tensor.py (two modes against the separate two-dimensional oracle in C,
the atom convention against explicit outer products, orthonormal dictionaries against hard
thresholding, the update against numpy lstsq on the stacked mode-d system).
"""
from __future__ import annotations

import numpy as np

STOP_REL = 1e-14
DEP_EPS = 1e-10
SPD_REL_TOL = 1e-12


class TensorOracleError(RuntimeError):
    pass


def kron_dictionary(Ds):
    """K = D_n (x) ... (x) D_1 (prod m_d x prod n_d)."""
    K = np.asarray(Ds[0], np.float64)
    for D in Ds[1:]:
        K = np.kron(np.asarray(D, np.float64), K)
    return K


def vec(T):
    """vec of a tensor, first index fastest."""
    return np.asarray(T, np.float64).flatten(order="F")


def mode_product(T, M, d):
    """T x_d M: mode d of T (size I_d) is replaced by M's rows (M is J x I_d)."""
    return np.moveaxis(np.tensordot(M, T, axes=(1, d)), 0, d)


def matricize(T, d):
    """Mode-d matricisation T_(d): rows = mode d, columns = the other modes, lowest first."""
    return np.moveaxis(T, d, 0).reshape(T.shape[d], -1, order="F")


def atom_multi_index(a, ns):
    idx = []
    for n in ns:
        idx.append(a % n)
        a //= n
    return idx


def _cholesky(G, rel_tol):
    """Plain Cholesky of a small SPD matrix; returns (L, pivots, first failing row or -1)."""
    n = G.shape[0]
    L = np.zeros_like(G)
    piv = np.zeros(n)
    for k in range(n):
        d = G[k, k] - np.dot(L[k, :k], L[k, :k])
        piv[k] = d
        if not (d > rel_tol * G[k, k]):
            return L, piv, k
        L[k, k] = np.sqrt(d)
        for i in range(k + 1, n):
            L[i, k] = (G[i, k] - np.dot(L[i, :k], L[k, :k])) / L[k, k]
    return L, piv, -1


def _chol_solve(L, b):
    n = len(b)
    z = np.zeros(n)
    for i in range(n):
        z[i] = (b[i] - np.dot(L[i, :i], z[:i])) / L[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (z[i] - np.dot(L[i + 1:, i], x[i + 1:])) / L[i, i]
    return x


def tensor_omp(Y, Ds, s, err2=0.0, stop_rel=STOP_REL, dep_eps=DEP_EPS):
    """Sparse codes of every signal.  Y: (N, m_1, ..., m_n).  Returns (supp (N, s) int32,
    coef (N, s), res2 (N,)); unused slots are -1 / 0."""
    Y = np.asarray(Y, np.float64)
    N = Y.shape[0]
    K = kron_dictionary(Ds)
    A = K.shape[1]
    supp = np.full((N, s), -1, np.int32)
    coef = np.zeros((N, s))
    res2 = np.zeros(N)
    for k in range(N):
        y = vec(Y[k])
        ynorm = np.linalg.norm(y)
        r = y.copy()
        S = []
        x = np.zeros(0)
        sel = np.zeros(A, bool)
        for _ in range(s):
            if err2 > 0.0 and np.dot(r, r) <= err2:
                break
            c = np.abs(K.T @ r)
            c[sel] = -1.0
            a = int(np.argmax(c))  # first maximum: ties go to the smaller atom
            if not (c[a] > stop_rel * ynorm):
                break
            T = S + [a]
            G = K[:, T].T @ K[:, T]
            L, piv, fail = _cholesky(G, 0.0)
            if fail >= 0 or piv[-1] <= dep_eps * G[-1, -1]:
                break
            S = T
            sel[a] = True
            x = _chol_solve(L, K[:, S].T @ y)
            r = y - K[:, S] @ x
        supp[k, :len(S)] = S
        coef[k, :len(S)] = x
        res2[k] = np.dot(r, r)
    return supp, coef, res2


def densify(supp, coef, ns):
    """Dense codes (N, n_1, ..., n_n) from (supp, coef)."""
    N, s = supp.shape
    X = np.zeros((N, int(np.prod(ns))))
    for k in range(N):
        for t in range(s):
            if supp[k, t] >= 0:
                X[k, supp[k, t]] += coef[k, t]
    return X.reshape((N,) + tuple(ns), order="F")


def reconstruct(supp, coef, Ds):
    """D-model of every signal: X_k x_1 D_1 ... x_n D_n, (N, m_1, ..., m_n)."""
    X = densify(supp, coef, [D.shape[1] for D in Ds])
    out = []
    for k in range(X.shape[0]):
        T = X[k]
        for d, D in enumerate(Ds):
            T = mode_product(T, D, d)
        out.append(T)
    return np.array(out).reshape((X.shape[0],) + tuple(D.shape[0] for D in Ds))


def tensor_sums(mode, Y, Ds, supp, coef):
    """(A, B) of the mode-`mode` update (mode counted from 1)."""
    Y = np.asarray(Y, np.float64)
    d = mode - 1
    X = densify(supp, coef, [D.shape[1] for D in Ds])
    na, mb = Ds[d].shape[1], Ds[d].shape[0]
    A = np.zeros((na, na))
    B = np.zeros((mb, na))
    for k in range(Y.shape[0]):
        W = X[k]
        for e, D in enumerate(Ds):
            if e != d:
                W = mode_product(W, D, e)
        Wd = matricize(W, d)
        A += Wd @ Wd.T
        B += matricize(Y[k], d) @ Wd.T
    return A, B


def tensor_update(mode, Y, Ds, supp, coef):
    """Remark 3's mode-`mode` dictionary update from the codes.  Returns (new list of dictionaries,
    rescaled coef, w)."""
    d = mode - 1
    A, B = tensor_sums(mode, Y, Ds, supp, coef)
    D = np.array(Ds[d], np.float64, copy=True)
    na = D.shape[1]
    U = [i for i in range(na) if A[i, i] > 0.0]
    w = np.ones(na)
    if U:
        L, _, fail = _cholesky(A[np.ix_(U, U)], SPD_REL_TOL)
        if fail >= 0:
            raise TensorOracleError("the mode-%d Gram sum is not positive definite" % mode)
        for p in range(D.shape[0]):
            row = _chol_solve(L, B[p, U])
            D[p, U] = row
        for i in U:
            nrm = np.linalg.norm(D[:, i])
            if nrm > 0.0:
                w[i] = nrm
                D[:, i] /= nrm
    out = [np.array(E, np.float64, copy=True) for E in Ds]
    out[d] = D
    c = np.array(coef, np.float64, copy=True)
    ns = [E.shape[1] for E in Ds]
    for k in range(c.shape[0]):
        for t in range(c.shape[1]):
            if supp[k, t] >= 0:
                c[k, t] *= w[atom_multi_index(int(supp[k, t]), ns)[d]]
    return out, c, w


def rmse(res2, signal_size):
    return float(np.sqrt(np.sum(res2) / (len(res2) * signal_size)))


def tensor_learn(Y, Ds, s, K, err2=0.0):
    """Algorithm 1 generalised to n modes for K iterations plus a final sweep.
    Returns dict(Ds, supp, coef, res2, rmse (K + 1 values))."""
    Y = np.asarray(Y, np.float64)
    Ds = [np.array(D, np.float64, copy=True) for D in Ds]
    M = int(np.prod(Y.shape[1:]))
    trace = []
    for _ in range(K):
        for d in range(len(Ds)):
            supp, coef, res2 = tensor_omp(Y, Ds, s, err2=err2)
            if d == 0:
                trace.append(rmse(res2, M))
            Ds, coef, _ = tensor_update(d + 1, Y, Ds, supp, coef)
    supp, coef, res2 = tensor_omp(Y, Ds, s, err2=err2)
    trace.append(rmse(res2, M))
    return dict(Ds=Ds, supp=supp, coef=coef, res2=res2, rmse=np.array(trace))
