"""FP64 CPU oracle for separable dictionary learning (2D-OMP + TMOD).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU
baseline may call it; the GPU library never does, and this package imports
nothing from it.  The arithmetic lives in ``sdlref.c`` (plain C99 loops, FP64);
this module marshals numpy arrays in math shape:

    Y   (N, m1, m2)   Y[k, i, j] = pixel (i, j) of signal k
    D1  (m1, n1), D2 (m2, n2)
    supp (N, s) int32 atom indices a = i + n1*j in selection order, -1 = unused
    coef (N, s) float64, res2 (N,) float64

Parity unpinned: nothing.  Every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` against closed forms, library least squares on the
explicit Kronecker dictionary, brute force and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdlref.c")
_LIB = os.path.join(_HERE, "libsdlref.so")

STOP_REL = 1e-14
DEP_EPS = 1e-10


def _compile(out: str, march: str) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    # ISO C mode: gcc contracts no a*b+c into FMA (-ffp-contract=off), so the results do not
    # depend on the target's instruction set
    subprocess.check_call(["gcc", "-O3", "-march=" + march, "-std=c99", "-fopenmp", "-fPIC", "-shared",
                           "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O3 for the x86-64-v3 level (AVX2 and FMA, which every host
    this runs on has), OpenMP for the shard split."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, "x86-64-v3")
    return _LIB


def build_native(directory: str) -> str:
    """The same source compiled with -O3 -march=native for the host it runs on, into
    ``directory`` (for timing the oracle on that host); returns the library path."""
    return _compile(os.path.join(directory, "libsdlref_native.so"), "native")


_libs = {}


def _load(path=None):
    path = path or _LIB
    if path not in _libs:
        if path == _LIB and not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(path)
        i32, i64, dp, ip, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double
        lib.sdlref_omp.argtypes = [i32, i32, i32, i32, i32, i32, i64, dp, dp, dp, ip, dp, dp, f64, f64, i32]
        lib.sdlref_omp_err.argtypes = [i32, i32, i32, i32, i32, i32, i64, dp, dp, dp, ip, dp, dp, f64, f64, f64, i32]
        lib.sdlref_tmod_sums.argtypes = [i32, i32, i32, i32, i32, i32, i64, dp, dp, dp, ip, dp, i32, dp, dp]
        lib.sdlref_tmod_update.argtypes = [i32, i32, i32, i32, i32, i32, i64, dp, dp, dp, ip, dp, i32, dp]
        lib.sdlref_learn.argtypes = [i32, i32, i32, i32, i32, i64, i32, i32, dp, dp, dp, ip, dp, dp, dp,
                                     f64, f64, i32]
        lib.sdlref_ortho_code.argtypes = [i32, i32, i32, i64, dp, dp, dp, ip, dp, dp, i32]
        lib.sdlref_procrustes_update.argtypes = [i32, i32, i32, i32, i64, dp, dp, dp, ip, dp, i32]
        lib.sdlref_learn_ortho.argtypes = [i32, i32, i32, i64, i32, dp, dp, dp, ip, dp, dp, dp, i32]
        for f in (lib.sdlref_omp, lib.sdlref_omp_err, lib.sdlref_tmod_sums, lib.sdlref_tmod_update, lib.sdlref_learn,
                  lib.sdlref_ortho_code, lib.sdlref_procrustes_update, lib.sdlref_learn_ortho):
            f.restype = ctypes.c_int
        _libs[path] = lib
    return _libs[path]


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__("oracle status %d" % status)
        self.status = status


def _cm(a):
    """math-shaped (..., r, c) -> contiguous column-major memory"""
    return np.ascontiguousarray(np.swapaxes(np.asarray(a, dtype=np.float64), -1, -2))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(st):
    if st != 0:
        raise OracleError(st)


def omp(Y, D1, D2, s, mode="separable", p=1, stop_rel=STOP_REL, dep_eps=DEP_EPS, err2=0.0):
    """2D-OMP of every signal.  Returns (supp, coef, res2).  err2 > 0: error-driven stop
    (Sec. IV's denoising runs): a signal takes no further atom once ||R_k||_F^2 <= err2."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    n1, n2 = D1.shape[1], D2.shape[1]
    Yc, D1c, D2c = _cm(Y), _cm(D1), _cm(D2)
    supp = np.empty((N, s), np.int32)
    coef = np.empty((N, s), np.float64)
    res2 = np.empty(N, np.float64)
    st = _load().sdlref_omp_err(0 if mode == "separable" else 1, m1, m2, n1, n2, s, N, _ptr(Yc), _ptr(D1c),
                                _ptr(D2c), _ptr(supp), _ptr(coef), _ptr(res2), stop_rel, dep_eps, err2, p)
    _check(st)
    return supp, coef, res2


def tmod_sums(side, Y, D1, D2, supp, coef, p=1):
    """Dense partial sums (A, B) of one TMOD half-step, math-shaped."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    n1, n2 = D1.shape[1], D2.shape[1]
    s = supp.shape[1]
    na, mb = (n1, m1) if side == 1 else (n2, m2)
    A = np.empty((na, na), np.float64)
    B = np.empty((na, mb), np.float64)  # memory of column-major (mb x na)
    st = _load().sdlref_tmod_sums(side, m1, m2, n1, n2, s, N, _ptr(_cm(Y)), _ptr(_cm(D1)), _ptr(_cm(D2)),
                                  _ptr(np.ascontiguousarray(supp, np.int32)),
                                  _ptr(np.ascontiguousarray(coef, np.float64)), p, _ptr(A), _ptr(B))
    _check(st)
    return A.T.copy(), B.T.copy()


def tmod_update(side, Y, D1, D2, supp, coef, p=1):
    """One dictionary update.  Returns (D1_new, D2_new, coef_rescaled, w)."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    n1, n2 = D1.shape[1], D2.shape[1]
    s = supp.shape[1]
    D1c, D2c = _cm(D1), _cm(D2)
    c = np.array(coef, np.float64, copy=True)
    w = np.empty(n1 if side == 1 else n2, np.float64)
    st = _load().sdlref_tmod_update(side, m1, m2, n1, n2, s, N, _ptr(_cm(Y)), _ptr(D1c), _ptr(D2c),
                                    _ptr(np.ascontiguousarray(supp, np.int32)), _ptr(c), p, _ptr(w))
    _check(st)
    return D1c.T.copy(), D2c.T.copy(), c, w


def learn(Y, D1, D2, s, K, schedule=0, p=1, stop_rel=STOP_REL, dep_eps=DEP_EPS, allow_singular=False, lib=None):
    """Algorithm 1 for K iterations plus a final OMP.  lib: path of another build of the same
    source (build_native), else the default one.

    Returns dict(D1, D2, supp, coef, res2, rmse, status)."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    n1, n2 = D1.shape[1], D2.shape[1]
    D1c, D2c = _cm(D1), _cm(D2)
    supp = np.empty((N, s), np.int32)
    coef = np.empty((N, s), np.float64)
    res2 = np.empty(N, np.float64)
    rmse = np.empty(K + 1, np.float64)
    st = _load(lib).sdlref_learn(m1, m2, n1, n2, s, N, K, schedule, _ptr(_cm(Y)), _ptr(D1c), _ptr(D2c),
                              _ptr(supp), _ptr(coef), _ptr(res2), _ptr(rmse), stop_rel, dep_eps, p)
    if st != 0 and not (allow_singular and st == -5):
        raise OracleError(st)
    return dict(D1=D1c.T.copy(), D2=D2c.T.copy(), supp=supp, coef=coef, res2=res2, rmse=rmse, status=st)


def ortho_code(Y, D1, D2, s, p=1):
    """Remark 1's codes for orthonormal D1 (m1 x m1), D2 (m2 x m2): X_k = T_s(D1^T Y_k D2).
    Returns (supp, coef, res2)."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    supp = np.empty((N, s), np.int32)
    coef = np.empty((N, s), np.float64)
    res2 = np.empty(N, np.float64)
    _check(_load().sdlref_ortho_code(m1, m2, s, N, _ptr(_cm(Y)), _ptr(_cm(D1)), _ptr(_cm(D2)), _ptr(supp),
                                     _ptr(coef), _ptr(res2), p))
    return supp, coef, res2


def procrustes_update(side, Y, D1, D2, supp, coef, p=1):
    """Remark 1's dictionary update (orthogonal Procrustes).  Returns (D1_new, D2_new)."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    s = supp.shape[1]
    D1c, D2c = _cm(D1), _cm(D2)
    _check(_load().sdlref_procrustes_update(side, m1, m2, s, N, _ptr(_cm(Y)), _ptr(D1c), _ptr(D2c),
                                            _ptr(np.ascontiguousarray(supp, np.int32)),
                                            _ptr(np.ascontiguousarray(coef, np.float64)), p))
    return D1c.T.copy(), D2c.T.copy()


def learn_ortho(Y, D1, D2, s, K, p=1):
    """Algorithm 1 with Remark 1's codes and updates.  Returns dict(D1, D2, supp, coef, res2, rmse)."""
    Y = np.asarray(Y, np.float64)
    N, m1, m2 = Y.shape
    D1c, D2c = _cm(D1), _cm(D2)
    supp = np.empty((N, s), np.int32)
    coef = np.empty((N, s), np.float64)
    res2 = np.empty(N, np.float64)
    rmse = np.empty(K + 1, np.float64)
    _check(_load().sdlref_learn_ortho(m1, m2, s, N, K, _ptr(_cm(Y)), _ptr(D1c), _ptr(D2c), _ptr(supp), _ptr(coef),
                                      _ptr(res2), _ptr(rmse), p))
    return dict(D1=D1c.T.copy(), D2=D2c.T.copy(), supp=supp, coef=coef, res2=res2, rmse=rmse)


def densify(supp, coef, n1, n2):
    """Dense codes X (N, n1, n2) from sparse (supp, coef)."""
    N, s = supp.shape
    X = np.zeros((N, n1 * n2))
    rows = np.repeat(np.arange(N), s)
    a = supp.reshape(-1)
    ok = a >= 0
    np.add.at(X, (rows[ok], a[ok]), coef.reshape(-1)[ok])
    # atom a = i + n1*j -> X[i, j]: column-major vec of X
    return X.reshape(N, n2, n1).transpose(0, 2, 1).copy()
