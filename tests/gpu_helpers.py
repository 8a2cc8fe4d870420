"""Helpers shared by the GPU parity tests (no method arithmetic of the GPU path here)."""
import numpy as np


def kron_cols(d1, d2):
    return np.kron(d2, d1)


def near_tie_ok(Y, d1, d2, prefix, gpu_atom, oracle_atom, band):
    """At the first diverging step, is the GPU's pick within ``band`` (relative) of the best
    unselected |correlation|?  Residual of the common prefix is taken by numpy lstsq on the
    explicit Kronecker columns, independently of both implementations."""
    K = kron_cols(d1, d2)
    y = Y.flatten("F")
    if prefix:
        x = np.linalg.lstsq(K[:, prefix], y, rcond=None)[0]
        r = y - K[:, prefix] @ x
    else:
        r = y
    c = np.abs(K.T @ r)
    c[prefix] = -1
    top = c.max()
    return c[gpu_atom] >= top * (1 - band) and c[oracle_atom] >= top * (1 - band)


def compare_codes(Y, d1, d2, supp_g, coef_g, supp_o, coef_o, band, coef_rtol):
    """Returns (n_agree, n_near_tie, n_bad, max coef rel err on agreeing signals)."""
    agree = np.all(supp_g == supp_o, axis=1)
    bad = 0
    ties = 0
    for k in np.nonzero(~agree)[0]:
        t = int(np.argmax(supp_g[k] != supp_o[k]))
        prefix = [int(a) for a in supp_o[k, :t]]
        ga, oa = int(supp_g[k, t]), int(supp_o[k, t])
        if ga >= 0 and oa >= 0 and near_tie_ok(Y[k], d1, d2, prefix, ga, oa, band):
            ties += 1
        else:
            bad += 1
    err = 0.0
    if agree.any():
        num = np.abs(coef_g[agree] - coef_o[agree]).max(axis=1)
        den = np.abs(coef_o[agree]).max(axis=1) + 1e-300
        err = float((num / den).max())
    return int(agree.sum()), ties, bad, err
