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


def full_size_checks(Ym, pr, s, fresh, n_each=1000, seed=11):
    """Checks of a problem coded at full size on the GPU (``pr``, after Algorithm 1), against
    the oracle on ``Ym`` (N, m1, m2): exactly the signal values the GPU read, in FP64.

    * Sampled final codes (the first and last ``n_each`` signals and ``n_each`` random ones)
      against the oracle's 2D-OMP at the GPU's final dictionaries.
    * One D1 update from the GPU's full-batch codes, on a fresh problem built by ``fresh``
      with the same dictionaries and codes, against the oracle's FP64 update.

    Returns (n_sampled, n_agree, n_near_tie, n_bad, max coef rel err, max |D1 diff|)."""
    import torch

    import oracle
    from paper_2007_03800_amd import api

    N = len(Ym)
    e1, e2 = pr.d1(), pr.d2()
    sg, cg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy()
    rs = np.random.default_rng(seed)
    k = min(n_each, N)
    idx = np.unique(np.concatenate([np.arange(k), np.arange(N - k, N), rs.choice(N, k, replace=False)]))
    so, co, _ = oracle.omp(Ym[idx], e1, e2, s, p=8)
    agree, ties, bad, err = compare_codes(Ym[idx], e1, e2, sg[idx], cg[idx], so, co, 1e-4, 1e-4)
    u1 = oracle.tmod_update(1, Ym, e1, e2, sg, cg, p=8)[0]
    pu = fresh()
    pu.D1.copy_(pr.D1)
    pu.D2.copy_(pr.D2)
    pu.supp.copy_(pr.supp)
    pu.coef.copy_(pr.coef)
    api.tmod_update(pu, sides=1)
    torch.cuda.synchronize()
    return len(idx), agree, ties, bad, err, float(np.abs(pu.d1() - u1).max())
