"""Helpers shared by the GPU parity tests (no method arithmetic of the GPU path here)."""
import numpy as np


def kron_cols(d1, d2):
    return np.kron(d2, d1)


# Coefficient error floor: a coefficient's error is measured relative to max(|x|, COEF_FLOOR * the
# largest |x| of its signal), so a coefficient far below its signal's scale is held to that scale.
COEF_FLOOR = 2e-2


def tie_gap(Y, d1, d2, prefix, gpu_atom, oracle_atom):
    """At the first diverging step: (|corr| of the best unselected atom - |corr| of the GPU's pick,
    the best |corr|, ||Y||_F).  The residual of the common prefix is taken by numpy lstsq on the
    explicit Kronecker columns, independently of both implementations."""
    return _tie_gap(Y, kron_cols(d1, d2), prefix, gpu_atom, oracle_atom)


def _tie_gap(Y, K, prefix, gpu_atom, oracle_atom):
    y = Y.flatten("F")
    if prefix:
        x = np.linalg.lstsq(K[:, prefix], y, rcond=None)[0]
        r = y - K[:, prefix] @ x
    else:
        r = y
    c = np.abs(K.T @ r)
    c[prefix] = -1
    top = c.max()
    return top - min(c[gpu_atom], c[oracle_atom]), top, float(np.linalg.norm(y))


def kron_all(Ds):
    """D_n (x) ... (x) D_1 for n-dimensional signals (first index fastest)."""
    K = Ds[0]
    for D in Ds[1:]:
        K = np.kron(D, K)
    return K


def code_stats(Y, d1, d2, supp_g, coef_g, supp_o, coef_o, band, K=None):
    """Supports and coefficients of the GPU against the oracle's.

    A signal whose support differs is a classified near-tie when, at the first step where the two
    selections diverge, both picks' exact correlations are within band * (the best one) of the best
    (band: 1e-9 for FP64 arithmetic, 1e-4 for FP32); otherwise it counts as bad.  Coefficients are
    compared on the signals whose supports agree, element by element:
    |x_gpu - x_ref| / max(|x_ref|, COEF_FLOOR * max_t |x_ref|)."""
    agree = np.all(supp_g == supp_o, axis=1)
    bad, ties, gaps = 0, 0, []
    for k in np.nonzero(~agree)[0]:
        t = int(np.argmax(supp_g[k] != supp_o[k]))
        prefix = [int(a) for a in supp_o[k, :t]]
        ga, oa = int(supp_g[k, t]), int(supp_o[k, t])
        if ga >= 0 and oa >= 0:
            gap, top, yn = _tie_gap(Y[k], K if K is not None else kron_cols(d1, d2), prefix, ga, oa)
            gaps.append((int(k), t, gap / top, gap / yn))
            if gap <= band * top:
                ties += 1
                continue
        else:
            gaps.append((int(k), t, float("nan"), float("nan")))
        bad += 1
    err, worst, norm_err = 0.0, None, 0.0
    if agree.any():
        ref = coef_o[agree]
        mx = np.abs(ref).max(axis=1, keepdims=True)
        scale = np.maximum(np.abs(ref), COEF_FLOOR * mx) + 1e-300
        e = np.abs(coef_g[agree] - ref) / scale
        err = float(e.max())
        i, t = np.unravel_index(int(np.argmax(e)), e.shape)
        worst = (float(np.abs(ref[i, t]) / (mx[i, 0] + 1e-300)), float(np.abs(coef_g[agree][i, t] - ref[i, t])
                                                                          / (mx[i, 0] + 1e-300)))
        norm_err = float((np.linalg.norm(coef_g[agree] - ref, axis=1) / (np.linalg.norm(ref, axis=1) + 1e-300)).max())
    return dict(agree=int(agree.sum()), ties=ties, bad=bad, coef_err=err, gaps=gaps, worst=worst,
                norm_err=norm_err)


def compare_codes(Y, d1, d2, supp_g, coef_g, supp_o, coef_o, band, coef_rtol=None, K=None):
    """Returns (n_agree, n_near_tie, n_bad, max element-wise coefficient error) as code_stats defines them.
    K: explicit dictionary for n-dimensional signals (then d1, d2 are unused)."""
    st = code_stats(Y, d1, d2, supp_g, coef_g, supp_o, coef_o, band, K=K)
    if st["bad"]:
        print("unclassified support mismatches (signal, step, gap/best, gap/||Y||):", st["gaps"][:10])
    print("coefficients: element-wise err %.2e (worst at |x|/max %.2e, |dx|/max %.2e), normwise err %.2e"
          % (st["coef_err"], *(st["worst"] or (0.0, 0.0)), st["norm_err"]))
    return st["agree"], st["ties"], st["bad"], st["coef_err"]


def full_size_checks(Ym, pr, s, fresh, n_each=1000, seed=11, band=1e-4, **opts):
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
    agree, ties, bad, err = compare_codes(Ym[idx], e1, e2, sg[idx], cg[idx], so, co, band)
    u1 = oracle.tmod_update(1, Ym, e1, e2, sg, cg, p=8)[0]
    pu = fresh()
    pu.D1.copy_(pr.D1)
    pu.D2.copy_(pr.D2)
    pu.supp.copy_(pr.supp)
    pu.coef.copy_(pr.coef)
    api.tmod_update(pu, sides=1, **opts)
    torch.cuda.synchronize()
    return len(idx), agree, ties, bad, err, float(np.abs(pu.d1() - u1).max())


def code_residual_energy(Y, d1, d2, supp, coef, chunk=20000):
    """FP64 energy of Y_k - sum_t coef[k, t] d1[:, i_t] d2[:, j_t]^T for every signal, from the
    returned code itself (math layouts: Y (N, m1, m2), d1 (m1, n1), d2 (m2, n2); supp -1 = unused)."""
    n1 = d1.shape[1]
    out = np.empty(len(Y))
    for k0 in range(0, len(Y), chunk):
        k1 = min(len(Y), k0 + chunk)
        s = supp[k0:k1]
        valid = s >= 0
        a = np.where(valid, s, 0)
        c = np.where(valid, coef[k0:k1], 0.0)
        A = np.transpose(d1[:, a % n1], (1, 2, 0)) * c[:, :, None]  # (n, S, m1)
        B = np.transpose(d2[:, a // n1], (1, 2, 0))                  # (n, S, m2)
        R = Y[k0:k1] - np.matmul(np.transpose(A, (0, 2, 1)), B)
        out[k0:k1] = np.sum(R * R, axis=(1, 2))
    return out
