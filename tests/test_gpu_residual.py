"""The residual energy each kernel reports (res2) is the energy of the residual of the code it
returns: Y_k - sum_t x_t d1_{i_t} d2_{j_t}^T recomputed in FP64 from the returned supports and
coefficients (and the FP32-rounded signals and dictionaries the FP32 kernels read), for every
signal of full-size batches, at FP32's bar (1e-4 relative, with an absolute floor of 1e-7 ||Y_k||^2
for residuals near zero) or FP64's (1e-10).  A property of any size: it needs no oracle run."""
import numpy as np
import pytest
import torch

from paper_2007_03800_amd import api, synth
from tests.gpu_helpers import code_residual_energy

pytestmark = pytest.mark.gpu


def _check(w, N, s, dtype, rtol, floor, **opts):
    Y = synth.signals(w, 0, N)
    d1, d2 = synth.true_dictionaries(w)
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
        d1r, d2r = (d.astype(np.float32).astype(np.float64) for d in (d1, d2))
    else:
        d1r, d2r = d1, d2
    pr = api.Problem.from_math(Y, d1, d2, s, dtype=dtype)
    api.sparse_code(pr, **opts)
    torch.cuda.synchronize()
    supp, coef, res2 = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy(), pr.res2.cpu().double().numpy()
    r64 = code_residual_energy(Y, d1r, d2r, supp, coef)
    yy = np.sum(Y * Y, axis=(1, 2))
    err = np.abs(res2 - r64) / np.maximum(r64, floor * yy)
    k = int(np.argmax(err))
    print("%s N %d s %d %s: max rel %.2e at signal %d (res2 %.6e, recomputed %.6e), nnz mean %.1f"
          % (w.name, N, s, opts, err[k], k, res2[k], r64[k], np.mean(np.sum(supp >= 0, axis=1))))
    assert err.max() <= rtol, (k, res2[k], r64[k])


def test_error_driven_fp32_full_batch():
    # the one-wave-per-signal kernel with the error-driven stop, all 100,000 signals
    w = synth.WORKLOADS["fp32_8x8_n16_s8"]
    m = w.m1 * w.m2
    err2 = float((1.15 * w.sigma() * np.sqrt(m)) ** 2)
    _check(w, w.N, m // 2, torch.float32, 1e-4, 1e-7, err2=err2)


def test_plain_fp32_full_batch():
    w = synth.WORKLOADS["fp32_8x8_n16_s8"]
    _check(w, w.N, w.s, torch.float32, 1e-4, 1e-7)


@pytest.mark.parametrize("dtype,rtol,floor,N", [(torch.float32, 1e-4, 1e-7, None), (torch.float64, 1e-10, 1e-14, 4000)])
def test_large_shape_wave_kernel(dtype, rtol, floor, N):
    # 32x24 signals, 48x36 atoms, s = 20: one wave per signal, correlations in 16x16 MFMA tiles (FP32)
    w = synth.WORKLOADS["uneven_p4_32x24_n48x36_s20"]
    _check(w, N or w.N, w.s, dtype, rtol, floor)
