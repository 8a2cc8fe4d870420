"""FP64 CPU oracle of the patch-denoising driver of the paper's Sec. IV (TEST INFRASTRUCTURE ONLY:
the tests, the smoke check and the benchmark may call it; the GPU library never does).

The denoising experiment codes every overlapping patch of a noisy image with the error-driven
2D-OMP (the oracle's own `omp(..., err2=...)`), rebuilds each patch as D1 X_k D2^T and puts the
image back together.  The paper fixes the patch size, the stop and the cap; it does not say how the
overlapping estimates are combined: reading, every pixel is the plain average of the estimates of
all patches covering it (no weighting with the noisy image, no mean removal).

Plain numpy, one patch offset at a time, by the definitions:
  extract_patches  all (H - m1 + 1)(W - m2 + 1) patches, stride 1, patch k = r (W - m2 + 1) + c
                   holds img[r + i, c + j] at (i, j)
  image_from_codes the average over covering patches of (D1 X_k D2^T)[i, j]
Parity unpinned: nothing (pinned by tests/test_oracle_denoise.py against brute force and exact
reconstructions).
"""
from __future__ import annotations

import numpy as np

from . import densify


def extract_patches(img, m1, m2):
    img = np.asarray(img, np.float64)
    H, W = img.shape
    R, C = H - m1 + 1, W - m2 + 1
    out = np.empty((R * C, m1, m2))
    for i in range(m1):
        for j in range(m2):
            out[:, i, j] = img[i:i + R, j:j + C].reshape(-1)
    return out


def image_from_codes(supp, coef, D1, D2, H, W):
    m1, n1 = D1.shape
    m2, n2 = D2.shape
    R, C = H - m1 + 1, W - m2 + 1
    X = densify(np.asarray(supp), np.asarray(coef, np.float64), n1, n2)
    P = np.einsum("pi,kij,qj->kpq", D1, X, D2).reshape(R, C, m1, m2)
    acc = np.zeros((H, W))
    cnt = np.zeros((H, W))
    for i in range(m1):
        for j in range(m2):
            acc[i:i + R, j:j + C] += P[:, :, i, j]
            cnt[i:i + R, j:j + C] += 1.0
    return acc / cnt


def psnr(ref, img, peak=255.0):
    mse = float(np.mean((np.asarray(ref, np.float64) - np.asarray(img, np.float64)) ** 2))
    return 10.0 * np.log10(peak * peak / mse) if mse > 0 else float("inf")
