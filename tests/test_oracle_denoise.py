"""Pins of the denoising driver's oracle (Sec. IV): patch extraction and the overlap average."""
import numpy as np

import oracle
from oracle import denoise


def test_extract_patches_brute_force(rng):
    img = rng.standard_normal((13, 11))
    P = denoise.extract_patches(img, 4, 3)
    R, C = 10, 9
    assert P.shape == (R * C, 4, 3)
    for k in rng.choice(R * C, 25, replace=False):
        r, c = divmod(int(k), C)
        np.testing.assert_array_equal(P[k], img[r:r + 4, c:c + 3])


def test_exact_codes_rebuild_the_image(rng):
    """With D1 = I, D2 = I and s = m1 m2 every patch is its own code, so the average of the
    rebuilt patches is the image itself."""
    img = rng.standard_normal((9, 10))
    m1, m2 = 3, 4
    P = denoise.extract_patches(img, m1, m2)
    N = len(P)
    supp = np.tile(np.arange(m1 * m2, dtype=np.int32), (N, 1))
    coef = np.stack([p.flatten("F") for p in P])  # atom a = i + m1 j
    out = denoise.image_from_codes(supp, coef, np.eye(m1), np.eye(m2), *img.shape)
    np.testing.assert_allclose(out, img, rtol=0, atol=1e-13)


def test_overlap_average_brute_force(rng):
    H, W, m1, m2, n1, n2, s = 7, 8, 3, 2, 4, 3, 2
    d1 = rng.standard_normal((m1, n1))
    d2 = rng.standard_normal((m2, n2))
    R, C = H - m1 + 1, W - m2 + 1
    supp = rng.integers(0, n1 * n2, (R * C, s)).astype(np.int32)
    coef = rng.standard_normal((R * C, s))
    out = denoise.image_from_codes(supp, coef, d1, d2, H, W)
    for y in range(H):
        for x in range(W):
            vals = []
            for r in range(max(0, y - m1 + 1), min(R, y + 1)):
                for c in range(max(0, x - m2 + 1), min(C, x + 1)):
                    k = r * C + c
                    X = np.zeros((n1, n2))
                    for a, v in zip(supp[k], coef[k]):
                        X[a % n1, a // n1] += v
                    vals.append((d1 @ X @ d2.T)[y - r, x - c])
            assert abs(out[y, x] - np.mean(vals)) <= 1e-12


def test_error_driven_denoising_improves_psnr():
    """Orthonormal DCT-like dictionaries on a smooth image: coding every patch with the error-driven
    stop at 1.15 sigma sqrt(m1 m2) removes most of the noise (PSNR rises)."""
    rng = np.random.default_rng(3)
    H = W = 40
    yy, xx = np.mgrid[0:H, 0:W]
    img = 100 + 50 * np.cos(2 * np.pi * yy / 20.0) * np.cos(2 * np.pi * xx / 25.0)
    sigma = 15.0
    noisy = img + sigma * rng.standard_normal(img.shape)
    m = 8
    k = np.arange(m)
    dct = np.cos(np.pi * (k[:, None] + 0.5) * k[None, :] / m)
    dct /= np.linalg.norm(dct, axis=0)
    P = denoise.extract_patches(noisy, m, m)
    err2 = (1.15 * sigma * m) ** 2
    supp, coef, _ = oracle.omp(P, dct, dct, m * m // 2, err2=err2)
    out = denoise.image_from_codes(supp, coef, dct, dct, H, W)
    assert denoise.psnr(img, out) > denoise.psnr(img, noisy) + 5.0
