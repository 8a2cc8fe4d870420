"""The patch-denoising driver of Sec. IV on the GPU against the oracle's composition
(extract_patches, omp with the error-driven stop, image_from_codes).

* Patch extraction is a copy: bit-exact, FP64 and FP32, square and non-square patches, an image of
  exactly one patch, ragged image sizes.
* Reconstruction from given codes (random supports with unused slots, random dictionaries):
  FP64 within 1e-12 of the largest pixel, FP32 within 1e-5 (a sum of at most m1 m2 s products per
  pixel in the element type, then one division).
* The whole driver on a synthetic noisy image with overcomplete-DCT dictionaries, eps = 1.15 sigma
  sqrt(m1 m2), cap m1 m2 / 2: codes against the oracle's codes as in the error-driven parity test
  (FP64: every support the oracle's except classified near-ties), the image against the oracle's
  reconstruction from the GPU's own codes (the bars above), and the PSNR gain over the noisy image
  equal to the oracle pipeline's within 0.01 dB.
* The full-size workload (512 x 512 image, all 255025 overlapping 8 x 8 patches, FP32): sampled
  patches' codes recomputed one by one by the oracle, sampled pixels rebuilt by brute force from
  the GPU's codes."""
import numpy as np
import pytest
import torch

import oracle
from oracle import denoise as oden
from paper_2007_03800_amd import api, synth
from tests.gpu_helpers import compare_codes

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _dicts(m1, m2, n1, n2):
    d1, d2 = synth.overcomplete_dct(m1, n1), synth.overcomplete_dct(m2, n2)
    return d1, d2, torch.as_tensor(d1.T.copy(), device=DEV), torch.as_tensor(d2.T.copy(), device=DEV)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,m1,m2", [(37, 29, 8, 8), (20, 31, 5, 7), (8, 8, 8, 8), (64, 40, 12, 12)])
def test_image_to_patches_bit_exact(H, W, m1, m2, dtype, rng):
    img = rng.standard_normal((H, W))
    if dtype == torch.float32:
        img = img.astype(np.float32).astype(np.float64)
    g = api.image_to_patches(torch.as_tensor(img, dtype=dtype, device=DEV), m1, m2)
    torch.cuda.synchronize()
    ref = oden.extract_patches(img, m1, m2)  # (N, m1, m2)
    assert g.shape == (len(ref), m2, m1)
    np.testing.assert_array_equal(g.double().cpu().numpy().transpose(0, 2, 1), ref)


def _rebuild(d1t, d2t, supp, coef, H, W, dtype):
    m1, m2 = d1t.shape[1], d2t.shape[1]
    N = (H - m1 + 1) * (W - m2 + 1)
    Y = torch.zeros((N, m2, m1), dtype=dtype, device=DEV)
    pr = api.Problem(Y, d1t, d2t, supp.shape[1], supp=torch.as_tensor(supp, device=DEV),
                     coef=torch.as_tensor(coef, dtype=dtype, device=DEV))
    out = api.patches_to_image(pr, H, W)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-12), (torch.float32, 1e-5)], ids=["fp64", "fp32"])
@pytest.mark.parametrize("H,W,m1,m2,n1,n2,s", [(40, 33, 8, 8, 16, 16, 6), (17, 23, 5, 7, 9, 11, 4),
                                                (12, 12, 12, 12, 20, 20, 10), (37, 20, 6, 6, 8, 8, 32),
                                                (40, 36, 32, 24, 64, 48, 20), (70, 70, 64, 64, 40, 40, 8)])
def test_patches_to_image_matches_oracle(H, W, m1, m2, n1, n2, s, dtype, bar, rng):
    """Also the rebuild's on-chip limits: up to 4 used slots per patch are kept on chip, patches
    with more are read from memory (20% unused slots at s = 6 and 10 mixes both, s = 32 has nearly
    every patch beyond it); the large patches keep 2, 1 or no slots on chip (the last one, 64 x 40
    FP64 dictionaries, needs more than 64 KiB of LDS)."""
    d1 = rng.standard_normal((m1, n1))
    d2 = rng.standard_normal((m2, n2))
    N = (H - m1 + 1) * (W - m2 + 1)
    supp = rng.integers(0, n1 * n2, (N, s)).astype(np.int32)
    supp[rng.random((N, s)) < 0.2] = -1          # unused slots of an early stop
    coef = rng.standard_normal((N, s))
    if dtype == torch.float32:
        coef = coef.astype(np.float32).astype(np.float64)
        d1c, d2c = d1.astype(np.float32).astype(np.float64), d2.astype(np.float32).astype(np.float64)
    else:
        d1c, d2c = d1, d2
    g = _rebuild(torch.as_tensor(d1.T.copy(), device=DEV), torch.as_tensor(d2.T.copy(), device=DEV), supp, coef,
                 H, W, dtype)
    ref = oden.image_from_codes(supp, coef, d1c, d2c, H, W)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print("rebuild err %.2e" % err)
    assert err <= bar


@pytest.mark.parametrize("dtype,band,ctol,bar", [(torch.float64, 1e-9, 1e-10, 1e-12), (torch.float32, 1e-4, 1e-4, 1e-5)],
                         ids=["fp64", "fp32"])
@pytest.mark.parametrize("m1,n1", [(8, 16), (8, 8)])
def test_denoise_matches_oracle(m1, n1, dtype, band, ctol, bar):
    H, W, sigma = 72, 64, 20.0
    clean = synth.synthetic_image(31, H, W)
    noisy = synth.noisy_image(clean, 31, sigma)
    if dtype == torch.float32:
        noisy = noisy.astype(np.float32).astype(np.float64)
    d1, d2, d1t, d2t = _dicts(m1, m1, n1, n1)
    s = m1 * m1 // 2
    err2 = (1.15 * sigma) ** 2 * m1 * m1
    out, pr = api.denoise(torch.as_tensor(noisy, dtype=dtype, device=DEV), d1t, d2t, sigma)
    torch.cuda.synchronize()
    g = out.double().cpu().numpy()
    sg, cg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy()
    P = oden.extract_patches(noisy, m1, m1)
    so, co, _ = oracle.omp(P, d1, d2, s, err2=err2, p=8)
    ng, no = np.sum(sg >= 0, axis=1), np.sum(so >= 0, axis=1)
    same = ng == no
    ks = np.nonzero(same)[0]
    agree, ties, bad, cerr = compare_codes(P[ks], d1, d2, sg[ks], cg[ks], so[ks], co[ks], band, ctol)
    print("%s n=%d: patches %d, nnz mean %.2f, count mismatches %d, agree %d, ties %d, bad %d, coef err %.1e"
          % (dtype, n1, len(P), no.mean(), int((~same).sum()), agree, ties, bad, cerr))
    assert bad == 0 and cerr <= ctol
    assert (~same).sum() <= (2 if dtype == torch.float64 else 0.01 * len(P))
    # the image from the GPU's codes, by the oracle's overlap average
    d1c, d2c = (d1, d2) if dtype == torch.float64 else (d1.astype(np.float32).astype(np.float64),
                                                        d2.astype(np.float32).astype(np.float64))
    ref = oden.image_from_codes(sg, cg, d1c, d2c, H, W)
    assert np.abs(g - ref).max() / np.abs(ref).max() <= bar
    p_gpu = oden.psnr(clean, g)
    p_ora = oden.psnr(clean, oden.image_from_codes(so, co, d1, d2, H, W))
    p_noisy = oden.psnr(clean, noisy)
    print("PSNR noisy %.3f, GPU %.3f, oracle %.3f" % (p_noisy, p_gpu, p_ora))
    assert abs(p_gpu - p_ora) <= 0.01 and p_gpu > p_noisy + 3.0


def test_denoise_full_size_sampled():
    """512 x 512, sigma 20, all 255025 overlapping 8 x 8 patches, 8 x 16 overcomplete-DCT
    dictionaries, FP32: 256 sampled patches' codes against the oracle one by one, 512 sampled
    pixels against a brute-force average over their covering patches from the GPU's codes."""
    H = W = 512
    sigma = 20.0
    clean = synth.synthetic_image(7)
    noisy = synth.noisy_image(clean, 7, sigma).astype(np.float32).astype(np.float64)
    d1, d2, d1t, d2t = _dicts(8, 8, 16, 16)
    err2 = (1.15 * sigma) ** 2 * 64
    out, pr = api.denoise(torch.as_tensor(noisy, dtype=torch.float32, device=DEV), d1t, d2t, sigma)
    torch.cuda.synchronize()
    assert pr.N == 255025
    g = out.double().cpu().numpy()
    sg, cg = pr.supp.cpu().numpy(), pr.coef.cpu().double().numpy()
    rs = np.random.default_rng(5)
    ks = rs.choice(pr.N, 256, replace=False)
    C = W - 7
    P = np.stack([noisy[k // C:k // C + 8, k % C:k % C + 8] for k in ks])
    so, co, _ = oracle.omp(P, d1, d2, 32, err2=err2)
    same = np.sum(sg[ks] >= 0, axis=1) == np.sum(so >= 0, axis=1)
    agree, ties, bad, cerr = compare_codes(P[same], d1, d2, sg[ks][same], cg[ks][same], so[same], co[same], 1e-4,
                                           1e-4)
    print("sampled patches: count mismatches %d, agree %d, ties %d, bad %d, coef err %.1e"
          % (int((~same).sum()), agree, ties, bad, cerr))
    assert (~same).sum() <= 3 and bad == 0 and cerr <= 1e-4
    d1c, d2c = d1.astype(np.float32).astype(np.float64), d2.astype(np.float32).astype(np.float64)
    worst = 0.0
    for p in rs.choice(H * W, 512, replace=False):
        y, x = divmod(int(p), W)
        acc, cnt = 0.0, 0
        for r in range(max(0, y - 7), min(y, H - 8) + 1):
            for c in range(max(0, x - 7), min(x, W - 8) + 1):
                k = r * C + c
                a = sg[k][sg[k] >= 0]
                acc += float(np.sum(cg[k][sg[k] >= 0] * d1c[y - r, a % 16] * d2c[x - c, a // 16]))
                cnt += 1
        worst = max(worst, abs(g[y, x] - acc / cnt))
    print("sampled pixels: max |err| %.2e" % worst)
    assert worst <= 1e-5 * 255
    assert oden.psnr(clean, g) > oden.psnr(clean, noisy) + 3.0
