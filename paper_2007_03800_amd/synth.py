"""Seeded synthetic inputs for separable dictionary learning.

Every random number is counter based: value = splitmix64(key(seed, stream) + index)
(splitmix64 as published by Steele, Lea and Flood, OOPSLA 2014), so any prefix of
the signal index space is reproducible on its own and the generator needs no
state.  Normals come from the Box-Muller transform of two such uniforms.

This module draws dictionaries, sparse codes and noise and forms the planted
signals Y_k = D1 X_k D2^T + E of the separable model (eq. (1) of the paper).  It
holds no step of the learning method (no sparse coding, no dictionary update):
both the FP64 CPU oracle and the GPU library are fed from here, and nothing here
depends on either of them.

Streams: 0 true D1, 1 true D2, 2 supports, 3 coefficients, 4 noise,
5 initial D1, 6 initial D2, 7 network initialisation, 8 batch order,
9 image content, 10 image noise, 11 training-patch choice.

Array conventions (numpy, "math shape"): Y is (N, m1, m2) with Y[k, i, j] the
pixel (i, j) of signal k; D1 is (m1, n1); D2 is (m2, n2); a code is a list of s
atom indices a = i + n1*j (the column of D2 (x) D1 under column-major vec) and
s coefficients.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_U64 = np.uint64


def _splitmix64(x):
    with np.errstate(over="ignore"):
        z = (x + _U64(0x9E3779B97F4A7C15)).astype(np.uint64)
        z = ((z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)).astype(np.uint64)
        z = ((z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)).astype(np.uint64)
        return z ^ (z >> _U64(31))


def _key(seed: int, stream: int):
    return _splitmix64(np.asarray(_U64(seed) * _U64(256) + _U64(stream), dtype=np.uint64))


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform doubles in (0, 1) for counter indices ``idx`` (any int array)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        u = _splitmix64(_key(seed, stream) + idx)
    return ((u >> _U64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def normal(seed: int, stream: int, idx) -> np.ndarray:
    """Standard normals; index i uses the uniforms at counters 2i and 2i+1."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform(seed, stream, idx * _U64(2))
    u2 = uniform(seed, stream, idx * _U64(2) + _U64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def unit_norm_dictionary(seed: int, stream: int, m: int, n: int) -> np.ndarray:
    """(m, n) matrix of i.i.d. N(0,1) entries (counter = p + m*i), columns scaled to unit norm."""
    d = normal(seed, stream, np.arange(m * n)).reshape(n, m).T.copy()
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return d


def orthonormal_dictionary(seed: int, stream: int, m: int) -> np.ndarray:
    """(m, m) orthogonal matrix: the Q factor of an i.i.d. N(0,1) matrix (counter = p + m*i), with
    the signs of R's diagonal moved into Q so that the draw is uniform (Haar) and unique."""
    g = normal(seed, stream, np.arange(m * m)).reshape(m, m).T
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))


def random_supports(seed: int, k0: int, k1: int, n_atoms: int, s: int) -> np.ndarray:
    """s distinct atoms per signal, uniform over all size-s subsets (Floyd's sampling).

    Returns int32 (k1-k0, s).  Signal k uses counters k*s .. k*s+s-1 of stream 2.
    """
    n = k1 - k0
    out = np.empty((n, s), dtype=np.int64)
    base = np.arange(k0, k1, dtype=np.int64) * s
    for t in range(s):
        j = n_atoms - s + t
        r = np.floor(uniform(seed, 2, base + t) * (j + 1)).astype(np.int64)
        r = np.minimum(r, j)
        dup = (out[:, :t] == r[:, None]).any(axis=1) if t else np.zeros(n, bool)
        out[:, t] = np.where(dup, j, r)
    return out.astype(np.int32)


def random_coefficients(seed: int, k0: int, k1: int, s: int, kind: str) -> np.ndarray:
    idx = np.arange(k0 * s, k1 * s, dtype=np.int64)
    if kind == "normal":
        c = normal(seed, 3, idx)
    elif kind == "signed_uniform":  # sign * U(0.5, 1.5)
        sign = np.where(uniform(seed, 3, 2 * idx) < 0.5, -1.0, 1.0)
        c = sign * (0.5 + uniform(seed, 3, 2 * idx + 1))
    else:
        raise ValueError(kind)
    return c.reshape(k1 - k0, s)


def _coef_power(kind: str) -> float:
    return 1.0 if kind == "normal" else 13.0 / 12.0  # E[c^2]


@dataclasses.dataclass
class Workload:
    """One separable dictionary problem of the synthetic benchmark family."""
    name: str
    m1: int
    m2: int
    n1: int
    n2: int
    s: int
    N: int
    snr_db: float
    coef_kind: str
    seed: int
    iters: int
    orthonormal: bool = False  # square dictionaries with orthonormal columns (Remark 1's variant)

    @property
    def n_atoms(self) -> int:
        return self.n1 * self.n2

    def sigma(self) -> float:
        """Noise level: expected clean power per pixel times 10^(-SNR/10).

        With unit-norm atoms and independent zero-mean coefficients the expected
        squared norm of a clean signal is s*E[c^2]; using the expectation (not a
        sample mean) keeps sigma independent of which prefix of signals is drawn.
        """
        p = self.s * _coef_power(self.coef_kind) / (self.m1 * self.m2)
        return math.sqrt(p * 10.0 ** (-self.snr_db / 10.0))


# The benchmark family: image-patch-shaped signals (the paper trains on 8x8 and
# 16x16 patches and on hyperspectral patches); synthetic stand-ins of the same shapes.
WORKLOADS = {
    "fp64_8x8_n12_s4": Workload("fp64_8x8_n12_s4", 8, 8, 12, 12, 4, 2_000, 20.0, "normal", 1000, 10),
    "fp32_8x8_n16_s8": Workload("fp32_8x8_n16_s8", 8, 8, 16, 16, 8, 100_000, 30.0, "normal", 1001, 20),
    "mixed_12x12_n24_s12": Workload("mixed_12x12_n24_s12", 12, 12, 24, 24, 12, 1_000_000, 25.0,
                                    "signed_uniform", 1002, 10),
    "uneven_p1_8x8_n16_s6": Workload("uneven_p1_8x8_n16_s6", 8, 8, 16, 16, 6, 200_000, 30.0, "normal", 1003, 10),
    "uneven_p2_12x12_n20_s10": Workload("uneven_p2_12x12_n20_s10", 12, 12, 20, 20, 10, 100_000, 30.0, "normal",
                                        1003, 10),
    "uneven_p3_16x16_n32_s16": Workload("uneven_p3_16x16_n32_s16", 16, 16, 32, 32, 16, 50_000, 30.0, "normal",
                                        1003, 10),
    "uneven_p4_32x24_n48x36_s20": Workload("uneven_p4_32x24_n48x36_s20", 32, 24, 48, 36, 20, 20_000, 30.0,
                                           "normal", 1003, 10),
    "learned_8x8_n16_s8": Workload("learned_8x8_n16_s8", 8, 8, 16, 16, 8, 1_500_000, 30.0, "normal", 1004, 0),
    # Remark 1's orthonormal variant at the size of the paper's m = n = 8, s = 8 timing (128,000 patches)
    "ortho_8x8_s8": Workload("ortho_8x8_s8", 8, 8, 8, 8, 8, 128_000, 30.0, "normal", 1005, 20, True),
}
UNEVEN_BATCH = ["uneven_p1_8x8_n16_s6", "uneven_p2_12x12_n20_s10", "uneven_p3_16x16_n32_s16",
                "uneven_p4_32x24_n48x36_s20"]


def _problem_seed(w: Workload) -> int:
    # the four problems of the uneven batch share one base seed; give each its own
    if w.name.startswith("uneven_p"):
        return w.seed * 16 + int(w.name[len("uneven_p")])
    return w.seed


def _dictionaries(w: Workload, s1: int, s2: int):
    sd = _problem_seed(w)
    if w.orthonormal:
        return orthonormal_dictionary(sd, s1, w.m1), orthonormal_dictionary(sd, s2, w.m2)
    return unit_norm_dictionary(sd, s1, w.m1, w.n1), unit_norm_dictionary(sd, s2, w.m2, w.n2)


def true_dictionaries(w: Workload):
    return _dictionaries(w, 0, 1)


def initial_dictionaries(w: Workload):
    return _dictionaries(w, 5, 6)


def planted_codes(w: Workload, k0: int, k1: int):
    sd = _problem_seed(w)
    supp = random_supports(sd, k0, k1, w.n_atoms, w.s)
    coef = random_coefficients(sd, k0, k1, w.s, w.coef_kind)
    return supp, coef


def signals(w: Workload, k0: int = 0, k1: int | None = None, dtype=np.float64,
            layout: str = "math", chunk: int = 65536) -> np.ndarray:
    """Signals k0..k1-1 of workload ``w``: Y_k = D1 X_k D2^T + sigma*E.

    layout "math": (n, m1, m2) with Y[k, i, j];  layout "colmajor": (n, m2, m1),
    i.e. each signal stored column-major, pixel (i, j) at offset i + m1*j.
    """
    if k1 is None:
        k1 = w.N
    d1, d2 = true_dictionaries(w)
    sd = _problem_seed(w)
    sigma = w.sigma()
    shape = (k1 - k0, w.m1, w.m2) if layout == "math" else (k1 - k0, w.m2, w.m1)
    out = np.empty(shape, dtype=dtype)
    for c0 in range(k0, k1, chunk):
        c1 = min(k1, c0 + chunk)
        supp, coef = planted_codes(w, c0, c1)
        ii, jj = supp % w.n1, supp // w.n1
        # clean part: sum_t coef_t * d1_{i_t} d2_{j_t}^T
        y = np.einsum("kt,pkt,qkt->kqp", coef, d1[:, ii], d2[:, jj], optimize=True)  # (n, m2, m1)
        pix = np.arange(c0 * w.m1 * w.m2, c1 * w.m1 * w.m2, dtype=np.int64)
        y += sigma * normal(sd, 4, pix).reshape(c1 - c0, w.m2, w.m1)
        if layout == "math":
            out[c0 - k0:c1 - k0] = y.transpose(0, 2, 1)
        else:
            out[c0 - k0:c1 - k0] = y
    return out


def to_colmajor(a: np.ndarray) -> np.ndarray:
    """Math-shaped (..., r, c) array -> C-contiguous (..., c, r) whose memory is column-major."""
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


def from_colmajor(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


def synthetic_image(seed: int, H: int = 512, W: int = 512) -> np.ndarray:
    """A (H, W) grey-level image in [0, 255] standing in for the paper's 512 x 512 test images:
    a smooth background (a few low-frequency cosines), 24 axis-aligned rectangles and 12 discs of
    random intensity, and a band of fine stripes, so that patches have flat areas, edges and texture."""
    u = lambda n, off: uniform(seed, 9, np.arange(off, off + n))
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((H, W), 110.0)
    c = u(12, 0)
    for k in range(3):
        fy, fx, ph = 1 + 3 * c[4 * k], 1 + 3 * c[4 * k + 1], 2 * math.pi * c[4 * k + 2]
        img += 25.0 * (c[4 * k + 3] - 0.5) * 2 * np.cos(2 * math.pi * (fy * yy / H + fx * xx / W) + ph)
    r = u(24 * 5, 100)
    for k in range(24):
        y0, x0 = int(r[5 * k] * H * 0.9), int(r[5 * k + 1] * W * 0.9)
        h, w = int(8 + r[5 * k + 2] * H * 0.25), int(8 + r[5 * k + 3] * W * 0.25)
        img[y0:y0 + h, x0:x0 + w] = 30.0 + 200.0 * r[5 * k + 4]
    d = u(12 * 4, 1000)
    for k in range(12):
        cy, cx, rad = d[4 * k] * H, d[4 * k + 1] * W, 6 + d[4 * k + 2] * H * 0.08
        img[(yy - cy) ** 2 + (xx - cx) ** 2 <= rad ** 2] = 20.0 + 215.0 * d[4 * k + 3]
    band = (yy > 0.70 * H) & (yy < 0.78 * H)
    img[band] += 30.0 * np.sign(np.sin(2 * math.pi * xx[band] / 6.0))
    return np.clip(img, 0.0, 255.0)


def noisy_image(img: np.ndarray, seed: int, sigma: float) -> np.ndarray:
    """img + sigma * N(0, 1) i.i.d. per pixel (stream 10)."""
    return img + sigma * normal(seed, 10, np.arange(img.size)).reshape(img.shape)


def training_patch_index(seed: int, n_patches: int, count: int) -> np.ndarray:
    """count distinct patch indices out of n_patches, uniformly (stream 11), sorted."""
    u = uniform(seed, 11, np.arange(4 * count))
    idx = np.unique(np.floor(u * n_patches).astype(np.int64))[:count]
    return np.sort(idx)


def overcomplete_dct(m: int, n: int) -> np.ndarray:
    """(m, n) dictionary of sampled cosines, column k = cos(pi (i + 1/2) k / n), i = 0..m-1, scaled
    to unit norm: the usual starting dictionary of patch-based dictionary learning (n = m gives the
    orthonormal DCT-II basis)."""
    i = np.arange(m)[:, None] + 0.5
    k = np.arange(n)[None, :]
    d = np.cos(np.pi * i * k / n)
    return d / np.linalg.norm(d, axis=0)


@dataclasses.dataclass
class TensorWorkload:
    """n-dimensional signals (Remark 3): Y_k = X_k x_1 D_1 ... x_n D_n + sigma E with s planted atoms
    per signal (uniform over prod n atoms), N(0,1) coefficients and unit-norm random dictionaries."""
    name: str
    ms: tuple
    ns: tuple
    s: int
    N: int
    snr_db: float
    seed: int
    iters: int

    def sigma(self) -> float:
        return math.sqrt(self.s / float(np.prod(self.ms)) * 10.0 ** (-self.snr_db / 10.0))


# three-mode stand-in for hyperspectral patches: 8 x 8 pixels x 4 bands
TENSOR_WORKLOADS = {
    "tensor_8x8x4_n12x12x6_s8": TensorWorkload("tensor_8x8x4_n12x12x6_s8", (8, 8, 4), (12, 12, 6), 8, 100_000,
                                               30.0, 1006, 10),
}


def tensor_dictionaries(w: TensorWorkload, initial: bool = False):
    base = 20 if initial else 12  # streams 12.. (true) and 20.. (starting dictionaries), one per mode
    return [unit_norm_dictionary(w.seed, base + d, m, n) for d, (m, n) in enumerate(zip(w.ms, w.ns))]


def tensor_signals(w: TensorWorkload, k0: int = 0, k1: int | None = None, chunk: int = 20000) -> np.ndarray:
    """Signals k0..k1-1 in math layout (n, m_1, ..., m_n); counters as for the two-mode workloads
    (supports stream 2, coefficients stream 3), noise from stream 4 at counter k * prod(m) + pixel."""
    k1 = w.N if k1 is None else k1
    Ds = tensor_dictionaries(w)
    M = int(np.prod(w.ms))
    K = Ds[0]
    for D in Ds[1:]:
        K = np.kron(D, K)
    out = np.empty((k1 - k0,) + tuple(w.ms))
    for c0 in range(k0, k1, chunk):
        c1 = min(k1, c0 + chunk)
        supp = random_supports(w.seed, c0, c1, int(np.prod(w.ns)), w.s)
        coef = random_coefficients(w.seed, c0, c1, w.s, "normal")
        y = np.einsum("mkt,kt->km", K[:, supp], coef, optimize=True)
        y += w.sigma() * normal(w.seed, 4, np.arange(c0 * M, c1 * M, dtype=np.int64)).reshape(c1 - c0, M)
        out[c0 - k0:c1 - k0] = y.reshape((c1 - c0,) + tuple(reversed(w.ms))).transpose(
            (0,) + tuple(range(len(w.ms), 0, -1)))
    return out
