"""The seeded generator: counter-based, prefix-stable, distinct supports, unit-norm atoms."""
import numpy as np

from paper_2007_03800_amd import synth


def test_prefix_stable_and_layouts():
    w = synth.WORKLOADS["fp64_8x8_n12_s4"]
    a = synth.signals(w, 0, 40)
    b = synth.signals(w, 10, 25)
    np.testing.assert_array_equal(a[10:25], b)
    c = synth.signals(w, 0, 40, layout="colmajor")
    np.testing.assert_array_equal(c, a.transpose(0, 2, 1))


def test_supports_distinct_and_uniform_marginals():
    supp = synth.random_supports(7, 0, 20000, 16, 5)
    assert supp.min() >= 0 and supp.max() < 16
    assert all(len(set(r)) == 5 for r in supp[:2000])
    counts = np.bincount(supp.ravel(), minlength=16) / supp.size
    np.testing.assert_allclose(counts, 1 / 16, atol=0.01)


def test_normals_moments_and_dictionaries():
    z = synth.normal(3, 4, np.arange(200000))
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    for w in synth.WORKLOADS.values():
        d1, d2 = synth.true_dictionaries(w)
        assert d1.shape == (w.m1, w.n1) and d2.shape == (w.m2, w.n2)
        np.testing.assert_allclose(np.linalg.norm(d1, axis=0), 1, rtol=1e-14)


def test_snr_matches_definition():
    w = synth.WORKLOADS["fp32_8x8_n16_s8"]
    y = synth.signals(w, 0, 20000)
    d1, d2 = synth.true_dictionaries(w)
    supp, coef = synth.planted_codes(w, 0, 20000)
    clean = np.einsum("kt,pkt,qkt->kpq", coef, d1[:, supp % 16], d2[:, supp // 16])
    snr = 10 * np.log10(np.sum(clean ** 2) / np.sum((y - clean) ** 2))
    assert abs(snr - w.snr_db) < 0.3


def test_orthonormal_workload_dictionaries():
    w = synth.WORKLOADS["ortho_8x8_s8"]
    for d in (*synth.true_dictionaries(w), *synth.initial_dictionaries(w)):
        np.testing.assert_allclose(d.T @ d, np.eye(d.shape[0]), atol=1e-14)
    a, b = synth.true_dictionaries(w)
    assert np.abs(a - b).max() > 0.1  # different streams
