"""Host-side helpers of bench.py: flop and byte counts, the support-agreement measure."""
import importlib.util
import os

import numpy as np

_spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_support_agreement_counts_sets_not_order():
    g = np.array([[3, 1, 2, -1], [5, 6, 7, 8], [1, 2, 3, 4]])
    o = np.array([[1, 2, 3, -1], [5, 6, 7, 9], [4, 3, 2, 1]])
    a = bench.support_agreement(g, o)
    assert a["support_agreement"] == 2 / 3
    assert a["atom_agreement"] == 10 / 11


def test_support_agreement_empty_slots_do_not_count_as_atoms():
    g = np.array([[0, -1, -1]])
    o = np.array([[1, -1, -1]])
    a = bench.support_agreement(g, o)
    assert a["support_agreement"] == 0.0 and a["atom_agreement"] == 0.0


def test_omp_flops_grow_with_sparsity():
    f = [bench.omp_flops_per_signal(8, 8, 16, 16, s) for s in (1, 4, 8)]
    assert f[0] < f[1] < f[2]
