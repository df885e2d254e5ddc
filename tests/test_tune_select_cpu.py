"""Parameter choice of the tuned miner (ym_tune_select, host only): the sweep
entry with the highest F1 against the reference pairs, ties to the first
entry in row-major order, checked against exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest


@pytest.fixture(scope="module")
def ym():
    from paper_1509_08639_amd import ymine
    return ymine


def _argmax_f1(nm, nc, truth):
    best, best_f = None, None
    for g in range(nm.shape[0]):
        for t in range(nm.shape[1]):
            d = int(nm[g, t]) + truth
            f = Fraction(2 * int(nc[g, t]), d) if d else Fraction(0)
            if best_f is None or f > best_f:
                best, best_f = (g, t), f
    return best, best_f


def test_choice_matches_exact_argmax(ym):
    r = np.random.default_rng(3)
    for trial in range(300):
        G, T = int(r.integers(1, 6)), int(r.integers(1, 8))
        truth = int(r.integers(0, 50))
        nm = r.integers(0, 60, (G, T)).astype(np.int64)
        nc = np.minimum(nm, r.integers(0, truth + 1, (G, T))).astype(np.int64)
        if trial % 3 == 0:  # many equal F1 values
            nm[:] = nm[0, 0]
            nc[:] = nc[0, 0]
            nm[-1, -1] = nm[0, 0]
        got = ym.tune_select(nm, nc, truth)
        (g, t), f = _argmax_f1(nm, nc, truth)
        assert (got["gap_index"], got["tau_index"]) == (g, t), (trial, nm, nc, truth)
        assert got["n_mined"] == nm[g, t] and got["n_correct"] == nc[g, t]
        assert got["f1"] == pytest.approx(float(f), rel=1e-15, abs=0.0)


def test_worked_example(ym):
    # 10 reference pairs; gap 0 finds 8 with 6 right (F1 12/18), gap 1 finds
    # 12 with 8 right (F1 16/22, the best), gap 2 finds 4 with 4 right (8/14)
    nm = np.array([[8], [12], [4]], np.int64)
    nc = np.array([[6], [8], [4]], np.int64)
    got = ym.tune_select(nm, nc, 10)
    assert (got["gap_index"], got["tau_index"]) == (1, 0)
    assert got["precision"] == 8 / 12 and got["recall"] == 0.8 and got["f1"] == 16 / 22
    # equal F1 (2/6 and 4/12 with 4 reference pairs): the first entry wins
    got = ym.tune_select(np.array([[2, 8]], np.int64), np.array([[1, 2]], np.int64), 4)
    assert got["f1"] == pytest.approx(1 / 3) and (got["gap_index"], got["tau_index"]) == (0, 0)
    got = ym.tune_select(np.array([[8], [2]], np.int64), np.array([[2], [1]], np.int64), 4)
    assert (got["gap_index"], got["tau_index"]) == (0, 0)
    # nothing mined and no reference pairs: F1 0 everywhere, entry 0
    got = ym.tune_select(np.zeros((2, 2), np.int64), np.zeros((2, 2), np.int64), 0)
    assert (got["gap_index"], got["tau_index"], got["f1"]) == (0, 0, 0.0)


def test_rejects_bad_counts(ym):
    for nm, nc, truth in [([[3]], [[4]], 10), ([[3]], [[-1]], 10), ([[5]], [[5]], 4), ([[1]], [[0]], -1)]:
        with pytest.raises(ym.YmError):
            ym.tune_select(np.array(nm, np.int64), np.array(nc, np.int64), truth)
    with pytest.raises(ym.YmError):
        ym.tune_select(np.zeros((0, 3), np.int64), np.zeros((0, 3), np.int64), 1)
