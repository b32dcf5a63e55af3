"""The selector trainer's host-side pieces: the dataset built from tuner points and the loss
weights that favour each point's fastest outputs."""
import math

import numpy as np

from paper_1503_04955_amd import learn


def test_dataset_targets_and_mask():
    pts = {(20.0, 1, 1): {3: 0.5, 9: 1.0, "thesis": 0.8},
           (14.0, 2, 16): {18: 0.01, 2: 0.02, "thesis": 0.05}}
    X, T, Mk, keys = learn.dataset(pts)
    assert keys == sorted(pts)
    i = keys.index((20.0, 1, 1))
    assert Mk[i].sum() == 2 and Mk[i, 3] == 1 and Mk[i, 9] == 1
    assert abs(T[i, 3] - math.log(0.5)) < 1e-6 and abs(T[i, 9] - math.log(1.0)) < 1e-6
    assert X.shape == (2, learn.dk.MLP_IN)


def test_decision_weights():
    T = np.log(np.array([[1.0, 1.2, 3.0, 100.0, 7.0]], np.float32))
    Mk = np.array([[1, 1, 1, 1, 0]], np.float32)
    W = learn.decision_weights(T, Mk, tau=0.3, floor=0.1)
    assert W[0, 0] == 1.0                                   # the fastest output
    assert abs(W[0, 1] - math.exp(-math.log(1.2) / 0.3)) < 1e-6
    assert W[0, 2] == np.float32(0.1) and W[0, 3] == np.float32(0.1)   # floored
    assert W[0, 4] == 0.0                                   # not measured
    # a point with nothing measured keeps all weights at zero
    assert not learn.decision_weights(T, np.zeros_like(Mk)).any()
