"""Training-loop ablations: host logic against the oracle (CPU) and a small
mini-batch training run with refresh on the GPU, tracked against FP64."""
import numpy as np
import pytest

from oracle import lr as LR
from paper_2006_10091_amd import ablations as A
from paper_2006_10091_amd import synth


def test_minibatches_and_refresh_schedule():
    assert A.minibatches(6000, 6000) == [(0, 6000)]
    assert A.minibatches(6000, 8000) == [(0, 6000)]
    mb = A.minibatches(6000, 128)
    assert len(mb) == 46 and mb[0] == (0, 128) and mb[-1] == (5760, 5888)
    assert A.schedule(12, 4) == [4, 8, 12]
    assert A.schedule(10, 4) == [4, 8, 10]
    assert A.schedule(3, 1) == [1, 2, 3]


def test_ls_sigmoid_matches_oracle_fit():
    c = LR.grad_poly_binomial(8.0)
    got = A.ls_sigmoid(8.0)
    assert got[0] == 0.5 and got[2] == 0.0
    assert abs(got[1] - c[1]) < 1e-12 and abs(got[3] - c[3]) < 1e-14


@pytest.mark.parametrize("coef", list(A.TABLE2.values()))
def test_plain_gradient_matches_oracle(coef):
    X, y = synth.small_data(1001, 300, 16)
    w = np.random.default_rng(3).uniform(-1, 1, 16)
    a = A.plain_gradient(X, y, w, coef, 0.01)
    b = LR.lr_gradient_fp64(X, y, w, coef, 0.01)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_table2_rows_match_golden():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_gradient_polynomials.txt")
    rows = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, *vals = line.split()
            rows[name] = [float(v) for v in vals]
    assert rows == A.TABLE2


@pytest.mark.gpu
def test_minibatch_training_with_refresh_tracks_fp64():
    """4 mini-batches of 128 on a 9-prime chain (refresh every 2 steps): after
    every refresh the server's weights are within 2^-20 of the two FP64 steps
    taken from its previous weights, and within 2^-16 of the whole FP64
    trajectory (step errors compound through the margins)."""
    X, y = synth.image_data(1002, 640)
    R = A.Run(9, X[:512], y[:512], 128)
    trace, acc_plain = R.train(A.ls_sigmoid(8.0), 1.0, 8, 2, X[512:], y[512:], mode=1)
    assert [t[0] for t in trace] == [2, 4, 6, 8]
    for k, el, acc, dev, dev_period in trace:
        assert dev_period < 2.0 ** -20, (k, dev_period)
        assert dev < 2.0 ** -16, (k, dev)
    assert abs(trace[-1][2] - acc_plain) <= 1.0 / 128
