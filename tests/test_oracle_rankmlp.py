"""Pins of the learned-rank oracle (CPU, FP64): features on hand-built boxes,
the pinball loss on special cases, backpropagated gradients against central
finite differences and against the closed form of a linear model, the first
Adam step in closed form, and the label set's consistency with the oracle's
adaptive construction."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import hss_oracle as O
from oracle import rank_mlp as R


def test_box_gap_and_features_hand_built():
    # boxes [0,1]^3 and [3,4]x[0,1]x[0,1]: gap 2 along x only
    assert R.box_gap(np.zeros(3), np.ones(3), np.array([3.0, 0, 0]), np.array([4.0, 1, 1])) == 2.0
    # touching boxes
    assert R.box_gap(np.zeros(3), np.ones(3), np.array([1.0, 0, 0]), np.array([2.0, 1, 1])) == 0.0
    # diagonal separation: gaps 1 and 2 -> sqrt(5)
    g = R.box_gap(np.zeros(2), np.ones(2), np.array([2.0, 3.0]), np.array([3.0, 4.0]))
    assert abs(g - math.sqrt(5.0)) < 1e-15
    f = R.feature_vector(1000, [0, 0, 0], [0.1, 0.4, 0.2], [0.5, 0, 0], [0.6, 0.4, 0.2], 0.2, 1e-6)
    assert abs(f[0] - math.log2(1000)) < 1e-12
    np.testing.assert_allclose(f[1:4], [2.0, 1.0, 0.5])
    assert abs(f[4] - 0.4 / 0.2) < 1e-12
    assert abs(f[5] - math.log10(0.2)) < 1e-15 and abs(f[6] - 6.0) < 1e-12
    # point count clipped; 2-D boxes padded with a zero extent
    f2 = R.feature_vector(2 ** 20, [0, 0], [0.3, 0.1], [0.3, 0], [0.6, 0.1], 0.1, 1e-2)
    assert f2[0] == 13.0 and f2[3] == 0.0 and f2[4] == 0.0


def test_node_features_follow_the_tree():
    X = synth.points_uniform(512, 3, 11)
    t = O.build_tree(X, 64)
    Xt = X[t.perm]
    F, idx = R.node_features(Xt, t, 0.25, 1e-4)
    assert F.shape == (2 ** (t.levels + 1) - 2, 7)
    for row, (l, i) in zip(F, idx):
        lo, hi = t.ranges[l][i]
        P = Xt[lo:hi]
        ext = np.sort(P.max(0) - P.min(0))[::-1] / 0.25
        np.testing.assert_allclose(row[1:4], ext, rtol=1e-14)
        assert abs(row[0] - math.log2(hi - lo)) < 1e-12


def test_pinball_special_cases():
    y = np.array([0.0, 1.0, 2.0, 3.0])
    t = np.array([1.0, 1.0, 1.0, 1.0])
    # tau = 1/2: half the mean absolute error
    assert abs(R.pinball_loss(y, t, 0.5) - 0.5 * np.mean(np.abs(t - y))) < 1e-15
    # under-prediction costs tau per unit, over-prediction (1 - tau)
    assert abs(R.pinball_loss(np.array([0.0]), np.array([1.0]), 0.9) - 0.9) < 1e-15
    assert abs(R.pinball_loss(np.array([2.0]), np.array([1.0]), 0.9) - 0.1) < 1e-15
    g = R.pinball_grad(np.array([0.0, 2.0]), np.array([1.0, 1.0]), 0.9)
    np.testing.assert_allclose(g, [-0.9 / 2, 0.1 / 2])


def _small_params(sizes, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((o, i)) * 0.7, rng.standard_normal(o) * 0.3) for i, o in zip(sizes[:-1], sizes[1:])]


def test_gradients_match_central_differences():
    sizes = (7, 6, 5, 4, 1)
    params = _small_params(sizes, 3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((40, 7))
    t = rng.standard_normal(40) * 2.0
    tau = 0.9
    loss, grads = R.gradients(params, X, t, tau)
    h = 1e-6
    checked = 0
    for li, (W, b) in enumerate(params):
        for arr_k, arr in enumerate((W, b)):
            flat = arr.ravel()
            for q in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[q]
                flat[q] = old + h
                lp = R.pinball_loss(R.forward(params, X)[0], t, tau)
                flat[q] = old - h
                lm = R.pinball_loss(R.forward(params, X)[0], t, tau)
                flat[q] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][arr_k].ravel()[q]
                # the loss is piecewise linear: a kink inside [-h, h] would spoil the difference
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (li, arr_k, q, fd, an)
                checked += 1
    assert checked >= 30


def test_linear_model_gradient_closed_form():
    rng = np.random.default_rng(5)
    W = rng.standard_normal((1, 7))
    b = rng.standard_normal(1)
    X = rng.standard_normal((30, 7))
    t = rng.standard_normal(30)
    tau = 0.7
    loss, grads = R.gradients([(W, b)], X, t, tau)
    y = X @ W[0] + b[0]
    g = np.where(t > y, -tau, 1 - tau) / 30
    np.testing.assert_allclose(grads[0][0][0], X.T @ g, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(grads[0][1], [g.sum()], rtol=1e-13)
    assert abs(loss - np.mean(np.maximum(tau * (t - y), (tau - 1) * (t - y)))) < 1e-15


def test_first_adam_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so p -= lr * g / (|g| + eps)
    p = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    g = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    opt = R.Adam(p, lr=0.01)
    q = opt.step(p, g)
    for (W0, b0), (gW, gb), (W1, b1) in zip(p, g, q):
        np.testing.assert_allclose(W1, W0 - 0.01 * gW / (np.abs(gW) + 1e-8), rtol=1e-14)
        np.testing.assert_allclose(b1, b0 - 0.01 * gb / (np.abs(gb) + 1e-8), rtol=1e-12)


def test_training_decreases_the_loss():
    params = [(W, b) for W, b in synth.mlp_init((7, 16, 16, 1), seed=12)]
    rng = np.random.default_rng(6)
    X = rng.uniform(0, 1, (256, 7))
    t = 3.0 * X[:, 0] + np.sin(4 * X[:, 1])
    order = synth.minibatch_order(256, 30, seed=13)
    loss0 = R.pinball_loss(R.forward(params, X)[0], t, 0.9)
    params, losses = R.train(params, X, t, order, 32, tau=0.9, lr=3e-3)
    loss1 = R.pinball_loss(R.forward(params, X)[0], t, 0.9)
    assert loss1 < 0.25 * loss0


def test_rank_mapping():
    y = R.rank_target([1, 15, 96, 128])
    np.testing.assert_array_equal(R.rank_from_output(y, 128), [1, 15, 96, 128])
    np.testing.assert_array_equal(R.rank_from_output([-3.0, 40.0, 4.01], 100), [1, 100, 16])


@pytest.mark.slow
def test_labels_match_the_adaptive_construction():
    """Rows of the stored label set are the oracle's adaptive ranks: problem 0 recomputed."""
    path = os.path.join(os.path.dirname(__file__), "golden", "rank_labels.npz")
    d = np.load(path)
    import importlib.util

    spec = importlib.util.spec_from_file_location("mk", os.path.join(os.path.dirname(__file__), "golden",
                                                                     "make_rank_labels.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    j, F, ranks = mk.run(3)
    sel = d["problem"] == 3
    np.testing.assert_allclose(d["features"][sel], F.astype(np.float32))
    np.testing.assert_array_equal(d["ranks"][sel], ranks)
