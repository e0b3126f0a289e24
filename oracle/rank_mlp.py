"""CPU FP64 oracle of the learned rank model: node features, the MLP that maps
them to a basis rank, its pinball loss, the hand-derived gradients and the Adam
update; plus the rank labels from the oracle's adaptive pivoted QR.

TEST INFRASTRUCTURE ONLY: the reference the GPU training and inference kernels
are checked against; only the test-suite, the smoke check and the committed
label-generation script use it. It shares no code with the HIP library.

The paper keeps a fixed maximum rank (its Results section); the learned model is
an addition of this implementation: a multilayer perceptron predicts, for each
tree node, the rank that the adaptive pivoted QR (Eq. 2 with a tolerance) would
choose, so that sample counts and workspaces can be sized before compression.

Readings (listed with the others of this implementation):
  * features of a node (7): log2 of its point count (clipped at 13, the largest
    training nodes, because the rank of a densely sampled box stops growing with
    the point count), the three extents of its bounding box sorted in decreasing
    order and divided by the kernel length, the gap between its box and its
    sibling's box divided by the kernel length, log10 of the kernel length, and
    -log10 of the tolerance. Missing dimensions have extent 0;
  * target: log2(1 + rank); prediction rank = ceil(2^y - 1 - 1e-3) clipped to
    [1, cap] (the slack absorbs rounding when y is exactly a target);
  * loss: pinball (quantile) loss with tau = 0.9, so that under-prediction, which
    costs a recompression, weighs nine times more than over-prediction;
  * network: 7 -> 128 -> 128 -> 128 -> 1, ReLU between layers, no activation on
    the output; weights column-major W (out x in), biases b (out);
  * optimizer: Adam (Kingma and Ba 2015) with the bias corrections of the
    published algorithm, lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8.

Parity status: forward, loss, gradients and Adam are pinned (finite differences,
closed-form gradient of a linear model, pinball special cases, the first Adam
step). Features are pinned on hand-built boxes. The label generator reuses the
pinned adaptive construction of hss_oracle.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import hss_oracle as O

NFEAT = 7
SIZES = (7, 128, 128, 128, 1)
NPTS_LOG2_CLIP = 13.0


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------


def _box(P: np.ndarray):
    lo = P.min(axis=0)
    hi = P.max(axis=0)
    return lo, hi


def box_gap(lo1, hi1, lo2, hi2) -> float:
    """Euclidean distance between two axis-aligned boxes (0 if they touch or overlap)."""
    d = np.maximum(0.0, np.maximum(lo2 - hi1, lo1 - hi2))
    return float(np.sqrt(np.sum(d * d)))


def feature_vector(npts: int, lo, hi, slo, shi, length: float, tol: float) -> np.ndarray:
    ext = np.sort(np.asarray(hi) - np.asarray(lo))[::-1]
    e = np.zeros(3)
    e[: min(3, ext.size)] = ext[:3]
    return np.array([
        min(math.log2(max(npts, 1)), NPTS_LOG2_CLIP),
        e[0] / length,
        e[1] / length,
        e[2] / length,
        box_gap(np.asarray(lo), np.asarray(hi), np.asarray(slo), np.asarray(shi)) / length,
        math.log10(length),
        -math.log10(tol),
    ])


def node_features(Xt: np.ndarray, tree: O.Tree, length: float, tol: float):
    """Features of every non-root node, level by level (1..L), left to right.
    Xt: points in tree order. Returns (F [count x 7], [(level, index)])."""
    feats, idx = [], []
    for l in range(1, tree.levels + 1):
        boxes = [_box(Xt[lo:hi]) for lo, hi in tree.ranges[l]]
        for i, (lo, hi) in enumerate(tree.ranges[l]):
            sib = i ^ 1
            feats.append(feature_vector(hi - lo, boxes[i][0], boxes[i][1], boxes[sib][0], boxes[sib][1], length, tol))
            idx.append((l, i))
    return np.array(feats).reshape(-1, NFEAT), idx


def rank_target(rank) -> np.ndarray:
    return np.log2(1.0 + np.asarray(rank, dtype=np.float64))


def rank_from_output(y, cap: int) -> np.ndarray:
    """ceil(2^y - 1), ignoring an excess below 1e-3 over an integer (so that a
    target reproduces its rank despite rounding), clipped to [1, cap]."""
    r = np.ceil(np.exp2(np.asarray(y, dtype=np.float64)) - 1.0 - 1e-3)
    return np.clip(r, 1, cap).astype(np.int64)


# ----------------------------------------------------------------------------
# the network
# ----------------------------------------------------------------------------


def forward(params, X: np.ndarray):
    """params: list of (W [out x in], b [out]); X: [B x 7]. Returns (y [B], cache)."""
    H = X.T  # in x B
    cache = [H]
    nl = len(params)
    for li, (W, b) in enumerate(params):
        Z = W @ H + b[:, None]
        if li < nl - 1:
            cache.append(Z)
            H = np.maximum(Z, 0.0)
            cache.append(H)
        else:
            H = Z
    return H[0], cache


def pinball_loss(y: np.ndarray, t: np.ndarray, tau: float) -> float:
    """mean over samples of max(tau (t - y), (tau - 1)(t - y))."""
    d = t - y
    return float(np.mean(np.maximum(tau * d, (tau - 1.0) * d)))


def pinball_grad(y: np.ndarray, t: np.ndarray, tau: float) -> np.ndarray:
    """d loss / d y (the subgradient -tau where t > y, 1 - tau elsewhere), divided by B."""
    g = np.where(t > y, -tau, 1.0 - tau)
    return g / y.size


def gradients(params, X: np.ndarray, t: np.ndarray, tau: float):
    """Loss and gradients [(dW, db)] of the mean pinball loss, by backpropagation."""
    y, cache = forward(params, X)
    loss = pinball_loss(y, t, tau)
    G = pinball_grad(y, t, tau)[None, :]  # 1 x B: dL/dZ of the output layer
    nl = len(params)
    grads = [None] * nl
    for li in range(nl - 1, -1, -1):
        W, _ = params[li]
        Hin = cache[2 * li]  # input activation of layer li
        grads[li] = (G @ Hin.T, G.sum(axis=1))
        if li > 0:
            dH = W.T @ G
            Zprev = cache[2 * li - 1]
            G = dH * (Zprev > 0.0)
    return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
        self.t = 0

    def step(self, params, grads):
        """theta -= lr * mhat / (sqrt(vhat) + eps) with mhat = m / (1 - beta1^t),
        vhat = v / (1 - beta2^t), m and v the running first and second moments."""
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for li, (pp, gg) in enumerate(zip(params, grads)):
            new = []
            for k in range(2):
                g = gg[k]
                self.m[li][k] = self.b1 * self.m[li][k] + (1.0 - self.b1) * g
                self.v[li][k] = self.b2 * self.v[li][k] + (1.0 - self.b2) * g * g
                new.append(pp[k] - self.lr * (self.m[li][k] / c1) / (np.sqrt(self.v[li][k] / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


def train(params, X, t, order, batch: int, tau: float = 0.9, lr: float = 1e-3):
    """Minibatch Adam over the sample order `order` (a flat index array whose
    consecutive `batch`-sized chunks are the minibatches; a short tail is a
    smaller batch). Returns (params, per-step losses)."""
    opt = Adam(params, lr=lr)
    losses = []
    for s0 in range(0, len(order), batch):
        sel = order[s0:s0 + batch]
        loss, g = gradients(params, X[sel], t[sel], tau)
        params = opt.step(params, g)
        losses.append(loss)
    return params, losses


# ----------------------------------------------------------------------------
# labels: adaptive pivoted-QR ranks of the scaled construction
# ----------------------------------------------------------------------------


def labelled_nodes(X: np.ndarray, leaf: int, kern: O.Kernel, tol: float, omega: np.ndarray, max_rank: int):
    """Features and adaptive ranks of every non-root node of one problem: the
    oracle's scaled construction at tolerance `tol` (ranks capped at max_rank,
    omega: N x s Gaussian test matrix in the caller's point order)."""
    tree = O.build_tree(X, leaf)
    Xt = X[tree.perm]
    h = O.construct_scaled(X, tree, kern, omega[tree.perm], tol=tol, max_rank=max_rank)
    F, idx = node_features(Xt, tree, kern.length, tol)
    ranks = np.array([h.rank[l][i] for (l, i) in idx], dtype=np.int64)
    return F, ranks
