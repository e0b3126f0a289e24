"""Writes rank_labels.npz: features and adaptive pivoted-QR ranks of tree nodes
from the oracle's scaled construction, the training set of the learned rank
model. Calls only the oracle and the seeded input generators.

Problems: N in {2048, 4096, 8192}, points uniform in the unit cube, kernels
exponential / Matern-3/2 / Gaussian with length ~ U[0.05, 0.3] and nuggets
1e-4 / 1e-6 / 1e-5, leaf in {64, 128, 256}, tolerance in {1e-2, 1e-4, 1e-6,
1e-8}, 136 Gaussian samples, ranks capped at 128. Problem j uses seeds
6000+j (parameters), 7000+j (points) and 8000+j (test matrix).

Usage: python tests/golden/make_rank_labels.py [problems] [processes]
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import hss_oracle as O  # noqa: E402
from oracle import rank_mlp as R  # noqa: E402

KERNELS = (("exponential", 1e-4), ("matern32", 1e-6), ("gaussian", 1e-5))


def problem(j):
    rng = np.random.default_rng(6000 + j)
    n = int(rng.choice([2048, 4096, 8192], p=[0.4, 0.4, 0.2]))
    leaf = int(rng.choice([64, 128, 256]))
    kname, nug = KERNELS[int(rng.integers(3))]
    length = float(rng.uniform(0.05, 0.3))
    tol = float(rng.choice([1e-2, 1e-4, 1e-6, 1e-8]))
    return n, leaf, kname, nug, length, tol


def run(j):
    n, leaf, kname, nug, length, tol = problem(j)
    X = synth.points_uniform(n, 3, 7000 + j)
    om = synth.test_matrix(n, 136, 8000 + j)
    F, ranks = R.labelled_nodes(X, leaf, O.Kernel(kname, length, nug), tol, om, 128)
    return j, F, ranks


if __name__ == "__main__":
    import multiprocessing as mp

    count = int(sys.argv[1]) if len(sys.argv) > 1 else 240
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    with mp.Pool(procs) as pool:
        res = sorted(pool.imap_unordered(run, range(count)), key=lambda r: r[0])
        feats = np.concatenate([r[1] for r in res])
        ranks = np.concatenate([r[2] for r in res])
        prob = np.concatenate([np.full(len(r[2]), r[0]) for r in res])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rank_labels.npz")
    np.savez_compressed(out, features=feats.astype(np.float32), ranks=ranks.astype(np.int32),
                        problem=prob.astype(np.int32))
    print(out, feats.shape, "rank histogram", np.bincount(np.minimum(ranks, 128) // 16))
