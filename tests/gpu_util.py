"""Helpers for the GPU tests: oracle HSS objects to binding dicts and back."""
import numpy as np


def oracle_to_dict(h, perm=None):
    return dict(n=h.n, levels=h.levels, ranges=h.ranges, rank=h.rank, D=h.D, U=h.U, E=h.E, S=h.S, perm=perm)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    """Elementwise gate: max |a - b| / max |b| (a few wrong entries cannot hide
    under a normwise difference)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
