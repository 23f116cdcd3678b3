"""Tiny NumPy brute force of Algorithm 1 and eq. (2.7)/(2.8) -- TEST
INFRASTRUCTURE ONLY.

An independent second reading of the same definitions as ``apd_oracle.c``,
written with whole-array NumPy operations (the full N x J cost matrix is
formed, so it is for small instances only: N*J up to a few million).  It
cross-checks the C oracle.
"""
from __future__ import annotations

import numpy as np


def centres(inst) -> np.ndarray:
    """Pixel centres of the regular grid, eq. (2.6): y = lo + (k + 1/2) s,
    row-major with the last axis fastest."""
    axes = []
    for d in range(inst.dim):
        s = (inst.hi[d] - inst.lo[d]) / inst.grid[d]
        axes.append(inst.lo[d] + (np.arange(inst.grid[d]) + 0.5) * s)
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def cost_matrix(inst, w, x=None) -> np.ndarray:
    """C[i, j] = (y_j - x_i)^T A_i (y_j - x_i) - w_i (Algorithm 1)."""
    x = inst.x if x is None else x
    y = centres(inst)
    d = y[None, :, :] - x[:, None, :]                    # (N, J, D)
    Ad = np.einsum("nab,njb->nja", inst.A, d)            # (N, J, D)
    q = np.einsum("nja,nja->nj", d, Ad)
    return q - np.asarray(w)[:, None]


def assign(inst, w, x=None):
    C = cost_matrix(inst, w, x)
    lab = np.argmin(C, axis=0)           # first minimum = lowest index
    return lab.astype(np.int32), C


def evaluate(inst, w, x=None):
    """(g~, grad, counts) per eq. (2.7)-(2.8), summed cell by cell as the
    equation is written: sum_i (v_i - m_i|P|) w_i + sum_{H_j = i} |P| |y_j - x_i|^2."""
    lab, C = assign(inst, w, x)
    n = C.shape[0]
    P = float(np.prod([(inst.hi[d] - inst.lo[d]) / inst.grid[d] for d in range(inst.dim)]))
    w = np.asarray(w, dtype=np.float64)
    counts = np.bincount(lab, minlength=n)
    q = C + w[:, None]                   # the squared A-distances
    qsel = q[lab, np.arange(C.shape[1])]
    per_cell = np.bincount(lab, weights=qsel, minlength=n)
    g = float(np.sum((inst.v - counts * P) * w + P * per_cell))
    grad = inst.v - counts * P
    return g, grad, counts
