"""Oracle for the rest of a training iteration (TEST INFRASTRUCTURE ONLY).

* Grid total variation of Eq. 9: the paper names the term without a formula
  or weight; this is the K-Planes form the kernels implement (for every plane
  of every scale, the mean squared neighbour difference along each of the
  plane's two axes, summed), written out directly in FP64 numpy.
* Adam (Kingma & Ba, "Adam: A Method for Stochastic Optimization"): the
  published update with bias correction, FP64 numpy.
"""
from __future__ import annotations

import numpy as np


def tv_loss(planes, weight: float = 1.0):
    """planes: list over scales of six arrays [n_b][n_a][F].  Returns the
    weighted TV value and its gradient (same nesting)."""
    total = 0.0
    grads = []
    for lv in planes:
        gl = []
        for R in lv:
            R = np.asarray(R, np.float64)
            da = R[:, 1:, :] - R[:, :-1, :]          # along a (columns)
            db = R[1:, :, :] - R[:-1, :, :]          # along b (rows)
            total += (da ** 2).mean() + (db ** 2).mean()
            g = np.zeros_like(R)
            g[:, 1:, :] += 2.0 * da / da.size
            g[:, :-1, :] -= 2.0 * da / da.size
            g[1:, :, :] += 2.0 * db / db.size
            g[:-1, :, :] -= 2.0 * db / db.size
            gl.append(weight * g)
        grads.append(gl)
    return weight * total, grads


def adam(p, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (step >= 1); returns the new (p, m, v)."""
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
