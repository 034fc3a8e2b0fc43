"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np


def rel_err_per_power(Y, Yref):
    """max over right-hand sides of ||Y_k - Yref_k||_2 / ||Yref_k||_2, per power k.

    Falls back to the absolute norm where the reference column is zero.
    """
    Y = np.asarray(Y, dtype=np.float64)
    Yref = np.asarray(Yref, dtype=np.float64)
    assert Y.shape == Yref.shape, (Y.shape, Yref.shape)
    p = Y.shape[0]
    out = np.zeros(p)
    for k in range(p):
        d = np.linalg.norm((Y[k] - Yref[k]).reshape(Y.shape[1], -1), axis=0)
        r = np.linalg.norm(Yref[k].reshape(Y.shape[1], -1), axis=0)
        out[k] = np.max(np.where(r > 0, d / np.where(r > 0, r, 1.0), d)) if d.size else 0.0
    return out


def read_golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows
