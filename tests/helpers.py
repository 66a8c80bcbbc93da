"""Shared test helpers: error metrics and layout conversion between the
oracle's [T, ...] arrays and the library's structure-of-arrays layout."""
import numpy as np


def rel_l2(x, ref):
    """The paper's error metric (Sec. 3.1): root-mean-squared difference
    normalised by the root-mean-squared reference value."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / den) if den > 0 else float(np.linalg.norm(x))


def to_np(t):
    return t.detach().cpu().numpy()
