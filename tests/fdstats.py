"""Multiple-comparison test used by the finite-difference gradient checks."""
import math

import numpy as np


def holm_rejections(D: np.ndarray, alpha: float = 0.01) -> list:
    """Holm's step-down procedure over the columns of D (samples x
    hypotheses): two-sided one-sample Student t tests of mean zero at
    family-wise level alpha; returns the rejected columns."""
    from scipy import stats
    D = np.asarray(D, dtype=np.float64)
    S, m = D.shape
    se = D.std(axis=0, ddof=1) / math.sqrt(S)
    t = np.where(se > 0, D.mean(axis=0) / np.where(se > 0, se, 1.0), 0.0)
    p = 2.0 * stats.t.sf(np.abs(t), S - 1)
    out = []
    for rank, j in enumerate(np.argsort(p, kind="stable")):
        if p[j] > alpha / (m - rank):
            break
        out.append(int(j))
    return out
