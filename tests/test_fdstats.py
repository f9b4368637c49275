"""Holm's procedure as used by the finite-difference gradient checks."""
import numpy as np

from fdstats import holm_rejections


def test_no_rejection_under_the_null():
    rng = np.random.default_rng(0)
    hits = sum(len(holm_rejections(rng.normal(size=(24, 98)))) > 0 for _ in range(200))
    assert hits <= 8                      # family-wise level 1 %: about 2 of 200


def test_rejects_shifted_columns_only():
    rng = np.random.default_rng(1)
    D = rng.normal(size=(40, 98))
    D[:, 7] += 1.5
    D[:, 50] -= 2.0
    assert sorted(holm_rejections(D)) == [7, 50]


def test_step_down_thresholds():
    # p-values just below alpha/m, alpha/(m-1), ... are all rejected; one just
    # above its threshold stops the procedure
    from scipy import stats
    S, m = 30, 5
    targets = [0.01 / 5 * 0.9, 0.01 / 4 * 0.9, 0.01 / 3 * 1.1, 0.5, 0.9]
    cols = []
    for k, p in enumerate(targets):
        z = np.random.default_rng(k).normal(size=S)
        z = (z - z.mean()) / z.std(ddof=1) * np.sqrt(S)     # mean 0, standard error 1
        cols.append(z + stats.t.isf(p / 2, S - 1))          # t statistic with p-value p
    D = np.array(cols).T
    assert holm_rejections(D) == [0, 1]
