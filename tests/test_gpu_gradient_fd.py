"""GPU: the score-function gradient against central finite differences.

On the lattice (1e6 histories), for the loss w . T (T the normalised mesh
tally), the replay backward's dL/dSigma_t and dL/dSigma_s are compared with
central differences of forward runs at Sigma (1 +- h) using common random
numbers (the same seed, so the same Philox streams).  Both estimate the
derivative of the expected loss; their difference is compared, over
independent seeds, with its own standard error.  With common random numbers
a step flips a few discrete collision outcomes, so the difference quotient's
variance grows like 1/(N h): h = 1e-4 is the step the method is specified
with, h = 1e-2 the one that gives the comparison power (standard errors
below the gradients themselves).
"""
import math

import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


@pytest.mark.parametrize("rel", [1e-4, 1e-2])
def test_score_function_matches_central_fd(mcx, rel):
    n = 1_000_000
    d0 = inputs.lattice_mg(n_histories=n)
    nb = inputs.n_bins(d0)
    w = np.random.default_rng(81).uniform(-1.0, 1.0, nb)
    scale = 2.0 ** -int(d0["tally_scale_log2"]) / n
    params = [0, 10, 24, 48]                     # (material, group) entries of the 7 x 7 tables
    st0 = np.asarray(d0["sigma_t"], dtype=np.float64)
    ss0 = np.asarray(d0["sigma_s"], dtype=np.float64)
    diffs_t, diffs_s = [], []
    for seed in range(1, 9):
        P = mcx.Problem(dict(d0, seed=seed))
        P.run(sched="async")
        gt, gs = P.backward(w, sched="async")

        def loss(st, ss):
            P.set_xs(0, st, ss)
            P.run(sched="async")
            return float(w @ (P.tallies().astype(np.float64) * scale))

        fd_t, fd_s = np.empty(len(params)), np.empty(len(params))
        for k, i in enumerate(params):
            for base, out, is_t in ((st0, fd_t, True), (ss0, fd_s, False)):
                step = rel * base[i]
                vals = []
                for sgn in (1.0, -1.0):
                    arr = base.copy()
                    arr[i] += sgn * step
                    vals.append(loss(arr, ss0) if is_t else loss(st0, arr))
                out[k] = (vals[0] - vals[1]) / (2.0 * step)
        P.set_xs(0, st0, ss0)
        diffs_t.append(gt[params] - fd_t)
        diffs_s.append(gs[params] - fd_s)
    for diffs in (np.array(diffs_t), np.array(diffs_s)):
        mean = diffs.mean(axis=0)
        se = diffs.std(axis=0, ddof=1) / math.sqrt(diffs.shape[0])
        assert np.all(np.abs(mean) < 4 * se + 1e-12), (mean, se)
