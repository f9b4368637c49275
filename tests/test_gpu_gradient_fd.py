"""GPU: score-function gradients through autograd against central finite
differences with common random numbers, on the 7 x 7 material-group lattice
(1e6 histories), for all 98 parameters (Sigma_t and Sigma_s of every
material and group).

Both sides estimate the derivative of an expected loss: the replay backward
through TransportFn, and the difference quotient of forward runs at
Sigma (1 +- h) that reuse the seed (the same Philox streams).  Their
per-seed difference is compared, over independent seeds, with its own
standard error by Student t tests, Holm-corrected over the 98 parameters at a
family-wise level of 1 %.

The target loss sum_b (T_b - tau_b)^2, tau_b = T_b(Sigma_0) (0.9 + 0.2 xi_b),
is taken at the expected tally: with 1e6 histories spread over 364140 bins
a bin's estimate is mostly noise, so the plug-in loss of one run has
expectation sum (E T - tau)^2 + sum Var T, and its autograd gradient
2 (T - tau) . dT and the difference quotient then differ in expectation by
(1/N) sum_b d E[f_b^2] / d Sigma (f_b one history's score in bin b): about
a factor 2 on this lattice.  The product of two independent runs,
sum (T1 - tau)(T2 - tau), is an unbiased estimate of the loss at E T; its
gradient through autograd and its difference quotient estimate the same
derivative.  That gradient is a zero-mean random combination of the bins, so
many parameters have gradients far below the noise: this test has little
power, and the positive-weight loss below supplies it (standard error below
a quarter of |gradient| for every parameter, at both steps).

With common random numbers a step flips a few discrete outcomes (collision
or surface, absorption or scatter), so the quotient's variance grows like
1/(N h): h = 1e-4 is the step the method is specified with and needs about
120 seeds for that bound, h = 1e-2 needs a few.
"""
import math

import numpy as np
import pytest

from fdstats import holm_rejections
from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu

N = 1_000_000


@pytest.fixture(scope="module")
def mcx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_00263_amd import mcx as M
    M.lib()
    return M


@pytest.fixture(scope="module")
def lattice():
    d0 = inputs.cfg4_lattice_grad(N)
    st0 = np.asarray(d0["sigma_t"], np.float64)
    ss0 = np.asarray(d0["sigma_s"], np.float64)
    return d0, st0, ss0, 2.0 ** -int(d0["tally_scale_log2"]) / N


def _perturbed(st0, ss0, k, rel, sgn):
    st, ss = st0.copy(), ss0.copy()
    arr = st if k < st0.size else ss
    i = k % st0.size
    step = rel * arr.flat[i]
    arr.flat[i] += sgn * step
    return st, ss, step


def _raw(P, st, ss):
    P.set_xs(0, st, ss)
    P.run(sched="async")
    return P.tallies()


@pytest.mark.parametrize("rel,seeds", [(1e-4, 24), (1e-2, 24)])
def test_cfg4_loss_through_autograd_matches_central_fd(mcx, lattice, rel, seeds):
    import torch
    from paper_2506_00263_amd.autograd import transport
    d0, st0, ss0, scale = lattice
    P0 = mcx.Problem(d0)
    P0.run(sched="async")
    tau = inputs.target_tally(P0.tallies().astype(np.float64) * scale)
    tau_t = torch.tensor(tau, device="cuda")
    npar = 2 * st0.size
    sf, fd = [], []
    for seed in range(1, seeds + 1):
        Ps = [mcx.Problem(dict(d0, seed=seed)), mcx.Problem(dict(d0, seed=100_000 + seed))]
        st = torch.tensor(st0, device="cuda", requires_grad=True)
        ss = torch.tensor(ss0, device="cuda", requires_grad=True)
        T1 = transport(st, ss, Ps[0], sched="async")
        T2 = transport(st, ss, Ps[1], sched="async")
        loss = ((T1 - tau_t) * (T2 - tau_t)).sum()
        loss.backward()
        sf.append(np.concatenate([st.grad.cpu().numpy().ravel(), ss.grad.cpu().numpy().ravel()]))
        q = np.empty(npar)
        for k in range(npar):
            o = {}
            for sgn in (1.0, -1.0):
                a, b, step = _perturbed(st0, ss0, k, rel, sgn)
                for r in (0, 1):
                    o[r, sgn] = _raw(Ps[r], a, b)
            # L+ - L- = sum (T1+ - T1-)(T2+ - tau) + (T1- - tau)(T2+ - T2-), from
            # exact integer differences
            d1 = (o[0, 1.0] - o[0, -1.0]).astype(np.float64) * scale
            d2 = (o[1, 1.0] - o[1, -1.0]).astype(np.float64) * scale
            q[k] = (float(d1 @ (o[1, 1.0] * scale - tau)) + float((o[0, -1.0] * scale - tau) @ d2)) / (2.0 * step)
        fd.append(q)
    sf, fd = np.array(sf), np.array(fd)
    D = sf - fd
    rejected = holm_rejections(D)
    se = D.std(axis=0, ddof=1) / math.sqrt(seeds)
    powered = float(np.mean(se < np.abs(sf.mean(axis=0)) / 4))
    print(f"cfg4 rel={rel:g}: {seeds} seeds, SE < |grad|/4 for {powered:.0%} of the 98 parameters, "
          f"Holm rejections {rejected}")
    assert rejected == [], (rejected, D.mean(axis=0)[rejected], se[rejected])


@pytest.mark.parametrize("rel,seeds", [(1e-2, 8), (1e-4, 128)])
def test_all_parameters_with_power(mcx, lattice, rel, seeds):
    # a loss with a strong gradient in every parameter: positive bin weights
    import torch
    from paper_2506_00263_amd.autograd import transport
    d0, st0, ss0, scale = lattice
    nb = inputs.n_bins(d0)
    w = 1.0 + np.random.default_rng(5).random(nb)
    w_t = torch.tensor(w, device="cuda")
    npar = 2 * st0.size
    sf, fd = [], []
    for seed in range(1, seeds + 1):
        P = mcx.Problem(dict(d0, seed=seed))
        st = torch.tensor(st0, device="cuda", requires_grad=True)
        ss = torch.tensor(ss0, device="cuda", requires_grad=True)
        loss = (w_t * transport(st, ss, P, sched="async")).sum()
        loss.backward()
        sf.append(np.concatenate([st.grad.cpu().numpy().ravel(), ss.grad.cpu().numpy().ravel()]))
        q = np.empty(npar)
        for k in range(npar):
            a, b, step = _perturbed(st0, ss0, k, rel, 1.0)
            hi = _raw(P, a, b)
            a, b, step = _perturbed(st0, ss0, k, rel, -1.0)
            lo = _raw(P, a, b)
            q[k] = float(w @ ((hi - lo).astype(np.float64) * scale)) / (2.0 * step)
        fd.append(q)
    sf, fd = np.array(sf), np.array(fd)
    D = sf - fd
    se = D.std(axis=0, ddof=1) / math.sqrt(seeds)
    g = np.abs(sf.mean(axis=0))
    powered = se < g / 4
    print(f"power rel={rel:g}: {seeds} seeds, SE < |grad|/4 for {powered.sum()} of 98, "
          f"largest SE/|grad| {float((se / g).max()):.3f}")
    assert powered.mean() >= 0.95, np.argsort(-(se / g))[:5]
    rejected = holm_rejections(D)
    assert rejected == [], (rejected, D.mean(axis=0)[rejected], se[rejected])
    # the test can see an error of a quarter of the gradient
    assert len(holm_rejections(sf * 0.75 - fd)) > 0
