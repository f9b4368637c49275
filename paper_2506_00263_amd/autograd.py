"""torch.autograd.Function over the transport library.

forward(Sigma_t, Sigma_s) uploads the multigroup cross sections of one
problem (mcx_set_xs), runs its histories (mcx_run) and returns the
normalised track-length tally T = (raw * 2^-S) / N (float64, on the device of
the inputs).  backward(dL/dT) calls the score-function replay
(mcx_backward), which returns dL/dSigma_t and dL/dSigma_s.  Torch provides
memory and streams; every transport step runs in the HIP library.

mcx_backward replays the handle's latest forward.  When anything has run on
the problem since this graph's forward (another forward, new cross sections,
an autotuner's calibration runs), backward first restores this forward's
cross sections and runs it again (same histories and keys, so the same
integers) before the replay; the handle's tallies then hold that forward.
"""
from __future__ import annotations

import torch

from . import mcx


class TransportFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma_t, sigma_s, problem: "mcx.Problem", index: int = 0, opts: dict | None = None):
        opts = dict(opts or {})
        problem.set_xs(index, sigma_t.detach().to(torch.float64).contiguous(),
                       sigma_s.detach().to(torch.float64).contiguous())
        stream = torch.cuda.current_stream(sigma_t.device) if sigma_t.is_cuda else None
        problem.run(stream=stream, **opts)
        info = problem.info(index)
        d = problem.descs[index]
        if sigma_t.is_cuda:
            raw = torch.empty(info["n_bins"], dtype=torch.int64, device=sigma_t.device)
            problem.tallies_into(index, raw)
        else:
            raw = torch.from_numpy(problem.tallies(index))
        n = opts.get("n") or (info["n_histories"] - opts.get("first", 0))
        ctx.problem, ctx.index = problem, index
        ctx.generation = problem.generation
        ctx.xs = (sigma_t.detach().to(torch.float64).contiguous().clone(),
                  sigma_s.detach().to(torch.float64).contiguous().clone())
        ctx.run_opts = {k: v for k, v in opts.items() if k != "stream"}
        ctx.opts = {k: v for k, v in opts.items() if k in ("sched", "decomp", "lookup", "waves_per_cu",
                                                                "stash_links", "block_size")}
        ctx.shape = sigma_t.shape
        # T = (raw * 2^-S) / N: an exact power-of-two scaling, then one division
        return raw.to(torch.float64) * (2.0 ** (-int(d["tally_scale_log2"]))) / float(n)

    @staticmethod
    def backward(ctx, grad_t):
        P = ctx.problem
        if P.generation != ctx.generation:
            # something else ran on the handle: redo this graph's forward
            P.set_xs(ctx.index, *ctx.xs)
            stream = torch.cuda.current_stream(ctx.xs[0].device) if ctx.xs[0].is_cuda else None
            P.run(stream=stream, **ctx.run_opts)
            ctx.generation = P.generation
        gt, gs = P.backward(grad_t.detach().contiguous(), problem=ctx.index, **ctx.opts)
        if not torch.is_tensor(gt):
            gt = torch.from_numpy(gt)
            gs = torch.from_numpy(gs)
        dev = grad_t.device
        return gt.to(dev).view(ctx.shape), gs.to(dev).view(ctx.shape), None, None, None


def transport(sigma_t, sigma_s, problem: "mcx.Problem", index: int = 0, **opts):
    """Normalised tally of problem `index` as a differentiable function of its
    [n_mat, n_grp] (or flat) Sigma_t and Sigma_s."""
    return TransportFn.apply(sigma_t, sigma_s, problem, index, opts)
