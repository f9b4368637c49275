"""GPU: torch.autograd.Function over the C ABI, and the autotuner."""
import numpy as np
import pytest

from paper_2506_00263_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_transport_fn_forward_backward(torch_gpu, oracle):
    torch = torch_gpu
    from paper_2506_00263_amd import mcx
    from paper_2506_00263_amd.autograd import transport
    d = inputs.lattice_mg(n_histories=5000)
    P = mcx.Problem(d)
    st = torch.tensor(d["sigma_t"], dtype=torch.float64, device="cuda").view(7, 7).requires_grad_(True)
    ss = torch.tensor(d["sigma_s"], dtype=torch.float64, device="cuda").view(7, 7).requires_grad_(True)
    T = transport(st, ss, P, sched="async")
    ref = oracle.run(d)
    assert np.array_equal(P.tallies(), ref["tally"])              # the exact quantity
    expect = ref["tally"].astype(np.float64) * 2.0 ** -32 / 5000
    # torch divides by a scalar through its reciprocal: allow 1 ulp
    np.testing.assert_allclose(T.detach().cpu().numpy(), expect, rtol=2.3e-16, atol=0)
    w = torch.tensor(np.random.default_rng(3).normal(size=T.numel()), dtype=torch.float64, device="cuda")
    loss = (w * T).sum()
    loss.backward()
    rb = oracle.backward(d, w.cpu().numpy())
    assert np.array_equal(st.grad.cpu().numpy().ravel(), rb["grad_sigma_t"])
    assert np.array_equal(ss.grad.cpu().numpy().ravel(), rb["grad_sigma_s"])


def test_transport_fn_new_parameters(torch_gpu, oracle):
    torch = torch_gpu
    from paper_2506_00263_amd import mcx
    from paper_2506_00263_amd.autograd import transport
    d = inputs.cfg1_box(4000)
    P = mcx.Problem(d)
    st = torch.tensor(d["sigma_t"], dtype=torch.float64, device="cuda") * 1.1
    ss = torch.tensor(d["sigma_s"], dtype=torch.float64, device="cuda") * 0.9
    T = transport(st, ss, P, sched="stack")
    d2 = dict(d, sigma_t=st.cpu().numpy(), sigma_s=ss.cpu().numpy())
    ref = oracle.run(d2)
    assert np.array_equal(P.tallies(), ref["tally"])
    np.testing.assert_allclose(T.cpu().numpy(), ref["tally"] * 2.0 ** -32 / 4000, rtol=2.3e-16, atol=0)


def test_autotune_invariant(torch_gpu, oracle):
    from paper_2506_00263_amd import autotune, mcx
    d = inputs.cfg2_lattice(20000)
    P = mcx.Problem(d)
    for sched, decomp in (("async", "fused"), ("stack", "fused"), ("async", "split")):
        best = autotune.tune(P, sched=sched, decomp=decomp, use_cache=False, reps=1)
        P.run(sched=sched, decomp=decomp, **best)
        assert np.array_equal(P.tallies(), oracle.run(d)["tally"])


def test_backward_after_another_forward(torch_gpu, oracle):
    # two forwards on one handle (the second with other cross sections and
    # another history range), then backward through the first graph: its
    # gradient must be the first forward's
    torch = torch_gpu
    from paper_2506_00263_amd import autotune, mcx
    from paper_2506_00263_amd.autograd import transport
    d = inputs.lattice_mg(n_histories=6000)
    P = mcx.Problem(d)
    st = torch.tensor(d["sigma_t"], dtype=torch.float64, device="cuda").view(7, 7).requires_grad_(True)
    ss = torch.tensor(d["sigma_s"], dtype=torch.float64, device="cuda").view(7, 7).requires_grad_(True)
    T1 = transport(st, ss, P, sched="async")
    T2 = transport(st.detach() * 1.05, ss.detach() * 0.95, P, sched="stack", first=1000, n=2000)
    autotune.tune(P, sched="async", use_cache=False, reps=1)       # calibration runs on the handle
    w = torch.tensor(np.random.default_rng(8).normal(size=T1.numel()), dtype=torch.float64, device="cuda")
    (w * T1).sum().backward()
    rb = oracle.backward(d, w.cpu().numpy())
    assert np.array_equal(st.grad.cpu().numpy().ravel(), rb["grad_sigma_t"])
    assert np.array_equal(ss.grad.cpu().numpy().ravel(), rb["grad_sigma_s"])
    assert np.array_equal(P.tallies(), oracle.run(d)["tally"])    # the first forward again
    del T2
