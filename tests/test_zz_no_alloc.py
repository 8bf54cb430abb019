"""holo2d_grad_noalloc (the batched gradient for callers that cannot
allocate: tables and workspace in the library's static device array)
against holo2d_grad with a caller workspace, through the C ABI: two calls in
a row, the second on a smaller batch, then the first batch again (each call
rewrites the shared array's tables and workspace)."""

import sys

import numpy as np
import pytest

from oracle import holo_oracle as O
from paper_2407_20304_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_20304_amd import holo
    holo.lib()


def batch_inputs(plan, seed0):
    """Evaluation point (roles 4/5) and oracle-simulated Poisson data of a
    truth (roles 1/2/3) for every instance of the plan."""
    import torch
    dev = torch.device("cuda:0")
    psi, q, amp, amp_ref = [], [], [], []
    for i, n in enumerate(plan.sizes):
        sd = lambda role: seed0 + role + 100 * i
        psi_t = synth.phase_object_2d(n, sd(1)).astype(np.complex128)
        q_t = synth.probe(n, n, sd(2)).astype(np.complex128)
        v = O.holo2d_forward(psi_t, q_t, synth.MAG_REL, synth.M0, synth.FRESNEL0)
        amp.append(synth.poisson_amplitude(np.abs(v) ** 2, sd(3)))
        amp_ref.append(synth.poisson_amplitude(
            np.abs(O.propagate(q_t, 1.0, synth.FRESNEL0)) ** 2, sd(3) + 50))
        psi.append(synth.phase_object_2d(n, sd(4)))
        q.append(synth.probe(n, n, sd(5)))
    return tuple(plan.pack(x, device=dev) for x in (psi, q, amp, amp_ref))


def compare(plan, inputs, tag):
    import torch
    psi, q, amp, amp_ref = inputs
    F0, gp0, gq0 = plan.holo2d_grad(psi, q, amp, amp_ref)
    F = torch.full((plan.n_inst,), float("nan"), dtype=torch.float64, device=psi.device)
    gp = torch.full_like(psi, float("nan"))
    gq = torch.full_like(q, float("nan"))
    plan.holo2d_grad_noalloc(psi, q, amp, amp_ref, F, gp, gq)
    torch.cuda.synchronize()
    eF = (F - F0).abs().max().item() / F0.abs().max().item()
    ep = O.rel_err(gp.cpu().numpy(), gp0.cpu().numpy())
    eq = O.rel_err(gq.cpu().numpy(), gq0.cpu().numpy())
    same = bool(torch.equal(F, F0) and torch.equal(gp, gp0) and torch.equal(gq, gq0))
    say("  %s: sizes %s, scratch %d bytes: F %.2e  g_psi %.2e  g_q %.2e  bitwise %s"
        % (tag, plan.sizes, plan.noalloc_bytes(), eF, ep, eq, same))
    assert eF < TOL and ep < TOL and eq < TOL
    assert same          # the same kernels on the same inputs


def test_noalloc_matches_workspace_call_on_consecutive_batches():
    from paper_2407_20304_amd import holo
    big = holo.Plan2D([256, 128, 192, 64, 512, 384], synth.MAG_REL, synth.M0, synth.FRESNEL0)
    small = holo.Plan2D([128, 64], synth.MAG_REL, synth.M0, synth.FRESNEL0)
    assert small.noalloc_bytes() < big.noalloc_bytes()
    in_big = batch_inputs(big, 7000)
    in_small = batch_inputs(small, 7500)
    compare(big, in_big, "first call")
    compare(small, in_small, "second call, smaller batch")
    compare(big, in_big, "third call, first batch again")
    big.close()
    small.close()
