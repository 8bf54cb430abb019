"""hipGraph capture of the library calls: replays (with eager work and
synchronisations in between) reproduce the eager results bit for bit."""

import sys

import numpy as np
import pytest

from tests import problems as PB
from paper_2407_20304_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_joint_gradient_graph_replay():
    import torch
    say("graph capture: joint gradient 64^3, 12 angles")
    p = PB.make_problem(64, 64, 12, config=0, shifts=True, chunk=5)
    u, q, amp, amp_ref = PB.to_gpu(p)
    plan = PB.gpu_plan(p)
    F = torch.empty(1, dtype=torch.float64, device="cuda")
    gu, gq = torch.empty_like(u), torch.empty_like(q)
    plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=gu, g_q=gq)   # eager (also uploads tables)
    torch.cuda.synchronize()
    ref = (F.clone(), gu.clone(), gq.clone())
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=gu, g_q=gq)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(3):
        F.zero_(), gu.zero_(), gq.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert F.item() == ref[0].item(), r
        assert bool((gu == ref[1]).all()) and bool((gq == ref[2]).all()), r
        # eager work between replays
        plan.holo_objective(u, q, amp, amp_ref)
        torch.cuda.synchronize()


def test_overlapped_forward_is_bitwise_the_serial_one_and_replays():
    """The overlapped forward (the next chunk's ray sums on the library's
    second stream) computes the same gradient bit for bit, eagerly and as a
    captured graph (the fork and join through events are part of the
    capture), over several chunks, with and without object shifts."""
    import torch
    for shifts in (False, True):
        say("overlapped forward: 64^3, 12 angles, chunk 3, shifts", shifts)
        p = PB.make_problem(64, 64, 12, config=0, shifts=shifts, chunk=3)
        u, q, amp, amp_ref = PB.to_gpu(p)
        plan = PB.gpu_plan(p)
        F = torch.empty(1, dtype=torch.float64, device="cuda")
        gu, gq = torch.empty_like(u), torch.empty_like(q)
        plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=gu, g_q=gq)
        torch.cuda.synchronize()
        ref = (F.clone(), gu.clone(), gq.clone())
        v_ref = plan.holo_fwd(u, q).clone()
        w = torch.randn_like(v_ref)
        a_ref = [t.clone() for t in plan.holo_adj(u, q, w)]
        F1_ref = plan.holo_objective(u, q, amp, amp_ref).clone()
        plan.set_tile("overlap", 1)
        # the forward fields, the adjoint, the objective and the one-sided
        # gradients take the overlapped path too
        assert bool((plan.holo_fwd(u, q) == v_ref).all())
        assert all(bool((x == y).all()) for x, y in zip(plan.holo_adj(u, q, w), a_ref))
        assert bool((plan.holo_objective(u, q, amp, amp_ref) == F1_ref).all())
        _, gu1 = plan.holo_grad_object(u, q, amp, amp_ref)
        _, gq1 = plan.holo_grad_probe(u, q, amp, amp_ref)
        assert bool((gu1 == ref[1]).all()) and bool((gq1 == ref[2]).all())
        for r in range(2):
            F.zero_(), gu.zero_(), gq.zero_()
            plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=gu, g_q=gq)
            torch.cuda.synchronize()
            assert F.item() == ref[0].item(), r
            assert bool((gu == ref[1]).all()) and bool((gq == ref[2]).all()), r
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                plan.holo_grad(u, q, amp, amp_ref, F=F, g_u=gu, g_q=gq)
        torch.cuda.current_stream().wait_stream(s)
        for r in range(3):
            F.zero_(), gu.zero_(), gq.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert F.item() == ref[0].item(), r
            assert bool((gu == ref[1]).all()) and bool((gq == ref[2]).all()), r
            plan.holo_objective(u, q, amp, amp_ref)
            torch.cuda.synchronize()
        del g
        plan.close()


def test_batch_gradient_graph_replay():
    import torch
    from paper_2407_20304_amd import holo
    say("graph capture: batched retrievals")
    sizes = [256, 128, 192, 64]
    rng = np.random.default_rng(3)
    plan = holo.Plan2D(sizes, synth.MAG_REL, synth.M0, synth.FRESNEL0)
    psi = plan.pack([synth.phase_object_2d(n, 10 + i) for i, n in enumerate(sizes)], device="cuda")
    q = plan.pack([synth.probe(n, n, 20 + i) for i, n in enumerate(sizes)], device="cuda")
    amp = plan.pack([rng.uniform(0.5, 1.5, (4, n, n)).astype(np.float32) for n in sizes], device="cuda")
    amp_ref = plan.pack([rng.uniform(0.5, 1.5, (n, n)).astype(np.float32) for n in sizes], device="cuda")
    F = torch.empty(len(sizes), dtype=torch.float64, device="cuda")
    gp, gq = torch.empty_like(psi), torch.empty_like(q)
    plan.holo2d_grad(psi, q, amp, amp_ref, F=F, g_psi=gp, g_q=gq)
    torch.cuda.synchronize()
    ref = (F.clone(), gp.clone(), gq.clone())
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.holo2d_grad(psi, q, amp, amp_ref, F=F, g_psi=gp, g_q=gq)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(3):
        F.zero_(), gp.zero_(), gq.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert bool((F == ref[0]).all()) and bool((gp == ref[1]).all()) and bool((gq == ref[2]).all()), r
        plan.holo2d_objective(psi, q, amp, amp_ref)
        torch.cuda.synchronize()
