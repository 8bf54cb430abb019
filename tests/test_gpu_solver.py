"""Parity of the solver entry points (initial probe, Dai-Yuan conjugate
gradients on the joint (u, q) objective) with the FP64 oracle.

The conjugate-gradient case starts from u = 0 and the back-propagated
reference, with an initial step whose line search halves 1, 0, 2 and 0 times
in the oracle.  Every trial of the oracle's line search is recorded and the
test first checks that each accept/reject decision has a relative margin of
at least 1e-2, far above the single-precision objective's error (~1e-6), so
the HIP path must take the same decisions; then the objective history, the
accepted steps and the final iterate are compared."""

import sys

import numpy as np
import pytest

from oracle import holo_oracle as O
from tests import problems as PB

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


@pytest.mark.parametrize("H,W", [(64, 64), (128, 256), (384, 128)])
def test_probe_init_parity(H, W):
    import torch
    say("probe init", H, W)
    from paper_2407_20304_amd import holo, synth
    amp_ref = np.abs(synth.probe(H, W, 31)).astype(np.float32) + 0.5
    plan = holo.Plan(H, W, [0.0, 1.0], synth.MAG_REL, synth.M0, synth.FRESNEL0, synth.KAPPA)
    q = plan.holo_probe_init(torch.from_numpy(amp_ref).cuda()).cpu().numpy()
    ref = O.probe_init(amp_ref.astype(np.float64), synth.FRESNEL0)
    assert O.rel_err(q, ref) < TOL, O.rel_err(q, ref)


CG = dict(H=64, W=64, n_angles=12, config=0, shifts=True, chunk=5)
CG_ITERS = 4
CG_STEP0 = 7e-11


@pytest.fixture(scope="module")
def cg_case():
    p = PB.make_problem(**CG)
    amp = p.amp.astype(np.float64)
    amp_ref = p.amp_ref.astype(np.float64)
    q0 = O.probe_init(amp_ref, p.geom.fresnel0)
    u0 = np.zeros((p.geom.H, p.geom.W, p.geom.W), np.complex128)
    trials = []
    f = lambda x: O.objective(x[0], x[1], amp, amp_ref, p.geom)

    def grad(x):
        F, gu, gq = O.gradient(x[0], x[1], amp, amp_ref, p.geom)
        return F, (gu, gq)

    def search(f_, x, eta, F, gamma_try):
        seen = []

        def f_rec(xt):
            Ft = f_(xt)
            seen.append(Ft)
            return Ft
        out = O.backtracking(f_rec, x, eta, F, gamma_try)
        trials.append((F, seen))
        return out
    x, hist, steps, halv = O.cg_dai_yuan(f, grad, (u0, q0), CG_ITERS, CG_STEP0,
                                         line_search=search)
    return p, u0, q0, x, hist, steps, halv, trials


def test_cg_oracle_decisions_have_margin(cg_case):
    *_, halv, trials = cg_case
    assert len(trials) == CG_ITERS
    for F, seen in trials:
        for Ft in seen:
            assert np.isfinite(Ft) and abs(Ft - F) / F > 1e-2, (F, seen)
    # the case exercises rejected trials and first-trial acceptances
    assert min(halv) == 0 and max(halv) >= 2 and 31 not in halv


def test_cg_parity(cg_case):
    import torch
    p, u0, q0, (u_or, q_or), hist, steps, halv, _ = cg_case
    say("CG parity 64^3, 12 angles, shifts, chunk 5, %d iterations" % CG_ITERS)
    plan = PB.gpu_plan(p)
    _, _, amp, amp_ref = PB.to_gpu(p)
    q_gpu0 = plan.holo_probe_init(amp_ref)
    assert O.rel_err(q_gpu0.cpu().numpy(), q0) < TOL
    u_gpu0 = torch.zeros((p.geom.H, p.geom.W, p.geom.W), dtype=torch.complex64, device="cuda")
    u, q, F_hist, st, hv = plan.holo_cg(u_gpu0, q_gpu0, amp, amp_ref, CG_ITERS, CG_STEP0)
    # the inputs are not touched unless in_place
    assert not torch.any(u_gpu0 != 0)
    say("  F_hist", list(F_hist), "oracle", hist)
    assert list(hv) == list(halv)
    assert list(st) == list(steps)
    for a, b in zip(F_hist, hist):
        assert abs(a - b) / b < TOL, (a, b)
    e_u = O.rel_err(u.cpu().numpy(), u_or)
    e_q = O.rel_err(q.cpu().numpy(), q_or)
    say("  rel err u %.3e q %.3e" % (e_u, e_q))
    assert e_u < TOL and e_q < TOL


def test_cg_zero_iterations_and_in_place(cg_case):
    import torch
    p, *_ = cg_case
    say("CG iters 0, in place")
    plan = PB.gpu_plan(p)
    u, q, amp, amp_ref = PB.to_gpu(p)
    u_in, q_in = u.clone(), q.clone()
    u2, q2, F_hist, st, hv = plan.holo_cg(u, q, amp, amp_ref, 0, 1e-3, in_place=True)
    assert u2 is u and q2 is q and len(F_hist) == 1 and len(st) == 0 and len(hv) == 0
    assert torch.equal(u, u_in) and torch.equal(q, q_in)
    F_ref = O.objective(PB.c128(p.u), PB.c128(p.q), p.amp.astype(np.float64),
                        p.amp_ref.astype(np.float64), p.geom)
    assert abs(F_hist[0] - F_ref) / F_ref < TOL


def test_cg_without_an_accepted_step_keeps_the_point(cg_case):
    """One NaN amplitude makes every objective NaN, so no trial passes the
    line search's test: each step is 0, each search reports 31 halvings and
    the point stays (bitwise)."""
    import torch
    p, *_ = cg_case
    say("CG no accepted step")
    plan = PB.gpu_plan(p)
    u, q, amp, amp_ref = PB.to_gpu(p)
    amp[3, 1, 7, 9] = float("nan")
    u2, q2, F_hist, st, hv = plan.holo_cg(u, q, amp, amp_ref, 2, 1e-10)
    assert list(hv) == [31, 31] and list(st) == [0.0, 0.0]
    assert np.all(np.isnan(F_hist))
    assert torch.equal(u2, u) and torch.equal(q2, q)
