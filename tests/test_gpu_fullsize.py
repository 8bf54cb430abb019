"""Parity at the full sizes -- the 1024^3 / 1800-angle volume in the launch
configuration the benchmark times (chunks of 64 angles), and the
2048^2 x 512-slice slab with 900 angles (chunks of 32) -- on outputs the
oracle can compute one angle at a time, plus properties that hold at any
size.

The oracle's ray sums are slice-local, so it runs slab by slab (printing
progress) on the same complex64 volume the GPU sees."""

import sys
import time

import numpy as np
import pytest

from oracle import holo_oracle as O

pytestmark = pytest.mark.gpu
TOL = 1e-5
K_SAMPLE = 1317          # an angle that walks along x (131.7 degrees)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield workload_inputs("vol1024_a1800")
    torch.cuda.empty_cache()


def workload_inputs(name):
    import torch
    from paper_2407_20304_amd import holo, synth
    wl = synth.WORKLOADS[name]
    dev = torch.device("cuda:0")
    sd = lambda role: synth.seed_of(wl.config, role)
    say("full-size inputs", name)
    u = synth.ellipsoid_volume(wl.W, wl.H, sd(4), device=dev)
    q_np = synth.probe(wl.H, wl.W, sd(5))
    q = torch.from_numpy(q_np).to(dev)
    amp = synth.synthetic_amplitudes(wl.n_angles, 4, wl.H, wl.W, sd(9), device=dev)
    amp_ref = synth.synthetic_amplitudes(1, 1, wl.H, wl.W, sd(9) + 500, device=dev)[0, 0].contiguous()
    return holo, synth, wl, u, q, q_np, amp, amp_ref


def oracle_radon(u_np, theta, slab=128):
    H = u_np.shape[0]
    out = []
    for z0 in range(0, H, slab):
        t = time.time()
        out.append(O.radon(u_np[z0:z0 + slab], theta))
        say("  oracle ray sums, slices %d-%d: %.1f s" % (z0, z0 + slab, time.time() - t))
    return np.concatenate(out, axis=0)


def oracle_radon_T(h, theta, W, slab=128):
    H = h.shape[0]
    out = []
    for z0 in range(0, H, slab):
        t = time.time()
        out.append(O.radon_T(h[z0:z0 + slab], theta, W))
        say("  oracle transpose, slices %d-%d: %.1f s" % (z0, z0 + slab, time.time() - t))
    return np.concatenate(out, axis=0)


def one_angle_parity(inputs, k, slab):
    import torch
    holo, synth, wl, u, q, q_np, amp, amp_ref = inputs
    theta = float(wl.theta[k])
    # GPU: the benchmark-style plan (all angles, the workload's chunks) for
    # the forward field of angle k, and a one-angle plan for the full
    # gradient.
    plan = holo.Plan.for_workload(wl)
    v_gpu = plan.holo_fwd(u, q, k, k + 1).cpu().numpy()[0]
    plan.close()
    plan1 = holo.Plan(wl.H, wl.W, [theta], wl.mag_rel, wl.m0, wl.fresnel0, wl.kappa)
    F_gpu, gu_gpu, gq_gpu = plan1.holo_grad(u, q, amp[k:k + 1].contiguous(), amp_ref)
    F_gpu = F_gpu.item()
    gq_gpu = gq_gpu.cpu().numpy()
    u_np = u.cpu().numpy()
    gu_gpu = gu_gpu.cpu().numpy()
    plan1.close()
    torch.cuda.empty_cache()

    say("oracle, angle %d of %s" % (k, wl.name))
    p = oracle_radon(u_np, theta, slab)
    psi = np.exp(1j * wl.kappa * p)
    del p
    qc = q_np.astype(np.complex128)
    a_k = amp[k].cpu().numpy().astype(np.float64)
    a_ref = amp_ref.cpu().numpy().astype(np.float64)
    v_ref = O.holo2d_forward(psi, qc, wl.mag_rel, wl.m0, wl.fresnel0)
    for j in range(4):
        e = O.rel_err(v_gpu[j], v_ref[j])
        say("  forward plane %d rel err %.2e" % (j, e))
        assert e < TOL
    F_ref, g_psi, gq_ref = O.holo2d_gradient(psi, qc, a_k, a_ref, wl.mag_rel, wl.m0, wl.fresnel0)
    h = -1j * wl.kappa * np.conj(psi) * g_psi
    del u_np
    gu_ref = oracle_radon_T(h, theta, wl.W, slab)
    eF = abs(F_gpu - F_ref) / F_ref
    eq = O.rel_err(gq_gpu, gq_ref)
    eu = O.rel_err(gu_gpu, gu_ref)
    say("  F %.2e  g_q %.2e  g_u %.2e" % (eF, eq, eu))
    assert eF < TOL and eq < TOL and eu < TOL


def test_one_angle_forward_and_gradient_at_full_size(full):
    one_angle_parity(full, K_SAMPLE, 128)


def test_full_workload_invariants(full):
    import torch
    holo, synth, wl, u, q, q_np, amp, amp_ref = full
    say("full workload: probe-phase invariance and finite differences")
    plan = holo.Plan.for_workload(wl)
    F, gu, gq = plan.holo_grad(u, q, amp, amp_ref)
    F = F.item()
    # F(u, e^{i a} q) = F(u, q)  =>  Re<g_q, i q> = 0
    F2 = plan.holo_objective(u, q * np.exp(0.9j), amp, amp_ref).item()
    assert abs(F2 - F) / F < 1e-6, (F, F2)
    inv = torch.vdot(gq.flatten(), (1j * q).flatten()).real.item()
    assert abs(inv) < 1e-4 * gq.norm().item() * q.norm().item()
    # central differences along two seeded directions (single-precision
    # forward model: 1e-3 relative)
    gen = torch.Generator(device=u.device)
    gen.manual_seed(3006)
    for d in range(2):
        # random direction plus an equal-norm part along the gradient (see
        # the autograd test), steps of 1e-3 of the variables' size
        hu = torch.randn(u.shape, dtype=torch.complex64, device=u.device, generator=gen)
        hu = hu / hu.norm() + gu / gu.norm()
        hu *= 1e-3 * u.norm() / hu.norm()
        hq = torch.randn(q.shape, dtype=torch.complex64, device=u.device, generator=gen)
        hq = hq / hq.norm() + gq / gq.norm()
        hq *= 1e-3 * q.norm() / hq.norm()
        up, um, qp, qm = u + hu, u - hu, q + hq, q - hq
        Fp = plan.holo_objective(up, qp, amp, amp_ref).item()
        Fm = plan.holo_objective(um, qm, amp, amp_ref).item()
        fd = (Fp - Fm) / 2.0
        # the perturbation actually applied: u + h and u - h are rounded to
        # complex64, which keeps only ~1e-4 of h where |u| >> |h|
        an = 0.0
        for z0 in range(0, u.shape[0], 64):     # slabs keep the float64 temporaries small
            h_eff = (up[z0:z0 + 64].to(torch.complex128) - um[z0:z0 + 64].to(torch.complex128)) / 2
            an += torch.vdot(gu[z0:z0 + 64].flatten().to(torch.complex128), h_eff.flatten()).real.item()
        hq_eff = (qp.to(torch.complex128) - qm.to(torch.complex128)) / 2
        an += torch.vdot(gq.flatten().to(torch.complex128), hq_eff.flatten()).real.item()
        del up, um
        say("  direction %d: analytic %.6e fd %.6e" % (d, an, fd))
        assert abs(an - fd) / abs(fd) < 1e-3


@pytest.fixture(scope="module")
def slab():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield workload_inputs("slab2048x512_a900")
    torch.cuda.empty_cache()


def test_one_angle_forward_and_gradient_on_the_2048_slab(slab):
    # 42.4 degrees: a walk along y whose 2048-wide row windows split the
    # angle groups; 2048-point row transforms, 512-point column transforms
    one_angle_parity(slab, 212, 32)
