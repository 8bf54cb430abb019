"""Parity with the FP64 oracle at the workloads' own shapes and launch
configurations, through the C ABI:

* many angles: 64^3 with 360 angles in chunks of 64, so the transpose
  kernel refills its per-angle set-up windows and flushes its angle
  partials many times (it keeps 64 angles of set-up per window);
* the 256^3 / 360-angle workload through the autograd function, in full;
* the 1024^3 / 1800-angle workload and the 2048^2 x 512 / 900-angle slab on
  their strided 64-angle subsets {floor(i N_theta / 64)}, run by a 64-angle
  plan with the workload's chunking (64 and 32 angles): F and g_q in full,
  g_u on three 16-slice slabs (bottom, middle, top) -- the oracle's
  transpose is slice-local, so a slab of g_u needs only that slab of the
  sinogram;
* a zero field: a strongly absorbing volume makes psi = 0 exactly (on both
  sides), so every frame of the unmagnified plane is exactly zero and the
  residual's |v| = 0 case (v/|v| := 0) runs on all its pixels.

Every comparison checks relative L2 and max-abs/max error (tests/problems.py).
The oracle's ray sums here are the C loops of oracle/joseph.c and the frame
stage runs on a thread pool; the comparisons print their progress."""

import sys
import time

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
    O._joseph()          # the oracle's C part must be built too


def test_many_angles_transpose_windows():
    # 360 angles > 2 x 64: the transpose reuses both set-up windows several
    # times and flushes 32-angle partials 12 times per voxel
    say("grad parity 64^3, 360 angles, chunk 64")
    t = time.time()
    p = PB.make_problem(64, 64, 360, config=0, chunk=64, threads=PB.oracle_threads())
    u, q, amp, amp_ref = PB.to_gpu(p)
    plan = PB.gpu_plan(p)
    F, gu, gq = plan.holo_grad(u, q, amp, amp_ref)
    F0, gu0, gq0 = PB.oracle_grad_many(p)
    say("  oracle %.1f s" % (time.time() - t))
    PB.assert_close_scalar(F.item(), F0)
    PB.assert_close(gu.cpu().numpy(), gu0, "g_u")
    PB.assert_close(gq.cpu().numpy(), gq0, "g_q")


def test_vol256_a360_autograd_against_oracle():
    # the 256^3 / 360-angle workload: objective and both gradients through
    # the torch.autograd.Function, data from the oracle's forward model at
    # the truth (Poisson, 1e4 photons), evaluated at an independent draw
    import torch
    from paper_2407_20304_amd import holo, synth
    wl = synth.WORKLOADS["vol256_a360"]
    say("vol256_a360 autograd vs oracle")
    t = time.time()
    p = PB.make_problem(wl.H, wl.W, wl.n_angles, config=wl.config, chunk=wl.chunk,
                        threads=PB.oracle_threads())
    say("  data %.1f s" % (time.time() - t))
    u, q, amp, amp_ref = PB.to_gpu(p)
    plan = PB.gpu_plan(p)
    ur = u.clone().requires_grad_(True)
    qr = q.clone().requires_grad_(True)
    F = holo.holo_loss(ur, qr, amp, amp_ref, plan)
    F.backward()
    torch.cuda.synchronize()
    t = time.time()
    F0, gu0, gq0 = PB.oracle_grad_many(p)
    say("  oracle %.1f s" % (time.time() - t))
    PB.assert_close_scalar(F.item(), F0)
    PB.assert_close(ur.grad.cpu().numpy(), gu0, "g_u")
    PB.assert_close(qr.grad.cpu().numpy(), gq0, "g_q")


SLAB = 16


def strided_subset_parity(name):
    import torch
    from paper_2407_20304_amd import holo, synth
    wl = synth.WORKLOADS[name]
    ks = wl.subset(64)
    theta = wl.theta[ks]
    dev = torch.device("cuda:0")
    sd = lambda role: synth.seed_of(wl.config, role)
    say("%s: strided 64-angle subset, chunk %d" % (name, wl.chunk))
    u = synth.ellipsoid_volume(wl.W, wl.H, sd(4), device=dev)
    q_np = synth.probe(wl.H, wl.W, sd(5))
    q = torch.from_numpy(q_np).to(dev)
    amp = synth.synthetic_amplitudes(64, 4, wl.H, wl.W, sd(9) + 64, device=dev)
    amp_ref = synth.synthetic_amplitudes(1, 1, wl.H, wl.W, sd(9) + 500, device=dev)[0, 0].contiguous()
    plan = holo.Plan.for_workload(wl, theta=theta)
    F, gu, gq = plan.holo_grad(u, q, amp, amp_ref)
    torch.cuda.synchronize()
    slabs = [(0, SLAB), (wl.H // 2 - SLAB // 2, wl.H // 2 + SLAB // 2), (wl.H - SLAB, wl.H)]
    gu_slabs = [gu[z0:z1].cpu().numpy() for z0, z1 in slabs]
    F, gq = F.item(), gq.cpu().numpy()
    u_np = u.cpu().numpy()
    amp_np = amp.cpu().numpy().astype(np.float64)
    amp_ref_np = amp_ref.cpu().numpy().astype(np.float64)
    plan.close()
    del u, gu, amp, amp_ref, plan
    torch.cuda.empty_cache()

    geom = O.Geometry(H=wl.H, W=wl.W, theta=theta, mag_rel=wl.mag_rel, m0=wl.m0,
                      fresnel0=wl.fresnel0, kappa=wl.kappa)
    t = time.time()
    F0, h, gq0 = O.gradient_projection_domain(
        u_np, q_np.astype(np.complex128), amp_np, amp_ref_np, geom, threads=PB.oracle_threads(),
        progress=lambda m: say("  oracle: %s (%.1f s)" % (m, time.time() - t)))
    say("  oracle forward + frames %.1f s" % (time.time() - t))
    del u_np
    PB.assert_close_scalar(F, F0)
    PB.assert_close(gq, gq0, "g_q")
    for (z0, z1), g in zip(slabs, gu_slabs):
        t = time.time()
        ref = O.radon_T_set(np.ascontiguousarray(h[:, z0:z1]), theta, wl.W)
        say("  oracle transpose, slices %d-%d: %.1f s" % (z0, z1, time.time() - t))
        PB.assert_close(g, ref, "g_u slices %d-%d" % (z0, z1))


@pytest.mark.timeout(900)
def test_vol1024_a1800_strided_subset():
    strided_subset_parity("vol1024_a1800")


@pytest.mark.timeout(900)
def test_slab2048x512_a900_strided_subset():
    strided_subset_parity("slab2048x512_a900")


def test_zero_field_residual_case():
    # u = delta + i (large beta): kappa Im(R u) is thousands of radians of
    # absorption on every ray, so exp underflows to psi = 0 exactly in float
    # and in double.  Plane 0 (m~ = 1, no shift) samples psi on the grid, so
    # phi = 1 + (psi - 1) = 0 and v = D(Q phi) = 0 exactly: the residual takes
    # v/|v| := 0 there (cost a^2, residual 0).  The magnified planes see free
    # space at their edges, so their fields and the probe gradient are not
    # zero; g_u is exactly zero (h = -i kappa conj(psi) g_psi = 0).
    import torch
    say("zero field: psi = 0, 64^3, 6 angles")
    p = PB.make_problem(64, 64, 6, config=0, chunk=4)
    rng = np.random.default_rng(41)
    u_np = (1e-5 * rng.random((64, 64, 64)) + 1.0j).astype(np.complex64)
    p.u = u_np
    u, q, amp, amp_ref = PB.to_gpu(p)
    plan = PB.gpu_plan(p)
    v = plan.holo_fwd(u, q).cpu().numpy()
    assert np.all(v[:, 0] == 0)                        # exactly zero frames
    assert np.all(np.abs(v[:, 1:]).max(axis=(2, 3)) > 0)
    F, gu, gq = plan.holo_grad(u, q, amp, amp_ref)
    F0, gu0, gq0 = PB.oracle_grad(p)
    assert np.all(gu0 == 0) and bool((gu == 0).all())
    PB.assert_close_scalar(F.item(), F0)
    PB.assert_close(gq.cpu().numpy(), gq0, "g_q")
    # the zero frames contribute exactly sum a^2 to F: removing them from the
    # data (a = 0 on plane 0) lowers F by that much on both sides
    amp2 = amp.clone()
    amp2[:, 0] = 0
    F2 = plan.holo_objective(u, q, amp2, amp_ref).item()
    a0 = p.amp[:, 0].astype(np.float64)
    PB.assert_close_scalar(F.item() - F2, np.sum(a0 * a0), "F(a) - F(a without plane 0)")
