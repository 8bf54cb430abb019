"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerance: 1e-5 relative error on the objective, and on each gradient and
field both 1e-5 relative L2 error and 1e-5 max-abs error over the largest
magnitude (tests/problems.py: assert_close), the bar the single-precision
path is held to."""

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


def rel(x, ref):
    return O.rel_err(x, ref)


# ---------------------------------------------------------------------------
# Propagation alone: u = 0 gives psi = 1, phi = 1 and v_kj = D_1 q exactly.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", [(64, 64), (128, 256), (192, 192), (384, 128), (256, 512),
                                 (1024, 1024), (512, 2048), (2048, 64)])
def test_zero_object_fields_are_the_propagated_probe(H, W):
    import torch
    say("zero-object fwd", H, W)
    from paper_2407_20304_amd import synth
    q = synth.probe(H, W, 77)
    theta = np.array([0.1, 1.2, 2.0])
    from paper_2407_20304_amd import holo
    plan = holo.Plan(H, W, theta, synth.MAG_REL, synth.M0, synth.FRESNEL0, synth.KAPPA)
    u = torch.zeros((H, W, W), dtype=torch.complex64, device="cuda")
    v = plan.holo_fwd(u, torch.from_numpy(q).cuda()).cpu().numpy()
    ref = O.propagate(PB.c128(q), 1.0, synth.FRESNEL0)
    for k in range(3):
        for j in range(4):
            PB.assert_close(v[k, j], ref, "v[%d,%d] %dx%d" % (k, j, H, W))


# ---------------------------------------------------------------------------
# Forward model, adjoint, objective, gradient
# ---------------------------------------------------------------------------

SMALL = dict(H=64, W=64, n_angles=12, config=0, shifts=True, chunk=5)


@pytest.fixture(scope="module")
def small():
    return PB.make_problem(**SMALL)


def test_fwd_parity(small):
    say("fwd parity 64^3, 12 angles, shifts, chunk 5")
    u, q, _, _ = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    v = plan.holo_fwd(u, q, 2, 11).cpu().numpy()
    ref = O.forward(PB.c128(small.u), PB.c128(small.q), small.geom, ks=range(2, 11))
    PB.assert_close(v, ref, "v")


def test_adj_parity(small):
    import torch
    say("adj parity 64^3")
    u, q, _, _ = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    rng = np.random.default_rng(5)
    w = (rng.standard_normal((7, 4, 64, 64)) + 1j * rng.standard_normal((7, 4, 64, 64))).astype(np.complex64)
    gu, gq = plan.holo_adj(u, q, torch.from_numpy(w).cuda(), 3, 10)
    ru, rq = O.adjoint(PB.c128(small.u), PB.c128(small.q), PB.c128(w), small.geom, ks=range(3, 10))
    PB.assert_close(gu.cpu().numpy(), ru, "gu")
    PB.assert_close(gq.cpu().numpy(), rq, "gq")


def test_adj_parity_angle_classes():
    """The transpose visits a call's angles in two classes (sin >= 0 or < 0
    once the rows of angles with cos < 0 are reversed), each padded to whole
    angle groups with dummies: shuffled angles over the whole circle, with
    the class boundaries 0, pi/2, pi and 3 pi/2 among them, over more than two
    set-up windows, a sub-range whose classes end mid-group and a single
    angle."""
    import torch
    from paper_2407_20304_amd import holo, synth
    say("adj parity 64^3, 150 shuffled angles over the circle")
    H = W = 64
    rng = np.random.default_rng(11)
    theta = rng.uniform(0.0, 2.0 * np.pi, 150)
    theta[[0, 17, 40, 77, 101]] = [0.0, np.pi / 2, np.pi, 1.5 * np.pi, np.pi / 4]
    geom = O.Geometry(H=H, W=W, theta=theta, mag_rel=synth.MAG_REL, m0=synth.M0,
                      fresnel0=synth.FRESNEL0, kappa=synth.KAPPA, shift=None)
    u = synth.ellipsoid_volume(W, H, 901).numpy()
    q = synth.probe(H, W, 902)
    plan = holo.Plan(H, W, theta, synth.MAG_REL, synth.M0, synth.FRESNEL0, synth.KAPPA, chunk=32)
    ug = torch.from_numpy(u).cuda()
    qg = torch.from_numpy(q).cuda()
    for k0, k1 in ((0, 150), (5, 14), (40, 41)):
        say("  angles [%d, %d)" % (k0, k1))
        w = (rng.standard_normal((k1 - k0, 4, H, W)) +
             1j * rng.standard_normal((k1 - k0, 4, H, W))).astype(np.complex64)
        gu, gq = plan.holo_adj(ug, qg, torch.from_numpy(w).cuda(), k0, k1)
        ru, rq = O.adjoint(PB.c128(u), PB.c128(q), PB.c128(w), geom, ks=range(k0, k1))
        PB.assert_close(gu.cpu().numpy(), ru, "gu [%d, %d)" % (k0, k1))
        PB.assert_close(gq.cpu().numpy(), rq, "gq [%d, %d)" % (k0, k1))


def test_objective_and_grad_parity(small):
    say("objective/grad parity 64^3")
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    F0, gu0, gq0 = PB.oracle_grad(small)
    Fo = plan.holo_objective(u, q, amp, amp_ref).item()
    F, gu, gq = plan.holo_grad(u, q, amp, amp_ref)
    assert abs(Fo - F0) / F0 < TOL
    assert abs(F.item() - F0) / F0 < TOL
    PB.assert_close(gu.cpu().numpy(), gu0, "gu")
    PB.assert_close(gq.cpu().numpy(), gq0, "gq")
    # the object-only and probe-only entry points agree with the joint one
    F1, gu1 = plan.holo_grad_object(u, q, amp, amp_ref)
    F2, gq2 = plan.holo_grad_probe(u, q, amp, amp_ref)
    assert F1.item() == F.item() and F2.item() == F.item()
    assert rel(gu1.cpu().numpy(), gu.cpu().numpy()) < 1e-6
    assert rel(gq2.cpu().numpy(), gq.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("H,W,n,chunk,shifts", [
    (64, 64, 90, 0, False),        # the 64^3, 90-angle workload
    (128, 256, 9, 4, True),        # rectangular, ragged last chunk
    (192, 192, 7, 3, True),        # radix-3 FFT lengths
    (64, 384, 5, 2, False),
    (1024, 64, 3, 2, True),        # 1024-point columns: one wavefront each, radix-16 stage
])
def test_grad_parity_shapes(H, W, n, chunk, shifts):
    say("grad parity", H, W, n, chunk, shifts)
    p = PB.make_problem(H, W, n, config=0, chunk=chunk, shifts=shifts)
    u, q, amp, amp_ref = PB.to_gpu(p)
    plan = PB.gpu_plan(p)
    F0, gu0, gq0 = PB.oracle_grad(p)
    F, gu, gq = plan.holo_grad(u, q, amp, amp_ref)
    assert abs(F.item() - F0) / F0 < TOL, (F.item(), F0)
    PB.assert_close(gu.cpu().numpy(), gu0, "gu")
    PB.assert_close(gq.cpu().numpy(), gq0, "gq")


def test_intensity_functional_parity(small):
    """F1 of Eq. (9): the plan switched to the intensity residual, data given
    as intensities (the squared amplitudes)."""
    import torch
    say("intensity functional 64^3, 12 angles, shifts, chunk 5")
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    plan.set_functional("intensity")
    d, d_ref = (amp * amp).contiguous(), (amp_ref * amp_ref).contiguous()
    F, g_u, g_q = plan.holo_grad(u, q, d, d_ref)
    Fo = plan.holo_objective(u, q, d, d_ref)
    # the same float32 intensities on both sides
    d64 = (small.amp * small.amp).astype(np.float64)
    dr64 = (small.amp_ref * small.amp_ref).astype(np.float64)
    Fr, gur, gqr = O.gradient(PB.c128(small.u), PB.c128(small.q), d64, dr64, small.geom,
                              functional="intensity")
    assert abs(F.item() - Fr) / Fr < TOL and abs(Fo.item() - Fr) / Fr < TOL
    PB.assert_close(g_u.cpu().numpy(), gur, "g_u")
    PB.assert_close(g_q.cpu().numpy(), gqr, "g_q")
    # and back to the amplitude functional on the same plan
    plan.set_functional("amplitude")
    F2, _, _ = plan.holo_grad(u, q, amp, amp_ref)
    Fo2, _, _ = PB.oracle_grad(small)
    assert abs(F2.item() - Fo2) / Fo2 < TOL


def test_conventional_functional_parity(small):
    """The flat-field functional of Eq. (16): the plan switched to the
    model with q = 1 and no reference term; the data stand for sqrt(d / d^r).
    F and g_u against the oracle's conventional functional, g_q exactly 0,
    the forward fields equal the joint model's with a unit probe."""
    import torch
    say("conventional functional 64^3, 12 angles, shifts, chunk 5")
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    plan.set_functional("conventional")
    F, g_u, g_q = plan.holo_grad(u, q, amp, amp_ref)
    Fo = plan.holo_objective(u, q, amp, amp_ref)
    v = plan.holo_fwd(u, q, 2, 7)
    Fr, gur = O.conventional_gradient(PB.c128(small.u), small.amp.astype(np.float64), small.geom)
    PB.assert_close_scalar(F.item(), Fr)
    PB.assert_close_scalar(Fo.item(), Fr, "F (objective call)")
    PB.assert_close(g_u.cpu().numpy(), gur, "g_u")
    assert bool((g_q == 0).all())
    ones = np.ones_like(PB.c128(small.q))
    vr = O.forward(PB.c128(small.u), ones, small.geom, ks=range(2, 7))
    PB.assert_close(v.cpu().numpy(), vr, "v (unit probe)")
    # and back to the amplitude functional on the same plan
    plan.set_functional("amplitude")
    F2, _, _ = plan.holo_grad(u, q, amp, amp_ref)
    Fo2, _, _ = PB.oracle_grad(small)
    PB.assert_close_scalar(F2.item(), Fo2, "F2 after switching back")


@pytest.mark.parametrize("H,W,n_angles,chunk,_unused",
                         [(64, 64, 12, 5, False), (128, 256, 9, 4, False), (1024, 64, 3, 2, False)])
def test_padded_propagation_parity(H, W, n_angles, chunk, _unused):
    from paper_2407_20304_amd import synth
    """Every propagation on the 2H x 2W grid with the field zero outside
    (reading P1): forward fields, objective, both gradients, the adjoint and
    the initial probe against the oracle with the same padding; object
    shifts (probe shifts are refused with padding)."""
    import torch
    say("padded propagation %dx%d, %d angles, chunk %d" % (H, W, n_angles, chunk))
    p = PB.make_problem(H, W, n_angles, config=0, chunk=chunk, shifts=True)
    p.geom.pad = 2
    plan = PB.gpu_plan(p)
    plan.set_padding(2)
    u, q, amp, amp_ref = PB.to_gpu(p)
    v = plan.holo_fwd(u, q, 1, n_angles).cpu().numpy()
    ref = O.forward(PB.c128(p.u), PB.c128(p.q), p.geom, ks=range(1, n_angles))
    PB.assert_close(v, ref, "v")
    F, g_u, g_q = plan.holo_grad(u, q, amp, amp_ref)
    Fo = plan.holo_objective(u, q, amp, amp_ref)
    F0, gu0, gq0 = PB.oracle_grad(p)
    PB.assert_close_scalar(F.item(), F0)
    PB.assert_close_scalar(Fo.item(), F0, "F (objective call)")
    PB.assert_close(g_u.cpu().numpy(), gu0, "g_u")
    PB.assert_close(g_q.cpu().numpy(), gq0, "g_q")
    rng = np.random.default_rng(5)
    w = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)).astype(np.complex64)
    au, aq = plan.holo_adj(u, q, torch.from_numpy(w).cuda(), 1, n_angles)
    au0, aq0 = O.adjoint(PB.c128(p.u), PB.c128(p.q), w.astype(np.complex128), p.geom,
                         ks=range(1, n_angles))
    PB.assert_close(au.cpu().numpy(), au0, "adj g_u")
    PB.assert_close(aq.cpu().numpy(), aq0, "adj g_q")
    q0 = plan.holo_probe_init(amp_ref).cpu().numpy()
    PB.assert_close(q0, O.probe_init(p.amp_ref.astype(np.float64), p.geom.fresnel0, pad=2),
                    "probe init")
    # the periodic propagation on the same plan gives the periodic result
    plan.set_padding(1)
    p.geom.pad = 1
    F1, _, _ = plan.holo_grad(u, q, amp, amp_ref)
    PB.assert_close_scalar(F1.item(), PB.oracle_grad(p)[0], "F periodic")


@pytest.mark.parametrize("H,W,angles,chunk", [
    (64, 64, "uniform12", 5),
    (256, 128, "scattered9", 4),     # unsorted, beyond pi, repeated modulo pi
    (64, 192, "uniform7", 3),
])
def test_fourier_slice_projector_parity(H, W, angles, chunk):
    """The Fourier-slice discretisation of R_k (reading F1) by gridding on
    the GPU against the oracle's exact sums: forward fields, objective, both
    gradients and the adjoint."""
    import torch
    if angles == "scattered9":
        theta = np.array([2.9, 0.1, 4.0, 1.3, np.pi / 2, 0.1 + np.pi, 5.5, 0.77, 3.05])
    else:
        n = int(angles[len("uniform"):])
        theta = np.arange(n) * (np.pi / n)
    say("fourier-slice projector %dx%d, angles %s, chunk %d" % (H, W, angles, chunk))
    p = PB.make_problem(H, W, len(theta), config=0, chunk=chunk, theta=theta, shifts=True)
    p.geom.projector = "fourier"
    plan = PB.gpu_plan(p)
    plan.set_projector("fourier")
    u, q, amp, amp_ref = PB.to_gpu(p)
    v = plan.holo_fwd(u, q, 1, len(theta)).cpu().numpy()
    ref = O.forward(PB.c128(p.u), PB.c128(p.q), p.geom, ks=range(1, len(theta)))
    PB.assert_close(v, ref, "v")
    F, g_u, g_q = plan.holo_grad(u, q, amp, amp_ref)
    Fo = plan.holo_objective(u, q, amp, amp_ref)
    F0, gu0, gq0 = PB.oracle_grad(p)
    PB.assert_close_scalar(F.item(), F0)
    PB.assert_close_scalar(Fo.item(), F0, "F (objective call)")
    PB.assert_close(g_u.cpu().numpy(), gu0, "g_u")
    PB.assert_close(g_q.cpu().numpy(), gq0, "g_q")
    rng = np.random.default_rng(6)
    w = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)).astype(np.complex64)
    au, aq = plan.holo_adj(u, q, torch.from_numpy(w).cuda(), 1, len(theta))
    au0, aq0 = O.adjoint(PB.c128(p.u), PB.c128(p.q), w.astype(np.complex128), p.geom,
                         ks=range(1, len(theta)))
    PB.assert_close(au.cpu().numpy(), au0, "adj g_u")
    PB.assert_close(aq.cpu().numpy(), aq0, "adj g_q")
    # switching back gives Joseph's sums again
    plan.set_projector("joseph")
    p.geom.projector = "joseph"
    F1, _, _ = plan.holo_grad(u, q, amp, amp_ref)
    PB.assert_close_scalar(F1.item(), PB.oracle_grad(p)[0], "F with Joseph's sums")


def test_tile_choices_and_their_autotuner(small):
    """The launch-shape parameters change no field: the column pass at half
    its default tile and the Fourier-slice projector at slab depths 2 and 8
    give bitwise-equal gradients (F up to the grouping of its partial sums);
    the tile autotuner picks a value among the candidates and the tuned plan
    still matches the oracle."""
    import torch
    say("tile choices 64^3, 12 angles, shifts, chunk 5")
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    F0, gu0, gq0 = [t.clone() for t in plan.holo_grad(u, q, amp, amp_ref)]
    plan.set_tile("col_tile", plan.default_col_tile() // 2)
    F1, gu1, gq1 = plan.holo_grad(u, q, amp, amp_ref)
    assert bool(torch.equal(gu0, gu1)) and bool(torch.equal(gq0, gq1))
    assert abs(F1.item() - F0.item()) <= 1e-12 * abs(F0.item())
    plan.set_tile("col_tile", 0)
    # the forward ray sums in 8-bin blocks (regrouped angles): the same sums
    # to rounding
    plan.set_tile("fwd_bins", 8)
    F2, gu2, gq2 = plan.holo_grad(u, q, amp, amp_ref)
    Fo, guo, gqo = PB.oracle_grad(small)
    PB.assert_close_scalar(F2.item(), Fo, "F (8-bin forward)")
    PB.assert_close(gu2.cpu().numpy(), guo, "g_u (8-bin forward)")
    PB.assert_close(gq2.cpu().numpy(), gqo, "g_q (8-bin forward)")
    plan.set_tile("fwd_bins", 16)
    plan.set_projector("fourier")
    plan.set_tile("fs_slab", 8)
    _, guf8, gqf8 = [t.clone() for t in plan.holo_grad(u, q, amp, amp_ref)]
    plan.set_tile("fs_slab", 2)
    _, guf2, gqf2 = plan.holo_grad(u, q, amp, amp_ref)
    assert bool(torch.equal(guf8, guf2)) and bool(torch.equal(gqf8, gqf2))
    choice = plan.autotune_tiles(u, q, amp, amp_ref, chunks=(4, 6, 12))
    say("  tuned: %s" % {k: v[0] for k, v in choice.items()})
    assert choice["chunk"][0] in (4, 6, 12) and choice["col_tile"][0] in (0, plan.default_col_tile() // 2)
    assert choice["fs_slab"][0] in (2, 4, 8)
    F, g_u, g_q = plan.holo_grad(u, q, amp, amp_ref)
    small.geom.projector = "fourier"
    try:
        Fo, guo, gqo = PB.oracle_grad(small)
    finally:
        small.geom.projector = "joseph"
    PB.assert_close_scalar(F.item(), Fo)
    PB.assert_close(g_u.cpu().numpy(), guo, "g_u")
    PB.assert_close(g_q.cpu().numpy(), gqo, "g_q")


def test_autotune_chunk_and_cache(small, tmp_path):
    """The chunk autotuner times one gradient per candidate, keeps the
    fastest, and the tuned plan's gradient still matches the oracle; a
    second call with the same cache file reuses the stored choice."""
    say("autotune chunk 64^3, 12 angles, candidates 4, 6, 12")
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    cache = str(tmp_path / "tune.json")
    best, times = plan.autotune(u, q, amp, amp_ref, candidates=(4, 6, 12), cache=cache)
    assert best in (4, 6, 12) and plan.chunk == best
    assert set(times) == {4, 6, 12} and all(t > 0 for t in times.values())
    assert times[best] == min(times.values())
    F, g_u, g_q = plan.holo_grad(u, q, amp, amp_ref)
    Fo, guo, gqo = PB.oracle_grad(small)
    assert abs(F.item() - Fo) / Fo < TOL
    PB.assert_close(g_u.cpu().numpy(), guo, "g_u")
    PB.assert_close(g_q.cpu().numpy(), gqo, "g_q")
    plan2 = PB.gpu_plan(small)
    best2, times2 = plan2.autotune(u, q, amp, amp_ref, candidates=(4, 6, 12), cache=cache)
    assert best2 == best and times2 is None and plan2.chunk == best


def test_probe_shift_parity(small):
    """Probe shifts s_kj (circular, Eq. 9) with object shifts: forward,
    objective and both gradients against the oracle; removing the shifts
    restores the unshifted gradient."""
    import torch
    say("probe shifts 64^3, 12 angles, shifts, chunk 5")
    g = small.geom
    ps = np.random.default_rng(61).uniform(-3.0, 3.0, (g.n_angles, g.n_dist, 2)).astype(np.float32)
    gs = O.Geometry(H=g.H, W=g.W, theta=g.theta, mag_rel=g.mag_rel, m0=g.m0, fresnel0=g.fresnel0,
                    kappa=g.kappa, shift=g.shift, probe_shift=ps.astype(np.float64))
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    plan.set_probe_shifts(ps)
    v = plan.holo_fwd(u, q, 0, 4).cpu().numpy()
    vref = O.forward(PB.c128(small.u), PB.c128(small.q), gs, ks=range(4))
    PB.assert_close(v, vref, "v")
    F, g_u, g_q = plan.holo_grad(u, q, amp, amp_ref)
    Fr, gur, gqr = O.gradient(PB.c128(small.u), PB.c128(small.q), small.amp.astype(np.float64),
                              small.amp_ref.astype(np.float64), gs)
    assert abs(F.item() - Fr) / Fr < TOL
    PB.assert_close(g_u.cpu().numpy(), gur, "g_u")
    PB.assert_close(g_q.cpu().numpy(), gqr, "g_q")
    plan.set_probe_shifts(None)
    F0, gu0, gq0 = plan.holo_grad(u, q, amp, amp_ref)
    Fo, guo, gqo = PB.oracle_grad(small)
    assert abs(F0.item() - Fo) / Fo < TOL
    PB.assert_close(gq0.cpu().numpy(), gqo, "g_q without probe shifts")


def test_repeat_calls_are_bitwise_identical(small):
    say("determinism")
    u, q, amp, amp_ref = PB.to_gpu(small)
    plan = PB.gpu_plan(small)
    a = plan.holo_grad(u, q, amp, amp_ref)
    b = plan.holo_grad(u, q, amp, amp_ref)
    assert a[0].item() == b[0].item()
    assert bool((a[1] == b[1]).all()) and bool((a[2] == b[2]).all())


def test_fwd_parity_fine_angles_across_walk_switch():
    # 0.1-degree spacing (as in the 1800-angle workload) around the 45 and
    # 90 degree switches of the walk direction, on a 512-wide detector: the
    # forward ray sums stage shared row windows for such angle groups.
    say("fwd parity 64x512x512, fine angles")
    deg = np.array([0.0, 0.1, 0.2, 44.8, 44.9, 45.0, 45.1, 45.2, 89.9, 90.0, 90.1, 135.0,
                    179.8, 179.9])
    p = PB.make_problem(64, 512, len(deg), config=0, theta=np.deg2rad(deg), chunk=6)
    u, q, _, _ = PB.to_gpu(p)
    plan = PB.gpu_plan(p)
    v = plan.holo_fwd(u, q).cpu().numpy()
    ref = O.forward(PB.c128(p.u), PB.c128(p.q), p.geom)
    for k in range(len(deg)):
        PB.assert_close(v[k], ref[k], "v at %.1f deg" % deg[k])


def test_dense_volume_with_poisoned_workspace():
    # A volume that is non-zero out to the corners, so the ray sums' staged
    # row windows and sinogram segments at and beyond the volume's edges
    # carry data, and a workspace filled with NaN bytes beforehand: the
    # zero padding the ray sums read outside the volume and the detector
    # must be written by the call itself.
    import torch
    say("dense volume, poisoned workspace, 64x128x128, 24 angles")
    deg = np.concatenate([np.arange(0.0, 180.0, 9.0), [44.9, 45.0, 45.1, 134.9]])
    p = PB.make_problem(64, 128, len(deg), config=0, theta=np.deg2rad(deg), chunk=7)
    rng = np.random.default_rng(11)
    u_np = (1e-5 * (rng.random((64, 128, 128)) + 0.1j * rng.random((64, 128, 128)))).astype(np.complex64)
    u = torch.from_numpy(u_np).cuda()
    q = torch.from_numpy(np.ascontiguousarray(p.q)).cuda()
    plan = PB.gpu_plan(p)
    plan.workspace(u.device).fill_(255)
    v = plan.holo_fwd(u, q).cpu().numpy()
    ref = O.forward(PB.c128(u_np), PB.c128(p.q), p.geom)
    for k in range(len(deg)):
        PB.assert_close(v[k], ref[k], "v at %.1f deg" % deg[k])
    w = (rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape)).astype(np.complex64)
    plan.workspace(u.device).fill_(255)
    gu, gq = plan.holo_adj(u, q, torch.from_numpy(w).cuda())
    ru, rq = O.adjoint(PB.c128(u_np), PB.c128(p.q), PB.c128(w), p.geom)
    PB.assert_close(gu.cpu().numpy(), ru, "gu")
    PB.assert_close(gq.cpu().numpy(), rq, "gq")
