"""Parity of the hierarchical schedule's pieces and of the whole schedule
with the FP64 oracle: intensity-averaging binning, replication to the denser
grid, and two levels (binned by 2, then unbinned) of conjugate gradients on
a 128^3 problem.  As for the single-level solver, every accept/reject
decision of the oracle's line searches is checked to have a relative margin
of at least 1e-2 before the histories are compared."""

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


@pytest.mark.parametrize("b", [2, 4])
@pytest.mark.parametrize("amplitude", [True, False])
def test_bin_frames_parity(b, amplitude):
    import torch
    from paper_2407_20304_amd import holo
    say("bin frames b=%d amplitude=%s" % (b, amplitude))
    rng = np.random.default_rng(41)
    a = (0.5 + rng.uniform(0, 1, (3, 4, 64, 192))).astype(np.float32)
    out = holo.bin_frames(torch.from_numpy(a).cuda(), b, amplitude=amplitude).cpu().numpy()
    ref = O.bin_frames(a.astype(np.float64), b, amplitude=amplitude)
    assert out.shape == ref.shape
    assert np.max(np.abs(out - ref) / ref) < 1e-6


@pytest.mark.parametrize("f", [2, 4])
def test_upsample_is_exact_replication(f):
    import torch
    from paper_2407_20304_amd import holo
    say("upsample f=%d" % f)
    rng = np.random.default_rng(42)
    q = (rng.standard_normal((2, 16, 24)) + 1j * rng.standard_normal((2, 16, 24))).astype(np.complex64)
    u = (rng.standard_normal((8, 12, 12)) + 1j * rng.standard_normal((8, 12, 12))).astype(np.complex64)
    qo = holo.upsample_frames(torch.from_numpy(q).cuda(), f).cpu().numpy()
    uo = holo.upsample_volume(torch.from_numpy(u).cuda(), f).cpu().numpy()
    assert np.array_equal(qo, O.upsample_frame(q, f))
    assert np.array_equal(uo, O.upsample_volume(u, f))


SCHEDULE = [(2, 2, 1e-10), (1, 2, 5e-11)]


@pytest.fixture(scope="module")
def mr_case():
    p = PB.make_problem(H=128, W=128, n_angles=8, config=0)
    trials = []

    def search(f, x, eta, F, gamma_try):
        seen = []

        def f_rec(xt):
            Ft = f(xt)
            seen.append(Ft)
            return Ft
        out = O.backtracking(f_rec, x, eta, F, gamma_try)
        trials.append((F, seen, out[3]))
        return out
    u, q, hists = O.multires_cg(p.amp.astype(np.float64), p.amp_ref.astype(np.float64), p.geom,
                                SCHEDULE, line_search=search)
    return p, u, q, hists, trials


def test_multires_schedule_parity(mr_case):
    import torch
    from paper_2407_20304_amd import multires
    p, u_or, q_or, hists, trials = mr_case
    for F, seen, _ in trials:
        for Ft in seen:
            assert np.isfinite(Ft) and abs(Ft - F) / F > 1e-2, (F, seen)
    say("multires schedule 128^3, 8 angles, levels 2 and 1, 2 iterations each")
    g = p.geom
    _, _, amp, amp_ref = PB.to_gpu(p)
    u, q, levels = multires.multires_cg(g.H, g.W, g.theta, g.mag_rel, g.m0, g.fresnel0, g.kappa,
                                        amp, amp_ref, SCHEDULE)
    halv_or = [t[2] for t in trials]
    halv = [int(h) for (_, _, _, hv) in levels for h in hv]
    assert halv == halv_or
    for (b, F_hist, _, _), h_or in zip(levels, hists):
        say("  level %d F_hist %s oracle %s" % (b, list(F_hist), h_or))
        for a, r in zip(F_hist, h_or):
            assert abs(a - r) / r < TOL, (b, a, r)
    e_u = O.rel_err(u.cpu().numpy(), u_or)
    e_q = O.rel_err(q.cpu().numpy(), q_or)
    say("  rel err u %.3e q %.3e" % (e_u, e_q))
    assert e_u < TOL and e_q < TOL
