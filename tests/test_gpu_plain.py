"""The plain unfused GPU form (the speed-up denominator) computes the same
function: its per-angle ray-sum kernels against the oracle's R and R^T, and
its whole gradient against the oracle's."""

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
    from paper_2407_20304_amd import plain
    plain.lib()


@pytest.mark.parametrize("H,W", [(8, 64), (16, 96)])
def test_plain_radon_and_transpose(H, W):
    import torch
    from paper_2407_20304_amd import plain
    say("plain R / R^T", H, W)
    rng = np.random.default_rng(3)
    u = (rng.standard_normal((H, W, W)) + 1j * rng.standard_normal((H, W, W))).astype(np.complex64)
    h = (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))).astype(np.complex64)
    pg = plain.PlainGrad(H, W, [0.0], [1.0], 300.0, 0.01, 1.0)
    ud, hd = torch.from_numpy(u).cuda(), torch.from_numpy(h).cuda()
    # axis-aligned, the walk switch at 45 degrees, oblique and past pi/2
    for th in (0.0, 0.3, np.pi / 4, np.pi / 4 + 1e-3, np.pi / 2, 2.0, 2.9):
        pg.theta = [float(th)]
        p = torch.empty((H, W), dtype=torch.complex64, device="cuda")
        pg.radon(ud, 0, p, None)
        pT = torch.empty_like(p)          # the mirrored sums on the transposed copy
        pg.radon(ud, 0, pT, None, ud.transpose(1, 2).contiguous())
        g = torch.zeros_like(ud)
        pg.radon_adj(hd, 0, g, None)
        torch.cuda.synchronize()
        ref_p = O.radon(u.astype(np.complex128), th)
        ref_g = O.radon_T(h.astype(np.complex128), th, W)
        assert O.rel_err(p.cpu().numpy(), ref_p) < TOL, (th, O.rel_err(p.cpu().numpy(), ref_p))
        assert O.rel_err(pT.cpu().numpy(), ref_p) < TOL, (th, O.rel_err(pT.cpu().numpy(), ref_p))
        assert O.rel_err(g.cpu().numpy(), ref_g) < TOL, (th, O.rel_err(g.cpu().numpy(), ref_g))


def test_plain_gradient_parity():
    import torch
    from paper_2407_20304_amd import plain
    say("plain gradient 64^3, 12 angles")
    p = PB.make_problem(H=64, W=64, n_angles=12, config=0)
    g = p.geom
    pg = plain.PlainGrad(g.H, g.W, g.theta, g.mag_rel, g.m0, g.fresnel0, g.kappa, chunk=5)
    u, q, amp, amp_ref = PB.to_gpu(p)
    F, g_u, g_q = pg.grad(u, q, amp, amp_ref)
    Fo, guo, gqo = PB.oracle_grad(p)
    assert abs(F.item() - Fo) / Fo < TOL
    assert O.rel_err(g_u.cpu().numpy(), guo) < TOL
    assert O.rel_err(g_q.cpu().numpy(), gqo) < TOL
