"""Host-side check of the forward ray sums' angle grouping (no GPU needed:
plans are built on the host).

For every angle group the plan forms, every block of NB bins (the plan's
bin block, 16 or 8) and every row, the kernel stages the columns
floor(mn) - 1 ... floor(mn) + 30 of the row (mn = the lowest tap of the
group's rays in the block) and clamps each thread's tap base to
[max(0, -span), 31 - max(0, span) - 0.01] (span = (NB/4 - 1) B, the thread's
NB/4 bins; four bin groups per block) so that a tap and its right neighbour
are always read inside the 32 staged columns.  The clamp exists for windows
moved into the zero padding (rays that miss the volume); for every other
window it must never act, or it would shift a tap.  This recomputes the
windows and the thread bases in double precision and checks that every tap
of an unmoved window lies below column 30, for the plan's own bin block and
for the other one."""

import math

import numpy as np
import pytest

from paper_2407_20304_amd import holo, synth

SEG, PAD = 32, 32


def angle_constants(theta, W):
    c = W / 2.0
    C, S = np.cos(theta), np.sin(theta)
    along_y = np.abs(C) >= np.abs(S)
    den = np.where(along_y, C, S)
    other = np.where(along_y, S, C)
    B = 1.0 / den
    D = -other / den
    A = c - c / den + c * other / den
    return A, B, D


def check_plan_windows(theta, W, nb=None):
    plan = holo.Plan(64, W, theta, synth.MAG_REL, synth.M0, synth.FRESNEL0, synth.KAPPA)
    if nb is not None:
        plan.set_tile("fwd_bins", nb)
    NB = plan.get_tile("fwd_bins")
    BPT = NB // 4
    groups = plan.ray_groups()
    plan.close()
    assert sum(n for _, n in groups) == len(theta)
    assert [f for f, _ in groups] == list(np.cumsum([0] + [n for _, n in groups[:-1]]))
    A, B, D = angle_constants(np.asarray(theta, np.float64), W)
    y = np.arange(W, dtype=np.float64)[None, None, :]
    sb = np.arange(0, W, NB, dtype=np.float64)[None, :, None]
    checked = 0
    for first, n in groups:
        a = slice(first, first + n)
        Aa, Ba, Da = (x[a][:, None, None] for x in (A, B, D))
        lo = np.minimum(Aa + sb * Ba + y * Da, Aa + (sb + NB - 1) * Ba + y * Da).min(axis=0)
        start = np.floor(lo) - 1
        moved = (start < -PAD) | (start > W + PAD - SEG)
        for bg in range(4):
            rel = Aa + (sb + BPT * bg) * Ba + y * Da - start          # (n, blocks, rows)
            span = (BPT - 1) * Ba.astype(np.float32).astype(np.float64)
            rel_lo = np.maximum(0.0, -span)
            rel_hi = (SEG - 1) - np.maximum(0.0, span) - 0.01
            bad = ((rel < rel_lo) | (rel > rel_hi)) & ~moved[None]
            assert not bad.any(), (first, n, np.argwhere(bad)[:3])
            # every tap of an unmoved window lies in [0, SEG - 2): it and its
            # right neighbour are inside the window with a column to spare
            for b in range(BPT):
                q = rel + b * Ba
                ok = (q >= 0) & (q < SEG - 2)
                assert (ok | moved[None]).all()
            checked += int((~moved).sum()) * n
    return groups, checked, NB


@pytest.mark.parametrize("name", ["vol64_a90", "vol256_a360", "vol1024_a1800",
                                  "slab2048x512_a900"])
@pytest.mark.parametrize("nb", [None, 16, 8])
def test_ray_group_windows_of_the_workloads(name, nb):
    wl = synth.WORKLOADS[name]
    groups, checked, NB = check_plan_windows(wl.theta, wl.W, nb)
    assert checked > 0
    mean = np.mean([n for _, n in groups])
    # the grouping still shares windows: at the 1024^3 workload's 0.1 degree
    # steps most groups hold the maximum of 4 angles with 16-bin blocks; on
    # the 2048-wide slab (0.2 degree steps) 8-bin blocks grow the groups
    # from about two to three or more angles on average
    if name == "vol1024_a1800" and NB == 16:
        assert mean > 3.5
    if name == "slab2048x512_a900" and NB == 8:
        assert mean >= 3.0


def test_ray_group_windows_near_the_walk_switches():
    deg = np.array([0.0, 0.1, 0.2, 44.8, 44.9, 45.0, 45.1, 45.2, 89.9, 90.0, 90.1, 135.0,
                    179.8, 179.9])
    for W in (64, 512, 2048):
        for nb in (16, 8):
            check_plan_windows(np.deg2rad(deg), W, nb)
    rng = np.random.default_rng(7)
    for nb in (16, 8):
        check_plan_windows(np.sort(rng.uniform(0, math.pi, 200)), 384, nb)
