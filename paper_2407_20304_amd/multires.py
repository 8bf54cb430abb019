"""Hierarchical schedule of the joint reconstruction (Sec. 4): conjugate
gradients on binned data, the result moved to a grid twice as dense as the
next level's start, less binning at each level, the last level unbinned.

A problem binned by b is the same dimensionless model on pixels b times
larger: an H/b x W/b detector and W/b x W/b x H/b volume, N_F0 b^2, kappa b,
shifts / b (angles, magnifications and m0 unchanged).  Data are binned by
averaging intensities (holo_bin_frames), the solution is moved to the denser
grid by replication (holo_upsample_volume / holo_upsample_frames); the first
level starts from u = 0 and the back-propagated binned reference.  Every
step runs in the library's kernels; this module only sequences the calls.
"""

import numpy as np

from . import holo


def level_plan(H, W, theta, mag_rel, m0, fresnel0, kappa, b, shift=None, chunk=64):
    """The holo.Plan of the problem binned by b."""
    return holo.Plan(H // b, W // b, theta, mag_rel, m0, fresnel0 * b * b, kappa * b,
                     shift=None if shift is None else np.asarray(shift, np.float32) / b,
                     chunk=chunk)


def multires_cg(H, W, theta, mag_rel, m0, fresnel0, kappa, amp, amp_ref, schedule,
                shift=None, chunk=64, stream=None):
    """Run the schedule [(b, iters, step0), ...] (b decreasing, each dividing
    the one before, H/b and W/b supported sizes) on amplitudes amp
    [n_angles][n_dist][H][W] and amp_ref [H][W] (float32, GPU).  Returns the
    final (u, q) and, per level, (b, F_hist, steps, halvings)."""
    import torch
    u = q = None
    prev = None
    levels = []
    for b, iters, step0 in schedule:
        if prev is not None and (b >= prev or prev % b):
            raise ValueError("binning factors must decrease, each dividing the one before")
        plan = level_plan(H, W, theta, mag_rel, m0, fresnel0, kappa, b, shift, chunk)
        a = holo.bin_frames(amp, b, stream=stream) if b > 1 else amp
        ar = holo.bin_frames(amp_ref, b, stream=stream) if b > 1 else amp_ref
        if u is None:
            u = torch.zeros((H // b, W // b, W // b), dtype=torch.complex64, device=amp.device)
            q = plan.holo_probe_init(ar, stream=stream)
        else:
            f = prev // b
            u = holo.upsample_volume(u, f, stream=stream)
            q = holo.upsample_frames(q, f, stream=stream)
        u, q, F_hist, steps, halv = plan.holo_cg(u, q, a, ar, iters, step0, in_place=True,
                                                 stream=stream)
        levels.append((b, F_hist, steps, halv))
        plan.close()
        prev = b
    return u, q, levels
