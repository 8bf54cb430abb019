"""Seeded test problems shared by the parity tests.

Inputs come from the generators module; data and expected values come from
the FP64 oracle only.  The GPU path receives the float32/complex64 versions
and the oracle receives the same values upcast, so a measured difference is
the GPU path's own arithmetic.
"""

from dataclasses import dataclass
from typing import Optional

import numpy as np

from oracle import holo_oracle as O
from paper_2407_20304_amd import synth


@dataclass
class Problem:
    geom: O.Geometry
    u: np.ndarray          # complex64 (H, W, W) evaluation point
    q: np.ndarray          # complex64 (H, W)
    amp: np.ndarray        # float32 (n_angles, n_dist, H, W)
    amp_ref: np.ndarray    # float32 (H, W)
    chunk: int = 0


def c128(x):
    return np.asarray(x).astype(np.complex128)


def make_problem(H, W, n_angles, config=0, chunk=0, theta=None, shifts=False,
                 mag_rel=synth.MAG_REL, kappa=synth.KAPPA, fresnel0=synth.FRESNEL0,
                 delta_max=1e-5, threads=None) -> Problem:
    """Truth from roles 1/2, Poisson data (role 3) of the oracle forward model
    at the truth, evaluation point from roles 4/5.  With `threads` the
    oracle's many-angle forward (C ray sums, threaded frames) makes the
    data."""
    sd = lambda role: synth.seed_of(config, role)
    if theta is None:
        theta = np.arange(n_angles) * (np.pi / n_angles)
    theta = np.asarray(theta, dtype=np.float64)
    sh = synth.random_shifts(len(theta), len(mag_rel), sd(8)) if shifts else None
    geom = O.Geometry(H=H, W=W, theta=theta, mag_rel=mag_rel, m0=synth.M0,
                      fresnel0=fresnel0, kappa=kappa, shift=sh)
    u_true = synth.ellipsoid_volume(W, H, sd(1), delta_max=delta_max).numpy()
    q_true = synth.probe(H, W, sd(2))
    if threads:
        v = O.forward_many(u_true, c128(q_true), geom, threads=threads)
    else:
        v = O.forward(c128(u_true), c128(q_true), geom)
    amp = synth.poisson_amplitude(np.abs(v) ** 2, sd(3))
    P = O.propagate(c128(q_true), 1.0, geom.fresnel0)
    amp_ref = synth.poisson_amplitude(np.abs(P) ** 2, sd(3) + 500)
    u = synth.ellipsoid_volume(W, H, sd(4), delta_max=delta_max).numpy()
    q = synth.probe(H, W, sd(5))
    return Problem(geom, u, q, amp, amp_ref, chunk)


def oracle_grad(p: Problem):
    return O.gradient(c128(p.u), c128(p.q), p.amp.astype(np.float64),
                      p.amp_ref.astype(np.float64), p.geom)


def oracle_threads():
    """Worker threads for the oracle's large checks: the host's cores, at
    most 16 (the share of a one-GPU machine)."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_grad_many(p: Problem, threads=None):
    """`oracle_grad` through the many-angle path (same definitions)."""
    threads = threads or oracle_threads()
    F, h, gq = O.gradient_projection_domain(p.u, c128(p.q), p.amp.astype(np.float64),
                                            p.amp_ref.astype(np.float64), p.geom,
                                            threads=threads)
    return F, O.radon_T_set(h, p.geom.theta, p.geom.W), gq


def gpu_plan(p: Problem):
    from paper_2407_20304_amd import holo
    g = p.geom
    return holo.Plan(g.H, g.W, g.theta, g.mag_rel, g.m0, g.fresnel0, g.kappa,
                     shift=None if g.shift is None else g.shift.astype(np.float32),
                     chunk=p.chunk)


def to_gpu(p: Problem):
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(p.u)).to(dev),
            torch.from_numpy(np.ascontiguousarray(p.q)).to(dev),
            torch.from_numpy(np.ascontiguousarray(p.amp)).to(dev),
            torch.from_numpy(np.ascontiguousarray(p.amp_ref)).to(dev))


TOL = 1e-5


def assert_close(x, ref, what="", tol=TOL, max_tol=TOL):
    """The parity bar: relative L2 error ||x - ref|| / ||ref|| below `tol`
    and max |x - ref| / max |ref| below `max_tol` (both in float64 against
    the oracle's values); prints both."""
    e2 = O.rel_err(x, ref)
    em = O.max_rel_err(x, ref)
    print("  %-28s rel L2 %.2e   max-abs/max %.2e" % (what, e2, em), flush=True)
    assert e2 < tol and em < max_tol, (what, e2, em)
    return e2, em


def assert_close_scalar(x, ref, what="F", tol=TOL):
    e = abs(float(x) - float(ref)) / abs(float(ref))
    print("  %-28s rel %.2e" % (what, e), flush=True)
    assert e < tol, (what, float(x), float(ref), e)
    return e
