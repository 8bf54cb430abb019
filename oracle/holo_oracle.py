"""FP64 CPU oracle for the joint object-and-probe holotomography gradient.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path (the HIP library
and its Python binding) never calls it and shares no code with it.

Everything here is the plain, slow definition of what the GPU path computes,
written in NumPy complex128/float64 so that a reader can check it against the
paper by eye:

  * Sec. 2, Eq. (8)   cone-beam forward model with probe: the field on the
                      detector for sample plane j is D_{zeta_j/m~_j^2}(
                      D_{omega_j}(q) . M_{1/m~_j}(psi)), after the rescaling
                      of the data by m0^2 M_{1/m0} (Eq. 9 text).
  * Sec. 2, Eq. (10)  the amplitude functional F2 with the reference term.
  * Sec. 2, Eq. (11)  and the display after it: the gradients with respect to
                      psi_k and q, including the adjoint L* = S_-t M*_{1/m~}
                      (conj(D_omega q) . D_{-zeta/m~^2}(.)).
  * Sec. 5, Eq. (17)  the joint model psi_k = exp(2 pi i/nu R_k u).
  * Sec. 2, Eq. (14)  R_k, the Radon transform at angle theta_k.
  * Appendix A, the Fresnel kernel P_Z and D_Z psi = psi * P_Z.

For problems too large for the NumPy loops (hundreds of angles on 256^3 to
1024^3 volumes) the same Joseph sums and transpose are available from
oracle/joseph.c (plain C loops in double precision, built by
oracle/build_oracle.py) through `radon_set` and `radon_T_set`; the pins hold
both implementations to the same facts.

Dimensionless units (one length unit = one detector pixel after the data
rescaling):  the Fresnel number of the first plane is N_F0 = Delta^2 /
(lambda zeta_0), every propagation distance is a multiple rho of zeta_0, and
kappa = 2 pi Delta / nu turns the voxel-unit ray sum of u into a phase.

Readings of points the paper leaves open (each one is listed with its reason
in the design notes of the repository):
  R1 R is Joseph's ray-driven discretisation: unit steps along the dominant
     axis, linear interpolation across it, path factor 1/max(|cos|,|sin|),
     zero outside the grid.  Voxel (ix, iy) sits at (ix - W/2, iy - W/2); bin i
     sits at s = i - W/2 with s = x cos(theta) + y sin(theta).
  R2 D_rho is the FFT transfer function exp(-i pi rho |k|^2 / N_F0) on the
     unpadded periodic H x W grid; the constant e^{ikZ}/(i lambda Z) is
     dropped, so D is unitary and D_a D_b = D_{a+b}.
  R3 M_{1/m~} S_t is bilinear sampling at src = c + m~ (x - c) - t about the
     grid centre c = n/2; outside the psi grid the transmission is 1 (free
     space), i.e. M(psi) = 1 + B(psi - 1).
  R4 v/|v| := 0 where |v| = 0.
  R5 Gradient convention g = dF/dRe + i dF/dIm (the paper's 2 L*(...)).
     The object gradient of the joint model follows by the chain rule:
     g_u = sum_k R_k^T(-i kappa conj(psi_k) g_psi_k).
  R6 Data are given directly as amplitudes a = sqrt(d~) on the computational
     grid (the m0^2 M_{1/m0} rescaling is the identity there).
  F1 The Fourier-slice discretisation of R_k (an option of the geometry,
     projector = "fourier"): the Fourier slice theorem evaluated exactly on
     the slice's discrete-time Fourier transform at W + 1 frequencies
     m (cos, sin), the two Nyquist terms at half weight, inverted at the W
     bins; equivalently p[i] = sum u[y, x] D_W(s_i - (x' cos + y' sin)) with
     the periodic sinc D_W(d) = sin(pi d) / (W tan(pi d / W)).  No path
     factor.  Without it (projector = "joseph") reading R1 holds.
  P1 Padded propagation (an option of the geometry, pad = 2): D_Z is a
     convolution over the whole plane, the fields are known on the H x W
     grid only and are taken as zero outside; each propagation sets the
     field in the centre of a 2H x 2W grid, applies that grid's transfer
     function (same pixel size) and cuts the centre out again.  Every
     propagation of the model (probe, detector, reference, adjoints) is
     padded when the option is set; its adjoint is the padded propagation
     by -rho.  Without it (pad = 1) reading R2 holds.

The solver around the gradient (Sec. 2, the CG iteration with the
Dai-Yuan formula, Eq. (12)-(13), and the initial probe):
  C1 The unknown is the joint vector x = (u, q) with the real inner product
     <a, b> = Re sum conj(a) b over both parts (the one in which -g is the
     steepest-descent direction, R5); one Dai-Yuan beta and one step length
     per iteration for the whole vector.
  C2 The line search is only required to keep F from increasing.  Here:
     halve a trial step until F(x + gamma eta) <= F(x); the first trial of
     the first iteration is given, later ones start at twice the previous
     accepted step; after 30 halvings the step is 0.
  C3 If the Dai-Yuan denominator <g_new - g_old, eta> is not positive, the
     direction restarts from -g (beta = 0).
  C4 The initial probe is the reference amplitude, with zero phase,
     propagated back to sample plane 0: q0 = D_{-1}(sqrt(d~r)).

Array layouts (the same ones the C ABI uses):
  u, g_u      (H, W, W) complex  -- u[z, y, x], z = detector row = slice
  q, g_q      (H, W) complex
  amp         (n_angles, n_dist, H, W) float
  amp_ref     (H, W) float
  frames v, w (n_angles, n_dist, H, W) complex
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------

def distances(m0: float, mag_rel: Sequence[float]):
    """Dimensionless propagation distances of Eq. (8) / Theorem A.3.

    With z_0 the first sample plane, m~_j = z_j / z_0 and m0 = Z / z_0:
      zeta_j / m~_j^2 (object-to-detector step)  ->  rho_det_j
      omega_j = (z_j - z_0) / m~_j (probe step)  ->  rho_probe_j
    both divided by zeta_0 = z_0 (Z - z_0) / Z, so the reference image is the
    probe propagated by rho = 1.
    """
    m = np.asarray(mag_rel, dtype=np.float64)
    rho_det = (m0 - m) / (m * (m0 - 1.0))
    rho_probe = m0 * (m - 1.0) / (m * (m0 - 1.0))
    return rho_det, rho_probe


@dataclass
class Geometry:
    """Parameters of one gradient evaluation (dimensionless, see module doc)."""
    H: int                      # detector rows = volume slices (z)
    W: int                      # detector columns = in-plane volume edge
    theta: np.ndarray           # (n_angles,) radians
    mag_rel: np.ndarray         # (n_dist,) m~_j = z_j / z_0, mag_rel[0] = 1
    m0: float = 300.0           # Z / z_0
    fresnel0: float = 0.01      # N_F0 of the first plane
    kappa: float = 4667.35      # phase per unit u per voxel of path
    shift: Optional[np.ndarray] = None   # (n_angles, n_dist, 2) = (t_y, t_x) px
    probe_shift: Optional[np.ndarray] = None   # (n_angles, n_dist, 2) = (s_y, s_x) px
    pad: int = 1                # 1: periodic propagation; 2: padded (reading P1)
    projector: str = "joseph"   # R_k: "joseph" (reading R1) or "fourier" (reading F1)

    def __post_init__(self):
        self.theta = np.asarray(self.theta, dtype=np.float64)
        self.mag_rel = np.asarray(self.mag_rel, dtype=np.float64)
        if self.shift is not None:
            self.shift = np.asarray(self.shift, dtype=np.float64)
        if self.probe_shift is not None:
            self.probe_shift = np.asarray(self.probe_shift, dtype=np.float64)

    @property
    def n_angles(self):
        return len(self.theta)

    @property
    def n_dist(self):
        return len(self.mag_rel)

    def t(self, k, j):
        if self.shift is None:
            return 0.0, 0.0
        return float(self.shift[k, j, 0]), float(self.shift[k, j, 1])

    def s(self, k, j):
        if self.probe_shift is None:
            return 0.0, 0.0
        return float(self.probe_shift[k, j, 0]), float(self.probe_shift[k, j, 1])


# ---------------------------------------------------------------------------
# Fresnel propagation (Appendix A: D_Z psi = psi * P_Z)
# ---------------------------------------------------------------------------

def transfer(n: int, rho: float, fresnel0: float) -> np.ndarray:
    """1-D factor of the Fresnel transfer function along an axis of length n.

    The Fourier transform of P_Z (with e^{-2 pi i x f}) is, up to the dropped
    constant, exp(-i pi lambda Z |f|^2); with f = k / (n Delta) and
    Z = rho zeta_0 this is exp(-i pi rho k^2 / (N_F0 n^2)).
    """
    k = np.fft.fftfreq(n) * n
    return np.exp(-1j * np.pi * rho * k * k / (fresnel0 * n * n))


def propagate(f: np.ndarray, rho: float, fresnel0: float, pad: int = 1) -> np.ndarray:
    """D_rho f on the last two axes (reading R2).

    With pad > 1, the padded propagation (reading P1): D_Z is a convolution
    over the whole plane (Appendix A), and the field is known on the H x W
    grid only; it is taken as zero outside, set in the centre of a grid pad
    times larger in each direction (same pixel size), propagated there with
    that grid's transfer function, and the centre H x W is cut out.  Its
    adjoint is the same with -rho (cutting out is the transpose of setting
    in)."""
    H, W = f.shape[-2:]
    if pad > 1:
        H2, W2 = pad * H, pad * W
        y0, x0 = (H2 - H) // 2, (W2 - W) // 2
        g = np.zeros(f.shape[:-2] + (H2, W2), dtype=np.complex128)
        g[..., y0:y0 + H, x0:x0 + W] = f
        return propagate(g, rho, fresnel0)[..., y0:y0 + H, x0:x0 + W]
    h = transfer(H, rho, fresnel0)[:, None] * transfer(W, rho, fresnel0)[None, :]
    return np.fft.ifft2(np.fft.fft2(f) * h)


# ---------------------------------------------------------------------------
# Radon transform R_k (Eq. 14), Joseph discretisation (reading R1)
# ---------------------------------------------------------------------------

def _joseph_taps(W: int, theta: float, step: int):
    """Taps of all rays for one step of the walk along the dominant axis.

    Returns (axis, idx0, w, scale): for bin i the ray crosses line `step` of
    the dominant axis at fractional index f_i = idx0_i + w_i of the other axis.
    axis = 0: the walk is along y (|cos| >= |sin|) and the taps index x.
    axis = 1: the walk is along x and the taps index y.
    """
    c = W / 2.0
    C, S = np.cos(theta), np.sin(theta)
    s = np.arange(W, dtype=np.float64) - c
    if abs(C) >= abs(S):
        f = c + (s - (step - c) * S) / C
        axis, scale = 0, 1.0 / abs(C)
    else:
        f = c + (s - (step - c) * C) / S
        axis, scale = 1, 1.0 / abs(S)
    i0 = np.floor(f).astype(np.int64)
    return axis, i0, f - i0, scale


def radon(u: np.ndarray, theta: float) -> np.ndarray:
    """p[z, i] = R_theta u: ray sums of every slice z at one angle.

    u is (H, W, W) = u[z, y, x]; the result is (H, W) = p[z, bin].
    """
    H, W, W2 = u.shape
    assert W == W2
    p = np.zeros((H, W), dtype=np.result_type(u.dtype, np.float64))
    for step in range(W):
        axis, i0, w, scale = _joseph_taps(W, theta, step)
        for idx, wt in ((i0, 1.0 - w), (i0 + 1, w)):
            ok = (idx >= 0) & (idx < W)
            if not ok.any():
                continue
            if axis == 0:
                vals = u[:, step, idx[ok]]
            else:
                vals = u[:, idx[ok], step]
            p[:, ok] += (wt[ok] * scale)[None, :] * vals
    return p


def radon_T(p: np.ndarray, theta: float, W: int) -> np.ndarray:
    """Literal transpose of `radon`: scatter each ray sum back with the same
    interpolation weights.  p is (H, W) = p[z, bin]; returns (H, W, W)."""
    H = p.shape[0]
    g = np.zeros((H, W, W), dtype=np.result_type(p.dtype, np.float64))
    for step in range(W):
        axis, i0, w, scale = _joseph_taps(W, theta, step)
        for idx, wt in ((i0, 1.0 - w), (i0 + 1, w)):
            ok = (idx >= 0) & (idx < W)
            if not ok.any():
                continue
            sel = idx[ok]
            contrib = (wt[ok] * scale)[None, :] * p[:, ok]
            where = (slice(None), step, sel) if axis == 0 else (slice(None), sel, step)
            # Consecutive bins are >= 1 index apart along a step (the slope
            # is 1/max(|cos|,|sin|) >= 1), so indices repeat only when
            # rounding lands a crossing exactly on an integer; np.add.at keeps
            # the scatter-add exact in that case too.
            if np.all(np.diff(sel) != 0):
                g[where] += contrib
            else:
                np.add.at(g, where, contrib)
    return g


# ---------------------------------------------------------------------------
# Fourier-slice discretisation of R_k (reading F1)
#
# The Fourier slice theorem: the 1-D Fourier transform of the projection at
# angle theta is the 2-D Fourier transform of the slice along the line
# through the origin at that angle.  Evaluated exactly on a slice's
# discrete-time Fourier transform F(xi) = sum u[y, x] e^{-2 pi i xi.(x', y')/W}
# at the W + 1 frequencies xi = m (cos, sin), m = -W/2 .. W/2 (the two
# Nyquist terms at half weight, so that R stays a real operator), and
# inverted with the W-point inverse DFT at the bins s_i = i - W/2, it gives
#   p[i] = sum_{y,x} u[y, x] D_W(s_i - (x' cos + y' sin)),
#   D_W(d) = (1/W) sum_m c_m e^{2 pi i m d / W} = sin(pi d) / (W tan(pi d / W)),
# D_W(0) = 1: the line integrals of the slice's trigonometric interpolant.
# No path factor appears (the integral has unit speed along the line).
# ---------------------------------------------------------------------------

def periodic_sinc(d, W: int) -> np.ndarray:
    """D_W(d) = sin(pi d) / (W tan(pi d / W)) for even W, 1 where d is a
    multiple of W."""
    d = np.asarray(d, dtype=np.float64)
    out = np.ones_like(d)
    t = np.tan(np.pi * d / W)
    nz = np.abs(np.sin(np.pi * d / W)) > 1e-14
    out[nz] = np.sin(np.pi * d[nz]) / (W * t[nz])
    return out


def fourier_slice_matrix(W: int, theta: float) -> np.ndarray:
    """The (W, W*W) matrix of the Fourier-slice projection of one slice:
    entry [i, y*W + x] = D_W(s_i - (x' cos(theta) + y' sin(theta)))."""
    c = W // 2
    xs = np.arange(W, dtype=np.float64) - c
    t = (xs[None, :] * np.cos(theta) + xs[:, None] * np.sin(theta)).ravel()   # [y, x]
    s = np.arange(W, dtype=np.float64) - c
    return periodic_sinc(s[:, None] - t[None, :], W)


def radon_fourier(u: np.ndarray, theta: float) -> np.ndarray:
    """p[z, i] of every slice of u (H, W, W) at one angle (reading F1)."""
    H, W, _ = u.shape
    A = fourier_slice_matrix(W, theta)
    return u.reshape(H, W * W) @ A.T


def radon_fourier_T(p: np.ndarray, theta: float, W: int) -> np.ndarray:
    """Transpose of `radon_fourier`: p (H, W) -> (H, W, W)."""
    A = fourier_slice_matrix(W, theta)
    return (p @ A).reshape(p.shape[0], W, W)


def project(u: np.ndarray, theta: float, projector: str = "joseph") -> np.ndarray:
    """R_theta u with the chosen discretisation."""
    return radon_fourier(u, theta) if projector == "fourier" else radon(u, theta)


def project_T(p: np.ndarray, theta: float, W: int, projector: str = "joseph") -> np.ndarray:
    """R_theta^T p with the chosen discretisation."""
    return radon_fourier_T(p, theta, W) if projector == "fourier" else radon_T(p, theta, W)


# ---------------------------------------------------------------------------
# Demagnification and shift M_{1/m~} S_t (reading R3)
# ---------------------------------------------------------------------------

def interp_matrix(n: int, mag: float, shift: float) -> np.ndarray:
    """Dense n x n linear-interpolation matrix of one axis:
    (B1 f)[i] = f sampled at c + mag (i - c) - shift, taps outside dropped."""
    c = n / 2.0
    src = c + mag * (np.arange(n, dtype=np.float64) - c) - shift
    i0 = np.floor(src).astype(np.int64)
    w = src - i0
    B = np.zeros((n, n))
    for idx, wt in ((i0, 1.0 - w), (i0 + 1, w)):
        ok = (idx >= 0) & (idx < n)
        B[np.nonzero(ok)[0], idx[ok]] += wt[ok]
    return B


def resample(f: np.ndarray, mag: float, ty: float = 0.0, tx: float = 0.0):
    """B f: bilinear sampling of an (H, W) frame (separable)."""
    H, W = f.shape
    return interp_matrix(H, mag, ty) @ f @ interp_matrix(W, mag, tx).T


def resample_T(g: np.ndarray, mag: float, ty: float = 0.0, tx: float = 0.0):
    """B^T g, the exact transpose of `resample`."""
    H, W = g.shape
    return interp_matrix(H, mag, ty).T @ g @ interp_matrix(W, mag, tx)


def transmit(psi: np.ndarray, mag: float, ty: float = 0.0, tx: float = 0.0):
    """M_{1/m~} S_t psi with free space (transmission 1) outside the grid."""
    return 1.0 + resample(psi - 1.0, mag, ty, tx)


# ---------------------------------------------------------------------------
# The joint model and its objective/gradient
# ---------------------------------------------------------------------------

def transmittance(u: np.ndarray, theta: float, kappa: float, projector: str = "joseph") -> np.ndarray:
    """psi_k = exp(i kappa R_k u) (Sec. 5, Eq. 17)."""
    return np.exp(1j * kappa * project(u, theta, projector))


def circular_shift_matrix(n: int, shift: float) -> np.ndarray:
    """n x n matrix of the circular linear-interpolation shift along one
    axis (reading R23): (S f)[i] = f sampled at i - shift, indices mod n."""
    src = np.arange(n, dtype=np.float64) - shift
    i0 = np.floor(src).astype(np.int64)
    w = src - i0
    S = np.zeros((n, n))
    S[np.arange(n), i0 % n] += 1.0 - w
    S[np.arange(n), (i0 + 1) % n] += w
    return S


def probe_shift_op(f: np.ndarray, sy: float, sx: float) -> np.ndarray:
    """S_s f on the last two axes (Eq. 9 with probe shifts, reading R23)."""
    H, W = f.shape[-2:]
    return circular_shift_matrix(H, sy) @ f @ circular_shift_matrix(W, sx).T


def probe_shift_op_T(g: np.ndarray, sy: float, sx: float) -> np.ndarray:
    """S_s^T, the literal transpose of `probe_shift_op`."""
    H, W = g.shape[-2:]
    return circular_shift_matrix(H, sy).T @ g @ circular_shift_matrix(W, sx)


def probe_frames(q: np.ndarray, geom: Geometry, k: int):
    """Q_kj = D_{rho_probe_j}(S_{s_kj} q): the probe at sample plane j for
    angle k (Eq. 9, shifting then propagating, as written)."""
    _, rho_p = distances(geom.m0, geom.mag_rel)
    return [propagate(probe_shift_op(q, *geom.s(k, j)), r, geom.fresnel0, geom.pad)
            for j, r in enumerate(rho_p)]


def probes(q: np.ndarray, geom: Geometry):
    """Q_j = D_{rho_probe_j} q: the probe at sample plane j (Eq. 8)."""
    _, rho_p = distances(geom.m0, geom.mag_rel)
    return [propagate(q, r, geom.fresnel0, geom.pad) for r in rho_p]


def _residual(v: np.ndarray, a: np.ndarray):
    """(|v| - a)^2 summed, and r = 2 (v - a v/|v|) (Eq. 11, reading R4)."""
    av = np.abs(v)
    unit = np.divide(v, av, out=np.zeros_like(v), where=av > 0)
    return float(np.sum((av - a) ** 2)), 2.0 * (v - a * unit)


def _residual_intensity(v: np.ndarray, d: np.ndarray):
    """Intensity functional F1 (Eq. 9): (|v|^2 - d)^2 summed, and its
    gradient in v, r = dF/dRe v + i dF/dIm v = 4 (|v|^2 - d) v."""
    e = np.abs(v) ** 2 - d
    return float(np.sum(e ** 2)), 4.0 * e * v


RESIDUALS = {"amplitude": _residual, "intensity": _residual_intensity}


def forward(u: np.ndarray, q: np.ndarray, geom: Geometry, ks=None) -> np.ndarray:
    """Detector fields v_kj of Eq. (17) for the angles `ks` (default: all)."""
    ks = range(geom.n_angles) if ks is None else ks
    rho_d, _ = distances(geom.m0, geom.mag_rel)
    Q = probes(q, geom)
    out = np.zeros((len(ks), geom.n_dist, geom.H, geom.W), dtype=np.complex128)
    for a, k in enumerate(ks):
        if geom.probe_shift is not None:
            Q = probe_frames(q, geom, k)
        psi = transmittance(u, geom.theta[k], geom.kappa, geom.projector)
        for j in range(geom.n_dist):
            phi = transmit(psi, geom.mag_rel[j], *geom.t(k, j))
            out[a, j] = propagate(Q[j] * phi, rho_d[j], geom.fresnel0, geom.pad)
    return out


def reference_term(q: np.ndarray, amp_ref: np.ndarray, fresnel0: float,
                   functional: str = "amplitude", pad: int = 1):
    """|| |D_1 q| - sqrt(d~r) ||^2 (or, for the intensity functional,
    || |D_1 q|^2 - d~r ||^2 with amp_ref holding d~r) and its probe gradient
    D_{-1}(r_ref)."""
    P = propagate(q, 1.0, fresnel0, pad)
    F, r = RESIDUALS[functional](P, amp_ref)
    return F, propagate(r, -1.0, fresnel0, pad)


def objective(u, q, amp, amp_ref, geom: Geometry, functional: str = "amplitude") -> float:
    """F(u, q) = F2(psi_k = exp(i kappa R_k u), q), Eq. (10) with Eq. (17);
    with functional="intensity" the F1 of Eq. (9) instead (amp and amp_ref
    then hold the intensities d~ and d~r)."""
    v = forward(u, q, geom)
    F = sum(RESIDUALS[functional](v[k, j], amp[k, j])[0]
            for k in range(v.shape[0]) for j in range(v.shape[1]))
    return F + reference_term(q, amp_ref, geom.fresnel0, functional, geom.pad)[0]


def _angle_terms(psi, k, Q, amp_k, geom: Geometry, functional: str = "amplitude"):
    """The frame stage of one angle k, given psi_k: forward to v_kj, residual
    r_kj (Eq. 11), w_kj = D_{-rho}(r_kj) (D* = D_{-z}), probe part
    conj(phi_kj) w_kj (display after Eq. 11), object part
    B^T(conj(Q_j) w_kj) (L* of Eq. 11).

    Returns (F_k, g_psi_k, G_k, gq_k): G_k[j] = conj(phi_kj) w_kj when there
    are no probe shifts (summed over k and propagated back by the caller),
    else None and gq_k = sum_j S^T D_{-rho_probe_j}(conj(phi_kj) w_kj)."""
    rho_d, rho_p = distances(geom.m0, geom.mag_rel)
    F = 0.0
    g_psi = np.zeros_like(psi)
    G = [] if geom.probe_shift is None else None
    gq = None if geom.probe_shift is None else np.zeros((geom.H, geom.W), np.complex128)
    for j in range(geom.n_dist):
        ty, tx = geom.t(k, j)
        phi = transmit(psi, geom.mag_rel[j], ty, tx)
        v = propagate(Q[j] * phi, rho_d[j], geom.fresnel0, geom.pad)
        Fk, r = RESIDUALS[functional](v, amp_k[j])
        F += Fk
        w = propagate(r, -rho_d[j], geom.fresnel0, geom.pad)
        if G is not None:
            G.append(np.conj(phi) * w)
        else:   # Q_kj = D S q: back through D, then S^T
            gq += probe_shift_op_T(propagate(np.conj(phi) * w, -rho_p[j], geom.fresnel0, geom.pad),
                                   *geom.s(k, j))
        g_psi += resample_T(np.conj(Q[j]) * w, geom.mag_rel[j], ty, tx)
    return F, g_psi, G, gq


def gradient(u, q, amp, amp_ref, geom: Geometry, with_reference=True,
             functional: str = "amplitude"):
    """F, g_u, g_q of the joint objective (F2, or F1 with
    functional="intensity").

    Per angle: psi_k, the frame stage `_angle_terms`, then the chain rule
    through the exponential and R^T (reading R5); after all angles the probe
    parts go back through D_{-rho_probe_j} and the reference term is added.
    """
    _, rho_p = distances(geom.m0, geom.mag_rel)
    Q = probes(q, geom)
    F = 0.0
    G = [np.zeros((geom.H, geom.W), np.complex128) for _ in range(geom.n_dist)]
    g_u = np.zeros(u.shape, np.complex128)
    g_q = np.zeros((geom.H, geom.W), np.complex128)
    for k in range(geom.n_angles):
        if geom.probe_shift is not None:
            Q = probe_frames(q, geom, k)
        psi = transmittance(u, geom.theta[k], geom.kappa, geom.projector)
        Fk, g_psi, Gk, gqk = _angle_terms(psi, k, Q, amp[k], geom, functional)
        F += Fk
        if Gk is not None:
            for j in range(geom.n_dist):
                G[j] += Gk[j]
        else:
            g_q += gqk
        h = -1j * geom.kappa * np.conj(psi) * g_psi
        g_u += project_T(h, geom.theta[k], geom.W, geom.projector)
    g_q = g_q + sum(propagate(G[j], -rho_p[j], geom.fresnel0, geom.pad) for j in range(geom.n_dist))
    if with_reference:
        Fr, gr = reference_term(q, amp_ref, geom.fresnel0, functional, geom.pad)
        F += Fr
        g_q = g_q + gr
    return F, g_u, g_q


def adjoint(u, q, w_frames, geom: Geometry, ks=None):
    """J^H w for J = d v / d(u, q) over the angles `ks`: (g_u, g_q).

    v is holomorphic in (u, q), so this is the vector-Jacobian product of a
    complex-linear map; with w = r it reproduces the gradient without the
    reference term.
    """
    ks = range(geom.n_angles) if ks is None else ks
    rho_d, rho_p = distances(geom.m0, geom.mag_rel)
    Q = probes(q, geom)
    G = [np.zeros((geom.H, geom.W), np.complex128) for _ in range(geom.n_dist)]
    g_u = np.zeros(u.shape, np.complex128)
    g_q = np.zeros((geom.H, geom.W), np.complex128)
    for a, k in enumerate(ks):
        if geom.probe_shift is not None:
            Q = probe_frames(q, geom, k)
        psi = transmittance(u, geom.theta[k], geom.kappa, geom.projector)
        g_psi = np.zeros_like(psi)
        for j in range(geom.n_dist):
            ty, tx = geom.t(k, j)
            phi = transmit(psi, geom.mag_rel[j], ty, tx)
            wb = propagate(w_frames[a, j], -rho_d[j], geom.fresnel0, geom.pad)
            if geom.probe_shift is None:
                G[j] += np.conj(phi) * wb
            else:
                g_q += probe_shift_op_T(propagate(np.conj(phi) * wb, -rho_p[j], geom.fresnel0, geom.pad),
                                        *geom.s(k, j))
            g_psi += resample_T(np.conj(Q[j]) * wb, geom.mag_rel[j], ty, tx)
        g_u += project_T(-1j * geom.kappa * np.conj(psi) * g_psi, geom.theta[k], geom.W,
                         geom.projector)
    g_q = g_q + sum(propagate(G[j], -rho_p[j], geom.fresnel0, geom.pad) for j in range(geom.n_dist))
    return g_u, g_q


# ---------------------------------------------------------------------------
# The conventional functional with division by the reference image (Sec. 3,
# Eq. 16): no probe, one independent functional per projection
# ---------------------------------------------------------------------------
#
# Reading F1 (flat field): Eq. 16 compares |D(S psi_k)|^2 with the square
# root of the flat-field-corrected data; amplitudes are taken on both sides
# (the data are square roots, as in F2).  The plane-j field is the model of
# Eq. 8 with q = 1 -- the paper's own remark that q = 1 turns its cone-beam
# model into the conventional one -- so psi is demagnified and shifted per
# plane exactly as in the joint model, and the data a_kj = sqrt(d_kj / d^r)
# are given on the computational grid (their rescaling is preprocessing, as
# R6).  There is no probe and no reference term.

def conventional_objective(u, amp, geom: Geometry) -> float:
    """sum_k sum_j || |D_{rho'_j}(M_j S_{t_kj} psi_k)| - a_kj ||^2 with
    psi_k = exp(i kappa R_k u)."""
    rho_d, _ = distances(geom.m0, geom.mag_rel)
    F = 0.0
    for k in range(geom.n_angles):
        psi = transmittance(u, geom.theta[k], geom.kappa, geom.projector)
        for j in range(geom.n_dist):
            v = propagate(transmit(psi, geom.mag_rel[j], *geom.t(k, j)), rho_d[j], geom.fresnel0,
                          geom.pad)
            F += float(np.sum((np.abs(v) - amp[k, j]) ** 2))
    return F


def conventional_gradient(u, amp, geom: Geometry):
    """F and g_u of `conventional_objective`: per plane the residual
    r = 2(v - a v/|v|) (v/|v| := 0 at |v| = 0), back through D_{-rho'_j}
    and the transposed resampling, then the chain rule through exp and R^T."""
    rho_d, _ = distances(geom.m0, geom.mag_rel)
    F = 0.0
    g_u = np.zeros(u.shape, np.complex128)
    for k in range(geom.n_angles):
        psi = transmittance(u, geom.theta[k], geom.kappa, geom.projector)
        g_psi = np.zeros_like(psi)
        for j in range(geom.n_dist):
            ty, tx = geom.t(k, j)
            v = propagate(transmit(psi, geom.mag_rel[j], ty, tx), rho_d[j], geom.fresnel0, geom.pad)
            av = np.abs(v)
            F += float(np.sum((av - amp[k, j]) ** 2))
            unit = np.divide(v, av, out=np.zeros_like(v), where=av > 0)
            w = propagate(2.0 * (v - amp[k, j] * unit), -rho_d[j], geom.fresnel0, geom.pad)
            g_psi += resample_T(w, geom.mag_rel[j], ty, tx)
        g_u += project_T(-1j * geom.kappa * np.conj(psi) * g_psi, geom.theta[k], geom.W,
                         geom.projector)
    return F, g_u


def holo2d_conventional_gradient(psi, amp, mag_rel, m0, fresnel0):
    """Eq. 16 for one projection with psi the unknown: F and g_psi."""
    rho_d, _ = distances(m0, mag_rel)
    F = 0.0
    g_psi = np.zeros(psi.shape, np.complex128)
    for j in range(len(mag_rel)):
        v = propagate(transmit(psi, mag_rel[j]), rho_d[j], fresnel0)
        av = np.abs(v)
        F += float(np.sum((av - amp[j]) ** 2))
        unit = np.divide(v, av, out=np.zeros_like(v), where=av > 0)
        w = propagate(2.0 * (v - amp[j] * unit), -rho_d[j], fresnel0)
        g_psi += resample_T(w, mag_rel[j])
    return F, g_psi


# ---------------------------------------------------------------------------
# Single-angle multi-distance retrieval (psi is the unknown; Eq. 10, N_theta=1)
# ---------------------------------------------------------------------------

def holo2d_forward(psi, q, mag_rel, m0, fresnel0):
    rho_d, rho_p = distances(m0, mag_rel)
    return np.stack([
        propagate(propagate(q, rho_p[j], fresnel0) * transmit(psi, mag_rel[j]),
                  rho_d[j], fresnel0)
        for j in range(len(mag_rel))])


def holo2d_gradient(psi, q, amp, amp_ref, mag_rel, m0, fresnel0, functional="amplitude"):
    """F2 of one projection with its own probe: F, g_psi, g_q (Eq. 10/11);
    functional="intensity" takes F1 (Eq. 9) instead, amp and amp_ref then
    holding intensities."""
    residual = RESIDUALS[functional]
    rho_d, rho_p = distances(m0, mag_rel)
    F = 0.0
    g_psi = np.zeros(psi.shape, np.complex128)
    g_q = np.zeros(q.shape, np.complex128)
    for j in range(len(mag_rel)):
        Qj = propagate(q, rho_p[j], fresnel0)
        phi = transmit(psi, mag_rel[j])
        v = propagate(Qj * phi, rho_d[j], fresnel0)
        Fj, r = residual(v, amp[j])
        F += Fj
        w = propagate(r, -rho_d[j], fresnel0)
        g_psi += resample_T(np.conj(Qj) * w, mag_rel[j])
        g_q += propagate(np.conj(phi) * w, -rho_p[j], fresnel0)
    Fr, gr = reference_term(q, amp_ref, fresnel0, functional)
    return F + Fr, g_psi, g_q + gr


# ---------------------------------------------------------------------------
# The solver: conjugate gradients with the Dai-Yuan formula (Sec. 2)
# ---------------------------------------------------------------------------

def inner(a, b) -> float:
    """<a, b> = Re sum conj(a) b over all parts of two tuples of arrays (C1)."""
    return float(sum(np.real(np.vdot(x, y)) for x, y in zip(a, b)))


def backtracking(f, x, eta, F, gamma_try, max_halvings=30):
    """Monotone line search (C2): halve gamma from gamma_try until
    f(x + gamma eta) <= F.  Returns (gamma, f at the new point, new point,
    number of halvings); gamma = 0 if no trial is accepted."""
    gamma = gamma_try
    for h in range(max_halvings + 1):
        xt = tuple(xi + gamma * ei for xi, ei in zip(x, eta))
        Ft = f(xt)
        if Ft <= F:
            return gamma, Ft, xt, h
        gamma *= 0.5
    return 0.0, F, x, max_halvings + 1


def dai_yuan_direction(g_new, g_old, eta):
    """The next search direction of Eq. (13): -g_new + beta eta with
    beta = ||g_new||^2 / <g_new - g_old, eta> (restart with beta = 0 when the
    denominator is not positive, C3).  Returns (direction, beta)."""
    den = inner(g_new, eta) - inner(g_old, eta)
    beta = inner(g_new, g_new) / den if den > 0.0 else 0.0
    return tuple(-gn + beta * ei for gn, ei in zip(g_new, eta)), beta


def cg_dai_yuan(f, grad, x0, iters, step0, line_search=None):
    """Conjugate gradients with the Dai-Yuan formula (Eq. 12-13):
    x_{m+1} = x_m + gamma_m eta_m, eta_0 = -g_0,
    eta_{m+1} = -g_{m+1} + ||g_{m+1}||^2 / <g_{m+1} - g_m, eta_m> eta_m.

    `f` and `grad` act on tuples of arrays; `grad` returns (F, g).  The line
    search (default: `backtracking`, C2) is called as
    line_search(f, x, eta, F, gamma_try) and returns
    (gamma, F_new, x_new, halvings).  Returns the final x, the objective
    after every iteration (F_0 first), the accepted steps and the halvings."""
    search = line_search or backtracking
    x = tuple(np.asarray(xi) for xi in x0)
    F, g = grad(x)
    eta = tuple(-gi for gi in g)
    hist, steps, halv = [F], [], []
    gamma_try = step0
    for _ in range(iters):
        gamma, F_new, x_new, h = search(f, x, eta, F, gamma_try)
        steps.append(gamma)
        halv.append(h)
        if gamma == 0.0:
            hist.append(F)
            continue
        x = x_new
        F, g_new = grad(x)
        eta, _ = dai_yuan_direction(g_new, g, eta)
        g = g_new
        hist.append(F)
        gamma_try = 2.0 * gamma
    return x, hist, steps, halv


def probe_init(amp_ref, fresnel0, pad: int = 1) -> np.ndarray:
    """Initial probe (C4): q0 = D_{-1}(sqrt(d~r)), the reference amplitude
    with zero phase propagated back to sample plane 0."""
    return propagate(np.asarray(amp_ref, dtype=np.complex128), -1.0, fresnel0, pad)


def holo_cg(u0, q0, amp, amp_ref, geom: Geometry, iters, step0, line_search=None):
    """`iters` Dai-Yuan CG iterations on the joint objective F(u, q)."""
    f = lambda x: objective(x[0], x[1], amp, amp_ref, geom)

    def grad(x):
        F, gu, gq = gradient(x[0], x[1], amp, amp_ref, geom)
        return F, (gu, gq)

    (u, q), hist, steps, halv = cg_dai_yuan(f, grad, (u0, q0), iters, step0, line_search)
    return u, q, hist, steps, halv


# ---------------------------------------------------------------------------
# Hierarchical binning and upsampling (Sec. 4, the speed-up schedule:
# iterate on binned data, move the result to a grid twice as dense, continue
# with less binning).  Readings:
#   M1  binning by b averages the intensities of b x b detector pixels; for
#       amplitude data a_b = sqrt(mean a^2);
#   M2  the binned problem is the same dimensionless model on pixels b times
#       larger: N_F0 -> b^2 N_F0 (N_F0 = Delta^2 / (lambda zeta_0)),
#       kappa -> b kappa (phase per voxel of path), H -> H / b, W -> W / b,
#       shifts -> shifts / b; angles, m~_j and m0 are unchanged;
#   M3  moving to a grid f times denser replicates every cell (f^3 voxels of
#       the volume, f^2 pixels of a frame).
# ---------------------------------------------------------------------------

def bin_frames(d: np.ndarray, b: int, amplitude: bool = True) -> np.ndarray:
    """M1 on the last two axes (sizes divisible by b)."""
    d = np.asarray(d, dtype=np.float64)
    H, W = d.shape[-2:]
    x = d * d if amplitude else d
    m = x.reshape(d.shape[:-2] + (H // b, b, W // b, b)).mean(axis=(-3, -1))
    return np.sqrt(m) if amplitude else m


def upsample_frame(q: np.ndarray, f: int) -> np.ndarray:
    """M3 for a frame (last two axes)."""
    return np.repeat(np.repeat(q, f, axis=-2), f, axis=-1)


def upsample_volume(u: np.ndarray, f: int) -> np.ndarray:
    """M3 for a volume [z][y][x]."""
    return np.repeat(np.repeat(np.repeat(u, f, axis=0), f, axis=1), f, axis=2)


def level_geometry(geom: Geometry, b: int) -> Geometry:
    """M2: the geometry of the problem binned by b."""
    return Geometry(H=geom.H // b, W=geom.W // b, theta=geom.theta, mag_rel=geom.mag_rel,
                    m0=geom.m0, fresnel0=geom.fresnel0 * b * b, kappa=geom.kappa * b,
                    shift=None if geom.shift is None else geom.shift / b,
                    probe_shift=None if geom.probe_shift is None else geom.probe_shift / b)


def multires_cg(amp, amp_ref, geom: Geometry, schedule, line_search=None):
    """The hierarchical schedule: for each (b, iters, step0) in order (b
    decreasing, each dividing the one before), bin the data by b (M1),
    start from the previous level's result moved to the denser grid (M3) --
    or, at the first level, from u = 0 and the back-propagated reference --
    and run `iters` conjugate-gradient iterations on the level's geometry
    (M2).  Returns the final (u, q) and each level's objective history."""
    u = q = None
    prev = None
    hists = []
    for b, iters, step0 in schedule:
        g = level_geometry(geom, b)
        a, ar = bin_frames(amp, b), bin_frames(amp_ref, b)
        if u is None:
            u = np.zeros((g.H, g.W, g.W), np.complex128)
            q = probe_init(ar, g.fresnel0)
        else:
            u, q = upsample_volume(u, prev // b), upsample_frame(q, prev // b)
        u, q, hist, _, _ = holo_cg(u, q, a, ar, g, iters, step0, line_search)
        hists.append(hist)
        prev = b
    return u, q, hists


# ---------------------------------------------------------------------------
# Error metric used by the parity tests
# ---------------------------------------------------------------------------

def rel_err(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 in float64 (0 if both are zero)."""
    x = np.asarray(x, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    if den == 0.0:
        return float(num)
    return float(num / den)


def max_rel_err(x, ref) -> float:
    """max |x - ref| / max |ref| over all elements, in float64 (0 if both
    are zero): a wrong value where |ref| is small, which the L2 metric can
    hide, shows here."""
    x = np.asarray(x, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(x - ref))) if ref.size else 0.0
    if den == 0.0:
        return num
    return num / den


# ---------------------------------------------------------------------------
# Problems too large for the NumPy ray sums (hundreds of angles, 256^3 to
# 1024^3 volumes): the same Joseph sums and transpose from oracle/joseph.c
# (plain C loops in double precision, slices in parallel), and the frame
# stage of several angles at once on a thread pool (NumPy's FFTs and
# products release the interpreter lock).  Same definitions, same steps.
# ---------------------------------------------------------------------------

_JOSEPH_LIB = None
JOSEPH_SO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libjoseph_oracle.so")


def _joseph():
    global _JOSEPH_LIB
    if _JOSEPH_LIB is None:
        if not os.path.exists(JOSEPH_SO):
            raise RuntimeError("oracle/libjoseph_oracle.so is not built (oracle/build_oracle.py)")
        L = ctypes.CDLL(JOSEPH_SO)
        P, I = ctypes.c_void_p, ctypes.c_int
        L.joseph_radon.argtypes = [P, I, I, P, I, I, I, P]
        L.joseph_radon_T.argtypes = [P, I, P, I, I, P]
        L.joseph_radon.restype = L.joseph_radon_T.restype = I
        _JOSEPH_LIB = L
    return _JOSEPH_LIB


def radon_set(u, thetas, z0: int = 0, nz: Optional[int] = None) -> np.ndarray:
    """p[k, z, i] = (R_{theta_k} u)[z0 + z, i] -- `radon` at every angle of
    `thetas` for the slices z0 .. z0 + nz - 1, computed by joseph.c.

    u is (H, W, W); it is read as complex64 (the inputs of the comparisons
    are single-precision values), every sum is formed in double."""
    u = np.ascontiguousarray(u, dtype=np.complex64)
    H, W, _ = u.shape
    nz = H - z0 if nz is None else nz
    th = np.ascontiguousarray(thetas, dtype=np.float64).ravel()
    p = np.empty((len(th), nz, W), np.complex128)
    rc = _joseph().joseph_radon(u.ctypes.data, H, W, th.ctypes.data, len(th), z0, nz,
                                p.ctypes.data)
    if rc != 0:
        raise RuntimeError("joseph_radon failed (%d)" % rc)
    return p


def radon_T_set(h, thetas, W: int) -> np.ndarray:
    """sum_k R_{theta_k}^T h[k] -- `radon_T` of every angle, summed, for the
    nz slices of h (n, nz, W); returns (nz, W, W) complex128."""
    h = np.ascontiguousarray(h, dtype=np.complex128)
    n, nz, W2 = h.shape
    assert W2 == W
    th = np.ascontiguousarray(thetas, dtype=np.float64).ravel()
    assert len(th) == n
    g = np.empty((nz, W, W), np.complex128)
    rc = _joseph().joseph_radon_T(h.ctypes.data, W, th.ctypes.data, n, nz, g.ctypes.data)
    if rc != 0:
        raise RuntimeError("joseph_radon_T failed (%d)" % rc)
    return g


def _pool_map(fn, items, threads):
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1), ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


def _ray_sums_all(u, geom: Geometry) -> np.ndarray:
    """p[k] = R_k u for every angle: joseph.c for Joseph's sums, the dense
    Fourier-slice matrices otherwise."""
    if geom.projector == "fourier":
        u = np.asarray(u, dtype=np.complex64).astype(np.complex128)
        return np.stack([radon_fourier(u, th) for th in geom.theta])
    return radon_set(u, geom.theta)


def forward_many(u, q, geom: Geometry, threads: int = 8) -> np.ndarray:
    """`forward` for all angles: ray sums from joseph.c, then the frames of
    each angle (psi_k, phi_kj = M S psi_k, v_kj = D_{rho_det_j}(Q_j phi_kj))."""
    rho_d, _ = distances(geom.m0, geom.mag_rel)
    p = _ray_sums_all(u, geom)

    def one(k):
        Q = probe_frames(q, geom, k) if geom.probe_shift is not None else probes(q, geom)
        psi = np.exp(1j * geom.kappa * p[k])
        return np.stack([propagate(Q[j] * transmit(psi, geom.mag_rel[j], *geom.t(k, j)),
                                   rho_d[j], geom.fresnel0, geom.pad)
                         for j in range(geom.n_dist)])

    return np.stack(_pool_map(one, range(geom.n_angles), threads))


def gradient_projection_domain(u, q, amp, amp_ref, geom: Geometry, threads: int = 8,
                               functional: str = "amplitude", progress=None):
    """`gradient` up to its last step: returns (F, h, g_q) with
    h[k] = -i kappa conj(psi_k) g_psi_k, so that g_u = sum_k R_k^T h[k]
    (`radon_T_set(h, geom.theta, W)`, slab by slab for large volumes).

    The ray sums come from joseph.c; the frame stage `_angle_terms` of each
    angle runs on a thread pool; F and the probe parts are summed in angle
    order.  `progress(message)`, if given, is called after the ray sums and
    after each batch of angles."""
    _, rho_p = distances(geom.m0, geom.mag_rel)
    p = _ray_sums_all(u, geom)
    if progress:
        progress("ray sums of %d angles done" % geom.n_angles)
    Q0 = probes(q, geom)

    def one(k):
        Q = probe_frames(q, geom, k) if geom.probe_shift is not None else Q0
        psi = np.exp(1j * geom.kappa * p[k])
        Fk, g_psi, Gk, gqk = _angle_terms(psi, k, Q, amp[k], geom, functional)
        p[k] = -1j * geom.kappa * np.conj(psi) * g_psi      # h_k replaces p_k
        return Fk, Gk, gqk

    F = 0.0
    G = [np.zeros((geom.H, geom.W), np.complex128) for _ in range(geom.n_dist)]
    g_q = np.zeros((geom.H, geom.W), np.complex128)
    batch = max(1, threads)
    for k0 in range(0, geom.n_angles, batch):
        for Fk, Gk, gqk in _pool_map(one, range(k0, min(k0 + batch, geom.n_angles)), threads):
            F += Fk
            if Gk is not None:
                for j in range(geom.n_dist):
                    G[j] += Gk[j]
            else:
                g_q += gqk
        if progress:
            progress("frames of angles %d-%d done" % (k0, min(k0 + batch, geom.n_angles) - 1))
    g_q = g_q + sum(propagate(G[j], -rho_p[j], geom.fresnel0, geom.pad) for j in range(geom.n_dist))
    Fr, gr = reference_term(q, amp_ref, geom.fresnel0, functional, geom.pad)
    return F + Fr, p, g_q + gr
