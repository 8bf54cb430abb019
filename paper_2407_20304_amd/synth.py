"""Seeded synthetic inputs and the workload definitions.

This module only draws random numbers and paints shapes: it holds none of the
method's arithmetic (no propagation, no ray sums, no objective).  The same
arrays feed the GPU path and the FP64 oracle.

Every generator takes an explicit seed; the convention is
seed = 1000 * config + role, with role 1 object, 2 probe, 3 Poisson noise,
4 evaluation object, 5 evaluation probe, 6 finite-difference directions,
7 size mix, 8 test shifts, 9 data amplitudes of the large workloads.

The paper's own inputs (the ALD phantom of Sec. 3, the NFP-recovered probe and
the beamline data of Sec. 4) are not public; these generators stand in for
them with the paper's shapes and value ranges: delta ~ 1e-6..1e-5 with
beta = delta / 100 (Sec. 3), a probe carrying horizontal and vertical line
structure from multilayer KB mirrors (Sec. 1, Fig. 1), four sample planes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Geometry of Table 1 (ID16A PXM): focal spot to detector Z and the four
# focal spot to sample distances z_j; wavelength of 17.05 keV X-rays (Sec. 3).
TABLE1_Z = 1.208
TABLE1_ZJ = (4.026e-3, 4.199e-3, 4.890e-3, 6.325e-3)
WAVELENGTH = 7.27183e-11

MAG_REL = (1.0, 1.08, 1.25, 1.5)     # m~_j of the synthetic workloads
M0 = 300.0                          # Z / z_0 (Table 1: m_0 = 300)
FRESNEL0 = 0.01                     # Fresnel number of the first plane


def kappa_for(fresnel0: float = FRESNEL0) -> float:
    """Phase per unit u per voxel, 2 pi Delta / nu, with the pixel size Delta
    fixed by N_F0 = Delta^2 / (nu zeta_0) and zeta_0 = z_0 (Z - z_0) / Z of
    Table 1."""
    z0 = TABLE1_ZJ[0]
    zeta0 = z0 * (TABLE1_Z - z0) / TABLE1_Z
    delta = math.sqrt(fresnel0 * WAVELENGTH * zeta0)
    return 2.0 * math.pi * delta / WAVELENGTH


KAPPA = kappa_for()


def seed_of(config: int, role: int) -> int:
    return 1000 * config + role


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    H: int                 # detector rows = volume slices
    W: int                 # detector columns = in-plane volume edge
    n_angles: int
    chunk: int
    mag_rel: tuple = MAG_REL
    m0: float = M0
    fresnel0: float = FRESNEL0
    kappa: float = KAPPA
    config: int = 0

    @property
    def theta(self) -> np.ndarray:
        """theta_k = k pi / N_theta: uniform over [0, pi)."""
        return np.arange(self.n_angles, dtype=np.float64) * (np.pi / self.n_angles)

    def subset(self, n: int) -> np.ndarray:
        """Indices of the strided n-angle subset floor(i N_theta / n)."""
        return (np.arange(n) * self.n_angles) // n


WORKLOADS = {
    # 64^3 volume, 90 angles, 64^2 detector (the small case)
    "vol64_a90": Workload("vol64_a90", 64, 64, 90, 90, config=0),
    # 256^3 volume, 360 angles, 256^2 detector
    "vol256_a360": Workload("vol256_a360", 256, 256, 360, 64, config=1),
    # 1024^3 volume, 1800 angles in chunks of 64, 1024^2 detector
    "vol1024_a1800": Workload("vol1024_a1800", 1024, 1024, 1800, 64, config=3),
    # 2048^2 x 512-slice slab, 900 angles in chunks of 32, 512 x 2048 detector
    "slab2048x512_a900": Workload("slab2048x512_a900", 512, 2048, 900, 32, config=4),
}


# ---------------------------------------------------------------------------
# Object: painter's-order random ellipsoids
# ---------------------------------------------------------------------------

def ellipsoid_params(W: int, H: int, seed: int, n: int = 10, delta_max: float = 1e-5):
    """Draw n ellipsoids: centre (x, y) ~ U(-0.2W, 0.2W), z ~ U(-0.2H, 0.2H);
    in-plane semi-axes U(0.05, 0.2) W, vertical U(0.05, 0.2) H; rotation about
    z ~ U(0, pi); delta ~ U(0, delta_max), beta = delta / 100."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        cx, cy = rng.uniform(-0.2 * W, 0.2 * W, size=2)
        cz = rng.uniform(-0.2 * H, 0.2 * H)
        ax, ay = rng.uniform(0.05, 0.2, size=2) * W
        az = rng.uniform(0.05, 0.2) * H
        rot = rng.uniform(0.0, np.pi)
        delta = rng.uniform(0.0, delta_max)
        out.append((cx, cy, cz, ax, ay, az, rot, delta))
    return out


def ellipsoid_volume(W: int, H: int, seed: int, device="cpu", n: int = 10,
                     delta_max: float = 1e-5):
    """Complex volume u = delta + i beta, shape (H, W, W) = u[z, y, x].

    Voxel (ix, iy, iz) sits at (ix - W/2, iy - W/2, iz - H/2); a voxel takes the
    value of the last ellipsoid (in drawing order) that contains its position.
    Returns a torch complex64 tensor on `device`.
    """
    import torch
    vol = torch.zeros((H, W, W), dtype=torch.complex64, device=device)
    for (cx, cy, cz, ax, ay, az, rot, delta) in ellipsoid_params(W, H, seed, n, delta_max):
        r = max(ax, ay)
        y0, y1 = max(0, int(math.floor(W / 2 + cy - r))), min(W, int(math.ceil(W / 2 + cy + r)) + 1)
        x0, x1 = max(0, int(math.floor(W / 2 + cx - r))), min(W, int(math.ceil(W / 2 + cx + r)) + 1)
        z0, z1 = max(0, int(math.floor(H / 2 + cz - az))), min(H, int(math.ceil(H / 2 + cz + az)) + 1)
        if y0 >= y1 or x0 >= x1 or z0 >= z1:
            continue
        f64 = torch.float64
        Y = torch.arange(y0, y1, dtype=f64, device=device)[:, None] - W / 2 - cy
        X = torch.arange(x0, x1, dtype=f64, device=device)[None, :] - W / 2 - cx
        Zc = torch.arange(z0, z1, dtype=f64, device=device) - H / 2 - cz
        c, s = math.cos(rot), math.sin(rot)
        xr = X * c + Y * s
        yr = -X * s + Y * c
        inplane = (xr / ax) ** 2 + (yr / ay) ** 2               # (ny, nx)
        inside = inplane[None, :, :] + ((Zc / az) ** 2)[:, None, None] <= 1.0
        val = torch.tensor(complex(delta, delta / 100.0), dtype=torch.complex64, device=device)
        block = vol[z0:z1, y0:y1, x0:x1]
        block[inside] = val
    return vol


# ---------------------------------------------------------------------------
# Probe: Gaussian beam with KB-mirror line structure
# ---------------------------------------------------------------------------

def _stripes(rng, n: int, count: int = 16) -> np.ndarray:
    """Sum of `count` sinusoids with periods U(2, 32) px, random phases and
    U(0, 1) weights, normalised to max |S| = 1."""
    periods = rng.uniform(2.0, 32.0, size=count)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=count)
    weights = rng.uniform(0.0, 1.0, size=count)
    x = np.arange(n, dtype=np.float64)
    S = (weights[:, None] * np.sin(2.0 * np.pi * x[None, :] / periods[:, None]
                                   + phases[:, None])).sum(axis=0)
    return S / np.max(np.abs(S))


def probe(H: int, W: int, seed: int) -> np.ndarray:
    """Complex probe q (H, W), complex64.

    Amplitude: Gaussian (sigma = 0.375 W across, 0.375 H down) times
    (1 + 0.05 S_x + 0.05 S_y) (+-10 % line modulation).  Phase: a smooth
    random field scaled to max 1 rad plus 0.15 T_x + 0.15 T_y (+-0.3 rad
    ripples)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    Sx, Sy = _stripes(rng, W), _stripes(rng, H)
    Tx, Ty = _stripes(rng, W), _stripes(rng, H)
    noise = rng.standard_normal((H, W))
    smooth = gaussian_filter(noise, sigma=min(H, W) / 8.0, mode="wrap")
    smooth /= np.max(np.abs(smooth))
    x = np.arange(W, dtype=np.float64) - W / 2
    y = np.arange(H, dtype=np.float64) - H / 2
    sx, sy = 0.375 * W, 0.375 * H
    amp = np.exp(-(x[None, :] ** 2) / (2 * sx * sx) - (y[:, None] ** 2) / (2 * sy * sy))
    amp = amp * (1.0 + 0.05 * Sx[None, :] + 0.05 * Sy[:, None])
    phase = smooth + 0.15 * Tx[None, :] + 0.15 * Ty[:, None]
    return (amp * np.exp(1j * phase)).astype(np.complex64)


# ---------------------------------------------------------------------------
# Data
# ---------------------------------------------------------------------------

def poisson_amplitude(intensity: np.ndarray, seed: int, photons: float = 1e4) -> np.ndarray:
    """a = sqrt(Poisson(photons * I) / photons) as float32."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(photons * np.asarray(intensity, dtype=np.float64))
    return np.sqrt(counts / photons).astype(np.float32)


def synthetic_amplitudes(n_angles: int, n_dist: int, H: int, W: int, seed: int,
                         device="cpu", photons: float = 1e4, out=None):
    """Data-like amplitudes for the workloads too large to simulate on a CPU.

    Frame (k, j) is sqrt(Poisson(photons * I_kj) / photons) with
    I_kj = G(z, s) (1 + 0.2 sin(2 pi (f_y z / H + f_x s / W) + c)), G the
    probe's Gaussian envelope and (f_y, f_x, c) drawn per frame: the value
    range and the smooth-envelope-times-fringes look of holograms, without
    simulating them.  Returns a torch float32 tensor (n_angles, n_dist, H, W).
    """
    import torch
    rng = np.random.default_rng(seed)
    fy = rng.uniform(1.0, 40.0, size=(n_angles, n_dist))
    fx = rng.uniform(1.0, 40.0, size=(n_angles, n_dist))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(n_angles, n_dist))
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    if out is None:
        out = torch.empty((n_angles, n_dist, H, W), dtype=torch.float32, device=device)
    y = torch.arange(H, dtype=torch.float32, device=device)[:, None]
    x = torch.arange(W, dtype=torch.float32, device=device)[None, :]
    env = torch.exp(-((x - W / 2) ** 2) / (2 * (0.375 * W) ** 2)
                    - ((y - H / 2) ** 2) / (2 * (0.375 * H) ** 2))
    # blocks of frames at a time (a few hundred MB of temporaries)
    per = max(1, (1 << 26) // (n_dist * H * W))
    for k0 in range(0, n_angles, per):
        k1 = min(n_angles, k0 + per)
        cy = torch.tensor(fy[k0:k1], dtype=torch.float32, device=device)[:, :, None, None]
        cx = torch.tensor(fx[k0:k1], dtype=torch.float32, device=device)[:, :, None, None]
        cp = torch.tensor(ph[k0:k1], dtype=torch.float32, device=device)[:, :, None, None]
        arg = 2 * math.pi * (cy * (y / H) + cx * (x / W)) + cp
        inten = env * (1.0 + 0.2 * torch.sin(arg))
        counts = torch.poisson(photons * inten, generator=gen)
        out[k0:k1] = torch.sqrt(counts / photons)
    return out


# ---------------------------------------------------------------------------
# Batched single-angle problems (96 uneven instances)
# ---------------------------------------------------------------------------

BATCH_SIZES = (128, 192, 256, 384, 512)


def batch_sizes(n: int = 96, seed: int = seed_of(2, 7)) -> List[int]:
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(BATCH_SIZES, size=n)]


def phase_object_2d(n: int, seed: int, count: int = 10) -> np.ndarray:
    """psi = exp((i - 0.01) phi), phi from `count` painter's-order ellipses
    with values U(0, 1) rad (centres within 0.3 n of the middle, semi-axes
    U(0.05, 0.25) n)."""
    rng = np.random.default_rng(seed)
    phi = np.zeros((n, n))
    y = np.arange(n, dtype=np.float64)[:, None] - n / 2
    x = np.arange(n, dtype=np.float64)[None, :] - n / 2
    for _ in range(count):
        cx, cy = rng.uniform(-0.3 * n, 0.3 * n, size=2)
        ax, ay = rng.uniform(0.05, 0.25, size=2) * n
        rot = rng.uniform(0.0, np.pi)
        val = rng.uniform(0.0, 1.0)
        c, s = math.cos(rot), math.sin(rot)
        xr = (x - cx) * c + (y - cy) * s
        yr = -(x - cx) * s + (y - cy) * c
        phi[(xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0] = val
    return np.exp((1j - 0.01) * phi).astype(np.complex64)


def random_shifts(n_angles: int, n_dist: int, seed: int, max_px: float = 2.0) -> np.ndarray:
    """Sample shifts t_kj = (t_y, t_x) ~ U(-max_px, max_px), float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-max_px, max_px, size=(n_angles, n_dist, 2)).astype(np.float32)
