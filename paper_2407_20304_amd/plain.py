"""The plain unfused GPU form of the gradient: the comparison baseline.

The same function as `holo_grad` (the joint objective, Eq. 10 with Eq. 17,
and its gradients in u and q), composed the obvious way: the ray sums and
their transpose are the per-angle kernels of libholo_plain.so (one thread
per ray or per voxel, taps from global memory, one launch per angle; rays
that walk along x read a transposed copy of u, so that every launch's taps
are contiguous across a wavefront), and
every frame step is a separate torch operation on materialised tensors --
exp, bilinear demagnification by gather with precomputed indices and
weights and its transpose by index_add_, probe products, Fresnel
propagation by torch.fft (rocFFT) times the transfer function, the
amplitude residual.  Nothing is fused or captured; all arithmetic is
float32 except the objective's sum.  Angles are processed in chunks only to
bound memory (every intermediate of a chunk is kept).

Used by bench.py as the denominator of the speed-up; it is not part of the
library's path.
"""

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PLAIN_LIB_PATH = os.path.join(_HERE, "libholo_plain.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(PLAIN_LIB_PATH):
            raise RuntimeError("libholo_plain.so is not built (run paper_2407_20304_amd/build.py)")
        L = ctypes.CDLL(PLAIN_LIB_PATH)
        for name in ("holo_plain_radon", "holo_plain_radon_adj"):
            fn = getattr(L, name)
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                           ctypes.c_void_p, ctypes.c_void_p]
            fn.restype = ctypes.c_int32
        _lib = L
    return _lib


def _call(fn, *args):
    st = fn(*args)
    if st != 0:
        raise RuntimeError("%s failed with status %d" % (fn.__name__, st))


class PlainGrad:
    """Objective and gradients of the joint model, plain form.

    Geometry as in holo.Plan: theta (radians), mag_rel = m~_j (first 1),
    m0 = Z / z_0, fresnel0 = N_F0, kappa; no shifts."""

    def __init__(self, H, W, theta, mag_rel, m0, fresnel0, kappa, chunk=64, device="cuda"):
        import torch
        self.H, self.W = int(H), int(W)
        self.theta = [float(t) for t in theta]
        self.m = [float(x) for x in mag_rel]
        self.m0, self.nf, self.kappa = float(m0), float(fresnel0), float(kappa)
        self.chunk = int(chunk)
        self.dev = torch.device(device)
        # Dimensionless distances (Thm A.3): object-to-detector step and
        # probe step of plane j, in units of zeta_0.
        self.rho_det = [(self.m0 - m) / (m * (self.m0 - 1.0)) for m in self.m]
        self.rho_probe = [self.m0 * (m - 1.0) / (m * (self.m0 - 1.0)) for m in self.m]
        self.taps = [self._bilinear(m) for m in self.m]

    # -- frame operators ----------------------------------------------------
    def transfer(self, rho):
        """exp(-i pi rho (ky^2/H^2 + kx^2/W^2) / N_F0) on the FFT grid."""
        import torch
        def axis(n):
            k = np.fft.fftfreq(n) * n
            return np.exp(-1j * math.pi * rho * k * k / (self.nf * n * n))
        t = np.outer(axis(self.H), axis(self.W)).astype(np.complex64)
        return torch.from_numpy(t).to(self.dev)

    def propagate(self, f, rho):
        import torch
        return torch.fft.ifft2(torch.fft.fft2(f) * self.transfer(rho))

    def _bilinear(self, m):
        """Gather taps of M_{1/m}: output pixel (y, x) samples the input at
        (c_H + m (y - c_H), c_W + m (x - c_W)); four corners, weights zero
        (index clamped) where a corner falls outside the grid."""
        import torch
        def axis(n):
            src = n / 2.0 + m * (np.arange(n) - n / 2.0)
            i0 = np.floor(src).astype(np.int64)
            w = src - i0
            out = []
            for idx, wt in ((i0, 1.0 - w), (i0 + 1, w)):
                ok = (idx >= 0) & (idx < n)
                out.append((np.where(ok, idx, 0), np.where(ok, wt, 0.0)))
            return out
        ys, xs = axis(self.H), axis(self.W)
        taps = []
        for iy, wy in ys:
            for ix, wx in xs:
                idx = (iy[:, None] * self.W + ix[None, :]).ravel()
                wt = (wy[:, None] * wx[None, :]).ravel().astype(np.float32)
                taps.append((torch.from_numpy(idx).to(self.dev),
                             torch.from_numpy(wt).to(self.dev)))
        return taps

    def demag(self, f, j):
        """B_j f for a batch (K, H, W) of complex frames (gather)."""
        import torch
        K = f.shape[0]
        fr = torch.view_as_real(f.reshape(K, -1))
        out = torch.zeros_like(fr)
        for idx, wt in self.taps[j]:
            out += wt[None, :, None] * fr[:, idx, :]
        return torch.view_as_complex(out).reshape(f.shape)

    def demag_T(self, g, j):
        """B_j^T g (scatter with index_add_)."""
        import torch
        K = g.shape[0]
        gr = torch.view_as_real(g.reshape(K, -1))
        out = torch.zeros_like(gr)
        for idx, wt in self.taps[j]:
            out.index_add_(1, idx, wt[None, :, None] * gr)
        return torch.view_as_complex(out).reshape(g.shape)

    # -- ray sums (one launch per angle) --------------------------------------
    def radon(self, u, k, out, st, uT=None):
        """out[z][bin] = R_theta_k u (overwrites out).

        For rays that walk along x (|cos| < |sin|) the taps u[z][i0][step]
        are W apart across a wavefront; given uT = u with x and y exchanged,
        the same sums are taken along y of uT at the mirrored angle
        pi/2 - theta (cos and sin exchange), whose taps are contiguous."""
        vol, th = self.ray_volume(k, u, uT)
        _call(lib().holo_plain_radon, ctypes.c_void_p(vol.data_ptr()), self.H, self.W,
              th, ctypes.c_void_p(out.data_ptr()), st)

    def ray_volume(self, k, u, uT):
        """(volume, angle) whose sums along y give R_theta_k u."""
        th = self.theta[k]
        if uT is not None and abs(math.cos(th)) < abs(math.sin(th)):
            return uT, 0.5 * math.pi - th
        return u, th

    def radon_adj(self, h, k, g_u, st):
        """g_u += R_theta_k^T h."""
        _call(lib().holo_plain_radon_adj, ctypes.c_void_p(h.data_ptr()), self.H, self.W,
              self.theta[k], ctypes.c_void_p(g_u.data_ptr()), st)

    # -- the gradient ---------------------------------------------------------
    def grad(self, u, q, amp, amp_ref, stream=None):
        """(F, g_u, g_q) at (u, q) for amplitudes amp [n_angles][n_dist][H][W]
        and amp_ref [H][W]; F is a float64 tensor of one element."""
        import torch
        for t, name in ((u, "u"), (q, "q")):
            if t.dtype != torch.complex64 or not t.is_contiguous():
                raise ValueError("%s must be contiguous complex64" % name)
        H, W, nd = self.H, self.W, len(self.m)
        st = None
        if self.dev.type == "cuda":
            st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        F = torch.zeros((), dtype=torch.float64, device=self.dev)
        g_u = torch.zeros_like(u)
        G = torch.zeros((nd, H, W), dtype=torch.complex64, device=self.dev)
        Q = [self.propagate(q, r) for r in self.rho_probe]
        uT = u.transpose(1, 2).contiguous()
        for k0 in range(0, len(self.theta), self.chunk):
            ks = list(range(k0, min(k0 + self.chunk, len(self.theta))))
            p = torch.empty((len(ks), H, W), dtype=torch.complex64, device=self.dev)
            for a, k in enumerate(ks):
                self.radon(u, k, p[a], st, uT)
            psi = torch.exp(1j * self.kappa * p)
            g_psi = torch.zeros_like(psi)
            for j in range(nd):
                phi = 1.0 + self.demag(psi - 1.0, j)
                x = Q[j] * phi
                v = self.propagate(x, self.rho_det[j])
                a_kj = amp[k0:k0 + len(ks), j]
                av = v.abs()
                F += ((av - a_kj) ** 2).sum(dtype=torch.float64)
                unit = torch.where(av > 0, v / torch.where(av > 0, av, torch.ones_like(av)),
                                   torch.zeros_like(v))
                r = 2.0 * (v - a_kj * unit)
                w = self.propagate(r, -self.rho_det[j])
                G[j] += (phi.conj() * w).sum(dim=0)
                g_psi += self.demag_T(Q[j].conj() * w, j)
            h = (-1j * self.kappa * psi.conj() * g_psi).resolve_conj().contiguous()
            for a, k in enumerate(ks):
                self.radon_adj(h[a], k, g_u, st)
        # reference term || |D_1 q| - a_ref ||^2 and its probe gradient
        P = self.propagate(q, 1.0)
        ap = P.abs()
        F += ((ap - amp_ref) ** 2).sum(dtype=torch.float64)
        unit = torch.where(ap > 0, P / torch.where(ap > 0, ap, torch.ones_like(ap)),
                           torch.zeros_like(P))
        g_q = self.propagate(2.0 * (P - amp_ref * unit), -1.0)
        for j in range(nd):
            g_q += self.propagate(G[j], -self.rho_probe[j])
        return F, g_u, g_q
