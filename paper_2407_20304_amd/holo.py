"""Python binding of libholo.so (C ABI in include/holo.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors are PyTorch CUDA/HIP tensors; their device pointers and the
current stream are handed to the library.  If the library is not built, every
call raises HoloError -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_size_t, c_void_p
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libholo.so")

# Every symbol declared in include/holo.h.
EXPORTS = (
    "holo_plan_create", "holo_plan_destroy", "holo_workspace_bytes", "holo_plan_set_functional",
    "holo_plan_set_chunk", "holo_plan_get_chunk", "holo_plan_autotune",
    "holo_plan_set_tile", "holo_plan_get_tile", "holo_plan_autotune_tile",
    "holo_plan_set_probe_shifts", "holo_plan_set_padding", "holo_plan_set_projector",
    "holo_fwd", "holo_adj", "holo_objective", "holo_grad",
    "holo_grad_object", "holo_grad_probe",
    "holo_probe_init", "holo_cg_workspace_bytes", "holo_cg",
    "holo_bin_frames", "holo_upsample_frames", "holo_upsample_volume",
    "holo2d_plan_create", "holo2d_plan_destroy", "holo2d_offsets", "holo2d_workspace_bytes",
    "holo2d_plan_set_functional", "holo2d_fwd", "holo2d_objective", "holo2d_grad",
    "holo2d_noalloc_bytes", "holo2d_grad_noalloc",
    "holo_timing_enable", "holo_timing_read", "holo_plan_ray_groups", "holo_last_error",
)

KERNEL_CLASSES = ("radon_fwd", "radon_adj", "pass_a", "pass_b", "pass_c", "pass_d", "probe",
                  "other", "solver")

STATUS = {0: "HOLO_OK", 1: "HOLO_ERR_INVALID_ARGUMENT", 2: "HOLO_ERR_UNSUPPORTED_SIZE",
          3: "HOLO_ERR_WORKSPACE_TOO_SMALL", 4: "HOLO_ERR_HIP", 5: "HOLO_ERR_OUT_OF_HOST_MEMORY"}


class HoloError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class holo_geom(ctypes.Structure):
    _fields_ = [
        ("det_rows", c_int32), ("det_cols", c_int32),
        ("n_angles", c_int32), ("n_dist", c_int32),
        ("theta", POINTER(c_double)), ("mag_rel", POINTER(c_double)),
        ("m0", c_double), ("fresnel0", c_double), ("kappa", c_double),
        ("shift", POINTER(c_float)), ("chunk", c_int32),
    ]


_lib = None


def lib():
    """Load libholo.so (raises HoloError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HoloError(-1, "libholo.so is not built (run paper_2407_20304_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    L.holo_plan_create.argtypes = [POINTER(holo_geom), POINTER(c_void_p)]
    L.holo_plan_destroy.argtypes = [P]
    L.holo_workspace_bytes.argtypes = [P, POINTER(c_size_t)]
    L.holo_plan_set_functional.argtypes = [P, c_int32]
    L.holo_plan_set_chunk.argtypes = [P, c_int32]
    L.holo_plan_set_probe_shifts.argtypes = [P, P]
    L.holo_plan_set_padding.argtypes = [P, c_int32]
    L.holo_plan_set_projector.argtypes = [P, c_int32]
    L.holo_plan_get_chunk.argtypes = [P, POINTER(c_int32)]
    L.holo_plan_autotune.argtypes = [P, P, P, P, P, P, P, P, P, c_int32, P, c_size_t, P, P, P]
    L.holo_plan_set_tile.argtypes = [P, c_int32, c_int32]
    L.holo_plan_get_tile.argtypes = [P, c_int32, POINTER(c_int32)]
    L.holo_plan_autotune_tile.argtypes = [P, c_int32, P, P, P, P, P, P, P, P, c_int32, P, c_size_t,
                                          P, P, P]
    L.holo_fwd.argtypes = [P, P, P, c_int32, c_int32, P, P, c_size_t, P]
    L.holo_adj.argtypes = [P, P, P, c_int32, c_int32, P, P, P, P, c_size_t, P]
    L.holo_objective.argtypes = [P, P, P, P, P, P, P, c_size_t, P]
    L.holo_grad.argtypes = [P, P, P, P, P, P, P, P, P, c_size_t, P]
    L.holo_grad_object.argtypes = [P, P, P, P, P, P, P, P, c_size_t, P]
    L.holo_grad_probe.argtypes = [P, P, P, P, P, P, P, P, c_size_t, P]
    L.holo_probe_init.argtypes = [P, P, P, P]
    L.holo_bin_frames.argtypes = [P, ctypes.c_int64, c_int32, c_int32, c_int32, c_int32, P, P]
    L.holo_upsample_frames.argtypes = [P, ctypes.c_int64, c_int32, c_int32, c_int32, P, P]
    L.holo_upsample_volume.argtypes = [P, c_int32, c_int32, c_int32, P, P]
    L.holo_cg_workspace_bytes.argtypes = [P, POINTER(c_size_t)]
    L.holo_cg.argtypes = [P, P, P, P, P, c_int32, c_double, P, P, P, P, c_size_t, P]
    L.holo2d_plan_create.argtypes = [c_int32, POINTER(c_int32), c_int32, POINTER(c_double),
                                     c_double, c_double, POINTER(c_void_p)]
    L.holo2d_plan_destroy.argtypes = [P]
    L.holo2d_plan_set_functional.argtypes = [P, c_int32]
    L.holo2d_offsets.argtypes = [P, POINTER(ctypes.c_int64), POINTER(ctypes.c_int64)]
    L.holo2d_workspace_bytes.argtypes = [P, POINTER(c_size_t)]
    L.holo2d_fwd.argtypes = [P, P, P, P, P, c_size_t, P]
    L.holo2d_objective.argtypes = [P, P, P, P, P, P, P, c_size_t, P]
    L.holo2d_grad.argtypes = [P, P, P, P, P, P, P, P, P, c_size_t, P]
    L.holo2d_noalloc_bytes.argtypes = [P, POINTER(c_size_t)]
    L.holo2d_grad_noalloc.argtypes = [P, P, P, P, P, P, P, P, P]
    L.holo_timing_enable.argtypes = [P, c_int32]
    L.holo_timing_read.argtypes = [P, c_int32, POINTER(c_double), POINTER(ctypes.c_int64)]
    L.holo_plan_ray_groups.argtypes = [P, P, P, c_int32, POINTER(c_int32)]
    for name in EXPORTS[:-1]:
        getattr(L, name).restype = c_int32
    L.holo_last_error.restype = c_char_p
    L.holo_last_error.argtypes = []
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise HoloError(status, lib().holo_last_error().decode())


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def bin_frames(t, b, amplitude=True, stream=None):
    """holo_bin_frames on a contiguous float32 GPU tensor [..., H, W]."""
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() < 2:
        raise ValueError("bin_frames needs a contiguous float32 GPU tensor [..., H, W]")
    H, W = t.shape[-2:]
    n = t.numel() // (H * W)
    out = torch.empty(t.shape[:-2] + (H // b, W // b), dtype=torch.float32, device=t.device)
    _check(lib().holo_bin_frames(_ptr(t), n, H, W, int(b), 1 if amplitude else 0, _ptr(out),
                                 _stream(stream)))
    return out


def upsample_frames(t, f, stream=None):
    """holo_upsample_frames on a contiguous complex64 GPU tensor [..., H, W]."""
    import torch
    if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() or t.dim() < 2:
        raise ValueError("upsample_frames needs a contiguous complex64 GPU tensor [..., H, W]")
    H, W = t.shape[-2:]
    n = t.numel() // (H * W)
    out = torch.empty(t.shape[:-2] + (H * f, W * f), dtype=torch.complex64, device=t.device)
    _check(lib().holo_upsample_frames(_ptr(t), n, H, W, int(f), _ptr(out), _stream(stream)))
    return out


def upsample_volume(t, f, stream=None):
    """holo_upsample_volume on a contiguous complex64 GPU tensor [H, W, W]."""
    import torch
    if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 3 \
            or t.shape[1] != t.shape[2]:
        raise ValueError("upsample_volume needs a contiguous complex64 GPU tensor [H, W, W]")
    H, W = t.shape[0], t.shape[1]
    out = torch.empty((H * f, W * f, W * f), dtype=torch.complex64, device=t.device)
    _check(lib().holo_upsample_volume(_ptr(t), H, W, int(f), _ptr(out), _stream(stream)))
    return out


class Plan:
    """A holo_plan plus the workspace it needs (allocated with torch)."""

    def __init__(self, H: int, W: int, theta: Sequence[float], mag_rel: Sequence[float],
                 m0: float, fresnel0: float, kappa: float, shift=None, chunk: int = 0):
        self.H, self.W = int(H), int(W)
        self._theta = np.ascontiguousarray(theta, dtype=np.float64)
        self._mag = np.ascontiguousarray(mag_rel, dtype=np.float64)
        self.n_angles, self.n_dist = len(self._theta), len(self._mag)
        self._shift = None if shift is None else np.ascontiguousarray(shift, dtype=np.float32)
        if self._shift is not None and self._shift.shape != (self.n_angles, self.n_dist, 2):
            raise ValueError("shift must have shape (n_angles, n_dist, 2)")
        g = holo_geom()
        g.det_rows, g.det_cols = self.H, self.W
        g.n_angles, g.n_dist = self.n_angles, self.n_dist
        g.theta = self._theta.ctypes.data_as(POINTER(c_double))
        g.mag_rel = self._mag.ctypes.data_as(POINTER(c_double))
        g.m0, g.fresnel0, g.kappa = float(m0), float(fresnel0), float(kappa)
        g.shift = (self._shift.ctypes.data_as(POINTER(c_float)) if self._shift is not None
                   else POINTER(c_float)())
        g.chunk = int(chunk)
        h = c_void_p()
        _check(lib().holo_plan_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h
        n = c_size_t()
        _check(lib().holo_workspace_bytes(h, ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        self._ws = None
        self.pad = 1
        self.projector = "joseph"

    @classmethod
    def for_workload(cls, wl, theta=None, shift=None):
        return cls(wl.H, wl.W, wl.theta if theta is None else theta, wl.mag_rel, wl.m0,
                   wl.fresnel0, wl.kappa, shift=shift, chunk=wl.chunk)

    def close(self):
        if getattr(self, "_h", None):
            lib().holo_plan_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device):
        import torch
        if self._ws is None or self._ws.device != torch.device(device):
            self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)
        return self._ws

    @property
    def chunk(self):
        c = c_int32()
        _check(lib().holo_plan_get_chunk(self._h, ctypes.byref(c)))
        return int(c.value)

    def set_chunk(self, chunk):
        """Angles per chunk; updates workspace_bytes (the workspace is
        reallocated on the next call if it grew)."""
        _check(lib().holo_plan_set_chunk(self._h, c_int32(int(chunk))))
        self._refresh_workspace_size()

    def set_probe_shifts(self, shifts):
        """Probe shifts s_kj, an (n_angles, n_dist, 2) array of (s_y, s_x)
        pixels, or None to remove them; updates workspace_bytes."""
        if shifts is None:
            _check(lib().holo_plan_set_probe_shifts(self._h, None))
            self._pshift = None
        else:
            a = np.ascontiguousarray(shifts, dtype=np.float32)
            if a.shape != (self.n_angles, self.n_dist, 2):
                raise ValueError("probe shifts must have shape (n_angles, n_dist, 2)")
            _check(lib().holo_plan_set_probe_shifts(self._h, a.ctypes.data_as(c_void_p)))
            self._pshift = a
        self._refresh_workspace_size()

    def _refresh_workspace_size(self):
        n = c_size_t()
        _check(lib().holo_workspace_bytes(self._h, ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        if self._ws is not None and self._ws.numel() < self.workspace_bytes:
            self._ws = None

    def tune_key(self, device):
        import torch
        return "%dx%dx%d_%dangles_%dplanes:%s" % (
            self.H, self.W, self.W, self.n_angles, self.n_dist,
            torch.cuda.get_device_name(torch.device(device)))

    def autotune(self, u, q, amp, amp_ref, candidates=(16, 32, 64, 128), cache=None,
                 stream=None):
        """Choose the chunk size by timing one gradient per candidate
        (holo_plan_autotune).  With `cache` (a JSON file path; default the
        HOLO_TUNE_CACHE environment variable, if set) a result stored for
        this geometry and device is reused without timing, and a new result
        is stored.  Returns (chunk, {candidate: ms} or None when cached)."""
        import json
        import torch
        self._check_data(u, q, amp, amp_ref)
        cache = cache or os.environ.get("HOLO_TUNE_CACHE")
        key = self.tune_key(u.device)
        cands = sorted({max(int(c), 1) for c in candidates})
        if cache and os.path.exists(cache):
            with open(cache) as f:
                entry = json.load(f).get(key)
            if entry is not None and int(entry["chunk"]) in cands:
                self.set_chunk(int(entry["chunk"]))
                return int(entry["chunk"]), None
        chunk0 = self.chunk
        need = 0
        for c in cands:
            self.set_chunk(c)
            need = max(need, self.workspace_bytes)
        self.set_chunk(chunk0)
        ws = torch.empty(need, dtype=torch.uint8, device=u.device)
        F = torch.empty((1,), dtype=torch.float64, device=u.device)
        g_u, g_q = torch.empty_like(u), torch.empty_like(q)
        arr = (c_int32 * len(cands))(*cands)
        times = (c_float * len(cands))()
        best = c_int32()
        _check(lib().holo_plan_autotune(self._h, _ptr(u), _ptr(q), _ptr(amp), _ptr(amp_ref),
                                        _ptr(F), _ptr(g_u), _ptr(g_q), arr, c_int32(len(cands)),
                                        _ptr(ws), c_size_t(ws.numel()), ctypes.byref(best),
                                        times, _stream(stream)))
        del ws, g_u, g_q
        self._ws = None
        self._refresh_workspace_size()
        result = {c: float(t) for c, t in zip(cands, times)}
        if cache:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = {"chunk": int(best.value), "ms": {str(c): t for c, t in result.items()}}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return int(best.value), result

    TILES = {"chunk": 0, "col_tile": 1, "fs_slab": 2, "fwd_bins": 3, "overlap": 4}

    def set_tile(self, name, value):
        """Set a launch-shape parameter ("chunk", "col_tile", "fs_slab",
        "fwd_bins", "overlap")."""
        _check(lib().holo_plan_set_tile(self._h, c_int32(self.TILES[name]), c_int32(int(value))))
        self._refresh_workspace_size()

    def get_tile(self, name):
        v = c_int32()
        _check(lib().holo_plan_get_tile(self._h, c_int32(self.TILES[name]), ctypes.byref(v)))
        return int(v.value)

    def autotune_tile(self, name, u, q, amp, amp_ref, candidates, stream=None):
        """Time one gradient per candidate value of a launch-shape parameter
        (holo_plan_autotune_tile) and keep the fastest.  Returns
        (value, {candidate: ms})."""
        import torch
        self._check_data(u, q, amp, amp_ref)
        cands = [int(c) for c in candidates]
        v0 = self.get_tile(name)
        need = 0
        for c in cands:
            self.set_tile(name, c)
            need = max(need, self.workspace_bytes)
        self.set_tile(name, v0)
        ws = torch.empty(need, dtype=torch.uint8, device=u.device)
        F = torch.empty((1,), dtype=torch.float64, device=u.device)
        g_u, g_q = torch.empty_like(u), torch.empty_like(q)
        arr = (c_int32 * len(cands))(*cands)
        times = (c_float * len(cands))()
        best = c_int32()
        _check(lib().holo_plan_autotune_tile(self._h, c_int32(self.TILES[name]), _ptr(u), _ptr(q),
                                             _ptr(amp), _ptr(amp_ref), _ptr(F), _ptr(g_u),
                                             _ptr(g_q), arr, c_int32(len(cands)), _ptr(ws),
                                             c_size_t(ws.numel()), ctypes.byref(best), times,
                                             _stream(stream)))
        del ws, g_u, g_q
        self._ws = None
        self._refresh_workspace_size()
        return int(best.value), {c: float(t) for c, t in zip(cands, times)}

    def autotune_tiles(self, u, q, amp, amp_ref, chunks=(16, 32, 64, 128), cache=None):
        """The chunk (autotune), then the column tile (default or half), the
        forward bin block (Joseph) or the slab depth (Fourier-slice, 2, 4,
        8), and the overlapped forward (Joseph), each timed with the others
        fixed.  Returns {name: (value, times)}; with a
        cache file the choices are stored and reused like the chunk's."""
        import json
        cache = cache or os.environ.get("HOLO_TUNE_CACHE")
        key = self.tune_key(u.device) + ":tiles:" + self.projector
        if cache and os.path.exists(cache):
            with open(cache) as f:
                entry = json.load(f).get(key)
            names = ("chunk", "col_tile", "fs_slab", "fwd_bins", "overlap")
            if entry is not None and all(n in entry for n in names):
                for name in names:
                    self.set_tile(name, int(entry[name]))
                return {name: (int(entry[name]), None) for name in names}
        out = {"chunk": self.autotune(u, q, amp, amp_ref, candidates=chunks)}
        out["col_tile"] = self.autotune_tile("col_tile", u, q, amp, amp_ref,
                                             [0, self.default_col_tile() // 2])
        if self.projector == "fourier":
            out["fs_slab"] = self.autotune_tile("fs_slab", u, q, amp, amp_ref, [2, 4, 8])
            out["fwd_bins"] = (self.get_tile("fwd_bins"), None)
        else:
            out["fs_slab"] = (self.get_tile("fs_slab"), None)
            bins = [b for b in (16, 8) if self._tile_ok("fwd_bins", b)]
            out["fwd_bins"] = self.autotune_tile("fwd_bins", u, q, amp, amp_ref, bins)
        out["overlap"] = (self.autotune_tile("overlap", u, q, amp, amp_ref, [0, 1])
                          if self.projector != "fourier" else (self.get_tile("overlap"), None))
        if cache:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = {name: v[0] for name, v in out.items()}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return out

    def _tile_ok(self, name, value):
        v0 = self.get_tile(name)
        ok = lib().holo_plan_set_tile(self._h, c_int32(self.TILES[name]), c_int32(int(value))) == 0
        lib().holo_plan_set_tile(self._h, c_int32(self.TILES[name]), c_int32(v0))
        return ok

    def default_col_tile(self):
        """The column pass's default columns per workgroup for this H."""
        return 4 if self.H >= 2048 else (8 if self.H >= 1024 else 16)

    FUNCTIONALS = {"amplitude": 0, "intensity": 1, "conventional": 2}

    PROJECTORS = {"joseph": 0, "fourier": 1}

    def set_projector(self, name):
        """"joseph" (ray-driven sums, default) or "fourier" (Fourier-slice
        gridding); updates workspace_bytes."""
        _check(lib().holo_plan_set_projector(self._h, c_int32(self.PROJECTORS[name])))
        self.projector = name
        self._refresh_workspace_size()

    def set_padding(self, pad):
        """1: periodic propagation (default); 2: padded propagation (fields
        zero outside the field of view, grids of 2H x 2W)."""
        _check(lib().holo_plan_set_padding(self._h, c_int32(int(pad))))
        self.pad = int(pad)

    def set_functional(self, name):
        """"amplitude" (F2, default; amp = sqrt(d)) or "intensity" (F1; amp
        and amp_ref then hold the intensities d)."""
        _check(lib().holo_plan_set_functional(self._h, c_int32(self.FUNCTIONALS[name])))
        self.functional = name

    # -- argument checks (shapes, dtypes, devices) -------------------------
    def _vol(self, t, name):
        import torch
        if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() \
                or tuple(t.shape) != (self.H, self.W, self.W):
            raise ValueError("%s must be a contiguous complex64 GPU tensor of shape (H, W, W)" % name)
        return t

    def _frame(self, t, name, dtype=None):
        import torch
        dtype = torch.complex64 if dtype is None else dtype
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() \
                or tuple(t.shape) != (self.H, self.W):
            raise ValueError("%s must be a contiguous %s GPU tensor of shape (H, W)" % (name, dtype))
        return t

    def _frames(self, t, n, name, dtype=None):
        import torch
        dtype = torch.complex64 if dtype is None else dtype
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() \
                or tuple(t.shape) != (n, self.n_dist, self.H, self.W):
            raise ValueError("%s must be a contiguous %s GPU tensor of shape (%d, n_dist, H, W)"
                             % (name, dtype, n))
        return t

    # -- entry points with the C ABI's names ------------------------------
    def holo_fwd(self, u, q, k0=0, k1=None, v=None, stream=None):
        import torch
        k1 = self.n_angles if k1 is None else k1
        self._vol(u, "u"), self._frame(q, "q")
        if v is None:
            v = torch.empty((k1 - k0, self.n_dist, self.H, self.W), dtype=torch.complex64,
                            device=u.device)
        self._frames(v, k1 - k0, "v")
        ws = self.workspace(u.device)
        _check(lib().holo_fwd(self._h, _ptr(u), _ptr(q), int(k0), int(k1), _ptr(v),
                              _ptr(ws), c_size_t(ws.numel()), _stream(stream)))
        return v

    def holo_adj(self, u, q, w, k0=0, k1=None, g_u=None, g_q=None, want_u=True, want_q=True,
                 stream=None):
        import torch
        k1 = self.n_angles if k1 is None else k1
        self._vol(u, "u"), self._frame(q, "q"), self._frames(w, k1 - k0, "w")
        if want_u and g_u is None:
            g_u = torch.empty_like(u)
        if want_q and g_q is None:
            g_q = torch.empty_like(q)
        ws = self.workspace(u.device)
        _check(lib().holo_adj(self._h, _ptr(u), _ptr(q), int(k0), int(k1), _ptr(w),
                              _ptr(g_u if want_u else None), _ptr(g_q if want_q else None),
                              _ptr(ws), c_size_t(ws.numel()), _stream(stream)))
        return g_u, g_q

    def holo_objective(self, u, q, amp, amp_ref, F=None, stream=None):
        import torch
        self._check_data(u, q, amp, amp_ref)
        if F is None:
            F = torch.empty((1,), dtype=torch.float64, device=u.device)
        ws = self.workspace(u.device)
        _check(lib().holo_objective(self._h, _ptr(u), _ptr(q), _ptr(amp), _ptr(amp_ref), _ptr(F),
                                    _ptr(ws), c_size_t(ws.numel()), _stream(stream)))
        return F

    def holo_grad(self, u, q, amp, amp_ref, F=None, g_u=None, g_q=None, want_F=True,
                  want_u=True, want_q=True, stream=None):
        import torch
        self._check_data(u, q, amp, amp_ref)
        if want_F and F is None:
            F = torch.empty((1,), dtype=torch.float64, device=u.device)
        if want_u and g_u is None:
            g_u = torch.empty_like(u)
        if want_q and g_q is None:
            g_q = torch.empty_like(q)
        ws = self.workspace(u.device)
        _check(lib().holo_grad(self._h, _ptr(u), _ptr(q), _ptr(amp), _ptr(amp_ref),
                               _ptr(F if want_F else None), _ptr(g_u if want_u else None),
                               _ptr(g_q if want_q else None), _ptr(ws), c_size_t(ws.numel()),
                               _stream(stream)))
        return (F if want_F else None), (g_u if want_u else None), (g_q if want_q else None)

    def holo_grad_object(self, u, q, amp, amp_ref, stream=None):
        F, g_u, _ = self.holo_grad(u, q, amp, amp_ref, want_q=False, stream=stream)
        return F, g_u

    def holo_grad_probe(self, u, q, amp, amp_ref, stream=None):
        F, _, g_q = self.holo_grad(u, q, amp, amp_ref, want_u=False, stream=stream)
        return F, g_q

    def holo_probe_init(self, amp_ref, q=None, stream=None):
        """Initial probe: the reference amplitude propagated back to sample
        plane 0 (complex64 (H, W) on amp_ref's device)."""
        import torch
        self._frame(amp_ref, "amp_ref", torch.float32)
        if q is None:
            q = torch.empty(amp_ref.shape, dtype=torch.complex64, device=amp_ref.device)
        self._frame(q, "q")
        _check(lib().holo_probe_init(self._h, _ptr(amp_ref), _ptr(q), _stream(stream)))
        return q

    def cg_workspace_bytes(self):
        n = c_size_t()
        _check(lib().holo_cg_workspace_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def holo_cg(self, u, q, amp, amp_ref, iters, step0, in_place=False, stream=None):
        """`iters` Dai-Yuan conjugate-gradient iterations on (u, q).  Returns
        (u, q, F_hist[iters + 1], steps[iters], halvings[iters]); u and q are
        overwritten when in_place, else copies are iterated."""
        import torch
        self._check_data(u, q, amp, amp_ref)
        if not in_place:
            u, q = u.clone(), q.clone()
        iters = int(iters)
        F_hist = np.zeros(max(iters + 1, 1), dtype=np.float64)
        steps = np.zeros(max(iters, 1), dtype=np.float64)
        halv = np.zeros(max(iters, 1), dtype=np.int32)
        ws = torch.empty(self.cg_workspace_bytes(), dtype=torch.uint8, device=u.device)
        _check(lib().holo_cg(self._h, _ptr(u), _ptr(q), _ptr(amp), _ptr(amp_ref),
                             c_int32(iters), c_double(step0),
                             F_hist.ctypes.data_as(c_void_p), steps.ctypes.data_as(c_void_p),
                             halv.ctypes.data_as(c_void_p), _ptr(ws), c_size_t(ws.numel()),
                             _stream(stream)))
        return u, q, F_hist[:iters + 1], steps[:iters], halv[:iters]

    def timing(self, on=True):
        """Record HIP events around every kernel launch of later calls."""
        _check(lib().holo_timing_enable(self._h, 1 if on else 0))

    def kernel_times(self):
        """{class: (total_ms, launches)} recorded since timing(True)."""
        out = {}
        for i, name in enumerate(KERNEL_CLASSES):
            ms, n = c_double(), ctypes.c_int64()
            _check(lib().holo_timing_read(self._h, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, int(n.value))
        return out

    def ray_groups(self):
        """[(first angle, count)] of the forward ray sums' angle groups."""
        n = c_int32()
        _check(lib().holo_plan_ray_groups(self._h, None, None, 0, ctypes.byref(n)))
        first = (c_int32 * max(n.value, 1))()
        count = (c_int32 * max(n.value, 1))()
        _check(lib().holo_plan_ray_groups(self._h, first, count, n.value, ctypes.byref(n)))
        return [(int(first[i]), int(count[i])) for i in range(n.value)]

    def _check_data(self, u, q, amp, amp_ref):
        import torch
        self._vol(u, "u"), self._frame(q, "q")
        self._frames(amp, self.n_angles, "amp", torch.float32)
        self._frame(amp_ref, "amp_ref", torch.float32)


class Plan2D:
    """A holo2d_plan: independent single-angle problems of uneven sizes in one
    packed layout (see include/holo.h)."""

    def __init__(self, sizes, mag_rel, m0, fresnel0):
        self.sizes = [int(n) for n in sizes]
        self.n_inst = len(self.sizes)
        self._mag = np.ascontiguousarray(mag_rel, dtype=np.float64)
        self.n_dist = len(self._mag)
        sz = (c_int32 * self.n_inst)(*self.sizes)
        h = c_void_p()
        _check(lib().holo2d_plan_create(self.n_inst, sz, self.n_dist,
                                        self._mag.ctypes.data_as(POINTER(c_double)),
                                        float(m0), float(fresnel0), ctypes.byref(h)))
        self._h = h
        offs = (ctypes.c_int64 * self.n_inst)()
        tot = ctypes.c_int64()
        _check(lib().holo2d_offsets(h, offs, ctypes.byref(tot)))
        self.offsets = [int(o) for o in offs]
        self.total = int(tot.value)
        n = c_size_t()
        _check(lib().holo2d_workspace_bytes(h, ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        self._ws = None
        self.functional = "amplitude"

    def set_functional(self, name):
        """"amplitude" (F2, default; amp = sqrt(d)) or "intensity" (F1; amp
        and amp_ref then hold the intensities d)."""
        _check(lib().holo2d_plan_set_functional(self._h, c_int32(Plan.FUNCTIONALS[name])))
        self.functional = name

    def close(self):
        if getattr(self, "_h", None):
            lib().holo2d_plan_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device):
        import torch
        if self._ws is None or self._ws.device != torch.device(device):
            self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)
        return self._ws

    # packing helpers (host-side list <-> packed tensor)
    def pack(self, frames, planes=False, dtype=None, device=None):
        import torch
        parts = []
        for f in frames:
            t = torch.as_tensor(np.ascontiguousarray(f))
            parts.append(t.reshape(-1))
        out = torch.cat(parts)
        if dtype is not None:
            out = out.to(dtype)
        return out.to(device) if device is not None else out

    def unpack(self, packed, planes=False):
        out = []
        k = self.n_dist if planes else 1
        for i, n in enumerate(self.sizes):
            o = k * self.offsets[i]
            blk = packed[o:o + k * n * n]
            out.append(blk.reshape((k, n, n) if planes else (n, n)))
        return out

    def _chk(self, t, planes, name, dtype):
        k = self.n_dist if planes else 1
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != k * self.total:
            raise ValueError("%s must be a contiguous packed %s GPU tensor of %d elements"
                             % (name, dtype, k * self.total))

    def holo2d_fwd(self, psi, q, v=None, stream=None):
        import torch
        self._chk(psi, False, "psi", torch.complex64)
        self._chk(q, False, "q", torch.complex64)
        if v is None:
            v = torch.empty(self.n_dist * self.total, dtype=torch.complex64, device=psi.device)
        self._chk(v, True, "v", torch.complex64)
        ws = self.workspace(psi.device)
        _check(lib().holo2d_fwd(self._h, _ptr(psi), _ptr(q), _ptr(v), _ptr(ws),
                                c_size_t(ws.numel()), _stream(stream)))
        return v

    def holo2d_objective(self, psi, q, amp, amp_ref, F=None, stream=None):
        import torch
        self._chk_data(psi, q, amp, amp_ref)
        if F is None:
            F = torch.empty(self.n_inst, dtype=torch.float64, device=psi.device)
        ws = self.workspace(psi.device)
        _check(lib().holo2d_objective(self._h, _ptr(psi), _ptr(q), _ptr(amp), _ptr(amp_ref),
                                      _ptr(F), _ptr(ws), c_size_t(ws.numel()), _stream(stream)))
        return F

    def holo2d_grad(self, psi, q, amp, amp_ref, F=None, g_psi=None, g_q=None, stream=None):
        import torch
        self._chk_data(psi, q, amp, amp_ref)
        if F is None:
            F = torch.empty(self.n_inst, dtype=torch.float64, device=psi.device)
        if g_psi is None:
            g_psi = torch.empty_like(psi)
        if g_q is None:
            g_q = torch.empty_like(q)
        ws = self.workspace(psi.device)
        _check(lib().holo2d_grad(self._h, _ptr(psi), _ptr(q), _ptr(amp), _ptr(amp_ref), _ptr(F),
                                 _ptr(g_psi), _ptr(g_q), _ptr(ws), c_size_t(ws.numel()),
                                 _stream(stream)))
        return F, g_psi, g_q

    def noalloc_bytes(self):
        """Bytes of the library's static scratch array that
        holo2d_grad_noalloc needs for this plan."""
        n = c_size_t()
        _check(lib().holo2d_noalloc_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def holo2d_grad_noalloc(self, psi, q, amp, amp_ref, F, g_psi, g_q, stream=None):
        """holo2d_grad through the allocation-free entry point: the library
        allocates nothing (its static scratch array holds the tables and the
        workspace); the outputs are the caller's preallocated tensors (F,
        g_psi, g_q; each may be None)."""
        import torch
        self._chk_data(psi, q, amp, amp_ref)
        if g_psi is not None:
            self._chk(g_psi, False, "g_psi", torch.complex64)
        if g_q is not None:
            self._chk(g_q, False, "g_q", torch.complex64)
        if F is not None and (F.dtype != torch.float64 or not F.is_cuda or F.numel() != self.n_inst):
            raise ValueError("F must be a float64 GPU tensor of %d elements" % self.n_inst)
        _check(lib().holo2d_grad_noalloc(self._h, _ptr(psi), _ptr(q), _ptr(amp), _ptr(amp_ref),
                                         _ptr(F), _ptr(g_psi), _ptr(g_q), _stream(stream)))
        return F, g_psi, g_q

    def _chk_data(self, psi, q, amp, amp_ref):
        import torch
        self._chk(psi, False, "psi", torch.complex64)
        self._chk(q, False, "q", torch.complex64)
        self._chk(amp, True, "amp", torch.float32)
        self._chk(amp_ref, False, "amp_ref", torch.float32)


def _make_autograd():
    import torch

    class HoloLoss(torch.autograd.Function):
        """F(u, q) as a differentiable scalar.

        Forward and backward share one sweep: the forward call runs holo_grad
        and keeps g_u and g_q; backward scales them by the incoming gradient.
        """

        @staticmethod
        def forward(ctx, u, q, amp, amp_ref, plan):
            need_u, need_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            F, g_u, g_q = plan.holo_grad(u.detach(), q.detach(), amp, amp_ref,
                                         want_u=need_u, want_q=need_q)
            ctx.save_for_backward(*(t for t in (g_u, g_q) if t is not None))
            ctx.have = (g_u is not None, g_q is not None)
            return F[0]

        @staticmethod
        def backward(ctx, grad_out):
            saved = list(ctx.saved_tensors)
            g_u = saved.pop(0) if ctx.have[0] else None
            g_q = saved.pop(0) if ctx.have[1] else None
            s = grad_out.to(torch.float32)
            return (None if g_u is None else g_u * s, None if g_q is None else g_q * s,
                    None, None, None)

    return HoloLoss


_HoloLoss = None


def holo_loss(u, q, amp, amp_ref, plan):
    """Differentiable objective F(u, q) (a 0-dim float64 tensor)."""
    global _HoloLoss
    if _HoloLoss is None:
        _HoloLoss = _make_autograd()
    return _HoloLoss.apply(u, q, amp, amp_ref, plan)
