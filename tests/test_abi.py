"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any device
work (plan creation is host-only)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2407_20304_amd import holo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "holo.h")

pytestmark = pytest.mark.skipif(not os.path.exists(holo.LIB_PATH),
                                reason="libholo.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(holo(?:2d)?_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(holo.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(holo.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def make_plan(**kw):
    args = dict(H=64, W=64, theta=np.linspace(0, np.pi, 10, endpoint=False),
                mag_rel=[1.0, 1.08, 1.25, 1.5], m0=300.0, fresnel0=0.01, kappa=4667.35)
    args.update(kw)
    return holo.Plan(**args)


def test_plan_and_workspace_size():
    p = make_plan(chunk=4)
    # frames: Q, G (4 each), reference, transposed volume, psi chunk, X chunk,
    # sinogram; all complex64 64 x 64
    fr = 64 * 64 * 8
    assert p.workspace_bytes >= fr * (4 + 4 + 1 + 64 + 4 + 16 + 10)
    p.close()


@pytest.mark.parametrize("kw,status", [
    (dict(H=100), 2), (dict(W=7 * 64), 2), (dict(H=32), 2), (dict(W=4096), 2),
    (dict(m0=1.0), 1), (dict(m0=float("nan")), 1), (dict(fresnel0=0.0), 1),
    (dict(mag_rel=[1.0, 0.9]), 1), (dict(mag_rel=[1.0] * 9), 1), (dict(mag_rel=[]), 1),
    (dict(theta=[]), 1), (dict(theta=[0.0, float("inf")]), 1), (dict(kappa=float("inf")), 1),
    (dict(chunk=-1), 1),
])
def test_plan_rejects_bad_geometry(kw, status):
    with pytest.raises(holo.HoloError) as e:
        make_plan(**kw)
    assert e.value.status == status
    assert holo.lib().holo_last_error().decode()


def test_plan_rejects_non_finite_shift():
    sh = np.zeros((10, 4, 2), np.float32)
    sh[3, 2, 1] = np.nan
    with pytest.raises(holo.HoloError) as e:
        make_plan(shift=sh)
    assert e.value.status == 1


def test_null_arguments_return_invalid_argument():
    L = holo.lib()
    assert L.holo_plan_create(None, None) == 1
    p = make_plan()
    n = ctypes.c_size_t()
    assert L.holo_workspace_bytes(None, ctypes.byref(n)) == 1
    # compute calls validate on the host before touching the device
    buf = ctypes.c_void_p(1)
    assert L.holo_fwd(p._h, None, buf, 0, 1, buf, buf, 1 << 40, None) == 1
    assert L.holo_fwd(p._h, buf, buf, 0, 11, buf, buf, 1 << 40, None) == 1
    assert L.holo_fwd(p._h, buf, buf, 3, 3, buf, buf, 1 << 40, None) == 1
    assert L.holo_adj(p._h, buf, buf, 0, 1, None, buf, buf, buf, 1 << 40, None) == 1
    assert L.holo_objective(p._h, buf, buf, None, buf, buf, buf, 1 << 40, None) == 1
    assert L.holo_grad(None, buf, buf, buf, buf, buf, buf, buf, buf, 1 << 40, None) == 1
    assert L.holo_grad_object(p._h, buf, buf, buf, buf, buf, None, buf, 1 << 40, None) == 1
    assert L.holo_grad_probe(p._h, buf, buf, buf, buf, buf, None, buf, 1 << 40, None) == 1
    # workspace checks come before any device work as well
    assert L.holo_grad(p._h, buf, buf, buf, buf, buf, buf, buf, None, 1 << 40, None) == 1
    assert L.holo_grad(p._h, buf, buf, buf, buf, buf, buf, buf, buf, 16, None) == 3
    assert L.holo_plan_destroy(None) == 0
    p.close()


def test_chunk_and_autotune_validate_on_the_host():
    L = holo.lib()
    p = make_plan(chunk=4)
    c = ctypes.c_int32()
    assert L.holo_plan_get_chunk(p._h, ctypes.byref(c)) == 0 and c.value == 4
    assert L.holo_plan_set_chunk(None, 8) == 1
    ws4 = p.workspace_bytes
    p.set_chunk(8)
    assert p.chunk == 8 and p.workspace_bytes > ws4
    p.set_chunk(100)                      # clamped to n_angles
    assert p.chunk == 10
    # a chunk below the largest forward angle group (>= 1) is rejected
    assert L.holo_plan_set_chunk(p._h, 0) == 1
    assert L.holo_plan_set_chunk(p._h, -5) == 1
    buf = ctypes.c_void_p(1)
    best = ctypes.c_int32()
    cands = (ctypes.c_int32 * 2)(4, 8)
    args = [p._h, buf, buf, buf, buf, buf, buf, buf]
    assert L.holo_plan_autotune(None, *args[1:], cands, 2, buf, 1 << 40, ctypes.byref(best), None, None) == 1
    assert L.holo_plan_autotune(*args, cands, 0, buf, 1 << 40, ctypes.byref(best), None, None) == 1
    assert L.holo_plan_autotune(*args, None, 2, buf, 1 << 40, ctypes.byref(best), None, None) == 1
    bad = (ctypes.c_int32 * 2)(0, 8)
    assert L.holo_plan_autotune(*args, bad, 2, buf, 1 << 40, ctypes.byref(best), None, None) == 1
    assert p.chunk == 10                  # a rejected call leaves the plan as it was
    assert L.holo_plan_autotune(*args, cands, 2, buf, 16, ctypes.byref(best), None, None) == 3
    p.close()


def test_binning_entry_points_validate_on_the_host():
    L = holo.lib()
    buf, buf2 = ctypes.c_void_p(1), ctypes.c_void_p(2)
    assert L.holo_bin_frames(None, 1, 8, 8, 2, 1, buf2, None) == 1
    assert L.holo_bin_frames(buf, 0, 8, 8, 2, 1, buf2, None) == 1
    assert L.holo_bin_frames(buf, 1, 8, 6, 4, 1, buf2, None) == 1   # 4 does not divide 6
    assert L.holo_bin_frames(buf, 1, 8, 8, 0, 1, buf2, None) == 1
    assert L.holo_bin_frames(buf, 1, 8, 8, 2, 1, buf, None) == 1    # aliasing
    assert L.holo_upsample_frames(buf, 1, 8, 8, 0, buf2, None) == 1
    assert L.holo_upsample_frames(buf, 1, 8, 8, 2, buf, None) == 1
    assert L.holo_upsample_volume(None, 8, 8, 2, buf2, None) == 1
    assert L.holo_upsample_volume(buf, 8, 0, 2, buf2, None) == 1


def test_probe_shifts_validate_and_grow_the_workspace():
    L = holo.lib()
    p = make_plan(chunk=4)
    ws0 = p.workspace_bytes
    assert L.holo_plan_set_probe_shifts(None, None) == 1
    bad = np.zeros((10, 4, 2), np.float32)
    bad[3, 1, 0] = np.nan
    assert L.holo_plan_set_probe_shifts(p._h, bad.ctypes.data_as(ctypes.c_void_p)) == 1
    p.set_probe_shifts(np.ones((10, 4, 2), np.float32))
    assert p.workspace_bytes == ws0 + 4 * 4 * 64 * 64 * 8   # chunk x n_dist frames
    with pytest.raises(ValueError):
        p.set_probe_shifts(np.ones((10, 3, 2)))
    p.set_probe_shifts(None)
    assert p.workspace_bytes == ws0
    p.close()


def test_functional_switch_validates_on_the_host():
    L = holo.lib()
    p = make_plan()
    assert L.holo_plan_set_functional(None, 0) == 1
    assert L.holo_plan_set_functional(p._h, 3) == 1
    assert L.holo_plan_set_functional(p._h, -1) == 1
    assert L.holo_plan_set_functional(p._h, 2) == 0
    assert L.holo_plan_set_functional(p._h, 1) == 0
    assert L.holo_plan_set_functional(p._h, 0) == 0
    p.set_functional("intensity")
    assert p.functional == "intensity"
    p.close()
    q = holo.Plan2D([128, 64], [1.0, 1.25], 300.0, 0.01)
    assert L.holo2d_plan_set_functional(None, 0) == 1
    assert L.holo2d_plan_set_functional(q._h, 3) == 1
    assert L.holo2d_plan_set_functional(q._h, 2) == 0
    assert L.holo2d_plan_set_functional(q._h, 1) == 0
    q.set_functional("amplitude")
    assert q.functional == "amplitude"
    q.close()


def test_solver_entry_points_validate_on_the_host():
    L = holo.lib()
    p = make_plan()
    buf = ctypes.c_void_p(1)
    F = (ctypes.c_double * 4)()
    n = ctypes.c_size_t()
    assert L.holo_cg_workspace_bytes(None, ctypes.byref(n)) == 1
    assert L.holo_cg_workspace_bytes(p._h, ctypes.byref(n)) == 0
    # three (u, q)-sized vectors beyond the gradient's own workspace
    assert n.value >= p.workspace_bytes + 3 * 8 * (64 ** 3 + 64 ** 2)
    big = n.value
    assert L.holo_cg(None, buf, buf, buf, buf, 2, 1e-3, F, None, None, buf, big, None) == 1
    assert L.holo_cg(p._h, None, buf, buf, buf, 2, 1e-3, F, None, None, buf, big, None) == 1
    assert L.holo_cg(p._h, buf, buf, None, buf, 2, 1e-3, F, None, None, buf, big, None) == 1
    assert L.holo_cg(p._h, buf, buf, buf, buf, 2, 1e-3, None, None, None, buf, big, None) == 1
    assert L.holo_cg(p._h, buf, buf, buf, buf, -1, 1e-3, F, None, None, buf, big, None) == 1
    for step0 in (0.0, -1.0, float("nan"), float("inf")):
        assert L.holo_cg(p._h, buf, buf, buf, buf, 2, step0, F, None, None, buf, big, None) == 1
    assert L.holo_cg(p._h, buf, buf, buf, buf, 2, 1e-3, F, None, None, None, big, None) == 1
    assert L.holo_cg(p._h, buf, buf, buf, buf, 2, 1e-3, F, None, None, buf, big - 1, None) == 3
    # the gradient's workspace alone is not enough
    assert L.holo_cg(p._h, buf, buf, buf, buf, 2, 1e-3, F, None, None, buf,
                     p.workspace_bytes, None) == 3
    assert L.holo_probe_init(None, buf, buf, None) == 1
    assert L.holo_probe_init(p._h, None, buf, None) == 1
    assert L.holo_probe_init(p._h, buf, None, None) == 1
    assert L.holo_probe_init(p._h, buf, buf, None) == 1
    p.close()


def test_plain_library_exports_and_validates():
    from paper_2407_20304_amd import plain
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "holo_plain.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(holo_plain_\w+)\s*\(", text)))
    assert names == ["holo_plain_radon", "holo_plain_radon_adj"]
    L = plain.lib()
    buf = ctypes.c_void_p(1)
    for fn in (L.holo_plain_radon, L.holo_plain_radon_adj):
        assert fn(None, 8, 64, 0.5, buf, None) == 1
        assert fn(buf, 8, 64, 0.5, None, None) == 1
        assert fn(buf, 0, 64, 0.5, buf, None) == 1
        assert fn(buf, 8, 1, 0.5, buf, None) == 1
        assert fn(buf, 8, 64, float("nan"), buf, None) == 1


def test_batch_plan_offsets_and_validation():
    p = holo.Plan2D([128, 192, 512, 64], [1.0, 1.08, 1.25, 1.5], 300.0, 0.01)
    assert p.offsets == [0, 128 ** 2, 128 ** 2 + 192 ** 2, 128 ** 2 + 192 ** 2 + 512 ** 2]
    assert p.total == 128 ** 2 + 192 ** 2 + 512 ** 2 + 64 ** 2
    fr = p.total * 8
    assert p.workspace_bytes >= fr * (4 + 1 + 4 + 4)
    p.close()
    for sizes, status in (([100], 2), ([2048], 2), ([], 1)):
        with pytest.raises(holo.HoloError) as e:
            holo.Plan2D(sizes, [1.0, 1.1], 300.0, 0.01)
        assert e.value.status == status
    with pytest.raises(holo.HoloError) as e:
        holo.Plan2D([128], [1.0, 0.5], 300.0, 0.01)
    assert e.value.status == 1
    L = holo.lib()
    q = holo.Plan2D([128], [1.0], 300.0, 0.01)
    buf = ctypes.c_void_p(1)
    assert L.holo2d_grad(q._h, None, buf, buf, buf, buf, buf, buf, buf, 1 << 40, None) == 1
    assert L.holo2d_grad(q._h, buf, buf, buf, buf, buf, buf, buf, buf, 8, None) == 3
    assert L.holo2d_fwd(q._h, buf, buf, None, buf, 1 << 40, None) == 1
    q.close()


def test_noalloc_batch_gradient_validates_on_the_host():
    # the batch of the benchmark needs more than the static scratch array:
    # rejected with WORKSPACE_TOO_SMALL before any device work
    L = holo.lib()
    sizes = [512] * 96
    big = holo.Plan2D(sizes, [1.0, 1.08, 1.25, 1.5], 300.0, 0.01)
    assert big.noalloc_bytes() > (128 << 20)
    buf = ctypes.c_void_p(1)
    assert L.holo2d_grad_noalloc(big._h, buf, buf, buf, buf, buf, buf, buf, None) == 3
    assert b"static array" in L.holo_last_error()
    small = holo.Plan2D([128, 64], [1.0, 1.08, 1.25, 1.5], 300.0, 0.01)
    assert big.workspace_bytes < big.noalloc_bytes()
    assert 0 < small.noalloc_bytes() < (128 << 20)
    assert L.holo2d_grad_noalloc(small._h, None, buf, buf, buf, buf, buf, buf, None) == 1
    assert L.holo2d_grad_noalloc(None, buf, buf, buf, buf, buf, buf, buf, None) == 1
    big.close()
    small.close()


def test_padding_switch_validates_on_the_host():
    L = holo.lib()
    p = make_plan()
    assert L.holo_plan_set_padding(None, 2) == 1
    assert L.holo_plan_set_padding(p._h, 3) == 1
    assert L.holo_plan_set_padding(p._h, 0) == 1
    n0 = p.workspace_bytes
    p.set_padding(2)
    assert p.pad == 2
    n = ctypes.c_size_t()
    assert L.holo_workspace_bytes(p._h, ctypes.byref(n)) == 0 and n.value == n0
    # probe shifts are refused on a padded plan, and padding on a shifted one
    sh = np.zeros((10, 4, 2), np.float32)
    assert L.holo_plan_set_probe_shifts(p._h, sh.ctypes.data_as(ctypes.c_void_p)) == 1
    p.set_padding(1)
    p.set_probe_shifts(sh)
    assert L.holo_plan_set_padding(p._h, 2) == 1
    p.set_probe_shifts(None)
    p.close()
    big = make_plan(W=2048)          # 2W = 4096 exceeds the padded transforms
    assert L.holo_plan_set_padding(big._h, 2) == 2
    assert L.holo_plan_set_padding(big._h, 1) == 0
    big.close()


def test_projector_switch_validates_on_the_host():
    L = holo.lib()
    p = make_plan()
    assert L.holo_plan_set_projector(None, 1) == 1
    assert L.holo_plan_set_projector(p._h, 2) == 1
    n0 = p.workspace_bytes
    p.set_projector("fourier")
    # 8 grids of (2W)^2 and 8 x n_angles x (W + 2) polar samples (complex64)
    # in place of the two slice-blocked volume copies (64 rows of 64 + 64)
    vol = 2 * 64 * 64 * (64 + 64) * 8
    assert p.workspace_bytes >= n0 - vol + 8 * (2 * 64) ** 2 * 8 + 8 * 10 * 66 * 8
    p.set_projector("joseph")
    assert p.workspace_bytes == n0
    p.close()
    big = make_plan(W=2048)
    assert L.holo_plan_set_projector(big._h, 1) == 2
    big.close()


def test_tile_parameters_validate_on_the_host():
    L = holo.lib()
    p = make_plan()          # 64 x 64: the column pass takes 16 columns, or 8
    v = ctypes.c_int32()
    assert L.holo_plan_set_tile(None, 1, 8) == 1
    assert L.holo_plan_set_tile(p._h, 5, 8) == 1          # unknown parameter
    # the overlapped forward: 0 or 1, and a second psi buffer (one chunk of
    # 64 x 64 frames) in the workspace when on
    n0 = p.workspace_bytes
    assert L.holo_plan_set_tile(p._h, 4, 2) == 1
    p.set_tile("overlap", 1)
    assert p.get_tile("overlap") == 1
    assert p.workspace_bytes >= n0 + p.get_tile("chunk") * 64 * 64 * 8
    p.set_tile("overlap", 0)
    assert p.workspace_bytes == n0
    assert L.holo_plan_set_tile(p._h, 3, 12) == 1         # forward bins are 16 or 8
    assert L.holo_plan_set_tile(p._h, 3, 8) == 0
    assert L.holo_plan_get_tile(p._h, 3, ctypes.byref(v)) == 0 and v.value == 8
    assert L.holo_plan_set_tile(p._h, 3, 16) == 0
    assert L.holo_plan_set_tile(p._h, 1, 4) == 1
    assert L.holo_plan_set_tile(p._h, 1, 8) == 0
    assert L.holo_plan_get_tile(p._h, 1, ctypes.byref(v)) == 0 and v.value == 8
    assert L.holo_plan_set_tile(p._h, 1, 0) == 0
    assert L.holo_plan_set_tile(p._h, 2, 3) == 1
    assert L.holo_plan_set_tile(p._h, 2, 4) == 0
    assert L.holo_plan_set_tile(p._h, 0, 2) == 0          # chunk 2 >= largest angle group
    assert L.holo_plan_get_tile(p._h, 0, ctypes.byref(v)) == 0 and v.value == 2
    assert p.default_col_tile() == 16
    buf = ctypes.c_void_p(1)
    cands = (ctypes.c_int32 * 2)(0, 3)
    best = ctypes.c_int32()
    # an invalid candidate is refused before any device work
    assert L.holo_plan_autotune_tile(p._h, 1, buf, buf, buf, buf, buf, buf, buf, cands, 2, buf,
                                     1 << 40, ctypes.byref(best), None, None) == 1
    p.close()
