"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/stencil.h declares, and rejects bad arguments
synchronously with the documented status codes."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")

sf = pytest.importorskip("paper_2103_09235_amd")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z0-9_]+)\s*\(", text)))


def test_header_and_exports_agree():
    decl = declared_symbols()
    assert decl, "no declarations parsed"
    assert sorted(sf.EXPORTS) == decl
    lib = ctypes.CDLL(sf.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_version_and_last_error():
    assert "gfx950" in sf.stencil_version()
    assert isinstance(sf.stencil_last_error(), str)


@pytest.mark.parametrize("args,code", [
    ((0, 1, sf.STENCIL_BOX), sf.STENCIL_E_ARG),
    ((4, 1, sf.STENCIL_BOX), sf.STENCIL_E_ARG),
    ((2, 0, sf.STENCIL_BOX), sf.STENCIL_E_ARG),
    ((2, 1, 7), sf.STENCIL_E_ARG),
])
def test_plan_create_rejects(args, code):
    dim, r, shape = args
    n = (2 * max(r, 1) + 1) ** max(min(dim, 3), 1)
    w = np.ones(n)
    out = ctypes.c_void_p()
    rc = sf.lib.stencil_plan_create(dim, r, shape, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    0, ctypes.byref(out))
    assert rc == code
    assert out.value is None
    assert sf.stencil_last_error()


def test_plan_create_rejects_nonfinite_and_off_axis_star():
    w = np.ones((3, 3))
    with pytest.raises(sf.StencilError) as e:
        sf.stencil_plan_create(2, 1, sf.STENCIL_STAR, w)
    assert e.value.code == sf.STENCIL_E_ARG
    w = synth.star2d_weights(0.6, 0.1)
    w[1, 1] = np.nan
    with pytest.raises(sf.StencilError) as e:
        sf.stencil_plan_create(2, 1, sf.STENCIL_STAR, w)
    assert e.value.code == sf.STENCIL_E_ARG
    h = sf.stencil_plan_create(2, 1, sf.STENCIL_STAR, synth.star2d_weights(0.6, 0.1),
                               sf.STENCIL_DIRICHLET)
    sf.stencil_plan_destroy(h)
    with pytest.raises(sf.StencilError) as e:
        sf.stencil_plan_create(2, 1, sf.STENCIL_STAR, synth.star2d_weights(0.6, 0.1), 7)
    assert e.value.code == sf.STENCIL_E_ARG
    rc = sf.lib.stencil_plan_create(2, 1, 0, None, 0, ctypes.byref(ctypes.c_void_p()))
    assert rc == sf.STENCIL_E_ARG


def test_plan_info_mode_and_profitability():
    p = sf.Plan(np.ones((3, 3)), sf.STENCIL_BOX)
    assert p.info() == {"dim": 2, "radius": 1, "m": 1, "folded_radius": 1, "mode": 0}
    # Section 3.2: 90 naive collect entries, 25 folded, for the 9-point box, m = 2
    assert p.profitability(2) == (90, 25)
    star = sf.Plan(synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR)
    assert star.profitability(2) == (30, 13)
    assert star.profitability(4) == (220, 41)
    p.set_mode(sf.STENCIL_MODE_MFMA_BF16X3)
    assert p.info()["mode"] == sf.STENCIL_MODE_MFMA_BF16X3
    with pytest.raises(sf.StencilError):
        p.set_mode(9)
    p3 = sf.Plan(np.ones((3, 3, 3)), sf.STENCIL_BOX)
    with pytest.raises(sf.StencilError) as e:
        p3.set_mode(sf.STENCIL_MODE_MFMA_BF16X3)
    assert e.value.code == sf.STENCIL_E_UNSUPPORTED
    with pytest.raises(sf.StencilError):
        p.profitability(0)
    p.set_fusion(0)
    p.set_fusion(3)
    with pytest.raises(sf.StencilError) as e:
        p.set_fusion(-1)
    assert e.value.code == sf.STENCIL_E_ARG
    p.set_graph(True)
    p.set_graph(False)
    assert sf.lib.stencil_plan_set_graph(p.handle, 2) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_plan_set_graph(None, 1) == sf.STENCIL_E_ARG
    # boundary values: Dirichlet plans only, finite
    p.set_boundary_value(0.0)
    assert sf.lib.stencil_plan_set_boundary_value(p.handle, 1.5) == sf.STENCIL_E_UNSUPPORTED
    d = sf.Plan(synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, sf.STENCIL_DIRICHLET)
    d.set_boundary_value(-2.25)
    assert sf.lib.stencil_plan_set_boundary_value(d.handle, float("nan")) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_plan_set_boundary_value(d.handle, float("inf")) == sf.STENCIL_E_ARG
    d.close()


def test_plan_f32_weights_start_unfolded():
    w = synth.WORKLOADS["box2d"].weights
    p = sf.Plan(w, sf.STENCIL_BOX)
    assert np.array_equal(p.weights_f32(), w.astype(np.float32))


def test_run_validation_before_device_work():
    p = sf.Plan(synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR)
    g = sf.stencil_grid()
    g.data = None
    g.dtype = sf.STENCIL_F32
    g.dim = 2
    g.shape[0] = g.shape[1] = 16
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 5) == sf.STENCIL_E_ARG
    g.data = 4096
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), -1) == sf.STENCIL_E_ARG
    g.dim = 3
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 5) == sf.STENCIL_E_ARG
    g.dim = 2
    g.dtype = 5
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 5) == sf.STENCIL_E_ARG
    g.dtype = sf.STENCIL_F32
    g.shape[1] = 2  # below 2*m*r + 1 = 3
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 5) == sf.STENCIL_E_UNSUPPORTED
    g.shape[1] = 16
    g.scratch = 4096 + 64  # overlaps data
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 5) == sf.STENCIL_E_ARG
    g.scratch = None
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 0) == sf.STENCIL_OK
    assert sf.lib.stencil_run(None, ctypes.byref(g), 1) == sf.STENCIL_E_ARG
    p.set_mode(sf.STENCIL_MODE_MFMA_BF16X3)
    g.dtype = sf.STENCIL_F64
    assert sf.lib.stencil_run(p.handle, ctypes.byref(g), 1) == sf.STENCIL_E_UNSUPPORTED


def test_residual_and_fold_validation():
    out = (ctypes.c_double * 3)()
    assert sf.lib.stencil_residual(None, None, 0, 10, None, out) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_residual(4096, None, 7, 10, None, out) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_residual(4096, None, 0, -1, None, out) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_residual(4096, None, 0, 0, None, out) == sf.STENCIL_OK
    p = sf.Plan(np.ones((3, 3)), sf.STENCIL_BOX)
    assert sf.lib.stencil_fold_weights(p.handle, 0, None, None) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_fold_weights(p.handle, 65, None, None) == sf.STENCIL_E_UNSUPPORTED


def test_batched_validation():
    assert sf.lib.stencil_run_batched(None, None, 0, 1, None) in (sf.STENCIL_OK, sf.STENCIL_E_ARG)
    p = sf.Plan(np.ones((3, 3)), sf.STENCIL_BOX)
    parr = (ctypes.c_void_p * 1)(p.handle.value)
    g = (sf.stencil_grid * 1)()
    g[0].dim = 2
    g[0].dtype = sf.STENCIL_F32
    g[0].shape[0] = g[0].shape[1] = 64
    g[0].data = None
    assert sf.lib.stencil_run_batched(parr, g, 1, 1, None) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_run_batched(parr, g, 1, -1, None) == sf.STENCIL_E_ARG


def _sched(plan, shape, T, dtype=None, data=1 << 20, scratch=None):
    dtype = sf.STENCIL_F32 if dtype is None else dtype
    return sf.stencil_run_schedule(plan.handle, shape, dtype, T, data, scratch)


def test_run_schedule_counts_launches():
    """Host-only launch plan: floor(T/m) folded then T mod m plain
    applications, fused up to the kernel's depth, an even launch count
    whenever a fusing pass can split once more, else a final copy."""
    star = sf.Plan(synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR)
    # 2D FP32 radius-1 star: up to 10 steps per launch; 1000 steps -> 100
    s = _sched(star, (8192, 8192), 1000)
    assert (s["plain_apps"], s["plain_launches"], s["final_copy"]) == (1000, 100, False)
    # radius-1 box: up to 8; 1000 steps -> 125 -> 126 (even)
    box = sf.Plan(synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX)
    s = _sched(box, (8192, 8192), 1000)
    assert (s["plain_apps"], s["plain_launches"], s["final_copy"]) == (1000, 126, False)
    # T = 8 would be one launch: split in two so no copy is needed
    assert _sched(star, (8192, 8192), 8)["plain_launches"] == 2
    assert _sched(star, (8192, 8192), 12)["plain_launches"] == 2
    # T = 1 cannot split: one launch and a copy
    s = _sched(star, (8192, 8192), 1)
    assert (s["plain_launches"], s["final_copy"]) == (1, True)
    # rows that are not whole 16-byte vectors, narrow grids, unaligned
    # buffers: one step per launch; FP64 grids up to 14 steps (radius-1 star)
    assert _sched(star, (8192, 8191), 10)["plain_launches"] == 10
    assert _sched(star, (64, 252), 10)["plain_launches"] == 10
    assert _sched(star, (512, 512), 12, sf.STENCIL_F64)["plain_launches"] == 2
    assert _sched(star, (512, 512), 10, data=(1 << 20) + 4)["plain_launches"] == 10
    assert _sched(star, (512, 512), 10, scratch=(1 << 30) + 8)["plain_launches"] == 10
    # the fusion cap
    star.set_fusion(1)
    assert _sched(star, (8192, 8192), 16)["plain_launches"] == 16
    star.set_fusion(3)
    assert _sched(star, (8192, 8192), 16)["plain_launches"] == 6
    star.set_fusion(0)
    # radius 4: up to 2 per launch (folded plans: the GPU tests)
    w4 = synth.random_positive_weights(2, 4, mask=synth.star_mask(2, 4))
    s = _sched(sf.Plan(w4, sf.STENCIL_STAR), (8192, 8192), 1001)
    assert (s["plain_launches"], s["final_copy"]) == (502, False)
    # zero-boundary plans: any axis >= 1, always a copy back; plain 2D
    # applications fuse on the padded grid (no even split needed), folded
    # ones and narrow padded grids do not
    dstar = sf.Plan(synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, sf.STENCIL_DIRICHLET)
    s = _sched(dstar, (8192, 8192), 16)
    assert (s["plain_launches"], s["final_copy"]) == (2, True)
    s = _sched(dstar, (8192, 8192), 13)
    assert (s["plain_launches"], s["final_copy"]) == (2, True)
    assert _sched(dstar, (1, 2), 3)["plain_launches"] == 3
    assert _sched(dstar, (100, 100), 10)["plain_launches"] == 10
    assert _sched(dstar, (8192, 8192), 14, sf.STENCIL_F64)["plain_launches"] == 1
    assert _sched(dstar, (8192, 8192), 15, sf.STENCIL_F64)["plain_launches"] == 2
    # boxes of radius 3 and more are not fused (FMA-issue bound already)
    b3 = synth.random_positive_weights(2, 3)
    assert _sched(sf.Plan(b3, sf.STENCIL_BOX), (8192, 8192), 10)["plain_launches"] == 10
    # modes other than VECTOR run one application per launch in 2D
    star.set_mode(sf.STENCIL_MODE_SYMMETRIC)
    assert _sched(star, (8192, 8192), 1000)["plain_launches"] == 1000
    # 1D fuses many steps per launch
    heat = sf.Plan(synth.heat1d_weights(), sf.STENCIL_STAR)
    assert _sched(heat, (1_000_000,), 100, sf.STENCIL_F64)["plain_launches"] < 10
    # short lines: wavefront spans of 1024 points, at most 51 steps per launch
    # at radius 1; long lines: workgroup spans of 4096, at most 102 (radius 1)
    # or 51 (radius 2); an even launch count saves the final copy
    assert _sched(heat, (1_000_000,), 100, sf.STENCIL_F64)["plain_launches"] == 2
    assert _sched(heat, (1_000_000,), 200, sf.STENCIL_F64)["plain_launches"] == 4
    assert _sched(heat, (20_000_000,), 200, sf.STENCIL_F64)["plain_launches"] == 2
    box5 = sf.Plan(synth.WORKLOADS["box1d5p"].weights, sf.STENCIL_BOX)
    assert _sched(box5, (10_240_000,), 1000, sf.STENCIL_F64)["plain_launches"] == 20
    # 3D FP32: the 27-point box two steps per launch (5 -> 3 launches, one
    # more for an even count), the 7-point star four; FP64 grids one; a
    # z-axis shorter than 2KR+1 planes takes fewer steps per launch
    box3 = sf.Plan(np.ones((3, 3, 3)) / 27, sf.STENCIL_BOX)
    s = _sched(box3, (64, 64, 64), 5)
    assert (s["plain_launches"], s["final_copy"]) == (4, False)
    star3 = sf.Plan(synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR)
    s = _sched(star3, (512, 512, 512), 200)
    assert (s["plain_launches"], s["final_copy"]) == (68, False)  # 3 steps per launch at most
    assert _sched(star3, (512, 512, 512), 200, sf.STENCIL_F64)["plain_launches"] == 200
    assert _sched(star3, (8, 512, 512), 8)["plain_launches"] == 4  # three per launch at most
    assert _sched(star3, (4, 512, 512), 4)["plain_launches"] == 4  # one per launch
    # (folded plans need the GPU to fold: the GPU tests cover them)
    with pytest.raises(sf.StencilError) as e:
        _sched(star, (8192, 8192), -1)
    assert e.value.code == sf.STENCIL_E_ARG
    with pytest.raises(sf.StencilError) as e:
        _sched(star, (2, 8192), 4)
    assert e.value.code == sf.STENCIL_E_UNSUPPORTED


def test_dirichlet_rejects_axes_beyond_int_range():
    """The fused zero-boundary kernels index the padded grid's interior box
    with 32-bit integers: axes whose padded extent would pass 2^31 are
    refused before any device work (a 1D line of 2^32 + 5 points would
    otherwise wrap to a 5-point interior)."""
    heat = sf.Plan(synth.heat1d_weights(), sf.STENCIL_STAR, sf.STENCIL_DIRICHLET)
    for n in ((1 << 32) + 5, (1 << 31) - 1):
        with pytest.raises(sf.StencilError) as e:
            _sched(heat, (n,), 10, sf.STENCIL_F64)
        assert e.value.code == sf.STENCIL_E_UNSUPPORTED
        assert "zero-boundary" in str(e.value)
    assert _sched(heat, ((1 << 31) - 67,), 10, sf.STENCIL_F64)["plain_launches"] >= 1
    # radius 2: the limit moves down by the wider pad
    box5 = sf.Plan(synth.WORKLOADS["box1d5p"].weights, sf.STENCIL_BOX, sf.STENCIL_DIRICHLET)
    with pytest.raises(sf.StencilError):
        _sched(box5, ((1 << 31) - 68,), 10, sf.STENCIL_F64)
    assert _sched(box5, ((1 << 31) - 69,), 10, sf.STENCIL_F64)["plain_launches"] >= 1
    # periodic lines of that length stay legal
    per = sf.Plan(synth.heat1d_weights(), sf.STENCIL_STAR)
    assert _sched(per, ((1 << 32) + 5,), 10, sf.STENCIL_F64)["plain_launches"] >= 1


def test_separable_rank_and_mode():
    """Rank of the operator by complete-pivoting elimination (host only) and
    when the separable form applies (rank 1 or 2, fewer FMAs than taps)."""
    unit = sf.Plan(np.ones((3, 3)) / 9.0, sf.STENCIL_BOX)
    assert unit.separable() == (1, True)
    assert sf.Plan(synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR).separable() == (2, False)
    assert sf.Plan(synth.random_positive_weights(2, 1), sf.STENCIL_BOX).separable() == (3, False)
    a = np.array([1.0, 2, 3, 2, 1])
    b = np.array([1.0, 0, 2, 0, 1])
    c = np.array([2.0, 1, 1, 1, 2])
    assert sf.Plan(np.outer(a, b) / 81, sf.STENCIL_BOX).separable() == (1, True)
    # rank 2 at radius 2: 2 * 2 * 5 = 20 FMAs < 25 taps
    assert sf.Plan((np.outer(a, b) + np.outer(c, a)) / 200, sf.STENCIL_BOX).separable() == (2, True)
    # rank 3 is never taken
    d = np.array([0.0, 1, 0, 1, 0])
    w3 = (np.outer(a, b) + np.outer(c, a) + np.outer(d, c)) / 300
    assert sf.Plan(w3, sf.STENCIL_BOX).separable() == (3, False)
    unit.set_mode(sf.STENCIL_MODE_SEPARABLE)
    assert unit.info()["mode"] == sf.STENCIL_MODE_SEPARABLE
    # 3D: products a (x) b (x) c (9 FMAs < 27 taps), not the random box or the star
    assert sf.Plan(np.ones((3, 3, 3)), sf.STENCIL_BOX).separable() == (1, True)
    p3 = np.einsum("i,j,k->ijk", a[1:4], c[1:4], b[1:4] + 1.0)
    assert sf.Plan(p3 / p3.sum(), sf.STENCIL_BOX).separable() == (1, True)
    assert sf.Plan(synth.random_positive_weights(3, 1), sf.STENCIL_BOX).separable() == (0, False)
    assert sf.Plan(synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR).separable() == (0, False)
    q3 = p3.copy()
    q3[0, 0, 0] *= 1.0 + 1e-9  # no longer a product
    assert sf.Plan(q3, sf.STENCIL_BOX).separable() == (0, False)
    sf.Plan(np.ones((3, 3, 3)), sf.STENCIL_BOX).set_mode(sf.STENCIL_MODE_SEPARABLE)
    with pytest.raises(sf.StencilError) as e:
        sf.Plan(synth.heat1d_weights(), sf.STENCIL_STAR).set_mode(sf.STENCIL_MODE_SEPARABLE)
    assert e.value.code == sf.STENCIL_E_UNSUPPORTED
    # SEPARABLE runs one application per launch
    s = sf.stencil_run_schedule(unit.handle, (1024, 1024), sf.STENCIL_F32, 16, 1 << 20)
    assert s["plain_launches"] == 16


def test_floor_and_life_validation():
    p2 = sf.Plan(np.ones((3, 3)) / 9, sf.STENCIL_BOX)
    assert sf.lib.stencil_plan_set_floor(p2.handle, 4096, sf.STENCIL_F32, 16) == \
        sf.STENCIL_E_UNSUPPORTED
    p1 = sf.Plan(synth.heat1d_weights(), sf.STENCIL_STAR)
    assert sf.lib.stencil_plan_set_floor(p1.handle, 4096, 9, 16) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_plan_set_floor(p1.handle, 4096, sf.STENCIL_F64, 0) == sf.STENCIL_E_ARG
    assert sf.lib.stencil_plan_set_floor(p1.handle, 4096, sf.STENCIL_F64, 16) == sf.STENCIL_OK
    # the floor must match the grid; and it makes folding unavailable
    g = sf.stencil_grid()
    g.data = 1 << 20
    g.dtype = sf.STENCIL_F64
    g.dim = 1
    g.shape[0] = 32
    assert sf.lib.stencil_run(p1.handle, ctypes.byref(g), 3) == sf.STENCIL_E_ARG
    p1.set_mode(sf.STENCIL_MODE_EXACT_ORDER)
    g.shape[0] = 16
    assert sf.lib.stencil_run(p1.handle, ctypes.byref(g), 3) == sf.STENCIL_E_UNSUPPORTED
    assert sf.lib.stencil_plan_set_floor(p1.handle, None, 0, 0) == sf.STENCIL_OK
    L = sf.lib.stencil_life
    assert L(None, 4096, 8, 8, 1, None) == sf.STENCIL_E_ARG
    assert L(1 << 20, 1 << 21, 0, 8, 1, None) == sf.STENCIL_E_ARG
    assert L(1 << 20, 1 << 21, 8, 8, -1, None) == sf.STENCIL_E_ARG
    assert L(1 << 20, (1 << 20) + 8, 8, 8, 1, None) == sf.STENCIL_E_ARG  # overlap
    assert L(1 << 20, 1 << 21, 8, 8, 0, None) == sf.STENCIL_OK


def test_life_launch_plan():
    # 5000^2 fits the last-level cache: 4 generations per launch
    assert sf.stencil_life_launches(5000, 5000, 1000) == 250
    assert sf.stencil_life_launches(5000, 5000, 7) == 3      # 4 + 2 + 1
    assert sf.stencil_life_launches(64, 96, 9) == 9          # too narrow: one per launch
    assert sf.stencil_life_launches(20, 1024, 9) == 9        # fewer than 33 rows: one per launch
    assert sf.stencil_life_launches(16384, 16384, 33) == 3   # 16 + 16 + 1
