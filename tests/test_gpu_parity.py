"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: kernels that keep the canonical operation order (every vector-mode and
exact-order kernel) are bit-exact against the oracle's FP32 mirror (and the
FP64 oracle itself for FP64 grids); every FP32 result is within 1e-5 (norm-
wise relative, infinity norm) of the FP64 oracle fed the FP32 weights.
Sizes span several tiles plus ragged tails; edge cases cover the smallest
legal sides (2*m*r+1), odd sweep counts and T = 0.
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2103_09235_amd as sf  # noqa: E402

DEV = torch.device("cuda:0")
MODES = {"vector": sf.STENCIL_MODE_VECTOR, "exact": sf.STENCIL_MODE_EXACT_ORDER}


def run_gpu(w, shape_kind, u0, T, m=1, mode=sf.STENCIL_MODE_VECTOR, scratch=False):
    plan = sf.Plan(w, shape_kind)
    if m > 1:
        plan.fold(m)
    plan.set_mode(mode)
    data = torch.from_numpy(np.ascontiguousarray(u0)).to(DEV)
    scr = torch.empty_like(data) if scratch else None
    plan.run(data, T, scr)
    torch.cuda.synchronize()
    out = data.cpu().numpy()
    plan.close()
    return out


CASES_2D = [
    # (name, weights, kind, shape, T, m)
    ("star2d", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (300, 517), 9, 1),
    ("star2d_m2", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (300, 517), 9, 2),
    ("star2d_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (257, 1031), 12, 4),
    ("box2d", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (190, 700), 7, 1),
    ("box2d_m4", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (190, 700), 8, 4),
    ("box2d_m8", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (140, 530), 16, 8),
    ("box2d_small_m3", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (7, 7), 7, 3),
    ("star2d_min_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (9, 9), 9, 4),
    ("star2d_aligned", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (256, 512), 5, 1),
    ("box2d_aligned_m2", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (128, 1024), 6, 2),
    ("star2d_aligned_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (136, 2048), 12, 4),
    ("star2d_aligned_m3", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (72, 520), 9, 3),
]

CASES_3D = [
    ("star3d", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (20, 33, 70), 5, 1),
    ("star3d_m2", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (20, 33, 70), 6, 2),
    ("box3d", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (19, 40, 64), 4, 1),
    ("box3d_m2", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (17, 36, 128), 5, 2),
    ("box3d_min_m2", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (5, 5, 5), 4, 2),
    # two rows per lane (radius-1 box): ragged 32-row and 64-column tiles
    ("box3d_ragged_tiles", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (7, 45, 130), 3, 1),
    ("box3d_one_row_tile", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (6, 3, 70), 3, 1),
]

CASES_1D = [
    ("heat1d", synth.heat1d_weights(), sf.STENCIL_STAR, (100_003,), 37, 1),
    ("heat1d_m3", synth.heat1d_weights(), sf.STENCIL_STAR, (4099,), 10, 3),
    ("box1d_r2", synth.random_positive_weights(1, 2), sf.STENCIL_BOX, (5000,), 13, 1),
    ("heat1d_min", synth.heat1d_weights(), sf.STENCIL_STAR, (3,), 5, 1),
]


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("case", CASES_1D + CASES_2D + CASES_3D, ids=lambda c: c[0])
def test_f32_bit_exact_vs_mirror(case, mode):
    name, w, kind, shape, T, m = case
    w = synth.to_f32_exact(w)
    u0 = synth.grid_f32(shape)
    print("case", name, mode, shape, "T", T, "m", m, flush=True)
    got = run_gpu(w, kind, u0, T, m, MODES[mode])
    ref = oracle.folded_reference_f32(w, u0, T, m)
    bad = np.count_nonzero(got != ref)
    assert bad == 0, "%d of %d elements differ" % (bad, got.size)
    ref64 = oracle.sweep(w, u0.astype(np.float64), T)
    assert oracle.errors(got, ref64)["e_rel"] < 1e-5


@pytest.mark.parametrize("case", [CASES_1D[0], CASES_1D[2], CASES_2D[1], CASES_3D[3]],
                         ids=lambda c: c[0])
def test_f64_vs_oracle(case):
    name, w, kind, shape, T, m = case
    u0 = synth.grid_f64(shape)
    got = run_gpu(w, kind, u0, T, m)
    if m == 1:
        ref = oracle.sweep(w, u0, T)
        assert np.array_equal(got, ref)
    else:
        q, s = oracle.schedule(T, m)
        ref = oracle.sweep(w, oracle.sweep(oracle.fold_weights(w, m), u0, q), s)
        ref_plain = oracle.sweep(w, u0, T)
        assert oracle.errors(got, ref)["e_rel"] < 1e-14
        assert oracle.errors(got, ref_plain)["e_rel"] < 1e-13


@pytest.mark.parametrize("name,m", [("star2d", 2), ("star2d", 4), ("box2d", 4), ("box2d", 8),
                                    ("star3d", 2), ("box3d", 2), ("heat1d", 6)])
def test_fold_weights_match_oracle(name, m):
    w = synth.WORKLOADS[name].weights
    kind = synth.WORKLOADS[name].shape_kind
    plan = sf.Plan(w, kind)
    W = plan.fold(m)
    ref = oracle.fold_weights(w, m)
    assert np.max(np.abs(W - ref)) <= 1e-16 * max(1.0, np.abs(ref).max()) * 8
    assert np.array_equal(plan.weights_f32(), oracle.fold_weights_f32(w, m))
    plan.close()


def test_fold_weights_integer_exact():
    plan = sf.Plan(np.ones((3, 3)), sf.STENCIL_BOX)
    assert np.array_equal(plan.fold(2), oracle.fold_weights(np.ones((3, 3)), 2))
    assert np.array_equal(plan.fold(5), oracle.fold_weights(np.ones((3, 3)), 5))
    plan.close()


def test_zero_steps_and_odd_sweeps_and_caller_scratch():
    w = synth.WORKLOADS["star2d"].weights
    u0 = synth.grid_f32((64, 96))
    assert np.array_equal(run_gpu(w, sf.STENCIL_STAR, u0, 0), u0)
    for T, m in [(1, 1), (3, 1), (5, 2), (7, 4)]:
        got = run_gpu(w, sf.STENCIL_STAR, u0, T, m, scratch=True)
        assert np.array_equal(got, oracle.folded_reference_f32(w, u0, T, m)), (T, m)


def test_split_runs_compose():
    """run(T1) then run(T2) equals run(T1 + T2) bit for bit when m divides T1."""
    w = synth.WORKLOADS["box2d"].weights
    u0 = synth.grid_f32((150, 333))
    plan = sf.Plan(w, sf.STENCIL_BOX)
    plan.fold(4)
    a = torch.from_numpy(u0).to(DEV)
    b = a.clone()
    plan.run(a, 8)
    plan.run(a, 6)
    plan.run(b, 14)
    torch.cuda.synchronize()
    # 14 = 3 folded + 2 plain; 8 + 6 = (2 folded) + (1 folded + 2 plain)
    assert torch.equal(a, b)
    plan.close()


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_translation_equivariance_bitwise(dim):
    shape = {1: (8191,), 2: (131, 257), 3: (24, 40, 72)}[dim]
    w = synth.to_f32_exact(synth.random_positive_weights(dim, 1))
    u0 = synth.grid_f32(shape)
    shift = {1: (77,), 2: (5, 131), 3: (3, 9, 33)}[dim]
    axes = tuple(range(dim))
    a = run_gpu(w, sf.STENCIL_BOX, np.roll(u0, shift, axes), 6, 2)
    b = np.roll(run_gpu(w, sf.STENCIL_BOX, u0, 6, 2), shift, axes)
    assert np.array_equal(a, b)


def test_residual_sums():
    u = synth.grid_f32((1000, 777))
    v = synth.grid_f32((1000, 777), stream=9)
    tu = torch.from_numpy(u).to(DEV)
    tv = torch.from_numpy(v).to(DEV)
    s, d, mx = sf.stencil_residual(tu, tv)
    assert abs(s - oracle.exact_sum(u)) <= 4 * 2.0 ** -53 * abs(s)
    diff = np.abs(u.astype(np.float64) - v.astype(np.float64))
    assert abs(d - oracle.exact_sum(diff)) <= 4 * 2.0 ** -53 * d
    assert mx == diff.max()
    u64 = synth.grid_f64((3, 5, 7))
    s2, _, _ = sf.stencil_residual(torch.from_numpy(u64).to(DEV))
    assert abs(s2 - oracle.exact_sum(u64)) <= 2 * 2.0 ** -53 * abs(s2)


def test_errors_surface_from_run():
    plan = sf.Plan(synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR)
    plan.fold(4)
    t = torch.zeros((8, 64), device=DEV)
    with pytest.raises(sf.StencilError) as e:
        plan.run(t, 4)
    assert e.value.code == sf.STENCIL_E_UNSUPPORTED
    host = torch.zeros((64, 64))
    g = sf.stencil_grid()
    g.data = host.data_ptr()
    g.dtype = sf.STENCIL_F32
    g.dim = 2
    g.shape[0] = g.shape[1] = 64
    import ctypes
    assert sf.lib.stencil_run(plan.handle, ctypes.byref(g), 4) == sf.STENCIL_E_ARG
    plan.close()


# ------------------------------------------------ BF16x3 matrix-core form

MFMA_CASES = [
    # (name, weights, kind, shape, T, m)
    ("box2d_m4", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (190, 700), 16, 4),
    ("box2d_m8", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (140, 530), 24, 8),
    ("box2d_m8_min", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (17, 17), 16, 8),
    ("box2d_m4_rem", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (257, 129), 18, 4),
    ("star2d_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (96, 260), 12, 4),
    ("box2d_plain", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (64, 64), 5, 1),
    ("box2d_m2_aligned", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (512, 1024), 8, 2),
    # whole 256-column strips only, with 16-byte loads and stores (the
    # launch the 16384^2 workload makes), several row segments
    ("box2d_m8_full", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (300, 768), 16, 8),
    # 8-byte loads, whole strips plus a 4-column remainder strip
    ("box2d_m6_rest", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (200, 516), 12, 6),
    # a grid narrower than one strip and shorter than the folded halo twice
    ("box2d_m3_narrow", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (9, 100), 9, 3),
]


@pytest.mark.parametrize("case", MFMA_CASES, ids=lambda c: c[0])
def test_mfma_bf16x3_within_1e3(case):
    """BF16 hi+lo products with FP32 accumulation: within 1e-3 (infinity-norm
    relative) of the FP64 oracle fed the FP32 weights; the matrix unit's own
    summation order makes bitwise parity unpinned."""
    name, w, kind, shape, T, m = case
    w = synth.to_f32_exact(w)
    u0 = synth.grid_f32(shape)
    print("case", name, shape, "T", T, "m", m, flush=True)
    got = run_gpu(w, kind, u0, T, m, sf.STENCIL_MODE_MFMA_BF16X3)
    ref64 = oracle.sweep(w, u0.astype(np.float64), T)
    e = oracle.errors(got, ref64)
    assert e["e_rel"] < 1e-3, e
    # and it is a real split: much closer than single-BF16 rounding of the input
    assert e["e_rel"] < 2.0 ** -12, e


def test_mfma_rejects_unsupported():
    plan = sf.Plan(synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX)
    plan.fold(9)
    plan.set_mode(sf.STENCIL_MODE_MFMA_BF16X3)
    t = torch.zeros((64, 64), device=DEV)
    with pytest.raises(sf.StencilError) as e:
        plan.run(t, 9)
    assert e.value.code == sf.STENCIL_E_UNSUPPORTED
    plan.fold(2)
    with pytest.raises(sf.StencilError) as e:
        plan.run(torch.zeros((64, 64), device=DEV, dtype=torch.float64), 2)
    assert e.value.code == sf.STENCIL_E_UNSUPPORTED
    plan.close()


# ----------------------------------------------------------- batched form

def _batch_inputs(count, seed_sides):
    sides, kinds, weights = synth.batched_recipe(count)
    # replace a few sides to cover the vector path (multiple of 4, >= 256) and
    # ragged small grids
    sides = sides.copy()
    sides[:3] = [256, 68, 301][: min(3, count)]
    grids = [synth.grid_f32((int(s), int(s)), stream=5 + i % 3) for i, s in enumerate(sides)]
    return sides, kinds, weights, grids


def _run_batched(kinds, weights, grids, T, tune_cache=None, autotune=False, use_graph=True,
                 max_m=1, repeats=1):
    plans = [sf.Plan(w, sf.STENCIL_STAR if k == synth.STAR else sf.STENCIL_BOX)
             for k, w in zip(kinds, weights)]
    datas = [torch.from_numpy(g).to(DEV) for g in grids]
    scr = [torch.empty_like(d) for d in datas]
    chosen = None
    for _ in range(repeats):
        chosen = sf.stencil_run_batched([p.handle for p in plans], datas, scr, T,
                                        autotune=autotune, tune_cache=tune_cache,
                                        use_graph=use_graph, max_m=max_m)
    torch.cuda.synchronize()
    outs = [d.cpu().numpy() for d in datas]
    for p in plans:
        p.close()
    return outs, chosen


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_plain_bit_exact(use_graph):
    sides, kinds, weights, grids = _batch_inputs(12, 0)
    T = 7  # odd: every grid ends after a copy-back
    outs, chosen = _run_batched(kinds, weights, grids, T, use_graph=use_graph)
    assert chosen == [1] * len(grids)
    for g, w, o in zip(grids, weights, outs):
        ref = oracle.folded_reference_f32(w, g, T, 1)
        assert np.array_equal(o, ref)


def test_batched_folded_from_tune_cache(tmp_path):
    sides, kinds, weights, grids = _batch_inputs(10, 1)
    cache = tmp_path / "tune.txt"
    # fold depth 2 for every (shape, r = 1, size class) this batch has
    lines = []
    for shape in (0, 1):
        for cls in range(5, 12):
            lines.append("stencil-batched-m %d 1 %d 2" % (shape, cls))
    cache.write_text("\n".join(lines) + "\n")
    T = 9  # 4 folded + 1 plain sweep per grid
    outs, chosen = _run_batched(kinds, weights, grids, T, tune_cache=str(cache), max_m=2)
    assert chosen == [2] * len(grids)
    for g, w, o in zip(grids, weights, outs):
        ref = oracle.folded_reference_f32(w, g, T, 2)
        assert np.array_equal(o, ref)


def test_batched_graph_replay_composes():
    sides, kinds, weights, grids = _batch_inputs(6, 2)
    outs, _ = _run_batched(kinds, weights, grids, 4, repeats=3)
    for g, w, o in zip(grids, weights, outs):
        assert np.array_equal(o, oracle.folded_reference_f32(w, g, 12, 1))


def test_batched_autotune_picks_valid_m(tmp_path):
    sides, kinds, weights, grids = _batch_inputs(5, 3)
    cache = tmp_path / "auto.txt"
    T = 8
    outs, chosen = _run_batched(kinds, weights, grids, T, tune_cache=str(cache), autotune=True,
                                max_m=2)
    assert all(m in (1, 2) for m in chosen)
    assert cache.exists() and "stencil-batched-m" in cache.read_text()
    for g, w, o, m in zip(grids, weights, outs, chosen):
        assert np.array_equal(o, oracle.folded_reference_f32(w, g, T, m))


def test_batched_cache_never_confuses_plans():
    """Plans destroyed and created between batched runs on the same tensors
    (a new plan may sit at a freed plan's address): every run must apply its
    own plan's operator, including a plan of the same kind and radius with
    other weights, whose cached tables would otherwise be reused."""
    sides = [96, 130, 64, 300]
    grids0 = [synth.grid_f32((s, s), stream=9 + i) for i, s in enumerate(sides)]
    datas = [torch.from_numpy(g).to(DEV) for g in grids0]
    scr = [torch.empty_like(d) for d in datas]
    T = 5
    for it in range(6):
        kind = synth.STAR if it % 3 != 2 else synth.BOX
        mask = synth.star_mask(2, 1) if kind == synth.STAR else None
        w = synth.to_f32_exact(synth.random_positive_weights(2, 1, offset=100 + 9 * it, mask=mask))
        plan = sf.Plan(w, sf.STENCIL_STAR if kind == synth.STAR else sf.STENCIL_BOX)
        for d, g in zip(datas, grids0):
            d.copy_(torch.from_numpy(g))
        sf.stencil_run_batched([plan.handle] * len(datas), datas, scr, T, use_graph=it % 2 == 0)
        torch.cuda.synchronize()
        for d, g in zip(datas, grids0):
            assert np.array_equal(d.cpu().numpy(), oracle.folded_reference_f32(w, g, T, 1)), it
        plan.close()


# ------------------------------------------- shared-partial-sum (symmetric)

def _symmetric_box():
    w = synth.random_positive_weights(2, 1)
    w = (w + w[::-1, :] + w[:, ::-1] + w[::-1, ::-1]) / 4.0
    return synth.to_f32_exact(w / w.sum())


SYM_CASES = [
    ("star2d_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (136, 2048), 12, 4, True),
    ("star2d_m2", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (100, 1024), 9, 2, True),
    ("star2d_plain", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (64, 512), 7, 1, True),
    ("symbox_m3", _symmetric_box(), sf.STENCIL_BOX, (90, 768), 9, 3, True),
    ("asym_box_m2", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (64, 512), 6, 2, False),
    ("star2d_ragged_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (77, 301), 8, 4, False),
]


@pytest.mark.parametrize("case", SYM_CASES, ids=lambda c: c[0])
def test_symmetric_mode(case):
    """Symmetric operators on vector-aligned grids: within 1e-5 of the FP64
    oracle (the order differs from the canonical one); everything else falls
    back to the canonical kernels and stays bit-exact."""
    name, w, kind, shape, T, m, shared = case
    w = synth.to_f32_exact(w)
    u0 = synth.grid_f32(shape)
    got = run_gpu(w, kind, u0, T, m, sf.STENCIL_MODE_SYMMETRIC)
    ref64 = oracle.sweep(w, u0.astype(np.float64), T)
    assert oracle.errors(got, ref64)["e_rel"] < 1e-5
    mirror = oracle.folded_reference_f32(w, u0, T, m)
    if not shared:
        assert np.array_equal(got, mirror)


# ------------------------------------------------- 2D temporal blocking

def _star_weights(r, offset):
    return synth.to_f32_exact(synth.random_positive_weights(2, r, offset=offset,
                                                            mask=synth.star_mask(2, r)))


def _box_weights(r, offset):
    return synth.to_f32_exact(synth.random_positive_weights(2, r, offset=offset))


TB_CASES = [
    # (name, weights, kind, shape, T, m, fusion): each launch fuses up to
    # `fusion` steps (0 = library choice); shapes span several 256-column
    # strips with a ragged last strip, and the minimum row count 2KR+1
    ("star_r1_k8", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (200, 1000), 16, 1, 8),
    ("star_r1_k10", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (200, 1000), 20, 1, 0),
    ("star_r1_k10_k11", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (90, 1284), 42, 1, 11),
    ("star_r1_k9_k10", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (64, 772), 38, 1, 10),
    ("star_r1_k10_min_rows", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (21, 512), 20, 1,
     0),
    ("star_r1_min_rows", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (17, 256), 8, 1, 8),
    ("box_r1_k7", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (150, 772), 14, 1, 7),
    ("box_r1_k5_k6", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (99, 516), 11, 1, 6),
    ("star_r1_k3_k4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (64, 260), 7, 1, 4),
    ("star_r1_k2", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (40, 300), 4, 1, 2),
    ("star_r2_plain", _star_weights(2, 100), sf.STENCIL_STAR, (120, 1024), 8, 1, 0),
    ("box_r2_plain_k3", _box_weights(2, 200), sf.STENCIL_BOX, (80, 520), 9, 1, 3),
    ("star2d_m2_fused", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (150, 768), 16, 2, 0),
    ("box2d_m2_fused", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (64, 2048), 14, 2, 0),
    ("star_r3_plain", _star_weights(3, 300), sf.STENCIL_STAR, (90, 512), 6, 1, 0),
    ("box2d_m3_not_fused", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (61, 764), 15, 3, 0),
    ("star2d_m4_fused", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (300, 1024), 16, 4, 0),
    ("box_r4_not_fused", _box_weights(4, 400), sf.STENCIL_BOX, (17, 256), 4, 1, 0),
]


@pytest.mark.parametrize("case", TB_CASES, ids=lambda c: c[0])
def test_temporal_blocking_bit_exact(case):
    """Several steps per launch (registers + LDS) equal one launch per step
    bit for bit: compared with the oracle's FP32 mirror of the schedule and
    with the same plan run unfused."""
    name, w, kind, shape, T, m, fusion = case
    w = synth.to_f32_exact(w)
    u0 = synth.grid_f32(shape)
    print("temporal blocking", name, shape, "T", T, "m", m, "fusion", fusion, flush=True)
    outs = []
    for fz in (fusion, 1):
        plan = sf.Plan(w, kind)
        if m > 1:
            plan.fold(m)
        plan.set_fusion(fz)
        data = torch.from_numpy(u0).to(DEV)
        plan.run(data, T, torch.empty_like(data))
        torch.cuda.synchronize()
        outs.append(data.cpu().numpy())
        plan.close()
    ref = oracle.folded_reference_f32(w, u0, T, m)
    assert np.array_equal(outs[0], ref)
    assert np.array_equal(outs[1], ref)


def _product3(a, b, c):
    w = np.einsum("i,j,k->ijk", np.asarray(a, float), np.asarray(b, float), np.asarray(c, float))
    return synth.to_f32_exact(w / w.sum())


SEP3_CASES = [
    # (name, weights, shape, T, m, separable): FP32 3D grids in SEPARABLE mode
    ("unitbox3d_plain", synth.to_f32_exact(np.full((3, 3, 3), 1.0 / 27)), (40, 70, 136), 6, 1, True),
    ("unitbox3d_m2", synth.to_f32_exact(np.full((3, 3, 3), 1.0 / 27)), (36, 40, 132), 8, 2, True),
    ("product3d_m2_ragged", _product3([1, 2, 1], [1, 1, 1], [0.2, 0.5, 0.3]), (33, 45, 70), 9, 2,
     True),
    ("product3d_m4", _product3([1, 2, 1], [3, 1, 2], [1, 1, 1]), (30, 40, 64), 8, 4, True),
    ("product3d_small", _product3([1, 2, 1], [3, 1, 2], [1, 1, 1]), (9, 7, 6), 5, 1, True),
    # not a product: the VECTOR kernels, canonical order
    ("randbox3d_fallback", synth.to_f32_exact(synth.random_positive_weights(3, 1)), (20, 30, 68), 4, 1,
     False),
]


@pytest.mark.parametrize("case", SEP3_CASES, ids=lambda c: c[0])
def test_separable_3d(case):
    """3D products a (x) b (x) c as an x-pass, a y-pass and a z-pass (the
    paper's vertical and horizontal folding, Section 3.3 Eq. 4-6, with a third
    axis): within 1e-5 of the FP64 oracle (another summation order); other
    operators fall back to the canonical kernels, bit-exact."""
    name, w, shape, T, m, sep = case
    u0 = synth.grid_f32(shape)
    print("3D separable", name, shape, "T", T, "m", m, flush=True)
    plan = sf.Plan(w, sf.STENCIL_BOX)
    if m > 1:
        plan.fold(m)
    assert plan.separable() == ((1, True) if sep else (0, False))
    plan.set_mode(sf.STENCIL_MODE_SEPARABLE)
    data = torch.from_numpy(u0).to(DEV)
    plan.run(data, T, torch.empty_like(data))
    torch.cuda.synchronize()
    got = data.cpu().numpy()
    plan.close()
    ref64 = oracle.sweep(w, u0.astype(np.float64), T)
    e = oracle.errors(got, ref64)
    assert e["e_rel"] < 1e-5, e
    mirror = oracle.folded_reference_f32(w, u0, T, m)
    if not sep:
        assert np.array_equal(got, mirror)
    else:
        assert not np.array_equal(got, mirror)  # the separable kernel ran


TB64_CASES = [
    # (name, weights, kind, shape, T, m, fusion, boundary): FP64 2D grids
    ("star_r1_k14", synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, (150, 772), 28, 1, 0,
     "periodic"),
    ("box_r1_k8", synth.random_positive_weights(2, 1), sf.STENCIL_BOX, (99, 516), 17, 1, 0,
     "periodic"),
    ("star_r1_ragged", synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, (37, 130), 14, 1, 0,
     "periodic"),
    ("star_r1_k3", synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, (40, 260), 7, 1, 3, "periodic"),
    ("star_m2_fused", synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, (64, 512), 9, 2, 0,
     "periodic"),
    ("box_m2_fused", synth.random_positive_weights(2, 1), sf.STENCIL_BOX, (70, 256), 8, 2, 0,
     "periodic"),
    ("star_r1_zero", synth.star2d_weights(0.6, 0.1), sf.STENCIL_STAR, (90, 300), 11, 1, 0, "zero"),
]


@pytest.mark.parametrize("case", TB64_CASES, ids=lambda c: c[0])
def test_temporal_blocking_fp64_bit_exact(case):
    """FP64 2D grids: several applications per launch (FP64 values moved
    between lanes as two 32-bit halves) equal one launch per application bit
    for bit, and the FP64 oracle's naive loop (periodic or zero ghosts) bit
    for bit when unfolded."""
    name, w, kind, shape, T, m, fusion, bc = case
    u0 = synth.grid_f64(shape)
    print("FP64 temporal blocking", name, shape, "T", T, "m", m, "fusion", fusion, flush=True)
    outs = []
    for fz in (fusion, 1):
        plan = sf.Plan(w, kind, sf.STENCIL_DIRICHLET if bc == "zero" else sf.STENCIL_PERIODIC)
        if m > 1:
            plan.fold(m)
        plan.set_fusion(fz)
        data = torch.from_numpy(u0).to(DEV)
        scr = torch.empty_like(data)
        sched = plan.schedule(data, T, scr)
        plan.run(data, T, scr)
        torch.cuda.synchronize()
        outs.append((data.cpu().numpy(), sched))
        plan.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    ref = oracle.sweep(w, u0, T, bc)
    if m == 1:
        assert np.array_equal(outs[0][0], ref)
    else:
        # the library's FP64 fold and the oracle's impulse-response fold agree
        # to a few ulps, not bit for bit
        assert oracle.errors(outs[0][0], ref)["e_rel"] < 1e-12
    s = outs[0][1]
    launches = s["folded_launches"] if m > 1 else s["plain_launches"]
    apps = s["folded_apps"] if m > 1 else s["plain_apps"]
    assert launches < apps, s


TB3_CASES = [
    # (name, weights, kind, shape, T, m, fusion); shapes span several 64 x TY
    # tiles and z-segments with ragged edges, rows of whole vectors or not
    ("star3d_k4", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (40, 48, 192), 8, 1, 0),
    ("star3d_k3k2_ragged", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (37, 41, 130), 9, 1,
     0),
    ("star3d_k3", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (33, 35, 68), 7, 1, 3),
    ("star3d_k2", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (30, 70, 136), 6, 1, 2),
    ("box3d_k2", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (36, 40, 132), 5, 1, 0),
    ("box3d_k2_ragged", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (20, 33, 70), 4, 1, 0),
    ("star3d_m2_fused", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (40, 36, 100), 9, 2, 0),
    ("box3d_m2_not_fused", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (24, 30, 68), 6, 2, 0),
    # tiles wider than the grid: every run wraps several times
    ("star3d_k4_tiny", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (9, 7, 6), 8, 1, 0),
    ("star3d_k4_narrow_vec", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (12, 10, 8), 8, 1,
     0),
]


@pytest.mark.parametrize("case", TB3_CASES, ids=lambda c: c[0])
def test_temporal_blocking_3d_bit_exact(case):
    """3D: K applications per launch streamed through K pipeline stages in
    LDS equal K single-step launches bit for bit (the oracle's FP32 mirror
    of the schedule, and the same plan unfused)."""
    name, w, kind, shape, T, m, fusion = case
    w = synth.to_f32_exact(w)
    u0 = synth.grid_f32(shape)
    print("3D temporal blocking", name, shape, "T", T, "m", m, "fusion", fusion, flush=True)
    outs = []
    for fz in (fusion, 1):
        plan = sf.Plan(w, kind)
        if m > 1:
            plan.fold(m)
        plan.set_fusion(fz)
        data = torch.from_numpy(u0).to(DEV)
        scr = torch.empty_like(data)
        sched = plan.schedule(data, T, scr)
        plan.run(data, T, scr)
        torch.cuda.synchronize()
        outs.append((data.cpu().numpy(), sched))
        plan.close()
    ref = oracle.folded_reference_f32(w, u0, T, m)
    assert np.array_equal(outs[0][0], ref)
    assert np.array_equal(outs[1][0], ref)
    fused = outs[0][1]
    if not name.endswith("not_fused"):
        launches = fused["folded_launches"] if m > 1 else fused["plain_launches"]
        apps = fused["folded_apps"] if m > 1 else fused["plain_apps"]
        assert launches < apps, fused  # several applications per launch


def test_run_schedule_folded_then_plain():
    """floor(T/m) applications of W_m (radius 4: two per launch), then the
    T mod m plain ones; the reported plan is the one stencil_run follows
    (same result as the oracle's mirror of the schedule)."""
    w = synth.WORKLOADS["star2d"].weights
    plan = sf.Plan(w, sf.STENCIL_STAR)
    plan.fold(4)
    u0 = synth.grid_f32((40, 512))
    data = torch.from_numpy(u0).to(DEV)
    scr = torch.empty_like(data)
    s = plan.schedule(data, 17, scr)
    # 2 + 1 launches would end in scratch: the folded pass splits once more
    assert (s["folded_apps"], s["folded_launches"], s["plain_apps"]) == (4, 3, 1)
    assert s["plain_launches"] == 1 and not s["final_copy"]
    plan.run(data, 17, scr)
    torch.cuda.synchronize()
    assert np.array_equal(data.cpu().numpy(), oracle.folded_reference_f32(w, u0, 17, 4))
    plan.close()


# ------------------------------------------------- separable (low-rank) form

def _rank2_box():
    a = np.array([1.0, 2, 3, 2, 1])
    b = np.array([1.0, 0, 2, 0, 1])
    c = np.array([2.0, 1, 1, 1, 2])
    # a dyadic scale keeps the FP32 weights exactly rank two
    return synth.to_f32_exact((np.outer(a, b) + np.outer(c, a)) / 256.0)


SEP_CASES = [
    # (name, weights, kind, shape, T, m, separable form used)
    ("unitbox_m1", np.full((3, 3), 1.0 / 9.0), sf.STENCIL_BOX, (70, 512), 7, 1, True),
    ("unitbox_m2", np.full((3, 3), 1.0 / 9.0), sf.STENCIL_BOX, (96, 768), 9, 2, True),
    ("unitbox_m4", np.full((3, 3), 1.0 / 9.0), sf.STENCIL_BOX, (130, 1024), 18, 4, True),
    ("unitbox_m8", np.full((3, 3), 1.0 / 9.0), sf.STENCIL_BOX, (120, 516), 19, 8, True),
    ("unitbox_m8_min", np.full((3, 3), 1.0 / 9.0), sf.STENCIL_BOX, (17, 20), 16, 8, True),
    ("rank2_r2", _rank2_box(), sf.STENCIL_BOX, (64, 260), 6, 1, True),
    ("star2d_m2_dense", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (64, 512), 6, 2, False),
    ("randbox_m4_dense", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (80, 512), 8, 4, False),
    ("unitbox_m4_ragged", np.full((3, 3), 1.0 / 9.0), sf.STENCIL_BOX, (75, 301), 8, 4, False),
]


@pytest.mark.parametrize("case", SEP_CASES, ids=lambda c: c[0])
def test_separable_mode(case):
    """Rank-one/two operators as horizontal then vertical passes: within
    1e-5 of the FP64 oracle (another summation order, factors rounded to
    FP32); operators without a cheaper separable form, and rows that are not
    whole vectors, run the canonical kernels and stay bit-exact."""
    name, w, kind, shape, T, m, used = case
    w = synth.to_f32_exact(w)
    u0 = synth.grid_f32(shape)
    plan = sf.Plan(w, kind)
    if m > 1:
        plan.fold(m)
    plan.set_mode(sf.STENCIL_MODE_SEPARABLE)
    print("separable", name, shape, "T", T, "m", m, plan.separable(), flush=True)
    if name != "unitbox_m4_ragged":
        assert plan.separable()[1] == used
    data = torch.from_numpy(u0).to(DEV)
    plan.run(data, T, torch.empty_like(data))
    torch.cuda.synchronize()
    got = data.cpu().numpy()
    plan.close()
    ref64 = oracle.sweep(w, u0.astype(np.float64), T)
    assert oracle.errors(got, ref64)["e_rel"] < 1e-5
    if not used:
        assert np.array_equal(got, oracle.folded_reference_f32(w, u0, T, m))


# ------------------------------------------------- zero Dirichlet boundaries

DIR_CASES = [
    # (name, weights, kind, shape, T, m, dtype)
    ("heat1d_plain_f64", synth.heat1d_weights(), sf.STENCIL_STAR, (1000,), 7, 1, "f64"),
    ("heat1d_m3_f32", synth.heat1d_weights(), sf.STENCIL_STAR, (37,), 10, 3, "f32"),
    ("star2d_plain", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (100, 130), 9, 1, "f32"),
    ("star2d_m4", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (64, 256), 13, 4, "f32"),
    ("star2d_m2_f64", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (50, 61), 7, 2, "f64"),
    ("box2d_m2", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (37, 41), 8, 2, "f32"),
    ("box2d_m8", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (90, 300), 17, 8, "f32"),
    ("tiny_band_everywhere", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (3, 5), 9, 4, "f32"),
    ("one_row", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (1, 9), 5, 2, "f32"),
    ("star3d_m2", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (12, 14, 18), 5, 2, "f32"),
    ("box3d_plain", synth.WORKLOADS["box3d"].weights, sf.STENCIL_BOX, (9, 10, 11), 3, 1, "f32"),
    # plain 2D FP32 applications fused on the padded grid (pad zeroed at
    # every stage): depths 10/9, 6/5, the 3-step remainder of a fold, and
    # the fewest padded rows a depth-12 star fuses with
    ("star2d_plain_fused", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (70, 300), 29, 1,
     "f32"),
    ("box2d_plain_fused", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (40, 260), 17, 1,
     "f32"),
    ("star2d_m4_rem3_fused", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (64, 256), 19, 4,
     "f32"),
    ("star2d_fused_min_rows", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (23, 510), 24, 1,
     "f32"),
    # plain 1D applications fused on the padded line (ghosts written at every
    # step): wavefront spans, a radius-2 box, the 3-step remainder of a fold,
    # and a line long enough for the workgroup spans
    ("heat1d_plain_fused_f32", synth.heat1d_weights(), sf.STENCIL_STAR, (5000,), 60, 1, "f32"),
    ("box1d_r2_fused_f64", synth.random_positive_weights(1, 2), sf.STENCIL_BOX, (3001,), 23, 1,
     "f64"),
    ("heat1d_m4_rem3_fused", synth.heat1d_weights(), sf.STENCIL_STAR, (777,), 15, 4, "f64"),
    ("heat1d_long_group_f64", synth.heat1d_weights(), sf.STENCIL_STAR, (4_000_000,), 50, 1, "f64"),
]


def _run_dirichlet(w, kind, u0, T, m, mode=sf.STENCIL_MODE_VECTOR, plan=None, ghost=None):
    own = plan is None
    if own:
        plan = sf.Plan(w, kind, sf.STENCIL_DIRICHLET)
        if m > 1:
            plan.fold(m)
        plan.set_mode(mode)
        if ghost is not None:
            plan.set_boundary_value(ghost)
    data = torch.from_numpy(np.ascontiguousarray(u0)).to(DEV)
    plan.run(data, T)
    torch.cuda.synchronize()
    if own:
        plan.close()
    return data.cpu().numpy()


@pytest.mark.parametrize("case", DIR_CASES, ids=lambda c: c[0])
def test_dirichlet_bit_exact_vs_mirror(case):
    """Zero-boundary runs (folded interior, plain-stepped band, zero pad
    restored per application) equal the oracle's mirror of the same reading
    bit for bit (canonical-order kernels), and the FP64 zero-ghost sweep
    within the FP32 gate."""
    name, w, kind, shape, T, m, dt = case
    print("dirichlet", name, shape, "T", T, "m", m, dt, flush=True)
    if dt == "f32":
        w = synth.to_f32_exact(w)
        u0 = synth.grid_f32(shape)
    else:
        u0 = synth.grid_f64(shape)
    got = _run_dirichlet(w, kind, u0, T, m)
    ref64 = oracle.sweep(w, u0.astype(np.float64), T, "zero")
    if dt == "f32":
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, m, f32=True))
        assert oracle.errors(got, ref64)["e_rel"] < 1e-5
    else:
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, m))
        assert oracle.errors(got, ref64)["e_rel"] < 1e-13


@pytest.mark.parametrize("mode,gate", [("exact", 0.0), ("symmetric", 1e-5), ("separable", 1e-5),
                                       ("mfma", 1e-3)])
def test_dirichlet_other_modes(mode, gate):
    w = np.full((3, 3), 1.0 / 9.0) if mode == "separable" else synth.WORKLOADS["star2d"].weights
    if mode == "mfma":
        w = synth.WORKLOADS["box2d"].weights
    w = synth.to_f32_exact(w)
    kind = sf.STENCIL_STAR if mode in ("exact", "symmetric") else sf.STENCIL_BOX
    code = {"exact": sf.STENCIL_MODE_EXACT_ORDER, "symmetric": sf.STENCIL_MODE_SYMMETRIC,
            "separable": sf.STENCIL_MODE_SEPARABLE, "mfma": sf.STENCIL_MODE_MFMA_BF16X3}[mode]
    u0 = synth.grid_f32((70, 256))
    T, m = 11, 4
    got = _run_dirichlet(w, kind, u0, T, m, code)
    if gate == 0.0:
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, m, f32=True))
    else:
        ref64 = oracle.sweep(w, u0.astype(np.float64), T, "zero")
        assert oracle.errors(got, ref64)["e_rel"] < gate


# ghost values: one exact in FP32, one rounded to FP32 on both sides
GHOSTS = {"heat1d_plain_f64": 0.3, "heat1d_m3_f32": -1.75, "star2d_plain": 0.3,
          "star2d_m4": -1.75, "star2d_m2_f64": -1.75, "box2d_m2": 0.3, "box2d_m8": 2.5,
          "tiny_band_everywhere": 0.3, "one_row": -1.75, "star3d_m2": 0.3, "box3d_plain": -1.75,
          "star2d_plain_fused": 0.3, "box2d_plain_fused": -1.75, "star2d_m4_rem3_fused": 2.5,
          "star2d_fused_min_rows": -1.75, "heat1d_plain_fused_f32": 0.3, "box1d_r2_fused_f64": -1.75,
          "heat1d_m4_rem3_fused": 2.5, "heat1d_long_group_f64": 0.3}


@pytest.mark.parametrize("case", DIR_CASES, ids=lambda c: c[0])
def test_dirichlet_ghost_value_bit_exact(case):
    """Ghosts of a nonzero value (the pad filled with it, the fused kernels
    writing it at every stage): bit for bit the oracle's folded reading with
    the same ghost, and the FP64 sweep with that ghost within the gate."""
    name, w, kind, shape, T, m, dt = case
    c = GHOSTS[name]
    print("dirichlet ghost", name, shape, "T", T, "m", m, dt, "ghost", c, flush=True)
    if dt == "f32":
        w = synth.to_f32_exact(w)
        u0 = synth.grid_f32(shape)
    else:
        u0 = synth.grid_f64(shape)
    got = _run_dirichlet(w, kind, u0, T, m, ghost=c)
    if dt == "f32":
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, m, f32=True, ghost=c))
        ref64 = oracle.sweep(w, u0.astype(np.float64), T, "zero", float(np.float32(c)))
        assert oracle.errors(got, ref64)["e_rel"] < 1e-5
    else:
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, m, ghost=c))
        ref64 = oracle.sweep(w, u0, T, "zero", c)
        assert oracle.errors(got, ref64)["e_rel"] < 1e-13


@pytest.mark.parametrize("mode,gate", [("exact", 0.0), ("symmetric", 1e-5), ("separable", 1e-5),
                                       ("mfma", 1e-3)])
def test_dirichlet_ghost_value_other_modes(mode, gate):
    w = np.full((3, 3), 1.0 / 9.0) if mode == "separable" else synth.WORKLOADS["star2d"].weights
    if mode == "mfma":
        w = synth.WORKLOADS["box2d"].weights
    w = synth.to_f32_exact(w)
    kind = sf.STENCIL_STAR if mode in ("exact", "symmetric") else sf.STENCIL_BOX
    code = {"exact": sf.STENCIL_MODE_EXACT_ORDER, "symmetric": sf.STENCIL_MODE_SYMMETRIC,
            "separable": sf.STENCIL_MODE_SEPARABLE, "mfma": sf.STENCIL_MODE_MFMA_BF16X3}[mode]
    u0 = synth.grid_f32((70, 256))
    T, m, c = 11, 4, -1.25
    print("dirichlet ghost mode", mode, flush=True)
    got = _run_dirichlet(w, kind, u0, T, m, code, ghost=c)
    if gate == 0.0:
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, m, f32=True, ghost=c))
    else:
        ref64 = oracle.sweep(w, u0.astype(np.float64), T, "zero", c)
        assert oracle.errors(got, ref64)["e_rel"] < gate


def test_dirichlet_ghost_value_changed_on_a_plan():
    """A plan's ghost value can change between runs: the pads of the kept
    buffers are refilled on every run."""
    w = synth.to_f32_exact(synth.WORKLOADS["star2d"].weights)
    plan = sf.Plan(w, sf.STENCIL_STAR, sf.STENCIL_DIRICHLET)
    plan.fold(2)
    u0 = synth.grid_f32((48, 300))
    for c in (1.5, 0.0, -0.5):
        plan.set_boundary_value(c)
        got = _run_dirichlet(w, sf.STENCIL_STAR, u0, 9, 2, plan=plan)
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, 9, 2, f32=True, ghost=c)), c
    plan.close()


def test_dirichlet_plan_reused_across_geometries():
    """The padded buffers are kept by the plan: a smaller grid after a larger
    one (stale data where the new pads lie) and the larger one again."""
    w = synth.WORKLOADS["star2d"].weights
    plan = sf.Plan(w, sf.STENCIL_STAR, sf.STENCIL_DIRICHLET)
    plan.fold(2)
    for shape, T in (((64, 200), 7), ((20, 33), 6), ((64, 200), 5)):
        u0 = synth.grid_f32(shape)
        got = _run_dirichlet(w, sf.STENCIL_STAR, u0, T, 2, plan=plan)
        assert np.array_equal(got, oracle.dirichlet_folded(w, u0, T, 2, f32=True)), shape
    plan.close()


# ------------------------------------------ nonlinear Table 1 workloads

def _apop_inputs(n, f32):
    u0 = synth.grid_f32((n,)) if f32 else synth.grid_f64((n,))
    x = np.arange(n, dtype=np.float64)
    payoff = np.maximum(0.6 - x / n, 0.0)
    return u0, payoff.astype(np.float32) if f32 else payoff


@pytest.mark.parametrize("n,T,f32,fusion", [(100_003, 37, False, 0), (37, 9, True, 0),
                                            (4099, 64, True, 0), (4099, 12, False, 1)])
def test_apop_floor_bit_exact(n, T, f32, fusion):
    """u <- maxNum(A u, payoff) every step (APOP, Table 1), several steps
    fused per launch: bit-exact against the oracle's step-by-step loop."""
    w = synth.to_f32_exact(np.array([0.3, 0.45, 0.249])) if f32 else np.array([0.3, 0.45, 0.249])
    u0, payoff = _apop_inputs(n, f32)
    plan = sf.Plan(w, sf.STENCIL_STAR)
    plan.set_fusion(fusion)
    fl = torch.from_numpy(payoff).to(DEV)
    plan.set_floor(fl)
    data = torch.from_numpy(u0).to(DEV)
    print("apop", n, T, f32, plan.schedule(data, T), flush=True)
    plan.run(data, T, torch.empty_like(data))
    torch.cuda.synchronize()
    got = data.cpu().numpy()
    plan.close()
    assert np.array_equal(got, oracle.floor_sweep(w, u0, payoff, T, f32=f32))


@pytest.mark.parametrize("shape,T", [((64, 96), 9), ((37, 41), 6), ((5000, 5000), 3),
                                     ((3, 4), 5), ((1, 8), 2),
                                     # fused generations (16, 8, 4, 2 per launch)
                                     ((300, 1024), 37), ((33, 256), 16), ((100, 260), 30),
                                     ((512, 5000), 19)])
def test_life_bit_exact(shape, T):
    g = np.random.default_rng(shape[0] * 7 + shape[1]).integers(0, 2, size=shape).astype(np.uint8)
    cells = torch.from_numpy(g).to(DEV)
    sf.stencil_life(cells, torch.empty_like(cells), T)
    torch.cuda.synchronize()
    assert np.array_equal(cells.cpu().numpy(), oracle.life(g, T))


def test_life_glider_on_gpu():
    g = np.zeros((32, 32), dtype=np.uint8)
    for y, x in ((0, 1), (1, 2), (2, 0), (2, 1), (2, 2)):
        g[y, x] = 1
    cells = torch.from_numpy(g).to(DEV)
    sf.stencil_life(cells, torch.empty_like(cells), 64)
    torch.cuda.synchronize()
    assert np.array_equal(cells.cpu().numpy(), np.roll(g, (16, 16), axis=(0, 1)))


@pytest.mark.parametrize("T,m", [(50, 1), (21, 2), (3, 1), (13, 1), (15, 2), (2, 1), (16, 1)])
def test_batched_fused_passes_bit_exact(tmp_path, T, m):
    """Fused passes (full passes of 8 plain applications at radius 1, 4 at
    radius 2, then one pass of the remainder, e.g. 50 = 6 x 8 + 2), then the
    plain remainder one step per launch; odd launch counts end in a copy
    back.  Every grid bit-exact against the oracle's mirror."""
    sides = [512, 1024, 260, 300, 64, 256]
    kinds = [synth.STAR, synth.BOX, synth.STAR, synth.BOX, synth.STAR, synth.BOX]
    weights = [synth.WORKLOADS["star2d"].weights, synth.WORKLOADS["box2d"].weights] * 3
    grids = [synth.grid_f32((s, s), stream=5 + i) for i, s in enumerate(sides)]
    cache = tmp_path / "m.txt"
    cache.write_text("".join("stencil-batched-m %d 1 %d %d\n" % (sh, c, m)
                             for sh in (0, 1) for c in range(5, 12)))
    outs, chosen = _run_batched(kinds, weights, grids, T, tune_cache=str(cache), max_m=m)
    assert chosen == [m] * len(grids)
    for g, w, o in zip(grids, weights, outs):
        assert np.array_equal(o, oracle.folded_reference_f32(w, g, T, m))


# (ny, nx) around every strip-layout threshold: 64-column strips from 55
# columns (radius 1 only), 128-column strips from 119, 256-column strips from
# 247, remainders covered by narrow strips, too few rows to fuse (16 < 17),
# radius-2 folds on grids too narrow for their strips (one step per launch)
NARROW_SHAPES = [(70, 55), (64, 54), (100, 119), (81, 118), (90, 247), (65, 246), (40, 290),
                 (33, 700), (17, 200), (16, 300), (257, 301), (120, 252), (96, 480), (50, 484)]


@pytest.mark.parametrize("T,m,rows,kc,narrow", [
    (50, 1, 0, 0, 0), (21, 2, 0, 0, 0), (13, 1, 32, 0, 0), (15, 2, 128, 0, 0), (9, 1, 16, 0, 0),
    # tuned caps on the applications of a fused pass (narrower borders) and
    # the narrow strip layout
    (17, 1, 0, 4, 0), (23, 1, 32, 2, 1), (19, 2, 0, 2, 1), (11, 1, 128, 3, 1), (26, 1, 0, 0, 1)])
def test_batched_narrow_strips_bit_exact(tmp_path, T, m, rows, kc, narrow):
    """Fused passes cover a grid's columns with 256-column strips and its
    last columns (or a whole narrow grid) with 128- and 64-column strips, of
    the tuned height (rows; 0 = the default 64), the tuned cap on a pass's
    applications (kc; 0 = the kernel's 8 at radius 1, 4 at radius 2) and
    layout (narrow: no 256-column strips); grids no layout fits run one step
    per launch.  Every grid bit-exact against the oracle's mirror, stars and
    boxes, rows of whole vectors or not."""
    kinds = [synth.STAR if i % 2 == 0 else synth.BOX for i in range(len(NARROW_SHAPES))]
    weights = [synth.WORKLOADS["star2d"].weights if k == synth.STAR
               else synth.WORKLOADS["box2d"].weights for k in kinds]
    grids = [synth.grid_f32(sh, stream=5 + i % 10) for i, sh in enumerate(NARROW_SHAPES)]
    print("batched narrow strips T", T, "m", m, "rows", rows, "kc", kc, "narrow", narrow,
          NARROW_SHAPES, flush=True)
    cache = tmp_path / "m.txt"
    cls = [(sh, c) for sh in (0, 1) for c in range(3, 12)]
    cache.write_text("".join("stencil-batched-m %d 1 %d %d\n" % (sh, c, m) for sh, c in cls) +
                     "".join("stencil-batched-rows %d 1 %d %d\n" % (sh, c, rows)
                             for sh, c in cls if rows) +
                     "".join("stencil-batched-kc %d 1 %d %d\n" % (sh, c, kc)
                             for sh, c in cls if kc) +
                     "".join("stencil-batched-narrow %d 1 %d 1\n" % (sh, c)
                             for sh, c in cls if narrow))
    outs, chosen = _run_batched(kinds, weights, grids, T, tune_cache=str(cache), max_m=m)
    assert chosen == [m] * len(grids)
    for g, w, o, sh in zip(grids, weights, outs, NARROW_SHAPES):
        assert np.array_equal(o, oracle.folded_reference_f32(w, g, T, m)), sh


GRAPH_CASES = [
    # (name, weights, kind, shape, T, m, mode, dtype, caller scratch); every
    # run makes more than 4 launches (shorter runs are never captured)
    ("star2d_fused_odd", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (300, 1024), 75, 1,
     "vector", np.float32, True),
    ("star2d_m4_plan_scratch", synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR, (257, 1031), 42,
     4, "vector", np.float32, False),
    ("box2d_m8_mfma", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (140, 530), 56, 8, "mfma",
     np.float32, True),
    ("heat1d_f64", synth.heat1d_weights(), sf.STENCIL_STAR, (100_003,), 237, 1, "vector", np.float64,
     True),
    ("star3d_m2", synth.WORKLOADS["star3d"].weights, sf.STENCIL_STAR, (20, 33, 70), 25, 2, "vector",
     np.float32, True),
    ("box2d_exact", synth.WORKLOADS["box2d"].weights, sf.STENCIL_BOX, (61, 99), 5, 1, "exact",
     np.float32, False),
]


@pytest.mark.parametrize("case", GRAPH_CASES, ids=lambda c: c[0])
def test_run_graph_replays_equal_direct_launches(case):
    """stencil_plan_set_graph: the captured time loop, replayed several times
    with other eager work and synchronisations in between, gives the direct
    launches' result bit for bit every time (and the oracle's where the
    kernels keep the canonical order)."""
    name, w, kind, shape, T, m, mode, dt, caller_scratch = case
    w = synth.to_f32_exact(w) if dt == np.float32 else w
    u0 = synth.grid_f32(shape) if dt == np.float32 else synth.grid_f64(shape)
    print("graph replay", name, shape, "T", T, "m", m, mode, flush=True)
    modes = {"vector": sf.STENCIL_MODE_VECTOR, "exact": sf.STENCIL_MODE_EXACT_ORDER,
             "mfma": sf.STENCIL_MODE_MFMA_BF16X3}
    plan = sf.Plan(w, kind)
    if m > 1:
        plan.fold(m)
    plan.set_mode(modes[mode])
    data = torch.from_numpy(u0).to(DEV)
    scr = torch.empty_like(data) if caller_scratch else None
    plan.run(data, T, scr)
    torch.cuda.synchronize()
    direct = data.cpu().numpy()
    if mode != "mfma":
        ref = (oracle.folded_reference_f32(w, u0, T, m) if dt == np.float32
               else oracle.sweep(w, u0, T))
        assert np.array_equal(direct, ref)
    sched = plan.schedule(data, T, scr)
    launches = sched["folded_launches"] + sched["plain_launches"] + sched["final_copy"]
    assert launches > 4, sched  # the run is captured, not launched directly
    plan.set_graph(True)
    other = sf.Plan(synth.WORKLOADS["star2d"].weights, sf.STENCIL_STAR)
    side = torch.from_numpy(synth.grid_f32((64, 80), stream=7)).to(DEV)
    for rep in range(4):
        data.copy_(torch.from_numpy(u0).to(DEV))
        plan.run(data, T, scr)
        # eager work of the program between replays
        other.run(side, 3)
        _ = (side * 2.0).sum().item()
        torch.cuda.synchronize()
        assert np.array_equal(data.cpu().numpy(), direct), "replay %d differs" % rep
    # a plan change drops the graph: fold depth 1 must give the plain result
    plan.fold(1)
    data.copy_(torch.from_numpy(u0).to(DEV))
    plan.run(data, T, scr)
    torch.cuda.synchronize()
    plain = data.cpu().numpy()
    plan.set_graph(False)
    data.copy_(torch.from_numpy(u0).to(DEV))
    plan.run(data, T, scr)
    torch.cuda.synchronize()
    assert np.array_equal(plain, data.cpu().numpy())
    other.close()
    plan.close()
