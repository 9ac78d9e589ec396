"""GPU parity at the measured workloads' full sizes, in the launch
configurations bench.py times.

The oracle cannot sweep a 16384^2 grid for hundreds of steps, so:
  * sampled outputs of short runs are computed one by one by the oracle on
    each sample's dependency window (the FP32 mirror of the same schedule, so
    vector kernels must match bit for bit; the matrix-core form within 1e-3 of
    the FP64 sweep);
  * long runs are checked through properties that hold at any size: mass
    (sum w)^T sum u0 against the FP64 compensated GPU sum, and bitwise
    translation equivariance of the whole grid.
"""

import functools
import math
import zlib

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


@functools.lru_cache(maxsize=2)
def full_grid(name):
    return synth.grid_f32(synth.WORKLOADS[name].shape)


def window(u0, p, reach):
    idx = [(int(c) + np.arange(-reach, reach + 1)) % n for c, n in zip(p, u0.shape)]
    return u0[np.ix_(*idx)]


def sampled_points(shape, k, seed):
    rng = np.random.default_rng(seed)
    pts = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(k)]
    pts.append(tuple(0 for _ in shape))
    pts.append(tuple(n - 1 for n in shape))
    return pts


def run(w, kind, u0, T, m, mode=sf.STENCIL_MODE_VECTOR):
    plan = sf.Plan(w, kind)
    if m > 1:
        plan.fold(m)
    plan.set_mode(mode)
    d = torch.from_numpy(u0).to(DEV)
    s = torch.empty_like(d)
    plan.run(d, T, s)
    torch.cuda.synchronize()
    plan.close()
    return d


@pytest.mark.parametrize("name,m,T,mode", [
    ("star2d", 1, 6, "vector"), ("star2d", 2, 6, "vector"), ("star2d", 4, 8, "vector"),
    ("box2d", 4, 8, "vector"), ("box2d", 8, 8, "vector"), ("box2d", 4, 8, "mfma"),
    ("box2d", 8, 16, "mfma"), ("star3d", 2, 4, "vector"), ("box3d", 2, 4, "vector"),
    ("box3d", 1, 3, "vector"), ("unitbox2d", 8, 16, "separable"), ("box2d", 1, 16, "vector"),
    # the headline launch geometry: two fused launches of 10 steps each
    # (strip height from the occupancy query), and the plain 7-point 3D star
    ("star2d", 1, 20, "vector"), ("star3d", 1, 3, "vector"),
    # 3D fused launches beside those the 512^3 runs make: four steps of the
    # 7-point star (a fused launch of three, then one plain step; four per
    # launch where STENCIL_TB3_STAR_K asks for them), two of the 27-point box
    ("star3d", 1, 4, "vector"), ("box3d", 1, 4, "vector"),
])
def test_sampled_outputs_full_size(name, m, T, mode):
    wl = synth.WORKLOADS[name]
    print("full size", name, wl.shape, "m", m, "T", T, mode, flush=True)
    u0 = full_grid(name)
    mcode = {"mfma": sf.STENCIL_MODE_MFMA_BF16X3, "separable": sf.STENCIL_MODE_SEPARABLE,
             "vector": sf.STENCIL_MODE_VECTOR}[mode]
    d = run(wl.weights, wl.shape_kind, u0, T, m, mcode)
    pts = sampled_points(wl.shape, 40, zlib.crc32(("%s-%d" % (name, m)).encode()))
    got = np.array([d[p].item() for p in pts], dtype=np.float32)
    reach = T * ((wl.weights.shape[0] - 1) // 2)
    centre = tuple([reach] * len(wl.shape))
    if mode == "vector":
        ref = np.array([oracle.folded_reference_f32(wl.weights, window(u0, p, reach), T, m)[centre]
                        for p in pts], dtype=np.float32)
        assert np.array_equal(got, ref)
    ref64 = np.array([oracle.sweep(wl.weights, window(u0, p, reach).astype(np.float64), T)[centre]
                      for p in pts])
    err = np.max(np.abs(got - ref64)) / np.max(np.abs(ref64))
    assert err < (1e-3 if mode == "mfma" else 1e-5), err
    if (name, m, T) == ("star2d", 1, 24):
        plan = sf.Plan(wl.weights, wl.shape_kind)
        sched = sf.stencil_run_schedule(plan.handle, wl.shape, sf.STENCIL_F32, T, 1 << 30, 1 << 34)
        assert (sched["plain_launches"], sched["final_copy"]) == (2, False)
        plan.close()
    if mode == "separable":
        plan = sf.Plan(wl.weights, wl.shape_kind)
        plan.fold(m)
        assert plan.separable() == (1, True)
        plan.close()


@pytest.mark.parametrize("name,m", [("star2d", 4), ("star2d", 1), ("star3d", 2), ("box2d", 8)])
def test_long_run_mass_full_size(name, m):
    """Full T: total mass equals (sum w)^T times the initial mass to within
    the FP32 rounding the run can accumulate (bound derived below)."""
    wl = synth.WORKLOADS[name]
    u0 = full_grid(name)
    d = torch.from_numpy(u0).to(DEV)
    s0 = sf.stencil_residual(d)[0]
    plan = sf.Plan(wl.weights, wl.shape_kind)
    if m > 1:
        plan.fold(m)
    s = torch.empty_like(d)
    plan.run(d, wl.T, s)
    torch.cuda.synchronize()
    s1 = sf.stencil_residual(d)[0]
    plan.close()
    sw = math.fsum(wl.weights.ravel().tolist())
    expect = sw ** wl.T * s0
    # each sweep rounds every output once per tap (relative 2^-24 each,
    # unbiased): the mean mass error of N points grows like
    # sweeps * taps * 2^-24 / sqrt(N); allow a bias of 2^-24 per sweep on top
    sweeps = wl.T // m + wl.T % m
    bound = sweeps * 2.0 ** -24 * 4
    assert abs(s1 - expect) / abs(expect) < bound, (s1, expect, bound)


@pytest.mark.parametrize("name,m", [("star2d", 4), ("box3d", 2)])
def test_translation_equivariance_full_size(name, m):
    wl = synth.WORKLOADS[name]
    u0 = full_grid(name)
    shift = tuple(n // 3 + 1 for n in wl.shape)
    axes = tuple(range(len(wl.shape)))
    T = 2 * m + 1
    a = run(wl.weights, wl.shape_kind, np.ascontiguousarray(np.roll(u0, shift, axes)), T, m)
    b = run(wl.weights, wl.shape_kind, u0, T, m)
    assert torch.equal(a, torch.roll(b, shift, axes))


def test_heat1d_full_size_bit_exact_fp64():
    wl = synth.WORKLOADS["heat1d"]
    u0 = synth.grid_f64(wl.shape)
    d = run(wl.weights, wl.shape_kind, u0, wl.T, 1)
    ref = oracle.sweep(wl.weights, u0, wl.T)
    assert np.array_equal(d.cpu().numpy(), ref)


@pytest.mark.parametrize("case", [
    # the 1D5P line (random positive 5-point box, FP64) and a long FP32 heat
    # line: both run the workgroup-owned 1D kernel (more than four wavefront
    # spans per SIMD), several steps fused per launch
    ("box1d5p", 10_240_000, 60, "f64"),
    ("heat_f32", 6_000_000, 53, "f32"),
    # a middle-length line: wavefront spans of 16 points per lane (shorter
    # lines take 8, longer ones the workgroup spans)
    ("heat_f64_mid", 3_000_000, 51, "f64"),
], ids=lambda c: c[0])
def test_1d_long_line_sampled_bit_exact(case):
    """Sampled points of a long line, bit-exact against the oracle's sweep of
    each point's window (2RT+1 points: exact at its centre after T steps)."""
    name, n, T, dt = case
    if name == "box1d5p":
        w, kind = synth.WORKLOADS["box1d5p"].weights, sf.STENCIL_BOX
    else:
        w, kind = synth.to_f32_exact(synth.heat1d_weights()), sf.STENCIL_STAR
    r = (len(w) - 1) // 2
    u0 = synth.grid_f64((n,)) if dt == "f64" else synth.grid_f32((n,))
    print("1d long line", name, n, "T", T, dt, flush=True)
    u = run(w, kind, u0, T, 1).cpu().numpy()
    for x in sampled_points((n,), 20, zlib.crc32(name.encode())):
        x = x[0]
        idx = (x + np.arange(-r * T, r * T + 1)) % n
        if dt == "f64":
            ref = oracle.sweep(w, u0[idx], T)[r * T]
        else:
            ref = oracle.sweep_f32(w, u0[idx], T)[r * T]
        assert u[x] == ref, x


def test_batched_full_size_sampled_grids(tmp_path):
    """The 4096-grid batch as bench.py runs it (autotuned m <= 2, graph):
    16 grids checked whole against the oracle's FP32 mirror of their fold
    depth."""
    count, T = 4096, 50
    sides, kinds, weights = synth.batched_recipe(count)
    npts = int(np.sum(sides.astype(np.int64) ** 2))
    flat = synth.uniform_f32(synth.SEED, synth.STREAM_GRID, npts)
    u0s, off = [], 0
    for s in sides:
        n = int(s) * int(s)
        u0s.append(flat[off:off + n].reshape(int(s), int(s)))
        off += n
    datas = [torch.from_numpy(u).to(DEV) for u in u0s]
    scr = [torch.empty_like(d) for d in datas]
    plans = [sf.Plan(w, sf.STENCIL_STAR if k == synth.STAR else sf.STENCIL_BOX)
             for k, w in zip(kinds, weights)]
    chosen = sf.stencil_run_batched([p.handle for p in plans], datas, scr, T, autotune=True,
                                    tune_cache=str(tmp_path / "t.txt"), use_graph=True, max_m=2)
    torch.cuda.synchronize()
    order = np.argsort(sides)
    pick = list(order[:10]) + list(order[count // 2: count // 2 + 4]) + list(order[-2:])
    for i in pick:
        ref = oracle.folded_reference_f32(weights[i], u0s[i], T, chosen[i])
        assert np.array_equal(datas[i].cpu().numpy(), ref), (i, int(sides[i]), chosen[i])
    for p in plans:
        p.close()


def test_dirichlet_sampled_outputs_full_size():
    """Zero boundaries at the measured size (8192^2, fold m = 4, T = 8):
    sampled points, corners and edges included, against the FP64 zero-ghost
    oracle on the point's window clipped to the grid (a window edge inside the
    grid perturbs points within T*r of it only, so the centre is exact)."""
    wl = synth.WORKLOADS["star2d_dirichlet"]
    u0 = full_grid("star2d")
    T, m = 8, 4
    plan = sf.Plan(wl.weights, wl.shape_kind, sf.STENCIL_DIRICHLET)
    plan.fold(m)
    d = torch.from_numpy(u0).to(DEV)
    plan.run(d, T)
    torch.cuda.synchronize()
    plan.close()
    ny, nx = wl.shape
    pts = sampled_points(wl.shape, 30, zlib.crc32(b"star2d_dirichlet"))
    pts += [(0, nx // 2), (ny // 2, 0), (ny - 1, nx // 2), (2, nx - 3), (ny - 4, 1)]
    reach = T * 1
    for p in pts:
        y0, y1 = max(0, p[0] - reach), min(ny, p[0] + reach + 1)
        x0, x1 = max(0, p[1] - reach), min(nx, p[1] + reach + 1)
        win = u0[y0:y1, x0:x1].astype(np.float64)
        ref = oracle.sweep(wl.weights, win, T, "zero")[p[0] - y0, p[1] - x0]
        got = d[p].item()
        assert abs(got - ref) <= 1e-5 * abs(ref), (p, got, ref)


def test_dirichlet_plain_fused_full_size():
    """Zero boundaries, plain sweep at the measured size (8192^2, T = 20: two
    launches of 10 fused steps on the padded grid): sampled points, corners
    and edges included, against the FP64 zero-ghost oracle on the point's
    window clipped to the grid."""
    wl = synth.WORKLOADS["star2d_dirichlet"]
    u0 = full_grid("star2d")
    T = 20
    plan = sf.Plan(wl.weights, wl.shape_kind, sf.STENCIL_DIRICHLET)
    d = torch.from_numpy(u0).to(DEV)
    sched = plan.schedule(d, T)
    assert sched["plain_launches"] == 2
    plan.run(d, T)
    torch.cuda.synchronize()
    plan.close()
    ny, nx = wl.shape
    pts = sampled_points(wl.shape, 30, zlib.crc32(b"star2d_dirichlet_plain"))
    pts += [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (5, nx // 3), (ny // 3, nx - 2)]
    reach = T * 1
    for p in pts:
        y0, y1 = max(0, p[0] - reach), min(ny, p[0] + reach + 1)
        x0, x1 = max(0, p[1] - reach), min(nx, p[1] + reach + 1)
        win = u0[y0:y1, x0:x1].astype(np.float64)
        ref = oracle.sweep(wl.weights, win, T, "zero")[p[0] - y0, p[1] - x0]
        got = d[p].item()
        assert abs(got - ref) <= 1e-5 * abs(ref), (p, got, ref)


def test_apop_full_size_sampled_bit_exact():
    """APOP at its Table 1 size (10,240,000 points, FP64), 40 steps fused as
    the library runs them: sampled points bit-exact against the oracle's loop
    on each point's window."""
    n, w = synth.APOP["n"], synth.APOP["weights"]
    T = 40
    payoff = synth.apop_payoff(n)
    plan = sf.Plan(w, sf.STENCIL_STAR)
    fl = torch.from_numpy(payoff).to(DEV)
    plan.set_floor(fl)
    d = torch.from_numpy(payoff.copy()).to(DEV)
    plan.run(d, T, torch.empty_like(d))
    torch.cuda.synchronize()
    u = d.cpu().numpy()
    plan.close()
    for x in sampled_points((n,), 20, 7) :
        x = x[0]
        idx = (x + np.arange(-T, T + 1)) % n
        assert u[x] == oracle.floor_sweep(w, payoff[idx], payoff[idx], T)[T], x
