#!/usr/bin/env python3
"""Benchmark: iterated stencil sweeps with temporal computation folding on one
MI355X, reported as GStencil/s (grid points x original time steps per second)
and as a fraction of the roofline that bounds the dominant kernel.

Default run: the five measured workloads, each with all of its forms (plain,
folded, matrix-core, batched), every result checked against the FP64 oracle:
  star2d   2D 5-point star (centre 0.6, neighbours 0.1), 8192^2 FP32, T=1000,
           plain and folds m=2, m=4 -- the headline of the JSON line;
  heat1d   1D 3-point heat (0.25, 0.5, 0.25), 1,000,000 points FP64, T=100;
  star3d   3D 7-point star (0.4; 0.1), 512^3 FP32, T=200, plain and m=2;
  box3d    3D 27-point random positive box, 512^3 FP32, T=200, plain and m=2;
  box2d    2D 9-point random positive box, 16384^2 FP32, T=400, plain, m=4
           (9x9) and m=8 (17x17), vector and BF16x3 matrix-core forms;
  batched  4096 periodic 2D grids, sides log-uniform in [64, 1024], 5-point
           star or 9-point box, FP32, T=50, one hipGraph of persistent and
           fused launches against one stencil_run per grid.
Inputs are synthetic (SplitMix64, seed 2103), uniform [0, 1).  One step of a
form = one stencil_run of all T original steps with the plan and folded
weights prepared beforehand and the grid resident in HBM.

The line's top-level fields describe star2d's fastest form; "configs" holds
the same fields for every workload.  --workload X runs one workload alone
(profiling runs), and also the extras: Table 1's box1d5p, apop1d and
life2d, the unit boxes unitbox2d and unitbox3d, the zero-boundary
star2d_dirichlet and the FP64 star star2d_f64.

Prints ONE JSON line on stdout.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0           # HBM3E
FP32_VECTOR_TFLOPS = 157.3      # FP32 vector (counts packed FP32 FMAs)
FP64_VECTOR_TFLOPS = 78.6       # FP64 vector
BF16_MFMA_TFLOPS = 2500.0       # dense BF16 matrix
# FP32 FMA issue rate without packed FP32 (the kernels are built with packed
# FP32 disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_FMA_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "GStencil/s and % HBM roofline, plain vs folded/MFMA/batched at stated error"
VALU32_TOPS = 256 * 64 * 2.4e9 / 1e12  # 32-bit VALU lane-operations per second (x1e12)
DEFAULT_SET = ("star2d", "heat1d", "star3d", "box3d", "box2d", "batched")
GATE = {"vector": 0.0, "vector_graph": 0.0, "vector_unfused": 0.0, "symmetric": 1e-5,
        "separable": 1e-5, "mfma_bf16x3": 1e-3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all",
                    choices=["all", "star2d", "heat1d", "star3d", "box3d", "box2d", "unitbox2d",
                             "star2d_dirichlet", "star2d_f64", "unitbox3d", "box1d5p", "apop1d",
                             "life2d", "batched"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the FP64 oracle reference (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=0.0,
                    help="CPU oracle sample per workload (default 10 s alone, 6 s in the "
                         "default run)")
    ap.add_argument("--only-m", type=int, default=0,
                    help="time only this fold depth (profiling runs)")
    ap.add_argument("--only-mode", default="",
                    choices=["", "vector", "vector_unfused", "symmetric", "separable",
                             "mfma_bf16x3", "vector_graph", "tuned"],
                    help="time only this kernel family (profiling runs)")
    ap.add_argument("--no-per-grid", action="store_true",
                    help="batched: skip the per-grid-launch baseline (profiling runs)")
    ap.add_argument("--tune-cache", default="",
                    help="batched: tuning cache file to use (and fill); default a fresh "
                         "temporary file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 256 MiB device copy (PMC byte-counter calibration)")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# Source files holding each kernel family's device code: a committed PMC
# summary stays valid while these are unchanged.
KERNEL_SOURCES = {
    "sweep1d": ("sweep1d.hip",),
    "sweep2d": ("sweep2d.hip", "sweep2d_common.h", "sweep2d_impl.h", "sweep2d_launch.h",
                "sweep2d_r1.hip", "sweep2d_r2.hip", "sweep2d_r3.hip", "sweep2d_r4.hip",
                "sweep2d_r5.hip", "sweep2d_r6.hip", "sweep2d_r7.hip", "sweep2d_r8.hip"),
    "sweep2dtb": ("sweep2d_tb.hip", "sweep2d_common.h"),
    "sweep3d": ("sweep3d.hip",),
    "sweep3dtb": ("sweep3d_tb.hip",),
    "sweep3dsep": ("sweep3d_sep.hip",),
    "mfma2d": ("mfma2d.hip",),
    "life": ("life.hip",),
    "batched": ("batched.hip", "sweep2d_common.h", "sweep2d_impl.h"),
}


def kernel_family(kernel_key: str) -> str:
    return kernel_key.split("_")[0]


def kernel_source_hash(family: str) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_09235_amd", "csrc")
    for name in KERNEL_SOURCES[family]:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key: str, workload: str, field: str = "hbm-bytes-per-launch"):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if one
    exists for this kernel and workload and the kernel's sources have not
    changed since it was taken (its 'source-hash' line)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (kernel_key, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source-hash:\s*(\w+)", text)
    if not m or m.group(1) != kernel_source_hash(kernel_family(kernel_key)):
        return None
    b = re.search(re.escape(field) + r":\s*([0-9.eE+]+)", text)
    return float(b.group(1)) if b else None


def roofline(algo_bytes: float, flops: float, dur_s: float, peak_tflops: float, basis: str,
             unit_kind: str = "alu", force_hbm: bool = False) -> dict:
    """The roofline of one launch against MI355X's published peaks: the
    kernel's algorithmic intensity (flops per algorithmic HBM byte) against
    the ridge peak / 8 TB/s decides the bound; frac = achieved / peak of that
    bound, which is also achieved / min(peak, intensity x 8 TB/s)."""
    intensity = flops / algo_bytes if algo_bytes else float("inf")
    ridge = peak_tflops * 1e12 / (HBM_PEAK_GBS * 1e9)
    gbs = algo_bytes / dur_s / 1e9
    tfl = flops / dur_s / 1e12
    if intensity < ridge or force_hbm:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        r = {"bound": unit_kind, "achieved": round(tfl, 2), "peak": peak_tflops,
             "unit": "TFLOP/s"}
    r["frac"] = round(r["achieved"] / r["peak"], 4)
    r["intensity_flop_per_byte"] = round(intensity, 3)
    r["compute_peak"] = {"tflops": peak_tflops, "basis": basis}
    r["attainable_tflops"] = round(min(peak_tflops, intensity * HBM_PEAK_GBS / 1e3), 2)
    r["achieved_gbs"] = round(gbs, 1)
    r["achieved_tflops"] = round(tfl, 2)
    r["launch_ms"] = round(dur_s * 1e3, 5)
    r["algorithmic_bytes_per_launch"] = int(algo_bytes)
    r["algorithmic_flops_per_launch"] = float(flops)
    return r


def time_runs(fn, steps, warmup):
    """Seconds of `steps` calls between two HIP events on the current stream
    (the stream the library launches on), after `warmup` untimed calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def cpu_baseline(w, shape_full, T_full, budget_s, boundary="periodic"):
    """The oracle as it stands, timed on a bounded sample of the workload: a
    smaller grid of the same dimension and distribution (the full grid when
    it fits the budget), for a number of original steps chosen to fill about
    budget_s seconds."""
    import numpy as np
    import oracle
    import synth
    shape = tuple(shape_full)
    u0 = synth.grid_f64(shape)
    oracle.sweep(w, u0, 1, boundary)  # warm: threads, page faults
    # per-step cost from two calls (each call also pays a fixed cost for its
    # FP64 copies of the grid)
    t0 = time.perf_counter()
    oracle.sweep(w, u0, 2, boundary)
    t2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.sweep(w, u0, 6, boundary)
    t6 = time.perf_counter() - t0
    per_step = max((t6 - t2) / 4, t6 / 12, 1e-6)
    fixed = max(0.0, t2 - 2 * per_step)
    T = int(max(1, min(T_full, (budget_s - fixed) / per_step)))
    t0 = time.perf_counter()
    oracle.sweep(w, u0, T, boundary)
    dt = time.perf_counter() - t0
    if dt < 0.7 * budget_s and T < T_full:
        # short runs overstate the per-step cost: size the timed sample again
        T = int(max(1, min(T_full, T * budget_s / max(dt, 1e-6))))
        t0 = time.perf_counter()
        oracle.sweep(w, u0, T, boundary)
        dt = time.perf_counter() - t0
    n = int(np.prod(shape))
    return {
        "value": round(n * T / dt / 1e9, 4),
        "unit": "GStencil/s",
        "cores": oracle.num_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": "FP64 naive sweep, grid %s, %d of the %d original steps, %.1f s" % (
            "x".join(map(str, shape)), T, T_full, dt),
    }


def oracle_reference(w, u0, T, boundary="periodic"):
    """u_T in FP64 from the oracle: the naive loop where it finishes in a few
    seconds (bit-exact definition), else its spectral form (the same operator
    diagonalised by the DFT, or by the sine transform for zero ghosts;
    rounding of order eps log N)."""
    import numpy as np
    import oracle
    u64 = np.asarray(u0, dtype=np.float64)
    taps = int(np.count_nonzero(w))
    if u64.size * T * taps <= 4e9:
        return oracle.sweep(w, u64, T, boundary), "oracle.sweep (naive FP64 loop, canonical order)"
    return (oracle.sweep_spectral(w, u64, T, boundary),
            "oracle.sweep_spectral (FP64, eigen-decomposition of the operator)")


def error_vs(ref64, got):
    """e_rel = max|u - ref| / max|ref| and e_detr = max|u - ref| / max|ref -
    mean(ref)| (the oracle's error metrics, evaluated on the GPU for full
    grids), and the count of elements equal to the reference."""
    import torch
    d = (got.double() - ref64).abs().max().item()
    nref = ref64.abs().max().item()
    mean = ref64.mean().item()
    ndet = (ref64 - mean).abs().max().item()
    same = int((got.double() == ref64).sum().item())
    return d / nref if nref > 0 else d, d / ndet if ndet > 0 else d, same


def budget_s(args, default_run):
    return args.cpu_seconds if args.cpu_seconds > 0 else (6.0 if default_run else 10.0)


def bench_grid(args, wl_name, default_run=False):
    """One single-grid workload: every form timed, each one's T-step result
    checked against the FP64 oracle, the fastest form within its error gate
    reported with the roofline of its dominant kernel."""
    import numpy as np
    import torch
    import synth
    import paper_2103_09235_amd as sf

    wl = synth.WORKLOADS[wl_name]
    shape, T, w = wl.shape, wl.T, wl.weights
    zero_bc = wl.extra.get("boundary") == "zero"
    bc = sf.STENCIL_DIRICHLET if zero_bc else sf.STENCIL_PERIODIC
    f32 = wl.dtype == "f32"
    esz = 4 if f32 else 8
    n = int(np.prod(shape))
    r = (w.shape[0] - 1) // 2
    # runs this short (the 1D heat line: 0.03 ms) are timed over enough of
    # them to fill several milliseconds; the others over --steps
    steps = max(args.steps, min(1000, -(-20_000_000_000 // (n * T))))
    log("[bench] workload %s: %s" % (wl_name, wl.note))
    u0 = synth.grid_f32(shape) if f32 else synth.grid_f64(shape)
    dev = torch.device("cuda:0")
    data = torch.from_numpy(u0).to(dev)
    scratch = torch.empty_like(data)
    s0, _, _ = sf.stencil_residual(data)

    ref64, ref_kind = None, None
    if not args.no_oracle:
        log("[bench] FP64 oracle reference of T=%d steps" % T)
        t0 = time.perf_counter()
        ref_host, ref_kind = oracle_reference(w, u0, T, "zero" if zero_bc else "periodic")
        ref64 = torch.from_numpy(ref_host).to(dev)
        del ref_host
        log("[bench]   %s, %.1f s" % (ref_kind, time.perf_counter() - t0))

    forms = {}
    best = None
    symmetric = wl.dim == 2 and np.array_equal(w, w[::-1, :]) and np.array_equal(w, w[:, ::-1])
    # extra fold depths beyond the workload's stated ones are reported under
    # "forms" but never chosen as the workload's result
    extra = {"star2d": (8,)}.get(wl_name, ())
    for m in tuple(wl.folds) + extra:
        if args.only_m and m != args.only_m:
            continue
        # (name, mode, fusion): VECTOR fuses several applications per launch
        # where the tiled kernel can (2D FP32 radius <= 4, 1D); "unfused" is
        # the same kernel family one application per launch
        form_modes = []
        if m not in extra:
            form_modes.append(("vector", sf.STENCIL_MODE_VECTOR, 0))
            if not zero_bc:
                # the same launches captured once in a hipGraph and replayed
                form_modes.append(("vector_graph", sf.STENCIL_MODE_VECTOR, 0))
            if wl.dim in (2, 3) and not zero_bc:
                form_modes.append(("vector_unfused", sf.STENCIL_MODE_VECTOR, 1))
        if symmetric:
            form_modes.append(("symmetric", sf.STENCIL_MODE_SYMMETRIC, 0))
        if (wl.dim == 2 and f32 and m > 1) or (wl.dim == 3 and f32):
            probe = sf.Plan(w, wl.shape_kind)
            if m > 1:
                probe.fold(m)
            if probe.separable()[1]:
                form_modes.append(("separable", sf.STENCIL_MODE_SEPARABLE, 0))
            probe.close()
        if wl_name in ("box2d", "unitbox2d") and m > 1:
            form_modes.append(("mfma_bf16x3", sf.STENCIL_MODE_MFMA_BF16X3, 0))
        for mode_name, mode, fusion in form_modes:
            if args.only_mode and mode_name != args.only_mode:
                continue
            plan = sf.Plan(w, wl.shape_kind, bc)
            if m > 1:
                plan.fold(m)
            try:
                plan.set_mode(mode)
            except sf.StencilError as e:
                log("[bench] skip m=%d %s: %s" % (m, mode_name, e))
                continue
            plan.set_fusion(fusion)
            plan.set_graph(mode_name.endswith("_graph"))
            data.copy_(torch.from_numpy(u0).to(dev))
            sched = plan.schedule(data, T, scratch)

            def step():
                plan.run(data, T, scratch)

            log("[bench] m=%d %s: timing %d steps of T=%d" % (m, mode_name, steps, T))
            try:
                el, wall = time_runs(step, steps, args.warmup)
            except sf.StencilError as e:
                log("[bench] skip m=%d %s: %s" % (m, mode_name, e))
                continue
            # mass after the timed runs: data has advanced (warmup+steps)*T steps
            total_T = (args.warmup + steps) * T
            s1, _, _ = sf.stencil_residual(data)
            expect = math.fsum(float(v) for v in w.ravel()) ** total_T * s0
            # (zero boundaries lose mass through the faces: not an invariant)
            mass_rel = None if zero_bc else abs(s1 - expect) / abs(expect)
            # one T-step run from u0 against the oracle
            data.copy_(torch.from_numpy(u0).to(dev))
            plan.run(data, T, scratch)
            err = err_detr = None
            same = None
            if ref64 is not None:
                err, err_detr, same = error_vs(ref64, data)
            gst = n * T * steps / el / 1e9
            launches = sched["folded_launches"] + sched["plain_launches"]
            # the dominant kernel: the folded pass when there is one
            dom = "folded" if sched["folded_launches"] else "plain"
            per_launch = sched[dom + "_apps"] / sched[dom + "_launches"]
            launch_s = el / steps / launches
            algo_bytes = 2 * esz * n
            taps = int(np.count_nonzero(plan.fold(m) if m > 1 else w))
            # flops the form executes per point: one FMA per tap, or for the
            # separable form 2 * rank * (2R+1) (a horizontal and a vertical
            # pass per rank-one term)
            fmas = taps
            if mode_name == "separable":
                fmas = (2 * plan.separable()[0] if wl.dim == 2 else 3) * (2 * m * r + 1)
            flops = 2 * fmas * n * per_launch
            key = "%s_m%d_%s" % (wl_name, m, mode_name)
            gate = (1e-3 if mode_name == "mfma_bf16x3" else 1e-5) if f32 else 1e-12
            forms[key] = {
                "m": m, "mode": mode_name, "gstencil_s": round(gst, 2),
                "ms_per_run": round(el / steps * 1e3, 4),
                "launches_per_run": launches,
                "applications_per_launch": round(per_launch, 3),
                "ms_per_launch": round(launch_s * 1e3, 5), "taps": taps,
                "fmas_per_point": fmas,
                "hbm_gbs_algorithmic": round(algo_bytes / launch_s / 1e9, 1),
                "hbm_frac": round(algo_bytes / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                "tflops": round(flops / launch_s / 1e12, 2),
                "e_rel_vs_oracle": err, "e_detrended_vs_oracle": err_detr,
                "equal_to_oracle": same, "gate": gate,
                "within_gate": None if err is None else bool(err <= gate),
                "mass_rel_drift": mass_rel, "mass_T": total_T,
                "wall_s": round(wall, 3),
            }
            log("[bench]   %.1f GStencil/s, %d launches of %.2f applications, %.4f ms/launch, "
                "e_rel %s (detrended %s), mass drift %s" % (
                    gst, launches, per_launch, launch_s * 1e3,
                    "n/a" if err is None else "%.2e" % err,
                    "n/a" if err_detr is None else "%.2e" % err_detr,
                    "n/a" if mass_rel is None else "%.2e" % mass_rel))
            forms[key]["stated_fold"] = m not in extra
            Rf = m * r
            if mode_name == "mfma_bf16x3":
                # matrix-core work issued: per input row and dy three 16x16x32
                # products (hi*hi, lo*hi, hi*lo) per 16-column block, 64 flop
                # per output point each, over 2R+1 values of dy
                issued = 3 * (2 * Rf + 1) * 64.0 * n * per_launch
                forms[key]["mfma_issued_flop_per_point"] = int(3 * (2 * Rf + 1) * 64)
                forms[key]["mfma_issued_tflops"] = round(issued / launch_s / 1e12, 1)
                forms[key]["mfma_issued_frac_of_bf16_peak"] = round(
                    issued / launch_s / 1e12 / BF16_MFMA_TFLOPS, 4)
            ok = err is None or err <= gate
            if m not in extra and ok and (best is None or gst > best[1]):
                best = (key, gst, el, launch_s, algo_bytes, flops, m, mode_name, taps,
                        per_launch)
            plan.close()
    key, gst, el, launch_s, algo_bytes, flops, m, mode_name, taps, per_launch = best
    if mode_name.startswith("mfma"):
        peak_t, basis, kind = BF16_MFMA_TFLOPS, "dense BF16 matrix, published", "mfma"
    elif f32:
        peak_t, basis, kind = FP32_VECTOR_TFLOPS, "FP32 vector, published", "alu"
    else:
        peak_t, basis, kind = FP64_VECTOR_TFLOPS, "FP64 vector, published", "alu"
    # the symmetric form executes fewer operations than its dense taps: it is
    # priced by its bytes only
    roof = roofline(algo_bytes, flops, launch_s, peak_t, basis, kind,
                    force_hbm=mode_name == "symmetric")
    if f32 and not mode_name.startswith("mfma"):
        # the FP32 FMA issue rate these kernels can reach (packed FP32 off)
        roof["fp32_fma_issue_frac"] = round(flops / launch_s / 1e12 / FP32_FMA_TFLOPS, 4)
        roof["fp32_fma_issue_basis"] = ("256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = "
                                        "78.6 TFLOP/s (FMAs, packed FP32 not used)")
    if mode_name.startswith("mfma"):
        roof["mfma_issued_frac_of_bf16_peak"] = forms[key]["mfma_issued_frac_of_bf16_peak"]
    fused = per_launch > 1 and wl.dim in (2, 3)
    tkey = {"vector": ("sweep%dd%s_m%d" % (wl.dim, "tb" if fused else "", m)),
            "vector_graph": ("sweep%dd%s_m%d" % (wl.dim, "tb" if fused else "", m)),
            "vector_unfused": "sweep%dd_m%d" % (wl.dim, m),
            "symmetric": "sweep%dd_m%d_symmetric" % (wl.dim, m),
            "separable": ("sweep%dd_m%d_separable" % (wl.dim, m) if wl.dim == 2
                          else "sweep3dsep_m%d" % m),
            "mfma_bf16x3": "mfma2d_m%d" % m}[mode_name]
    roof["traffic"] = traffic_from_profiles(tkey, wl_name)
    kname = ("k_sweep%dd_tb" % wl.dim) if fused else ("k_mfma2d" if mode_name.startswith("mfma")
                                                      else "k_sweep%dd" % wl.dim)
    if mode_name == "separable" and wl.dim == 3:
        kname = "k_sweep3d_sep"
    roof["kernel"] = "%s R=%d (%s, %d taps, %.2f applications per launch)" % (
        kname,
        m * r, mode_name, taps, per_launch)
    roof["flops_basis"] = ("2 x FMAs per point (dense taps; 2 x rank x (2R+1) for the 2D separable "
                           "form, 3 x (2R+1) for the 3D one) x points x applications per launch")
    # speedups of the folded / matrix-core forms over the plain sweep
    plain_fused = forms.get("%s_m1_vector" % wl_name, {}).get("gstencil_s")
    plain_unfused = (forms.get("%s_m1_vector_unfused" % wl_name, {}).get("gstencil_s")
                     or plain_fused)
    speedups = {}
    for k, f in forms.items():
        if f["m"] > 1 or f["mode"] not in ("vector", "vector_unfused"):
            if plain_unfused:
                speedups[k] = {"vs_plain_one_step_launches": round(f["gstencil_s"] / plain_unfused, 3)}
                if plain_fused:
                    speedups[k]["vs_plain_fused"] = round(f["gstencil_s"] / plain_fused, 3)
    res = {
        "metric": METRIC,
        "value": round(gst, 2),
        "unit": "GStencil/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl.note, "grid": list(shape), "T": T, "fold_m": m,
                   "mode": mode_name, "points": n},
        "roofline": roof,
        "error_vs_oracle": {"e_rel": forms[key]["e_rel_vs_oracle"],
                            "e_detrended": forms[key]["e_detrended_vs_oracle"],
                            "equal_elements": forms[key]["equal_to_oracle"],
                            "gate": forms[key]["gate"], "reference": ref_kind},
        "forms": forms,
        "speedups": speedups,
    }
    del ref64
    if not args.no_cpu:
        log("[bench] timing the CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(w, shape, T, budget_s(args, default_run),
                                           "zero" if zero_bc else "periodic")
    return res


def bench_batched(args, default_run=False):
    """4096 independent periodic 2D grids, sides log-uniform in [64, 1024],
    each a 5-point star or 9-point box with random positive weights summing
    to 1, FP32, T = 50.  Forms: one persistent launch per (folded) sweep in a
    hipGraph with autotuned fold depth (the headline), the same with m = 1,
    and the per-grid baseline (one stencil_run per grid, 4096 x 50 kernel
    launches)."""
    import numpy as np
    import tempfile
    import torch
    import oracle
    import synth
    import paper_2103_09235_amd as sf

    count, T = 4096, 50
    sides, kinds, weights = synth.batched_recipe(count)
    npts = int(np.sum(sides.astype(np.int64) ** 2))
    log("[bench] batched: %d grids, %d points, T=%d; generating inputs" % (count, npts, T))
    dev = torch.device("cuda:0")
    flat = synth.uniform_f32(synth.SEED, synth.STREAM_GRID, npts)
    datas, u0s = [], []
    off = 0
    for s in sides:
        n = int(s) * int(s)
        u0s.append(flat[off:off + n].reshape(int(s), int(s)))
        off += n
    datas = [torch.from_numpy(u).to(dev) for u in u0s]
    scr = [torch.empty_like(d) for d in datas]
    plans = [sf.Plan(w, sf.STENCIL_STAR if k == synth.STAR else sf.STENCIL_BOX)
             for k, w in zip(kinds, weights)]
    handles = [p.handle for p in plans]
    cache = args.tune_cache or os.path.join(tempfile.mkdtemp(prefix="stencil_tune_"), "tune.txt")

    def reset():
        for d, u in zip(datas, u0s):
            d.copy_(torch.from_numpy(u).to(dev), non_blocking=True)

    forms = {}
    chosen = {}

    def run_form(name, fn, steps, warmup):
        reset()
        el, wall = time_runs(fn, steps, warmup)
        gst = npts * T * steps / el / 1e9
        forms[name] = {"gstencil_s": round(gst, 2), "ms_per_run": round(el / steps * 1e3, 3),
                       "wall_s": round(wall, 3)}
        log("[bench]   %s: %.1f GStencil/s, %.3f ms per T=%d run" % (name, gst, el / steps * 1e3, T))
        return el / steps

    # the call's arguments marshalled once (ctypes descriptors of 4096 grids);
    # every timed call still runs the whole C entry point
    batch = sf.BatchedRun(handles, datas, scr)
    log("[bench] persistent + graph, autotuned (fold depth up to 2, strip height, pass cap, "
        "layout, timed on the whole batch)")
    t0 = time.perf_counter()
    chosen["tuned"] = batch.run(T, autotune=True, tune_cache=cache, use_graph=True, max_m=2)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    log("[bench]   tuning and first run: %.1f s" % tune_s)
    t_tuned = run_form("persistent_graph_tuned", lambda: batch.run(
        T, tune_cache=cache, use_graph=True, max_m=2), args.steps, args.warmup)
    t_m1 = None
    if args.only_mode != "tuned":
        log("[bench] persistent + graph, default choices (m = 1, 64-row strips, widest layout)")
        t_m1 = run_form("persistent_graph_default", lambda: batch.run(
            T, use_graph=True, max_m=1), args.steps, args.warmup)
    stream = torch.cuda.current_stream(dev)

    def per_grid():
        for p, d, s in zip(plans, datas, scr):
            sf.stencil_run(p.handle, d, T, s, stream)
    t_pg = None
    if not args.no_per_grid and args.only_mode != "tuned":
        log("[bench] per-grid launches (4096 x stencil_run, m = 1)")
        t_pg = run_form("per_grid_launches_m1", per_grid, 1, 0)
    # correctness of the headline form: mass of every grid after one run
    reset()
    s0 = [sf.stencil_residual(d)[0] for d in datas[:64]]
    batch.run(T, tune_cache=cache, use_graph=True, max_m=2)
    drift = 0.0
    for i in range(64):
        w32 = weights[i].astype(np.float32).astype(np.float64)
        expect = math.fsum(float(v) for v in w32.ravel()) ** T * s0[i]
        drift = max(drift, abs(sf.stencil_residual(datas[i])[0] - expect) / abs(expect))
    # the same run against the FP64 oracle on every 64th grid
    err = {"e_rel_max": None, "grids_checked": 0}
    if not args.no_oracle:
        log("[bench] FP64 oracle on every 64th grid")
        worst = worst_d = 0.0
        checked = 0
        for i in range(0, count, 64):
            ref, kind = oracle_reference(weights[i], u0s[i], T)
            e = oracle.errors(datas[i].cpu().numpy(), ref)
            worst = max(worst, e["e_rel"])
            worst_d = max(worst_d, e["e_detr"])
            checked += 1
        err = {"e_rel_max": worst, "e_detrended_max": worst_d, "grids_checked": checked,
               "gate": 1e-5, "reference": kind}
    ms = chosen["tuned"]
    # The time loop is one graph of fused passes (several applications per
    # launch, grids of >= 256 columns), one-step launches and a copy back of
    # grids with an odd launch count, so its work is accounted over the whole
    # run: algorithmic bytes = every grid read and written once per launch
    # that passes over it (the library reports these per grid), algorithmic
    # flops = 2 x taps x points x applications (folded and plain).
    batch.run(T, tune_cache=cache, use_graph=True, max_m=2)
    passes = list(batch.passes)
    taps_of = {}  # (stencil kind, m) -> nonzero taps of the operator applied
    bytes_total = flops_total = 0
    for p, k, s, m, ps in zip(plans, kinds, sides, ms, passes):
        for mm in {1, m}:
            if (k, mm) not in taps_of:
                probe = sf.Plan(p.fold(1), sf.STENCIL_STAR if k == synth.STAR else sf.STENCIL_BOX)
                taps_of[(k, mm)] = int(np.count_nonzero(probe.fold(mm)))
                probe.close()
        n2 = int(s) * int(s)
        apps_f, apps_p = (T // m, T % m) if m > 1 else (0, T)
        flops_total += 2 * n2 * (apps_f * taps_of[(k, m)] + apps_p * taps_of[(k, 1)])
        bytes_total += 2 * 4 * n2 * ps
    run_s = t_tuned
    # the whole run as one launch unit (its fused, one-step and copy
    # launches together), priced against the published FP32 peak
    roof = roofline(bytes_total, flops_total, run_s, FP32_VECTOR_TFLOPS,
                    "FP32 vector, published", "alu")
    roof["fp32_fma_issue_frac"] = round(flops_total / run_s / 1e12 / FP32_FMA_TFLOPS, 4)
    roof["fp32_fma_issue_basis"] = ("256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = "
                                    "78.6 TFLOP/s (FMAs, packed FP32 not used)")
    roof["traffic"] = traffic_from_profiles("batched", "batched", "hbm-bytes-per-run")
    roof["traffic_unit"] = "HBM bytes per run (PMC FETCH_SIZE + WRITE_SIZE, calibrated)"
    roof["kernel"] = ("whole time loop: k_batched_tb fused passes + k_batched one-step "
                      "launches + copy back (one hipGraph)")
    roof["launch_unit"] = "one T-step run (all of its launches)"
    roof["passes_per_grid_mean"] = round(sum(passes) / len(passes), 3)
    # the tuned choices per (stencil, radius, size class), from the cache
    tuned = {}
    if os.path.exists(cache):
        for line in open(cache):
            f = line.split()
            if len(f) == 5 and f[0].startswith("stencil-batched-"):
                cls = "%s_r%s_class%s" % ("star" if f[1] == "0" else "box", f[2], f[3])
                tuned.setdefault(cls, {"m": 1, "rows": 64, "pass_cap": 0, "narrow": 0})
                fld = {"m": "m", "rows": "rows", "kc": "pass_cap", "narrow": "narrow"}[
                    f[0][len("stencil-batched-"):]]
                tuned[cls][fld] = int(f[4])
    res = {
        "metric": METRIC,
        "value": forms["persistent_graph_tuned"]["gstencil_s"],
        "unit": "GStencil/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": forms["persistent_graph_tuned"]["ms_per_run"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched: 4096 periodic 2D grids, sides log-uniform in [64, 1024], "
                               "5-point star or 9-point box (random positive weights), FP32, T=50",
                   "points": npts, "T": T,
                   "fold_m_histogram": {str(m): int(sum(1 for x in ms if x == m)) for m in sorted(set(ms))},
                   "tuned_per_class": tuned, "tuning_wall_s": round(tune_s, 1)},
        "roofline": roof,
        "forms": forms,
        "taps": {"%s_m%d" % ("star" if k == synth.STAR else "box", m): t
                 for (k, m), t in sorted(taps_of.items())},
        "speedup_vs_per_grid_launches": round(t_pg / t_tuned, 2) if t_pg else None,
        "speedup_tuned_vs_default": round(t_m1 / t_tuned, 3) if t_m1 else None,
        "mass_rel_drift_max_64_grids": drift,
        "error_vs_oracle": err,
    }
    for p in plans:
        p.close()
    if not args.no_cpu:
        log("[bench] timing the CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline_batched(weights, u0s, T, budget_s(args, default_run))
    return res


def cpu_baseline_batched(weights, grids, T, budget_s):
    """The oracle on the batch itself: grids in batch order, each advanced by
    all T steps, until about budget_s seconds have been spent."""
    import numpy as np
    import oracle
    oracle.sweep(weights[0], grids[0].astype(np.float64), 1)  # warm: threads
    pts = 0
    spent = 0.0
    k = 0
    while k < len(grids) and spent < budget_s:
        u0 = grids[k].astype(np.float64)
        t0 = time.perf_counter()
        oracle.sweep(weights[k], u0, T)
        spent += time.perf_counter() - t0
        pts += u0.size
        k += 1
    return {
        "value": round(pts * T / spent / 1e9, 4),
        "unit": "GStencil/s",
        "cores": oracle.num_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": "FP64 naive sweep of the batch's first %d grids (%d points, sides %d..%d), "
                  "all %d steps each, %.1f s" % (k, pts, min(g.shape[0] for g in grids[:k]),
                                                 max(g.shape[0] for g in grids[:k]), T, spent),
    }


def bench_apop(args):
    """Table 1's APOP: N = 10,240,000 option values (FP64), T = 1000 steps of
    u <- maxNum(A u, payoff) with a 3-point discounted stencil, several steps
    fused per launch.  Algorithmic bytes per launch: the values read and
    written once and the payoff read once (24 per point)."""
    import numpy as np
    import torch
    import synth
    import paper_2103_09235_amd as sf
    n, T, w = synth.APOP["n"], synth.APOP["T"], synth.APOP["weights"]
    payoff = synth.apop_payoff(n)
    dev = torch.device("cuda:0")
    fl = torch.from_numpy(payoff).to(dev)
    data = torch.from_numpy(payoff.copy()).to(dev)
    scratch = torch.empty_like(data)
    plan = sf.Plan(w, sf.STENCIL_STAR)
    plan.set_floor(fl)
    sched = plan.schedule(data, T, scratch)
    log("[bench] apop1d: N=%d FP64 T=%d, %s" % (n, T, sched))
    el, wall = time_runs(lambda: plan.run(data, T, scratch), args.steps, args.warmup)
    gst = n * T * args.steps / el / 1e9
    launches = sched["plain_launches"]
    launch_ms = el / args.steps / launches * 1e3
    algo = 24 * n
    # correctness of one run: sampled points against the oracle's FP64 loop on
    # each point's window (T*r on each side: a window edge perturbs points
    # within T*r of it only, so the centre is exact), bit for bit
    import oracle
    data.copy_(torch.from_numpy(payoff).to(dev))
    plan.run(data, T, scratch)
    u = data.cpu().numpy()
    plan.close()
    ok = True
    for x in (0, 1, 12345, n // 3, n // 2, n - 2, n - 1):
        idx = (x + np.arange(-T, T + 1)) % n
        ref = oracle.floor_sweep(w, payoff[idx], payoff[idx], T)[T]
        ok = ok and bool(u[x] == ref)
    # per step and point: 3 FMAs and a max (counted as 2 x 3 flops)
    flops = 2 * 3 * n * (T / launches)
    dur = launch_ms / 1e3
    if flops / algo < FP64_VECTOR_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        roof = {"bound": "hbm", "achieved": round(algo / dur / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": round(flops / dur / 1e12, 2),
                "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "peak_basis": "FP64 vector, published"}
    roof.update({"kernel": "k_sweep1d<double, 1, 16, floor> (%.1f steps per launch)" % (
                     T / launches),
                 "launch_ms": round(launch_ms, 5), "algorithmic_bytes_per_launch": algo,
                 "algorithmic_flops_per_launch": flops, "hbm_frac": round(
                     algo / dur / 1e9 / HBM_PEAK_GBS, 4), "traffic": None})
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    res = {"metric": METRIC, "value": round(gst, 2), "unit": "GStencil/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "APOP (Table 1): 1D 3-point discounted stencil floored by the "
                                  "put payoff, N=10,240,000 FP64, T=1000, plain (not foldable)",
                      "points": n, "T": T},
           "roofline": roof, "sampled_points_match_oracle": ok, "wall_s": round(wall, 3)}
    if not args.no_cpu:
        m = 1 << 20
        oracle.floor_sweep(w, payoff[:m], payoff[:m], 1)
        t0 = time.perf_counter()
        oracle.floor_sweep(w, payoff[:m], payoff[:m], 2)
        per = (time.perf_counter() - t0) / 2
        Ts = int(max(1, min(T, budget_s(args, False) / per)))
        t0 = time.perf_counter()
        oracle.floor_sweep(w, payoff[:m], payoff[:m], Ts)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(m * Ts / dt / 1e9, 4), "unit": "GStencil/s",
                               "cores": oracle.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
                               "sample": "FP64 floor sweep on the first %d points (periodic), "
                                         "%d of the %d steps, %.1f s" % (m, Ts, T, dt)}
    return res


def bench_life(args):
    """Table 1's Game of Life: 5000 x 5000 cells (uint8), T = 1000
    generations, one generation per launch; 2 algorithmic bytes per cell per
    generation (read and write once)."""
    import numpy as np
    import torch
    import synth
    import oracle
    import paper_2103_09235_amd as sf
    shape, T = synth.LIFE["shape"], synth.LIFE["T"]
    g0 = synth.life_cells(shape)
    dev = torch.device("cuda:0")
    cells = torch.from_numpy(g0).to(dev)
    scratch = torch.empty_like(cells)
    n = int(np.prod(shape))
    log("[bench] life2d: %s T=%d" % (shape, T))
    el, wall = time_runs(lambda: sf.stencil_life(cells, scratch, T), args.steps, args.warmup)
    gst = n * T * args.steps / el / 1e9
    launches = sf.stencil_life_launches(shape[0], shape[1], T)
    launch_ms = el / args.steps / launches * 1e3
    # correctness: 4 generations against the oracle
    cells.copy_(torch.from_numpy(g0).to(dev))
    sf.stencil_life(cells, scratch, 4)
    ok = bool(np.array_equal(cells.cpu().numpy(), oracle.life(g0, 4)))
    # Integer VALU work: the wavefront VALU instructions one launch issues
    # (rocprofv3 SQ_INSTS_VALU of the fused kernel, from the committed
    # counter summary while life.hip is unchanged), 64 lanes each, priced
    # against the 32-bit VALU issue rate; the issue includes the strips'
    # discarded border work.
    gens = T / launches
    dur = launch_ms / 1e3
    insts = traffic_from_profiles("life", "life2d", field="valu-insts-per-launch")
    achieved = round(insts * 64 / dur / 1e12, 2) if insts else None
    roof = {"bound": "alu", "achieved": achieved,
            "peak": VALU32_TOPS, "unit": "Tlane-op/s",
            "peak_basis": "32-bit VALU issue: 256 CUs x 64 lanes x 2.4 GHz",
            "achieved_basis": ("rocprofv3 SQ_INSTS_VALU per launch x 64 lanes / launch duration "
                               "(profiles/life_life2d_pmc.txt)"),
            "kernel": "k_life_tb (%.2f generations per launch)" % gens,
            "launch_ms": round(launch_ms, 5), "algorithmic_bytes_per_launch": 2 * n,
            "hbm_frac": round(2 * n / dur / 1e9 / HBM_PEAK_GBS, 4), "traffic": None}
    roof["frac"] = round(achieved / roof["peak"], 4) if achieved else None
    res = {"metric": METRIC, "value": round(gst, 2), "unit": "GStencil/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "Game of Life (Table 1), 5000x5000 uint8 cells, periodic, "
                                  "T=1000 generations, plain (not foldable)",
                      "points": n, "T": T},
           "roofline": roof, "matches_oracle_4_generations": ok, "wall_s": round(wall, 3)}
    if not args.no_cpu:
        sample = g0[:1000, :1000]
        oracle.life(sample, 1)
        t0 = time.perf_counter()
        oracle.life(sample, 2)
        per = (time.perf_counter() - t0) / 2
        Ts = int(max(1, min(T, budget_s(args, False) / per)))
        t0 = time.perf_counter()
        oracle.life(sample, Ts)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(sample.size * Ts / dt / 1e9, 4),
                               "unit": "GStencil/s", "cores": 1, "cpu_model": cpu_model(), "kind": "oracle",
                               "sample": "numpy Game of Life on a 1000x1000 corner, %d of the "
                                         "%d generations, %.1f s" % (Ts, T, dt)}
    return res



def config_entry(res: dict) -> dict:
    """The per-workload record of the default run: the workload's JSON line
    without the fields that only the top level carries."""
    drop = ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
            "data")
    return {k: v for k, v in res.items() if k not in drop}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(a grid would shard by slabs with one halo exchange per folded sweep; "
              "not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        n = 64 << 20
        x = torch.rand(n, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "copy calibration", "bytes_read_per_launch": 4 * n,
                          "bytes_written_per_launch": 4 * n, "launches": 4}), flush=True)
        return

    def one(name, default_run):
        if name == "batched":
            return bench_batched(args, default_run)
        if name == "apop1d":
            return bench_apop(args)
        if name == "life2d":
            return bench_life(args)
        return bench_grid(args, name, default_run)

    if args.workload != "all":
        print(json.dumps(one(args.workload, False)), flush=True)
        return
    t_start = time.perf_counter()
    results = {}
    for name in DEFAULT_SET:
        t0 = time.perf_counter()
        # the headline keeps the full CPU-oracle sample (about 10 s), the
        # other lines a shorter one so that the run stays within minutes
        results[name] = one(name, name != "star2d")
        torch.cuda.empty_cache()
        log("[bench] %s done: %.1f GStencil/s (%.0f s)" % (name, results[name]["value"],
                                                          time.perf_counter() - t0))
    res = dict(results["star2d"])
    res["configs"] = {name: config_entry(r) for name, r in results.items()}
    res["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
