"""Oracle functions (test infrastructure only; see the package docstring).

Every function states the passage of the paper it follows.  The arithmetic
of the sweep runs in ``stencil_oracle.c`` (plain loops, FP64, canonical FMA
order); the rest is plain numpy / Python on small arrays.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.oracle_sweep_f64.argtypes = [ctypes.c_int, i64p, ctypes.c_int, dp, dp,
                                     ctypes.c_int64, dp]
    lib.oracle_sweep_f64.restype = ctypes.c_int
    lib.oracle_sweep_f32.argtypes = [ctypes.c_int, i64p, ctypes.c_int, fp, fp,
                                     ctypes.c_int64, fp]
    lib.oracle_sweep_f32.restype = ctypes.c_int
    lib.oracle_sweep_bc_f64.argtypes = [ctypes.c_int, i64p, ctypes.c_int, dp, dp,
                                        ctypes.c_int64, ctypes.c_int, dp]
    lib.oracle_sweep_bc_f64.restype = ctypes.c_int
    lib.oracle_sweep_bc_f32.argtypes = [ctypes.c_int, i64p, ctypes.c_int, fp, fp,
                                        ctypes.c_int64, ctypes.c_int, fp]
    lib.oracle_sweep_bc_f32.restype = ctypes.c_int
    lib.oracle_sweep_gv_f64.argtypes = [ctypes.c_int, i64p, ctypes.c_int, dp, dp,
                                        ctypes.c_int64, ctypes.c_int, ctypes.c_double, dp]
    lib.oracle_sweep_gv_f64.restype = ctypes.c_int
    lib.oracle_sweep_gv_f32.argtypes = [ctypes.c_int, i64p, ctypes.c_int, fp, fp,
                                        ctypes.c_int64, ctypes.c_int, ctypes.c_float, fp]
    lib.oracle_sweep_gv_f32.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def available() -> bool:
    try:
        _load()
        return True
    except OSError:
        return False


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _radius_of(w: np.ndarray, dim: int) -> int:
    if w.ndim != dim:
        raise ValueError("weights must have the grid's dimension")
    side = w.shape[0]
    if any(s != side for s in w.shape) or side % 2 != 1:
        raise ValueError("weights must be a (2r+1)^dim array")
    return (side - 1) // 2


BOUNDARIES = {"periodic": 0, "zero": 1}


def sweep(w, u0, T: int, boundary: str = "periodic", ghost: float = 0.0) -> np.ndarray:
    """u_T = A^T u_0 in FP64 (paper, Section 1: the naive (d+1)-loop stencil,
    time outermost; canonical FMA order).  boundary "periodic" wraps every
    axis; "zero" holds every point outside the grid at the value ghost, 0 by
    default (Dirichlet ghosts; the paper states no boundary, so both are
    readings)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    dim = u0.ndim
    r = _radius_of(w, dim)
    shape = (ctypes.c_int64 * dim)(*u0.shape)
    out = np.empty_like(u0)
    rc = _load().oracle_sweep_gv_f64(
        dim, shape, r, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        u0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(T), BOUNDARIES[boundary],
        float(ghost), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_sweep_gv_f64 rejected its arguments")
    return out


def sweep_f32(w32, u0, T: int, boundary: str = "periodic", ghost: float = 0.0) -> np.ndarray:
    """The same loop and operation order in FP32 (fmaf; the ghost value
    rounded to FP32): the bit-exact reference for kernels that keep the
    canonical order."""
    u0 = np.ascontiguousarray(u0, dtype=np.float32)
    w32 = np.ascontiguousarray(w32, dtype=np.float32)
    dim = u0.ndim
    r = _radius_of(w32, dim)
    shape = (ctypes.c_int64 * dim)(*u0.shape)
    out = np.empty_like(u0)
    rc = _load().oracle_sweep_gv_f32(
        dim, shape, r, w32.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
        u0.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(T), BOUNDARIES[boundary],
        float(np.float32(ghost)), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if rc != 0:
        raise ValueError("oracle_sweep_gv_f32 rejected its arguments")
    return out


def sweep_window(w, u0, T: int, points, f32: bool = False) -> np.ndarray:
    """Selected outputs of ``sweep`` (or ``sweep_f32``) computed one by one.

    After T steps a point depends only on the inputs within T*r of it along
    every axis (the dependency cone of the naive loop).  Each sample runs the
    same loop on the (2Tr+1)-wide periodic window around it (the whole axis
    where the window would cover it), which yields bit-for-bit the value the
    full-grid loop gives, because every value in the cone is formed by the
    same taps in the same order.
    """
    u0 = np.asarray(u0)
    w = np.asarray(w)
    dim = u0.ndim
    r = _radius_of(w, dim)
    reach = int(T) * r
    vals = []
    for p in points:
        idx = []
        centre = []
        for a in range(dim):
            n = u0.shape[a]
            if 2 * reach + 1 >= n:
                idx.append(np.arange(n))
                centre.append(int(p[a]) % n)
            else:
                idx.append((int(p[a]) + np.arange(-reach, reach + 1)) % n)
                centre.append(reach)
        win = u0[np.ix_(*idx)]
        res = sweep_f32(w, win, T) if f32 else sweep(w, win, T)
        vals.append(res[tuple(centre)])
    return np.array(vals, dtype=np.float32 if f32 else np.float64)


def _cpow(z: np.ndarray, T: int) -> np.ndarray:
    """z**T for an integer T >= 0 by binary exponentiation (about 2 log2 T
    complex products, each rounded once per component)."""
    out = np.ones_like(z)
    base = z.copy()
    e = int(T)
    while e:
        if e & 1:
            out *= base
        e >>= 1
        if e:
            base *= base
    return out


def sweep_spectral(w, u0, T: int, boundary: str = "periodic", workers: int | None = None) -> np.ndarray:
    """u_T = A^T u_0 in FP64 through the eigen-decomposition of A, for grids
    too large for the naive loop (Section 1's sweep; the same operator as
    ``sweep``, evaluated in another order).

    periodic: A is circulant (correlation with w, every axis wrapped), so the
    discrete Fourier transform diagonalises it: with
    u_hat(k) = sum_x u[x] e^{-2 pi i k.x/n}, (A u)_hat(k) = lambda(k) u_hat(k)
    where lambda(k) = sum_o w[o] e^{+2 pi i k.o/n}; hence
    u_T = IDFT(DFT(u_0) lambda^T).  Offsets that alias on short axes add up,
    as in the circulant matrix.

    zero (Dirichlet ghosts 0; radius 1, weights unchanged by reversing any
    axis): A is a sum of Kronecker products of I and the truncated
    nearest-neighbour operator J (ones next to the diagonal), both diagonalised
    by the type-I discrete sine transform, J having the eigenvalues
    2 cos(pi j/(n+1)), j = 1..n; so lambda(j) = sum_o w[o] prod_a c(o_a, j_a)
    with c(0, j) = 1 and c(+-1, j) = cos(pi j/(n+1)) (each of the two
    mirrored taps takes one half of J's eigenvalue).

    Rounding: one forward and one inverse transform (error of order
    eps log2 N relative to ||u_0||) and lambda^T by binary powering
    (about 2 log2 T roundings); far below the FP32 and BF16 tolerances it
    is used for, but not bit-exact (the naive loop is the bit-exact one)."""
    import scipy.fft as sfft
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    dim = u0.ndim
    r = _radius_of(w, dim)
    if T < 0:
        raise ValueError("T >= 0")
    workers = workers or os.cpu_count() or 1
    shape = u0.shape
    if boundary == "periodic":
        # per axis: phases e^{2 pi i k o / n} for o in [-r, r] over the axis's
        # transform frequencies (the last axis: the n//2+1 of the real DFT),
        # angle from (k*o mod n) so each is rounded once
        phases = []
        for a, n in enumerate(shape):
            k = np.arange(n // 2 + 1 if a == dim - 1 else n, dtype=np.int64)
            rows = []
            for o in range(-r, r + 1):
                rows.append(np.exp(2j * np.pi * ((k * o) % n) / n))
            phases.append(rows)
        lam = None
        for idx in np.ndindex(*w.shape):
            wo = w[idx]
            if wo == 0.0:
                continue
            term = None
            for a in range(dim):
                v = phases[a][idx[a]]
                sh = [1] * dim
                sh[a] = v.size
                v = v.reshape(sh)
                term = v if term is None else term * v
            term = wo * term
            lam = term if lam is None else lam + term
        if lam is None:
            return np.zeros_like(u0) if T > 0 else u0.copy()
        lam = np.broadcast_to(lam, tuple(shape[:-1]) + (shape[-1] // 2 + 1,))
        uh = sfft.rfftn(u0, workers=workers)
        uh *= _cpow(np.ascontiguousarray(lam), T)
        return sfft.irfftn(uh, s=shape, workers=workers)
    if boundary == "zero":
        if r != 1:
            raise ValueError("the sine-transform form needs radius 1")
        for a in range(dim):
            if not np.array_equal(w, np.flip(w, axis=a)):
                raise ValueError("the sine-transform form needs weights symmetric in every axis")
        lam = np.zeros((1,) * dim)
        for idx in np.ndindex(*w.shape):
            wo = w[idx]
            if wo == 0.0:
                continue
            term = np.ones((1,) * dim)
            for a, n in enumerate(shape):
                sh = [1] * dim
                sh[a] = n
                if idx[a] != 1:
                    c = np.cos(np.pi * np.arange(1, n + 1) / (n + 1)).reshape(sh)
                    term = term * c
            lam = lam + wo * term
        lam = np.broadcast_to(lam, shape)
        uh = sfft.dstn(u0, type=1, norm="ortho", workers=workers)
        uh *= _rpow(np.ascontiguousarray(lam), T)
        return sfft.dstn(uh, type=1, norm="ortho", workers=workers)
    raise ValueError("boundary must be periodic or zero")


def _rpow(x: np.ndarray, T: int) -> np.ndarray:
    """x**T (real) by binary exponentiation."""
    out = np.ones_like(x)
    base = x.copy()
    e = int(T)
    while e:
        if e & 1:
            out *= base
        e >>= 1
        if e:
            base *= base
    return out


def fold_weights(w, m: int) -> np.ndarray:
    """Folded weights W_m of m steps (Section 3.1 and Section 3.3: the m-step
    expansion with merged terms and reassigned weights, the "folding matrix";
    Eq. 4-6 give the 2D 9-point, m = 2 instance).

    Obtained as the impulse response of m plain steps, independent of any
    convolution routine: on a periodic grid of side L = 2mr+1 per axis (wide
    enough that nothing aliases) start from a unit impulse at index 0, run m
    oracle steps, and read W_m[o] = u_m[(-o) mod L], because
    (A^m delta_0)[x] = sum_o W_m[o] delta_0[x + o] = W_m[-x].
    """
    w = np.asarray(w, dtype=np.float64)
    dim = w.ndim
    r = _radius_of(w, dim)
    if m < 1:
        raise ValueError("m >= 1")
    R = m * r
    L = 2 * R + 1
    u0 = np.zeros((L,) * dim, dtype=np.float64)
    u0[(0,) * dim] = 1.0
    um = sweep(w, u0, m)
    sel = (-(np.arange(L) - R)) % L
    return um[np.ix_(*([sel] * dim))].copy()


def fold_weights_f32(w, m: int) -> np.ndarray:
    """FP32 folded weights as the FP32 kernels hold them.

    Reading (the paper works in double and never rounds weights): each FP64
    W_m[o] is rounded to nearest-even FP32.  For m >= 2 the centre weight is
    then replaced by fl32(S - sum_{o != 0} fl32(W_m[o])), where S is (sum w)^m
    (the sum taken sequentially in row-major order, the power by repeated
    multiplication, all in FP64) and the inner sum is sequential in row-major
    order over the widened FP32 weights; this keeps the FP32 operator's total
    weight at the folded operator's, so the mean mode does not drift over
    many folded sweeps.  A centre that rounds to zero is left alone.  m = 1
    returns fl32(w) unchanged.
    """
    w = np.asarray(w, dtype=np.float64)
    Wm = fold_weights(w, m)
    W32 = Wm.astype(np.float32)
    if m == 1:
        return W32
    s1 = 0.0
    for v in w.ravel():
        s1 += float(v)
    target = 1.0
    for _ in range(m):
        target *= s1
    centre = tuple([(W32.shape[0] - 1) // 2] * W32.ndim)
    if W32[centre] == 0.0:
        return W32
    flat = W32.ravel()
    cidx = int(np.ravel_multi_index(centre, W32.shape))
    rest = 0.0
    for k in range(flat.size):
        if k != cidx:
            rest += float(flat[k])
    W32[centre] = np.float32(target - rest)
    return W32


def bf16_rne(x32) -> np.ndarray:
    """Round FP32 to bfloat16 (nearest, ties to even), returned as the FP32
    values it represents.  Reading for the split-precision contraction form,
    which the paper does not have: hi = bf16(x), lo = bf16(x - hi)."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    out = (rounded << np.uint64(16)).astype(np.uint32).view(np.float32)
    return out.reshape(np.shape(x32))


def bf16_split(x32):
    """(hi, lo) with hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32."""
    x32 = np.asarray(x32, dtype=np.float32)
    hi = bf16_rne(x32)
    lo = bf16_rne((x32 - hi).astype(np.float32))
    return hi, lo


def schedule(T: int, m: int):
    """Reading for T not divisible by m (the paper only runs m = 2 with even
    T): floor(T/m) folded sweeps first, then T mod m plain sweeps."""
    if m < 1 or T < 0:
        raise ValueError("m >= 1 and T >= 0")
    return T // m, T % m


def folded_reference_f32(w, u0, T: int, m: int) -> np.ndarray:
    """FP32 mirror of a folded run: the folded sweeps with the FP32 folded
    weights, then the plain remainder with fl32(w), canonical order."""
    q, s = schedule(T, m)
    u = np.asarray(u0, dtype=np.float32)
    if q:
        u = sweep_f32(fold_weights_f32(w, m), u, q)
    if s:
        u = sweep_f32(np.asarray(w, dtype=np.float64).astype(np.float32), u, s)
    return u


def band_mask(shape, width: int) -> np.ndarray:
    """Points closer than `width` to a face: min(i, n-1-i) < width along some
    axis."""
    mask = np.zeros(shape, dtype=bool)
    for a, n in enumerate(shape):
        i = np.arange(n)
        near = np.minimum(i, n - 1 - i) < width
        sh = [1] * len(shape)
        sh[a] = n
        mask |= near.reshape(sh)
    return mask


def dirichlet_folded(w, u0, T: int, m: int, f32: bool = False, ghost: float = 0.0) -> np.ndarray:
    """Folding with Dirichlet ghosts of value ghost, 0 by default (a reading:
    the paper states no boundary).  Each of the floor(T/m) folded
    applications (Section 3.3) uses W_m (its taps outside the grid reading
    the ghost value) at points at least (m-1)r from every face, where no
    intermediate point of the m plain steps it replaces lies outside the grid
    (the j-th intermediate point of a path lies within j*r of the output; only
    the final reads of the initial state reach the ghosts, which hold the
    same value at every step), and takes m plain steps of w in the band closer
    than (m-1)r; the T mod m remaining steps are plain.  In exact arithmetic
    this is sweep(w, u0, T, "zero", ghost).  f32: the FP32 mirror (FP32
    folded weights and ghost, canonical order), the bit-exact reference of the
    library's canonical-order kernels."""
    q, s = schedule(T, m)
    w = np.asarray(w, dtype=np.float64)
    r = (w.shape[0] - 1) // 2
    if f32:
        u = np.asarray(u0, dtype=np.float32)
        Wm, w1, run = fold_weights_f32(w, m), w.astype(np.float32), sweep_f32
    else:
        u = np.asarray(u0, dtype=np.float64)
        Wm, w1, run = fold_weights(w, m), w, sweep
    band = band_mask(u.shape, (m - 1) * r)
    for _ in range(q):
        u = np.where(band, run(w1, u, m, "zero", ghost), run(Wm, u, 1, "zero", ghost))
    if s:
        u = run(w1, u, s, "zero", ghost)
    return u


def floor_sweep(w, u0, floor, T: int, f32: bool = False) -> np.ndarray:
    """T steps of u <- max(A u, floor) (IEEE maxNum, elementwise): the
    American put option pricing benchmark of Table 1 (APOP: a 1D 3-point
    stencil over two arrays, the option value and its exercise payoff, whose
    update keeps the larger).  Periodic, like the plain sweep.  The max
    makes the update nonlinear, so it is never folded.  f32: the same steps
    in FP32 (sweep_f32, then fmax), the bit-exact reference."""
    if f32:
        u = np.asarray(u0, dtype=np.float32)
        fl = np.asarray(floor, dtype=np.float32)
        w1 = np.asarray(w, dtype=np.float64).astype(np.float32)
        step = sweep_f32
    else:
        u = np.asarray(u0, dtype=np.float64)
        fl = np.asarray(floor, dtype=np.float64)
        w1 = np.asarray(w, dtype=np.float64)
        step = sweep
    for _ in range(T):
        u = np.fmax(step(w1, u, 1), fl)
    return u


def life(cells, T: int) -> np.ndarray:
    """T generations of Conway's Game of Life (Table 1: each cell's update
    depends on its 8 neighbours) on a periodic grid of 0/1 cells: a cell is
    alive next iff it has exactly 3 live neighbours, or 2 and is alive."""
    c = np.asarray(cells, dtype=np.uint8)
    for _ in range(T):
        n = np.zeros(c.shape, dtype=np.int32)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dy or dx:
                    n += np.roll(c, (dy, dx), axis=(0, 1))
        c = ((n == 3) | ((c == 1) & (n == 2))).astype(np.uint8)
    return c


def exact_sum(u) -> float:
    """Correctly rounded sum of all values (math.fsum)."""
    return math.fsum(np.asarray(u, dtype=np.float64).ravel().tolist())


def errors(u, ref) -> dict:
    """Error of a result against the oracle, in FP64:
    e_rel  = ||u - ref||_inf / ||ref||_inf (the gate),
    e_detr = ||u - ref||_inf / ||ref - mean(ref)||_inf,
    max_abs, and the count of bitwise-equal elements (same dtype only:
    identical bit patterns, so -0.0 differs from +0.0; 0 when the dtypes
    differ).  A NaN anywhere in u - ref makes every norm NaN, which fails
    any "< gate" comparison.  A zero reference norm leaves the absolute
    error in place of the relative one."""
    u = np.asarray(u)
    ref = np.asarray(ref)
    if u.shape != ref.shape:
        raise ValueError("errors: shapes differ")
    d = np.abs(u.astype(np.float64) - ref.astype(np.float64))
    max_abs = float(d.max()) if d.size else 0.0
    nref = float(np.abs(ref.astype(np.float64)).max()) if d.size else 0.0
    mean = exact_sum(ref) / ref.size if ref.size else 0.0
    ndet = float(np.abs(ref.astype(np.float64) - mean).max()) if d.size else 0.0
    if u.dtype == ref.dtype and u.dtype.kind == "f":
        ui = np.ascontiguousarray(u).view(np.dtype("u%d" % u.dtype.itemsize))
        ri = np.ascontiguousarray(ref).view(np.dtype("u%d" % ref.dtype.itemsize))
        same = int(np.count_nonzero(ui == ri))
    elif u.dtype == ref.dtype:
        same = int(np.count_nonzero(u == ref))
    else:
        same = 0
    return {
        "e_rel": max_abs / nref if nref > 0 else max_abs,
        "e_detr": max_abs / ndet if ndet > 0 else max_abs,
        "max_abs": max_abs,
        "bit_equal": same,
        "n": int(u.size),
    }


def _support(w) -> set:
    w = np.asarray(w)
    r = (w.shape[0] - 1) // 2
    return {tuple(int(i) - r for i in idx) for idx in zip(*np.nonzero(w))}


def _minkowski(a: set, b: set) -> set:
    return {tuple(x + y for x, y in zip(p, q)) for p in a for q in b}


def collect_counts(w, m: int):
    """Scalar profitability analysis (Section 3.2, Eq. 1-3) by enumeration.

    Naive m-step expression: every distinct point needed at each intermediate
    level j = 0..m-1 (S^(+j), the j-fold sum set of the stencil's support S,
    with S^(+0) = {0}) is one |S|-way weighted sum, so |C(E)| = |S| * sum_j
    |S^(+j)|.  Folded expression: one term per point of S^(+m), so
    |C(E_Lambda)| = |S^(+m)|.  Returns (|C(E)|, |C(E_Lambda)|, ratio)."""
    S = _support(w)
    dim = np.asarray(w).ndim
    level = {(0,) * dim}
    naive = 0
    for _ in range(m):
        naive += len(S) * len(level)
        level = _minkowski(level, S)
    folded = len(level)
    return naive, folded, naive / folded
