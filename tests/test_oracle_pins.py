"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: the references are exact
rational brute force (a dense circulant operator, applied with Python
integers / fractions), closed forms (Fourier modes, the FFT diagonalisation,
binomial coefficients), invariants (constant fields, mass, the maximum
principle, translation equivariance) and the values printed in the paper's
worked example (tests/golden/paper_box9_m2.txt).
"""

import itertools
import zlib
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_box9_m2.txt")
EPS64 = 2.0 ** -53


def read_golden(path=GOLDEN):
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = [float(t) for t in v.split()]
    return out


def brute_force(w, u0, T):
    """A^T u0 with A the dense circulant correlation operator built as a
    sparse matrix (aliased offsets summed into one entry), exact arithmetic
    on Python ints / Fractions."""
    shape = u0.shape
    dim = len(shape)
    r = (w.shape[0] - 1) // 2
    rows = []
    for x in itertools.product(*[range(n) for n in shape]):
        row = {}
        for o in itertools.product(range(-r, r + 1), repeat=dim):
            wo = w[tuple(oi + r for oi in o)]
            if wo == 0:
                continue
            col = tuple((xi + oi) % ni for xi, oi, ni in zip(x, o, shape))
            c = int(np.ravel_multi_index(col, shape))
            row[c] = row.get(c, 0) + wo
        rows.append(row)
    vec = list(u0.ravel())
    for _ in range(T):
        vec = [sum(wv * vec[c] for c, wv in row.items()) for row in rows]
    return np.array(vec, dtype=object).reshape(shape)


def exact(a):
    return np.vectorize(lambda v: Fraction(float(v)), otypes=[object])(np.asarray(a))


def rng(seed):
    return np.random.default_rng(seed)


SMALL_SHAPES = [
    (1,), (2,), (3,), (5,), (7,), (12,),
    (1, 1), (2, 3), (3, 3), (5, 2), (8, 9),
    (1, 1, 1), (2, 3, 3), (4, 5, 6),
]


@pytest.mark.parametrize("shape", SMALL_SHAPES)
@pytest.mark.parametrize("r", [1, 2])
def test_brute_force_integer_bit_exact(shape, r):
    dim = len(shape)
    if dim == 3 and r == 2 and np.prod(shape) > 60:
        pytest.skip("kept small")
    g = rng(hash((shape, r)) % 2**32)
    w = g.integers(-3, 4, size=(2 * r + 1,) * dim).astype(np.int64)
    w[(r,) * dim] = 2
    u0 = g.integers(0, 16, size=shape).astype(np.int64)
    T = 3
    ref = brute_force(w.astype(object), u0.astype(object), T)
    got = oracle.sweep(w.astype(np.float64), u0.astype(np.float64), T)
    assert np.all(np.abs(ref.astype(np.float64)) < 2 ** 53)
    assert np.array_equal(got, ref.astype(np.float64))


@pytest.mark.parametrize("shape", [(7,), (3, 5), (8, 9), (3, 4, 5)])
def test_brute_force_float_within_bound(shape):
    dim = len(shape)
    g = rng(7 + len(shape))
    w = g.random((3,) * dim)
    w /= w.sum()
    u0 = g.random(shape)
    T = 4
    ref = brute_force(exact(w), exact(u0), T)
    got = oracle.sweep(w, u0, T)
    taps = w.size
    bound = 4 * T * taps * EPS64 * float(np.abs(w).sum()) ** T * float(np.abs(u0).max())
    err = max(abs(Fraction(float(a)) - b) for a, b in zip(got.ravel(), ref.ravel()))
    assert float(err) <= bound


def test_brute_force_decimal_weights_rationals():
    # the 2D heat stencil with exact decimal weights 3/5 and 1/10
    w = np.zeros((3, 3), dtype=object)
    w[1, 1] = Fraction(3, 5)
    w[0, 1] = w[2, 1] = w[1, 0] = w[1, 2] = Fraction(1, 10)
    u0 = rng(3).integers(0, 100, size=(6, 7))
    T = 5
    ref = brute_force(w, u0.astype(object), T)
    got = oracle.sweep(synth.star2d_weights(0.6, 0.1), u0.astype(np.float64), T)
    err = max(abs(Fraction(float(a)) - b) for a, b in zip(got.ravel(), ref.ravel()))
    assert float(err) <= 8 * T * 5 * EPS64 * 100


def fourier_closed_form(w, shape, k, T):
    dim = len(shape)
    r = (w.shape[0] - 1) // 2
    lam = 0j
    for o in itertools.product(range(-r, r + 1), repeat=dim):
        wo = w[tuple(oi + r for oi in o)]
        lam += wo * np.exp(2j * np.pi * sum(ki * oi / ni for ki, oi, ni in zip(k, o, shape)))
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = 2 * np.pi * sum(ki * gi / ni for ki, gi, ni in zip(k, grids, shape))
    u0 = np.cos(phase)
    uT = np.real(lam ** T * np.exp(1j * phase))
    return u0, uT, lam


@pytest.mark.parametrize("case", ["heat1d", "star2d", "star3d", "box2d_random"])
def test_fourier_mode_decay(case):
    if case == "heat1d":
        w, shape, k = synth.heat1d_weights(), (96,), (5,)
    elif case == "star2d":
        w, shape, k = synth.star2d_weights(0.6, 0.1), (48, 40), (3, 7)
    elif case == "star3d":
        w, shape, k = synth.star3d_weights(0.4, 0.1), (12, 10, 8), (1, 2, 3)
    else:
        w, shape, k = synth.random_positive_weights(2, 1), (30, 26), (4, 3)
    T = 40
    u0, uT, lam = fourier_closed_form(w, shape, k, T)
    if case == "heat1d":
        assert abs(lam - math.cos(math.pi * k[0] / shape[0]) ** 2) < 1e-15
    got = oracle.sweep(w, u0, T)
    assert np.max(np.abs(got - uT)) < 1e-12


def test_fft_closed_form_random_input():
    shape = (32, 40)
    w = synth.random_positive_weights(2, 1)
    u0 = synth.grid_f64(shape)
    T = 25
    K = np.zeros(shape)
    for oy in range(-1, 2):
        for ox in range(-1, 2):
            K[(-oy) % shape[0], (-ox) % shape[1]] += w[oy + 1, ox + 1]
    lam = np.fft.fft2(K)
    ref = np.real(np.fft.ifft2(np.fft.fft2(u0) * lam ** T))
    got = oracle.sweep(w, u0, T)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_constant_field_dyadic_bit_exact(dim):
    if dim == 1:
        w, shape, c = synth.heat1d_weights(), (33,), 0.75
    elif dim == 2:
        w, shape, c = synth.star2d_weights(0.5, 0.125), (9, 11), 0.375
    else:
        w, shape, c = synth.star3d_weights(0.25, 0.125), (5, 4, 6), 0.625
    got = oracle.sweep(w, np.full(shape, c), 60)
    assert np.all(got == c)


def test_constant_field_decimal_weights_bound():
    T = 200
    got = oracle.sweep(synth.star2d_weights(0.6, 0.1), np.full((8, 8), 0.5), T)
    assert np.max(np.abs(got - 0.5)) <= T * 5 * 2 * EPS64 * 0.5 * 2


@pytest.mark.parametrize("name", ["heat1d", "star2d", "box2d", "star3d", "box3d"])
def test_mass_and_maximum_principle(name):
    wl = synth.WORKLOADS[name]
    shape = {1: (257,), 2: (37, 41), 3: (9, 10, 11)}[wl.dim]
    u0 = synth.grid_f64(shape)
    T = 30
    got = oracle.sweep(wl.weights, u0, T)
    sw = oracle.exact_sum(wl.weights)
    expect = sw ** T * oracle.exact_sum(u0)
    assert abs(oracle.exact_sum(got) - expect) <= 4 * T * wl.weights.size * EPS64 * oracle.exact_sum(np.abs(u0))
    slack = 1e-12
    assert got.min() >= u0.min() - slack and got.max() <= u0.max() + slack


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_translation_equivariance_bitwise(dim):
    shape = {1: (50,), 2: (17, 23), 3: (7, 8, 9)}[dim]
    w = synth.random_positive_weights(dim, 1)
    u0 = synth.grid_f64(shape)
    shift = {1: (5,), 2: (3, -4), 3: (1, 2, -3)}[dim]
    axes = tuple(range(dim))
    a = oracle.sweep(w, np.roll(u0, shift, axes), 9)
    b = np.roll(oracle.sweep(w, u0, 9), shift, axes)
    assert np.array_equal(a, b)


# ----------------------------------------------------------------- fold pins

def test_paper_worked_fold_example():
    g = read_golden()
    W2 = oracle.fold_weights(np.ones((3, 3)), 2)
    lam = {1: np.array(g["lambda1"]), 2: np.array(g["lambda2"]), 3: np.array(g["lambda3"])}
    assert np.array_equal(lam[2], 2 * lam[1]) and np.array_equal(lam[3], 3 * lam[1])
    # column at horizontal offset t carries counterpart c - |t| (Eq. 5)
    for j, n in enumerate(g["column_counterpart"]):
        assert np.array_equal(W2[:, j], lam[int(n)])
    assert np.array_equal(W2, np.outer(lam[1], lam[1]))
    # counterpart count: distinct column vectors up to symmetry <= m + 1
    distinct = {tuple(W2[:, j]) for j in range(W2.shape[1])}
    assert len(distinct) <= int(g["max_counterparts"][0])
    # counterpart reuse weights (Section 3.5): c2 = 2 c1, c3 = 0 c2 + 3 c1
    c1, c2, c3 = W2[:, 0], W2[:, 1], W2[:, 2]
    o2 = g["omega2"]
    o3 = g["omega3"]
    assert np.array_equal(c2, o2[0] * c1)
    assert np.array_equal(c3, o3[0] * c2 + o3[1] * c1)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 8])
def test_folded_operator_ranks(m):
    """The separable structure the separable mode relies on, checked on the
    oracle's folds: the unit box folds to the outer product of the 1D folds
    (rank one; its m = 2 instance is the paper's vertical then horizontal
    folding, Eq. 4-6), a product stencil a b^T to (a^{*m})(b^{*m})^T, and the
    5-point star, delta x h + v x delta with h, v 1D, to rank m + 1
    (W_m = sum_k C(m,k) (v^{*k}) x (h^{*(m-k)}) with independent terms)."""
    one = np.ones(3)
    Wu = oracle.fold_weights(np.ones((3, 3)), m)
    u1 = oracle.fold_weights(one, m)
    assert np.array_equal(Wu, np.outer(u1, u1))
    a, b = np.array([1.0, 2.0, 1.0]), np.array([3.0, 1.0, 2.0])
    Wp = oracle.fold_weights(np.outer(a, b), m)
    assert np.array_equal(Wp, np.outer(oracle.fold_weights(a, m), oracle.fold_weights(b, m)))
    star = np.array([[0.0, 1, 0], [2, 3, 5], [0, 7, 0]])
    Ws = oracle.fold_weights(star, m)
    assert np.linalg.matrix_rank(Ws) == m + 1
    assert np.linalg.matrix_rank(Wu) == 1


def test_paper_profitability_counts():
    g = read_golden()
    naive, folded, ratio = oracle.collect_counts(np.ones((3, 3)), 2)
    assert naive == g["collect_naive"][0]
    assert folded == g["collect_folded"][0]
    assert abs(ratio - g["profitable_index"][0]) < 1e-12


@pytest.mark.parametrize("m", range(1, 11))
def test_binomial_closed_form_heat1d(m):
    W = oracle.fold_weights(synth.heat1d_weights(), m)
    ref = np.array([math.comb(2 * m, m + j) / 4.0 ** m for j in range(-m, m + 1)])
    assert np.array_equal(W, ref)


@pytest.mark.parametrize("dim,m", [(1, 3), (2, 2), (2, 4), (3, 2)])
def test_dft_identity(dim, m):
    w = synth.random_positive_weights(dim, 1, offset=17)
    Wm = oracle.fold_weights(w, m)
    n = 2 * m + 5

    def dft(arr, r):
        K = np.zeros((n,) * dim)
        for o in itertools.product(range(-r, r + 1), repeat=dim):
            K[tuple((-oi) % n for oi in o)] += arr[tuple(oi + r for oi in o)]
        return np.fft.fftn(K)

    assert np.max(np.abs(dft(Wm, m) - dft(w, 1) ** m)) < 1e-13


@pytest.mark.parametrize("name,m,count", [
    ("star2d", 2, 13), ("star2d", 4, 41), ("star3d", 2, 25),
    ("box3d", 2, 125), ("box2d", 4, 81), ("box2d", 8, 289)])
def test_support_counts_and_mass(name, m, count):
    w = synth.WORKLOADS[name].weights
    Wm = oracle.fold_weights(w, m)
    assert int(np.count_nonzero(Wm)) == count
    assert abs(oracle.exact_sum(Wm) - oracle.exact_sum(w) ** m) < 1e-14


def conv_full(a, b):
    out = np.zeros(tuple(x + y - 1 for x, y in zip(a.shape, b.shape)), dtype=a.dtype)
    for ia in itertools.product(*[range(n) for n in a.shape]):
        if a[ia] == 0:
            continue
        sl = tuple(slice(i, i + n) for i, n in zip(ia, b.shape))
        out[sl] += a[ia] * b
    return out


@pytest.mark.parametrize("a,b", [(1, 1), (1, 2), (2, 3)])
def test_semigroup_integer_weights(a, b):
    w = np.array([[1, 2, 0], [3, 5, 1], [0, 1, 2]], dtype=np.float64)
    lhs = conv_full(oracle.fold_weights(w, a), oracle.fold_weights(w, b))
    assert np.array_equal(lhs, oracle.fold_weights(w, a + b))


def test_fold_m1_is_identity():
    w = synth.random_positive_weights(3, 1)
    assert np.array_equal(oracle.fold_weights(w, 1), w)


def test_fold_identity_integer_exact():
    w = np.ones((3, 3))
    u0 = rng(11).integers(0, 16, size=(10, 12)).astype(np.float64)
    for m, T in [(2, 4), (4, 4), (3, 6)]:
        a = oracle.sweep(w, u0, T)
        b = oracle.sweep(oracle.fold_weights(w, m), u0, T // m)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,m", [("star2d", 4), ("box3d", 2), ("heat1d", 5)])
def test_fold_identity_float_bound(name, m):
    wl = synth.WORKLOADS[name]
    shape = {1: (101,), 2: (30, 33), 3: (8, 9, 10)}[wl.dim]
    u0 = synth.grid_f64(shape)
    T = 4 * m
    a = oracle.sweep(wl.weights, u0, T)
    b = oracle.sweep(oracle.fold_weights(wl.weights, m), u0, T // m)
    assert np.max(np.abs(a - b)) < 64 * T * EPS64 * 9 ** wl.dim


# ------------------------------------------------------ precision readings

@pytest.mark.parametrize("name,m", [("star2d", 1), ("star2d", 2), ("star2d", 4),
                                    ("box2d", 8), ("box3d", 2), ("star3d", 2)])
def test_fold_weights_f32_rounding(name, m):
    w = synth.WORKLOADS[name].weights
    Wm = oracle.fold_weights(w, m)
    W32 = oracle.fold_weights_f32(w, m)
    c = tuple([m] * w.ndim)
    other = np.ones(Wm.shape, bool)
    other[c] = False
    assert np.array_equal(W32[other], Wm[other].astype(np.float32))
    if m == 1:
        assert np.array_equal(W32, w.astype(np.float32))
    else:
        target = oracle.exact_sum(w) ** m
        s = oracle.exact_sum(W32.astype(np.float64))
        ulp = np.spacing(np.float32(W32[c]))
        assert abs(s - target) <= 0.5 * float(ulp) + 1e-15


def frac_round_sig(x: float, bits: int) -> float:
    """Round a float to ``bits`` significant bits, ties to even, with exact
    rationals (independent of bit manipulation)."""
    if x == 0:
        return 0.0
    f = Fraction(x)
    e = math.floor(math.log2(abs(x)))
    while Fraction(2) ** e > abs(f):
        e -= 1
    while Fraction(2) ** (e + 1) <= abs(f):
        e += 1
    q = f / Fraction(2) ** (e - bits + 1)
    fl = math.floor(q)
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return float(fl * Fraction(2) ** (e - bits + 1))


def test_bf16_rounding_against_rationals():
    vals = np.concatenate([
        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -0.1, 0.6, 3.0e-5], dtype=np.float32),
        synth.uniform_f32(5, 9, 2000) * np.float32(4) - np.float32(2),
    ]).astype(np.float32)
    got = oracle.bf16_rne(vals)
    ref = np.array([frac_round_sig(float(v), 8) for v in vals], dtype=np.float32)
    assert np.array_equal(got, ref)
    assert got[1] == 1.0 and got[2] == np.float32(1 + 2 ** -6)
    hi, lo = oracle.bf16_split(vals)
    assert np.array_equal(hi, got)
    resid = vals.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64)
    assert np.all(np.abs(resid) <= np.abs(vals.astype(np.float64)) * 2.0 ** -16)


def test_schedule_reading():
    assert oracle.schedule(1000, 4) == (250, 0)
    assert oracle.schedule(50, 4) == (12, 2)
    assert oracle.schedule(7, 1) == (7, 0)
    assert oracle.schedule(0, 3) == (0, 0)


# ---------------------------------------------------------- FP32 mirror pins

def test_f32_mirror_integer_exact_and_close():
    g = rng(5)
    w = g.integers(-2, 3, size=(3, 3)).astype(np.float32)
    u0 = g.integers(0, 8, size=(9, 7)).astype(np.float32)
    ref = brute_force(w.astype(np.int64).astype(object), u0.astype(np.int64).astype(object), 3)
    got = oracle.sweep_f32(w, u0, 3)
    assert np.array_equal(got, ref.astype(np.float32))
    wl = synth.WORKLOADS["box2d"]
    u = synth.grid_f32((40, 44))
    a = oracle.sweep_f32(wl.weights.astype(np.float32), u, 50)
    b = oracle.sweep(wl.weights, u.astype(np.float64), 50)
    assert oracle.errors(a, b)["e_rel"] < 50 * 9 * 2.0 ** -24


def test_f32_mirror_matches_explicit_fmaf_chain():
    # one step evaluated with a literal per-tap fused multiply-add chain in
    # exact rationals rounded to FP32 after every tap
    w = synth.WORKLOADS["box2d"].weights.astype(np.float32)
    u0 = synth.grid_f32((5, 6))
    got = oracle.sweep_f32(w, u0, 1)
    for y in range(5):
        for x in range(6):
            acc = np.float32(0.0)
            for oy in range(-1, 2):
                for ox in range(-1, 2):
                    exact_v = (Fraction(float(w[oy + 1, ox + 1]))
                               * Fraction(float(u0[(y + oy) % 5, (x + ox) % 6]))
                               + Fraction(float(acc)))
                    acc = np.float32(round_exact_to_f32(exact_v))
            assert got[y, x] == acc


def round_exact_to_f32(q: Fraction) -> float:
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = 0
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    scale = Fraction(2) ** (e - 23)
    t = a / scale
    fl = math.floor(t)
    rem = t - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * float(fl * scale)


def test_sweep_window_matches_full_grid_bitwise():
    wl = synth.WORKLOADS["star2d"]
    u0 = synth.grid_f32((64, 80))
    T = 6
    full = oracle.sweep_f32(wl.weights.astype(np.float32), u0, T)
    pts = [(0, 0), (63, 79), (10, 40), (32, 1)]
    got = oracle.sweep_window(wl.weights.astype(np.float32), u0, T, pts, f32=True)
    assert np.array_equal(got, np.array([full[p] for p in pts]))
    full64 = oracle.sweep(wl.weights, u0.astype(np.float64), T)
    got64 = oracle.sweep_window(wl.weights, u0.astype(np.float64), T, pts)
    assert np.array_equal(got64, np.array([full64[p] for p in pts]))


# ------------------------------------------------- planted-mistake checks

def test_pins_catch_orientation_and_transpose_mistakes():
    """A flipped offset (u[x-o] instead of u[x+o]) or transposed weights give
    different values than the exact brute force for an asymmetric stencil."""
    g = rng(9)
    w = g.integers(1, 5, size=(3, 3)).astype(np.float64)
    u0 = g.integers(0, 9, size=(5, 6)).astype(np.float64)
    ref = brute_force(w.astype(np.int64).astype(object), u0.astype(np.int64).astype(object), 2).astype(np.float64)
    assert np.array_equal(oracle.sweep(w, u0, 2), ref)
    assert not np.array_equal(oracle.sweep(w[::-1, ::-1].copy(), u0, 2), ref)
    assert not np.array_equal(oracle.sweep(w.T.copy(), u0, 2), ref)


def test_pins_catch_dropped_fold_term():
    W = oracle.fold_weights(np.ones((3, 3)), 2)
    bad = W.copy()
    bad[0, 0] = 0.0
    u0 = rng(2).integers(0, 10, size=(8, 8)).astype(np.float64)
    good = oracle.sweep(np.ones((3, 3)), u0, 2)
    assert np.array_equal(oracle.sweep(W, u0, 1), good)
    assert not np.array_equal(oracle.sweep(bad, u0, 1), good)


# ------------------------------------------- zero Dirichlet ghosts (a reading)

def brute_force_dirichlet(w, u0, T):
    """A^T u0 with A the dense correlation operator whose taps that leave the
    grid are dropped (points outside hold 0), exact arithmetic."""
    shape = u0.shape
    dim = len(shape)
    r = (w.shape[0] - 1) // 2
    rows = []
    for x in itertools.product(*[range(n) for n in shape]):
        row = {}
        for o in itertools.product(range(-r, r + 1), repeat=dim):
            wo = w[tuple(oi + r for oi in o)]
            col = tuple(xi + oi for xi, oi in zip(x, o))
            if wo == 0 or any(c < 0 or c >= n for c, n in zip(col, shape)):
                continue
            row[int(np.ravel_multi_index(col, shape))] = wo
        rows.append(row)
    vec = list(u0.ravel())
    for _ in range(T):
        vec = [sum(wv * vec[c] for c, wv in row.items()) for row in rows]
    return np.array(vec, dtype=object).reshape(shape)


@pytest.mark.parametrize("shape", [(1,), (2,), (5,), (9,), (1, 1), (3, 4), (6, 5), (2, 3, 4)])
@pytest.mark.parametrize("r", [1, 2])
def test_dirichlet_brute_force_integer_bit_exact(shape, r):
    g = rng(zlib.crc32(repr((shape, r, "dirichlet")).encode()))
    w = g.integers(-3, 4, size=(2 * r + 1,) * len(shape)).astype(np.float64)
    u0 = g.integers(-5, 6, size=shape).astype(np.float64)
    T = 3
    ref = brute_force_dirichlet(w.astype(int).astype(object), u0.astype(int).astype(object), T)
    got = oracle.sweep(w, u0, T, "zero")
    assert np.array_equal(got, ref.astype(np.float64))


@pytest.mark.parametrize("n,k", [(31, 1), (31, 5), (64, 17)])
def test_dirichlet_sine_modes_heat1d(n, k):
    """With zero ghosts, sin(pi k (i+1)/(n+1)) is an eigenvector of the 1D
    heat operator (1/4, 1/2, 1/4) with eigenvalue cos^2(pi k / (2(n+1)))."""
    i = np.arange(n)
    v = np.sin(np.pi * k * (i + 1) / (n + 1))
    lam = np.cos(np.pi * k / (2 * (n + 1))) ** 2
    T = 40
    got = oracle.sweep(synth.heat1d_weights(), v, T, "zero")
    assert np.max(np.abs(got - lam ** T * v)) < 4 * T * 3 * EPS64


def test_dirichlet_sine_modes_star2d():
    """2D 5-point star (centre c, neighbours n): the product of sine modes is
    an eigenvector with eigenvalue c + 2n (cos(theta_y) + cos(theta_x))."""
    ny, nx, ky, kx = 21, 34, 3, 7
    ty, tx = np.pi * ky / (ny + 1), np.pi * kx / (nx + 1)
    v = np.outer(np.sin(ty * (np.arange(ny) + 1)), np.sin(tx * (np.arange(nx) + 1)))
    c, nb = 0.6, 0.1
    lam = c + 2 * nb * (np.cos(ty) + np.cos(tx))
    T = 30
    got = oracle.sweep(synth.star2d_weights(c, nb), v, T, "zero")
    assert np.max(np.abs(got - lam ** T * v)) < 4 * T * 5 * EPS64


@pytest.mark.parametrize("dim,r,m,shape", [
    (1, 1, 2, (13,)), (1, 1, 4, (5,)), (1, 2, 3, (40,)),
    (2, 1, 2, (9, 14)), (2, 1, 4, (17, 30)), (2, 2, 3, (23, 11)), (2, 1, 8, (12, 40)),
    (3, 1, 2, (6, 7, 9)), (3, 1, 3, (11, 8, 10)),
])
def test_dirichlet_folding_reading_exact(dim, r, m, shape):
    """The folded Dirichlet reading (W_m at least (m-1)r from every face, m
    plain steps in the band) equals the plain zero-ghost sweep exactly on
    integer data, for any T (folded applications then the remainder),
    including grids narrower than twice the band."""
    g = rng(dim * 100 + r * 10 + m)
    w = g.integers(-2, 3, size=(2 * r + 1,) * dim).astype(np.float64)
    u0 = g.integers(-4, 5, size=shape).astype(np.float64)
    for T in (m, 2 * m + 1, 3 * m - 1):
        assert np.array_equal(oracle.dirichlet_folded(w, u0, T, m), oracle.sweep(w, u0, T, "zero"))


def test_dirichlet_pins_catch_a_narrow_band():
    """A band one r narrower than (m-1)r (planted here, on the CPU) breaks
    the exact equality the previous pin checks."""
    w = np.array([[0.0, 1, 0], [2, 3, 1], [0, 2, 0]])
    u0 = (np.arange(20 * 25).reshape(20, 25) % 7).astype(np.float64)
    m, T = 4, 8
    band = oracle.band_mask(u0.shape, (m - 2) * 1)
    u = u0
    for _ in range(T // m):
        u = np.where(band, oracle.sweep(w, u, m, "zero"),
                     oracle.sweep(oracle.fold_weights(w, m), u, 1, "zero"))
    assert not np.array_equal(u, oracle.sweep(w, u0, T, "zero"))


def brute_force_ghost(w, u0, T, ghost):
    """A^T u0 for Dirichlet ghosts of value ghost: each step sums the taps
    inside the grid over the current values and the taps outside over the
    ghost value (the affine map u -> A_0 u + ghost * b), exact arithmetic."""
    shape = u0.shape
    dim = len(shape)
    r = (w.shape[0] - 1) // 2
    rows, outs = [], []
    for x in itertools.product(*[range(n) for n in shape]):
        row, out = {}, 0
        for o in itertools.product(range(-r, r + 1), repeat=dim):
            wo = w[tuple(oi + r for oi in o)]
            col = tuple(xi + oi for xi, oi in zip(x, o))
            if any(c < 0 or c >= n for c, n in zip(col, shape)):
                out += wo
            elif wo != 0:
                row[int(np.ravel_multi_index(col, shape))] = wo
        rows.append(row)
        outs.append(out)
    vec = list(u0.ravel())
    for _ in range(T):
        vec = [sum(wv * vec[c] for c, wv in row.items()) + ghost * b for row, b in zip(rows, outs)]
    return np.array(vec, dtype=object).reshape(shape)


@pytest.mark.parametrize("shape", [(1,), (4,), (9,), (1, 1), (3, 4), (6, 5), (2, 3, 4)])
@pytest.mark.parametrize("r", [1, 2])
def test_ghost_value_brute_force_integer_bit_exact(shape, r):
    """Dirichlet ghosts of a nonzero value: integer weights, values and
    ghost, exact against the affine brute force."""
    g = rng(zlib.crc32(repr((shape, r, "ghost")).encode()))
    w = g.integers(-3, 4, size=(2 * r + 1,) * len(shape)).astype(np.float64)
    u0 = g.integers(-5, 6, size=shape).astype(np.float64)
    ghost = int(g.integers(-4, 5)) or 3
    T = 3
    ref = brute_force_ghost(w.astype(int).astype(object), u0.astype(int).astype(object), T, ghost)
    got = oracle.sweep(w, u0, T, "zero", ghost)
    assert np.array_equal(got, ref.astype(np.float64))
    assert np.array_equal(oracle.sweep_f32(w, u0, T, "zero", ghost), ref.astype(np.float32))


def test_ghost_value_affine_shift_exact():
    """Weights summing to 1: holding the ghosts at c is the zero-ghost sweep
    of u0 - c, shifted by c (exact with dyadic weights and values)."""
    w = synth.heat1d_weights()
    w2 = np.outer([0.25, 0.5, 0.25], [0.25, 0.5, 0.25])
    g = rng(77)
    for wt, shape in ((w, (23,)), (w2, (9, 12))):
        u0 = g.integers(0, 16, size=shape).astype(np.float64)
        c = 3.0
        for T in (1, 4, 7):
            got = oracle.sweep(wt, u0, T, "zero", c)
            assert np.array_equal(got, oracle.sweep(wt, u0 - c, T, "zero") + c)


def test_ghost_value_constant_field_stays():
    """A field equal to the ghost value everywhere stays at it (weights
    summing to 1, dyadic), in FP64 and in the FP32 mirror."""
    w2 = np.outer([0.25, 0.5, 0.25], [0.25, 0.5, 0.25])
    u0 = np.full((7, 10), 2.5)
    assert np.array_equal(oracle.sweep(w2, u0, 9, "zero", 2.5), u0)
    assert np.array_equal(oracle.sweep_f32(w2, u0.astype(np.float32), 9, "zero", 2.5),
                          u0.astype(np.float32))


@pytest.mark.parametrize("dim,r,m,shape", [(1, 1, 3, (14,)), (2, 1, 2, (9, 14)), (2, 1, 4, (17, 30)),
                                           (2, 2, 3, (23, 11)), (3, 1, 2, (6, 7, 9))])
def test_ghost_value_folding_reading_exact(dim, r, m, shape):
    """The folded reading with ghosts of a nonzero value equals the plain
    sweep exactly on integer data."""
    g = rng(dim * 1000 + r * 10 + m)
    w = g.integers(-2, 3, size=(2 * r + 1,) * dim).astype(np.float64)
    u0 = g.integers(-4, 5, size=shape).astype(np.float64)
    for T in (m, 2 * m + 1):
        assert np.array_equal(oracle.dirichlet_folded(w, u0, T, m, ghost=-2.0),
                              oracle.sweep(w, u0, T, "zero", -2.0))


def test_ghost_value_pin_catches_a_dropped_ghost():
    """Ignoring the ghost value (zero ghosts, planted here) fails the brute
    force the pins above use."""
    w = np.array([[0, 1, 0], [2, 3, 1], [0, 2, 0]])
    u0 = (np.arange(4 * 5).reshape(4, 5) % 7)
    ref = brute_force_ghost(w.astype(object), u0.astype(object), 2, 5)
    planted = oracle.sweep(w.astype(np.float64), u0.astype(np.float64), 2, "zero", 0.0)
    assert not np.array_equal(planted, ref.astype(np.float64))


def test_dirichlet_mirror_f32_close_to_fp64():
    w = synth.WORKLOADS["star2d"].weights
    u0 = synth.grid_f32((40, 52))
    got = oracle.dirichlet_folded(w, u0, 9, 4, f32=True)
    ref = oracle.sweep(w, u0.astype(np.float64), 9, "zero")
    assert oracle.errors(got, ref)["e_rel"] < 1e-6


# ------------------------------------------------- nonlinear Table 1 workloads

def _life_brute(cells, T):
    """Game of Life by explicit loops over cells and neighbours (tiny grids)."""
    ny, nx = cells.shape
    c = [[int(v) for v in row] for row in cells]
    for _ in range(T):
        nxt = [[0] * nx for _ in range(ny)]
        for y in range(ny):
            for x in range(nx):
                k = sum(c[(y + dy) % ny][(x + dx) % nx]
                        for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx)
                nxt[y][x] = 1 if (k == 3 or (k == 2 and c[y][x])) else 0
        c = nxt
    return np.array(c, dtype=np.uint8)


def test_life_known_patterns():
    g = np.zeros((8, 8), dtype=np.uint8)
    g[3, 2:5] = 1  # blinker: period 2
    assert np.array_equal(oracle.life(g, 2), g) and not np.array_equal(oracle.life(g, 1), g)
    b = np.zeros((6, 6), dtype=np.uint8)
    b[2:4, 2:4] = 1  # block: still life
    assert np.array_equal(oracle.life(b, 5), b)
    gl = np.zeros((10, 10), dtype=np.uint8)
    for y, x in ((0, 1), (1, 2), (2, 0), (2, 1), (2, 2)):  # glider: (+1, +1) per 4
        gl[y, x] = 1
    assert np.array_equal(oracle.life(gl, 4), np.roll(gl, (1, 1), axis=(0, 1)))
    assert np.array_equal(oracle.life(gl, 40), np.roll(gl, (10, 10), axis=(0, 1)))


@pytest.mark.parametrize("shape", [(5, 7), (9, 4), (3, 3), (1, 6)])
def test_life_brute_force(shape):
    g = rng(sum(shape)).integers(0, 2, size=shape).astype(np.uint8)
    assert np.array_equal(oracle.life(g, 6), _life_brute(g, 6))


def test_floor_sweep_reduces_and_bounds():
    """APOP reading: with a floor below every reachable value it is the plain
    sweep; with dyadic weights summing to 1 and a constant floor above the
    data every step lands exactly on the floor; the result never drops
    below the floor nor below the plain sweep (positive weights)."""
    w = np.array([0.25, 0.5, 0.25])
    u0 = rng(3).random(64)
    low = np.full(64, -10.0)
    assert np.array_equal(oracle.floor_sweep(w, u0, low, 7), oracle.sweep(w, u0, 7))
    high = np.full(64, 2.0)
    assert np.array_equal(oracle.floor_sweep(w, u0, high, 3), high)
    payoff = np.maximum(0.5 - np.arange(64) / 64.0, 0.0)
    got = oracle.floor_sweep(w, u0, payoff, 9)
    assert np.all(got >= payoff) and np.all(got >= oracle.sweep(w, u0, 9))


def test_floor_sweep_rational_brute_force():
    w = [Fraction(1, 5), Fraction(1, 2), Fraction(1, 4)]
    g = rng(11)
    n = 9
    u = [Fraction(int(v), 8) for v in g.integers(0, 8, size=n)]
    fl = [Fraction(int(v), 8) for v in g.integers(0, 6, size=n)]
    ref = list(u)
    for _ in range(4):
        ref = [max(sum(w[o + 1] * ref[(i + o) % n] for o in (-1, 0, 1)), fl[i]) for i in range(n)]
    got = oracle.floor_sweep(np.array([float(v) for v in w]), np.array([float(v) for v in u]),
                             np.array([float(v) for v in fl]), 4)
    assert np.max(np.abs(got - np.array([float(v) for v in ref]))) < 16 * EPS64


# ------------------------------------------- error metrics (the parity gate)

def _errors_expected_case():
    """Hand-computed metrics: ref = (2, -4, 2, 12) has max |ref| = 12 and
    exact mean 3, so max |ref - mean| = 9; u = (2, -6, 2, 15) differs by 2 at
    the second element and by 3 at the last, so max_abs = 3,
    e_rel = 3 / 12 = 0.25 and e_detr = 3 / 9; two elements are bitwise
    equal."""
    ref = np.array([2.0, -4.0, 2.0, 12.0])
    u = np.array([2.0, -6.0, 2.0, 15.0])
    return u, ref, {"e_rel": 0.25, "e_detr": 3.0 / 9.0, "max_abs": 3.0, "bit_equal": 2, "n": 4}


def test_errors_hand_computed():
    u, ref, want = _errors_expected_case()
    assert oracle.errors(u, ref) == want
    # the same values in 2D and in FP32 (all dyadic, exact in both)
    got32 = oracle.errors(u.astype(np.float32).reshape(2, 2), ref.astype(np.float32).reshape(2, 2))
    assert got32 == want
    # mixed dtypes: the norms hold, no element counts as bitwise equal
    mixed = oracle.errors(u.astype(np.float32), ref)
    assert mixed["e_rel"] == 0.25 and mixed["bit_equal"] == 0


def test_errors_special_cases():
    # identical arrays: zero error, every element bitwise equal
    a = synth.grid_f32((7, 5))
    e = oracle.errors(a, a.copy())
    assert e["e_rel"] == 0.0 and e["e_detr"] == 0.0 and e["max_abs"] == 0.0
    assert e["bit_equal"] == 35
    # -0.0 against +0.0: numerically equal, not bitwise equal
    z = oracle.errors(np.array([-0.0, 1.0]), np.array([0.0, 1.0]))
    assert z["max_abs"] == 0.0 and z["bit_equal"] == 1
    # a constant reference: detrended norm 0, so e_detr falls back to max_abs
    c = oracle.errors(np.array([2.0, 2.25, 2.0]), np.array([2.0, 2.0, 2.0]))
    assert c["e_rel"] == 0.125 and c["e_detr"] == 0.25
    # a zero reference: e_rel is the absolute error
    zr = oracle.errors(np.array([0.5, 0.0]), np.zeros(2))
    assert zr["e_rel"] == 0.5
    # a NaN anywhere must fail every gate
    n = oracle.errors(np.array([1.0, np.nan]), np.array([1.0, 1.0]))
    assert not (n["e_rel"] < 1e-5)
    with pytest.raises(ValueError):
        oracle.errors(np.zeros(3), np.zeros(4))


def test_errors_pin_catches_wrong_norms():
    """Plausible mistakes in the metric (normalising by u instead of ref, a
    2-norm, per-element relative error, the mean of u, a metric that
    returns 0, a value-equality count) each give a different value on the
    hand-computed case, so the pin above would catch them."""
    u, ref, want = _errors_expected_case()
    d = np.abs(u - ref)
    mutants = {
        "norm of u": d.max() / np.abs(u).max(),
        "2-norm": np.linalg.norm(d) / np.linalg.norm(ref),
        "elementwise relative": (d / np.abs(ref)).max(),
        "zero": 0.0,
    }
    for name, val in mutants.items():
        assert val != want["e_rel"], name
    assert d.max() / np.abs(u - u.mean()).max() != want["e_detr"]
    assert d.max() / np.abs(ref - np.median(ref)).max() != want["e_detr"]
    assert int(np.count_nonzero(np.array([-0.0]) == np.array([0.0]))) == 1  # value equality would count it


# -------------------------------------- FP32 mirror of a folded run (reading 3)

@pytest.mark.parametrize("dim,m,T,shape", [
    (1, 3, 7, (19,)), (2, 2, 5, (9, 11)), (2, 3, 7, (10, 12)), (2, 4, 6, (13, 9)), (3, 2, 3, (5, 6, 7)),
])
def test_folded_reference_f32_exact_on_integer_data(dim, m, T, shape):
    """Integer weights and inputs with every intermediate value below 2^24:
    every FP32 operation is exact, so the mirror of floor(T/m) folded sweeps
    and T mod m plain ones must equal the exact rational brute force of T
    plain steps (T not divisible by m, so the remainder is exercised), and
    the FP64 oracle."""
    g = rng(100 + dim * 10 + m)
    w = g.integers(0, 2, size=(3,) * dim).astype(np.int64)
    w[(1,) * dim] = 1
    u0 = g.integers(0, 3, size=shape).astype(np.int64)
    assert int(np.abs(w).sum()) ** T * 2 < 2 ** 24
    ref = brute_force(w.astype(object), u0.astype(object), T).astype(np.float64)
    got = oracle.folded_reference_f32(w.astype(np.float64), u0.astype(np.float32), T, m)
    assert got.dtype == np.float32
    assert np.array_equal(got.astype(np.float64), ref)
    assert np.array_equal(got.astype(np.float64), oracle.sweep(w.astype(np.float64), u0.astype(np.float64), T))


def test_folded_reference_f32_m1_is_the_plain_mirror():
    w = synth.WORKLOADS["box2d"].weights
    u0 = synth.grid_f32((12, 17))
    got = oracle.folded_reference_f32(w, u0, 9, 1)
    # exact FP32 chain: pinned separately against a per-tap rational FMA chain
    assert np.array_equal(got, oracle.sweep_f32(w.astype(np.float32), u0, 9))


@pytest.mark.parametrize("name,m,T", [("star2d", 2, 41), ("star2d", 4, 42), ("box2d", 4, 30),
                                       ("box2d", 8, 35), ("heat1d", 5, 23), ("box3d", 2, 7)])
def test_folded_reference_f32_within_derived_bound(name, m, T):
    """Against the FP64 oracle on the same (FP32-exact) weights.  Positive
    weights summing to 1 give ||W||_1 = 1 for every fold, so errors do not
    grow from sweep to sweep.  Per folded sweep: each weight rounded to FP32
    (|dW| <= u |W|), the mass-compensated centre off by at most the other
    weights' rounding plus its own (<= 2u ||W||_1 in all), and a chain of
    n = |S_m| FMAs with error <= gamma_n = n u / (1 - n u) times
    sum |W| |v| <= ||v||_inf; per plain sweep gamma_|S| + u.  With
    u = 2^-24 the absolute error after q folded and s plain sweeps is at most
    (q (gamma_|S_m| + 3u) + s (gamma_|S| + u)) (1 + 3u)^(q+s) ||u0||_inf."""
    wl = synth.WORKLOADS[name]
    w = synth.to_f32_exact(wl.weights)
    dim = w.ndim
    shape = {1: (61,), 2: (23, 29), 3: (9, 10, 11)}[dim]
    u0 = synth.grid_f32(shape)
    got = oracle.folded_reference_f32(w, u0, T, m)
    ref = oracle.sweep(w, u0.astype(np.float64), T)
    q, s = oracle.schedule(T, m)
    u = 2.0 ** -24
    nS = int(np.count_nonzero(w))
    nSm = int(np.count_nonzero(oracle.fold_weights(w, m)))
    gamma = lambda n: n * u / (1 - n * u)  # noqa: E731
    bound = (q * (gamma(nSm) + 3 * u) + s * (gamma(nS) + u)) * (1 + 3 * u) ** (q + s) * float(np.abs(u0).max())
    err = oracle.errors(got, ref)["max_abs"]
    assert 0 < err <= bound
    # a dropped remainder (floor(T/m) folded sweeps only) breaks the bound
    if s:
        short = oracle.sweep_f32(oracle.fold_weights_f32(w, m), u0, q)
        assert oracle.errors(short, ref)["max_abs"] > bound


# ------------------------------------------------- FP32 branch of the floor sweep

def test_floor_sweep_f32_exact_on_dyadic_data():
    """Dyadic weights (1/4, 1/2, 1/4) and inputs on a grid of 2^-4 keep every
    FP32 step exact for T steps (numerators below 2^(4 + 2T) < 2^24), so the
    FP32 branch must equal the exact rational brute force of
    u <- max(A u, floor), and the FP64 branch."""
    n, T = 17, 8
    g = rng(21)
    u = [Fraction(int(v), 16) for v in g.integers(0, 16, size=n)]
    fl = [Fraction(int(v), 16) for v in g.integers(0, 10, size=n)]
    w = [Fraction(1, 4), Fraction(1, 2), Fraction(1, 4)]
    ref = list(u)
    for _ in range(T):
        ref = [max(sum(w[o + 1] * ref[(i + o) % n] for o in (-1, 0, 1)), fl[i]) for i in range(n)]
    wf = np.array([0.25, 0.5, 0.25])
    u32 = np.array([float(v) for v in u], dtype=np.float32)
    fl32 = np.array([float(v) for v in fl], dtype=np.float32)
    got = oracle.floor_sweep(wf, u32, fl32, T, f32=True)
    assert got.dtype == np.float32
    assert np.array_equal(got.astype(np.float64), np.array([float(v) for v in ref]))
    assert np.array_equal(got.astype(np.float64),
                          oracle.floor_sweep(wf, u32.astype(np.float64), fl32.astype(np.float64), T))
    # the floor taken before the stencil instead of after it gives another result
    wrong = u32.copy()
    for _ in range(T):
        wrong = oracle.sweep_f32(wf.astype(np.float32), np.fmax(wrong, fl32), 1)
    assert not np.array_equal(wrong, got)


def test_floor_sweep_f32_close_to_fp64():
    """Non-dyadic weights (the APOP discount): each FP32 step adds at most
    (gamma_3 + u) ||v||_inf of error before the max, and max(., floor) is
    1-Lipschitz, so after T steps |u32 - u64| <= T (gamma_3 + u) ||u0||_inf
    plus the floor's own rounding (u ||floor||_inf)."""
    w = synth.to_f32_exact(synth.APOP["weights"])
    n, T = 200, 60
    u0 = synth.apop_payoff(n).astype(np.float32)
    fl = u0.copy()
    got = oracle.floor_sweep(w, u0, fl, T, f32=True)
    ref = oracle.floor_sweep(w, u0.astype(np.float64), fl.astype(np.float64), T)
    u = 2.0 ** -24
    bound = (T * (3 * u / (1 - 3 * u) + u) + u) * float(np.abs(u0).max())
    err = oracle.errors(got, ref)["max_abs"]
    assert err <= bound
    assert np.all(got >= fl)


# ------------------------------------- spectral form (full-size error reference)

@pytest.mark.parametrize("shape,r", [((1,), 1), ((2,), 1), ((5,), 2), ((7,), 1), ((3, 5), 1),
                                     ((4, 3), 2), ((2, 3, 4), 1)])
def test_spectral_against_rational_brute_force(shape, r):
    """Random real weights (asymmetric, so the orientation matters) on tiny
    grids, including sides shorter than 2r+1 where offsets alias: the
    spectral form agrees with the exact rational value of A^T u0 to a few
    ulps of the data's scale."""
    dim = len(shape)
    g = rng(hash((shape, r, "spec")) % 2**32)
    w = g.random((2 * r + 1,) * dim)
    w /= w.sum()
    u0 = g.random(shape)
    T = 5
    ref = brute_force(exact(w), exact(u0), T)
    got = oracle.sweep_spectral(w, u0, T)
    err = max(abs(Fraction(float(a)) - b) for a, b in zip(got.ravel(), ref.ravel()))
    assert float(err) <= 64 * EPS64 * float(np.abs(u0).max())


@pytest.mark.parametrize("name,shape,T", [("heat1d", (1000,), 100), ("star2d", (96, 130), 250),
                                          ("box2d", (64, 96), 100), ("star3d", (20, 24, 28), 40),
                                          ("box3d", (16, 18, 20), 30)])
def test_spectral_against_naive_sweep(name, shape, T):
    """The naive loop (pinned above by brute force) and the spectral form
    agree to the FFT's rounding on the workloads' own stencils, the random
    2D box being asymmetric."""
    w = synth.to_f32_exact(synth.WORKLOADS[name].weights)
    u0 = synth.grid_f64(shape)
    a = oracle.sweep(w, u0, T)
    b = oracle.sweep_spectral(w, u0, T)
    assert np.max(np.abs(a - b)) <= 1e-13 * float(np.abs(u0).max())


def test_spectral_fourier_mode_and_planted_conjugate():
    """A single Fourier mode decays by |lambda(k)|^T and turns by T arg
    lambda(k) (the closed form); conjugating lambda (the flipped
    orientation u[x-o]) misses it for the asymmetric random box."""
    w = synth.WORKLOADS["box2d"].weights
    for k, T in (((5, 7), 9), ((1, 2), 4), ((2, 1), 30)):
        u0, want, _ = fourier_closed_form(w, (24, 30), k, T)
        scale = float(np.abs(want).max())
        got = oracle.sweep_spectral(w, u0, T)
        assert np.max(np.abs(got - want)) < 1e-13
        flipped = oracle.sweep_spectral(w[::-1, ::-1].copy(), u0, T)
        assert np.max(np.abs(flipped - want)) > 1e-2 * scale


def test_spectral_zero_boundary():
    """Zero ghosts through the sine transform: equal to the naive zero-ghost
    loop (pinned by brute force with dropped taps), and a sine mode decays by
    its closed-form eigenvalue; asymmetric or wider stencils are refused."""
    w = synth.star2d_weights(0.6, 0.1)
    u0 = synth.grid_f64((30, 41))
    for T in (1, 6, 57):
        a = oracle.sweep(w, u0, T, "zero")
        b = oracle.sweep_spectral(w, u0, T, "zero")
        assert np.max(np.abs(a - b)) <= 1e-13
    box = np.array([[0.05, 0.1, 0.05], [0.1, 0.4, 0.1], [0.05, 0.1, 0.05]])
    assert np.max(np.abs(oracle.sweep(box, u0, 8, "zero") - oracle.sweep_spectral(box, u0, 8, "zero"))) < 1e-13
    n, kk, T = 31, 4, 12
    x = np.arange(1, n + 1)
    mode = np.sin(np.pi * kk * x / (n + 1))
    lam = 0.5 + 0.5 * np.cos(np.pi * kk / (n + 1))
    got = oracle.sweep_spectral(np.array([0.25, 0.5, 0.25]), mode, T, "zero")
    assert np.max(np.abs(got - lam ** T * mode)) < 1e-14
    with pytest.raises(ValueError):
        oracle.sweep_spectral(synth.WORKLOADS["box2d"].weights, u0, 2, "zero")
    with pytest.raises(ValueError):
        oracle.sweep_spectral(np.ones((5, 5)) / 25, u0, 2, "zero")
