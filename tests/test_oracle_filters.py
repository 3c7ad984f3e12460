"""Pins of the oracle's local filters and Marschner-Lobb function (CPU only).

The filters are checked against what their definitions fix: partition of
unity, interpolation of the samples (trilinear, Catmull-Rom), polynomial
reproduction (multilinear for trilinear, quadratics for Catmull-Rom inside
the grid, linear functions for the cubic B-spline filter, which turns x^2
into x^2 + h^2/3), the cubic B-spline weights against the Cox-de Boor basis
of uniform knots, Catmull-Rom against its Hermite form, gradients against
central differences, the support of each filter (samples outside the
stencil of the cell floor(g) do not matter) and the convex hull of the
non-negative filters.  The Marschner-Lobb function against closed-form
values and its gradient against central differences.
"""
import numpy as np
import pytest

from oracle import bspline as ob
from oracle import filters as of

KINDS = [of.TRILINEAR, of.CATMULL_ROM, of.BSPLINE3]


@pytest.mark.parametrize("kind", KINDS)
def test_weights_partition_of_unity_and_derivatives(kind):
    t = np.linspace(0.0, 1.0, 101)
    w, dw = of.weights(kind, t)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(dw.sum(axis=1), 0.0, rtol=0, atol=1e-14)
    eps = 1e-6
    tm = np.linspace(0.1, 0.9, 9)
    fd = (of.weights(kind, tm + eps)[0] - of.weights(kind, tm - eps)[0]) / (2 * eps)
    np.testing.assert_allclose(of.weights(kind, tm)[1], fd, rtol=0, atol=1e-8)


def test_cubic_bspline_weights_equal_cox_de_boor_basis():
    """On uniform knots ..., -1, 0, 1, 2, ... the four cubic B-splines alive
    on [0, 1) at t are the filter's weights (library-independent basis)."""
    T = np.arange(-3.0, 5.0)                       # knots -3 .. 4
    t = np.linspace(0.0, 0.999, 37)
    N, _ = ob.basis_and_derivs(T, 3, np.full(t.shape, 3), t)
    w, _ = of.weights(of.BSPLINE3, t)
    np.testing.assert_allclose(w, N, rtol=0, atol=1e-14)


def test_catmull_rom_equals_hermite_form():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(4)                     # samples c-1, c, c+1, c+2
    t = np.linspace(0.0, 1.0, 21)
    m0, m1 = (v[2] - v[0]) / 2, (v[3] - v[1]) / 2
    h00, h10 = 2 * t ** 3 - 3 * t ** 2 + 1, t ** 3 - 2 * t ** 2 + t
    h01, h11 = -2 * t ** 3 + 3 * t ** 2, t ** 3 - t ** 2
    want = h00 * v[1] + h10 * m0 + h01 * v[2] + h11 * m1
    w, _ = of.weights(of.CATMULL_ROM, t)
    np.testing.assert_allclose(w @ v, want, rtol=0, atol=1e-14)


def _grid(N, lo, hi):
    return [lo[a] + np.arange(N[a]) * ((hi[a] - lo[a]) / (N[a] - 1)) for a in range(3)]


@pytest.mark.parametrize("kind", [of.TRILINEAR, of.CATMULL_ROM])
def test_interpolating_filters_reproduce_the_samples(kind):
    rng = np.random.default_rng(kind)
    N, lo, hi = (7, 9, 6), (0.0, -1.0, 2.0), (1.0, 3.0, 2.5)
    V = rng.standard_normal(N)
    ax = _grid(N, lo, hi)
    X = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    f, _ = of.grid_field(V, lo, hi, kind)(X)
    np.testing.assert_allclose(f, V.ravel(), rtol=0, atol=1e-12)


def test_polynomial_reproduction_and_bspline_smoothing():
    rng = np.random.default_rng(11)
    N, lo, hi = (12, 10, 11), (0.0, 0.0, 0.0), (2.0, 1.5, 1.0)
    h = [(hi[a] - lo[a]) / (N[a] - 1) for a in range(3)]
    ax = _grid(N, lo, hi)
    G = np.meshgrid(*ax, indexing="ij")
    # points inside the grid, two cells away from the faces (no edge repeats)
    x = np.stack([lo[a] + 2 * h[a] + rng.random(400) * (hi[a] - lo[a] - 4 * h[a]) for a in range(3)], 1)
    multilin = lambda X, Y, Z: 0.3 + 1.2 * X - 0.7 * Y + 0.5 * Z + 0.9 * X * Y - 0.4 * Y * Z + 0.2 * X * Y * Z
    f, g = of.grid_field(multilin(*G), lo, hi, of.TRILINEAR)(x)
    np.testing.assert_allclose(f, multilin(x[:, 0], x[:, 1], x[:, 2]), rtol=0, atol=1e-12)
    quad = lambda X, Y, Z: 1.0 + X - 2 * Y + 3 * X * X - Y * Z + 0.5 * Z * Z
    f, g = of.grid_field(quad(*G), lo, hi, of.CATMULL_ROM)(x)
    np.testing.assert_allclose(f, quad(x[:, 0], x[:, 1], x[:, 2]), rtol=0, atol=1e-12)
    gq = np.stack([1 + 6 * x[:, 0], -2 - x[:, 2], -x[:, 1] + x[:, 2]], 1)
    np.testing.assert_allclose(g, gq, rtol=0, atol=1e-11)
    lin = lambda X, Y, Z: 0.5 - X + 2 * Y + 0.25 * Z
    f, g = of.grid_field(lin(*G), lo, hi, of.BSPLINE3)(x)
    np.testing.assert_allclose(f, lin(x[:, 0], x[:, 1], x[:, 2]), rtol=0, atol=1e-12)
    np.testing.assert_allclose(g, np.tile([-1.0, 2.0, 0.25], (400, 1)), rtol=0, atol=1e-12)
    # the cubic B-spline filter of x^2 is x^2 + h^2 / 3 (its second moment)
    f, _ = of.grid_field(G[0] ** 2, lo, hi, of.BSPLINE3)(x)
    np.testing.assert_allclose(f, x[:, 0] ** 2 + h[0] ** 2 / 3, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_gradients_equal_central_differences(kind):
    rng = np.random.default_rng(20 + kind)
    N, lo, hi = (9, 8, 10), (0.0, 0.0, 0.0), (1.0, 2.0, 1.5)
    V = rng.standard_normal(N)
    fn = of.grid_field(V, lo, hi, kind)
    h = np.array([(hi[a] - lo[a]) / (N[a] - 1) for a in range(3)])
    # points at cell centres +- 0.3 cells (away from cell faces, where the
    # trilinear gradient jumps)
    c = np.stack([rng.integers(0, N[a] - 1, 300) for a in range(3)], 1)
    x = np.asarray(lo) + (c + 0.5 + rng.uniform(-0.3, 0.3, (300, 3))) * h
    _, g = fn(x)
    eps = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        fd = (fn(x + e)[0] - fn(x - e)[0]) / (2 * eps)
        np.testing.assert_allclose(g[:, a], fd, rtol=0, atol=1e-6 * (1 + np.abs(fd).max()))


def test_marschner_lobb_closed_forms_and_gradient():
    f, _ = of.ml_value_grad(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 3.0],
                                      [1.0, 0.0, 0.0]]))
    # rho(0) = cos(12 pi) = 1; sin(pi/2) = 1; sin(3 pi/2) = -1; rho(1) = cos(2 pi 6 cos(pi/2)) = 1
    np.testing.assert_allclose(f, [1.5 / 2.5, 0.5 / 2.5, 2.5 / 2.5, 1.5 / 2.5], rtol=0, atol=1e-12)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.05, 6.95, size=(500, 3))
    v, g = of.ml_value_grad(x)
    assert v.min() >= 0.0 and v.max() <= 1.0
    eps = 1e-7
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        fd = (of.ml_value_grad(x + e)[0] - of.ml_value_grad(x - e)[0]) / (2 * eps)
        np.testing.assert_allclose(g[:, a], fd, rtol=0, atol=1e-5)
    S = of.ml_samples(9)
    assert S.shape == (9, 9, 9)
    np.testing.assert_allclose(S[0, 0, 0], 0.6, atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_support_and_convex_hull(kind):
    """The value at g depends only on the samples of the stencil of the
    cell floor(g) (c .. c+1 for trilinear, c-1 .. c+2 for the cubics), and
    the non-negative filters (trilinear, cubic B-spline) stay within the
    range of those samples."""
    rng = np.random.default_rng(30 + kind)
    N, lo, hi = (10, 10, 10), (0.0, 0.0, 0.0), (9.0, 9.0, 9.0)       # h = 1: g = x
    V = rng.standard_normal(N)
    x = rng.uniform(2.0, 6.99, size=(200, 3))
    f0, _ = of.grid_field(V, lo, hi, kind)(x)
    a0, a1 = (0, 1) if kind == of.TRILINEAR else (-1, 2)
    for q in range(len(x)):
        c = np.floor(x[q]).astype(int)
        sl = tuple(slice(c[a] + a0, c[a] + a1 + 1) for a in range(3))
        W = V.copy()
        mask = np.ones(N, dtype=bool)
        mask[sl] = False
        W[mask] += 10.0                                  # every sample outside the stencil
        f1, _ = of.grid_field(W, lo, hi, kind)(x[q:q + 1])
        assert f1[0] == pytest.approx(f0[q], abs=1e-12)
        if kind != of.CATMULL_ROM:
            assert V[sl].min() - 1e-12 <= f0[q] <= V[sl].max() + 1e-12


def test_input_generator_samples_equal_the_oracle_function():
    import synth
    for N in (5, 16):
        np.testing.assert_array_equal(synth.marschner_lobb_samples(N),
                                      of.ml_samples(N).astype(np.float32))
