"""Pins of the oracle's fixed-knot encoding (CPU only).

The oracle computes the least-squares control points by three mode products
with per-axis pseudo-inverses.  Each test checks it against something other
than that formula: the dense Kronecker least-squares problem solved directly
on tiny grids (brute force), exact reproduction of a spline of the same
space, reproduction of polynomials of degree <= p, and the normal equations
(the residual is orthogonal to every basis function of the model).
"""
import numpy as np
import pytest

import synth
from oracle import bspline as ob
from oracle import encode as oe


def nonuniform_knots(n, p, rng):
    inner = np.sort(rng.uniform(0.05, 0.95, size=n - p - 1))
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def spaced_knots(n, p, rng):
    """Non-uniform clamped knots whose spans are 0.4 to 1.6 times the mean
    span, so that a uniform grid of 3n samples puts samples in every span
    (the collocation matrices then have full column rank)."""
    m = n - p
    inner = (np.arange(1, m) + rng.uniform(-0.3, 0.3, size=m - 1)) / m
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def grid_params(N, rng, kind):
    if kind == "uniform":
        return np.arange(N, dtype=np.float64) / (N - 1)
    u = np.sort(rng.random(N))
    u[0], u[-1] = 0.0, 1.0
    return u


def kron_design(axis_u, degree, knots, n_ctrl):
    """Dense design matrix of the tensor grid, rows in C order of the samples
    and columns in C order of the control points, built point by point from
    the oracle's scalar basis (not from the collocation routine)."""
    rows = []
    for u0 in axis_u[0]:
        for u1 in axis_u[1]:
            for u2 in axis_u[2]:
                vals = []
                for a, u in enumerate((u0, u1, u2)):
                    T, p, n = knots[a], degree[a], n_ctrl[a]
                    s = ob.find_span(T, p, n, np.array([u]))
                    N, _ = ob.basis_and_derivs(T, p, s, np.array([u]))
                    v = np.zeros(n)
                    v[s[0] - p:s[0] + 1] = N[0]
                    vals.append(v)
                rows.append(np.einsum("i,j,k->ijk", *vals).ravel())
    return np.array(rows)


@pytest.mark.parametrize("kind", ["uniform", "random"])
@pytest.mark.parametrize("degree", [(3, 3, 3), (2, 3, 1), (4, 2, 3)])
def test_fit_equals_dense_kronecker_least_squares(kind, degree):
    rng = np.random.default_rng(sum(degree) + (kind == "random"))
    res = (9, 7, 8)
    n_ctrl = [degree[a] + 2 + a for a in range(3)]
    knots = [nonuniform_knots(n_ctrl[a], degree[a], rng) if kind == "random"
             else synth.clamped_uniform_knots(n_ctrl[a], degree[a]) for a in range(3)]
    axis_u = [grid_params(res[a], rng, kind) for a in range(3)]
    F = rng.standard_normal(res)
    P = oe.fit_grid(F, axis_u, degree, knots, n_ctrl)
    A = kron_design(axis_u, degree, knots, n_ctrl)
    want, *_ = np.linalg.lstsq(A, F.ravel(), rcond=None)
    np.testing.assert_allclose(P.ravel(), want, rtol=0, atol=1e-10 * np.abs(want).max())


@pytest.mark.parametrize("p", [2, 3, 5])
def test_fit_reproduces_a_spline_of_the_same_space(p):
    rng = np.random.default_rng(40 + p)
    n = (p + 5, p + 3, p + 7)
    knots = [spaced_knots(n[a], p, rng) for a in range(3)]
    C = rng.standard_normal(n)
    model = synth.single_block_model(C, [p] * 3, knots)
    axis_u = [grid_params(3 * n[a], rng, "uniform") for a in range(3)]
    F = ob.decode_grid(model, axis_u)[..., 0]          # samples of the spline itself
    P = oe.fit_grid(F, axis_u, [p] * 3, knots, n)
    np.testing.assert_allclose(P, C, rtol=0, atol=1e-9 * np.abs(C).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_fit_reproduces_polynomials_up_to_degree_p(p):
    rng = np.random.default_rng(50 + p)
    n = (p + 4, p + 6, p + 5)
    knots = [synth.clamped_uniform_knots(n[a], p) for a in range(3)]
    axis_u = [grid_params(2 * n[a] + 1, rng, "uniform") for a in range(3)]
    coef = rng.standard_normal((p + 1, p + 1, p + 1))

    def poly(x, y, z):
        out = 0.0
        for i in range(p + 1):
            for j in range(p + 1 - i):
                for k in range(p + 1 - i - j):
                    out = out + coef[i, j, k] * x ** i * y ** j * z ** k
        return out

    g = np.meshgrid(*axis_u, indexing="ij")
    P = oe.fit_grid(poly(*g), axis_u, [p] * 3, knots, n)
    model = synth.single_block_model(P, [p] * 3, knots)
    x = rng.random((500, 3))
    f = ob.evaluate(model, x)["f"]
    np.testing.assert_allclose(f, poly(x[:, 0], x[:, 1], x[:, 2]), rtol=0, atol=1e-10)


def test_residual_satisfies_the_normal_equations():
    rng = np.random.default_rng(60)
    p, n, res = 3, (11, 9, 13), (40, 31, 45)
    knots = [nonuniform_knots(n[a], p, rng) for a in range(3)]
    axis_u = [grid_params(res[a], rng, "random") for a in range(3)]
    F = rng.standard_normal(res)
    P = oe.fit_grid(F, axis_u, [p] * 3, knots, n)
    model = synth.single_block_model(P, [p] * 3, knots)
    R = ob.decode_grid(model, axis_u)[..., 0] - F
    G = R
    for a in range(3):                                  # B^T applied along every axis
        T = knots[a]
        s = ob.find_span(T, p, n[a], axis_u[a])
        N, _ = ob.basis_and_derivs(T, p, s, axis_u[a])
        Bt = np.zeros((n[a], res[a]))
        for r in range(p + 1):
            Bt[s - p + r, np.arange(res[a])] = N[:, r]
        G = np.moveaxis(np.tensordot(Bt, G, axes=([1], [a])), 0, a)
    assert np.abs(G).max() < 1e-10 * np.abs(F).max() * np.prod(res)


def test_collocation_rows_partition_unity_and_band():
    rng = np.random.default_rng(70)
    for p in (1, 3, 5):
        n = p + 9
        T = nonuniform_knots(n, p, rng)
        u = grid_params(50, rng, "random")
        B = oe.collocation(T, p, n, u)
        np.testing.assert_allclose(B.sum(axis=1), 1.0, rtol=0, atol=1e-14)
        assert np.all(B >= 0.0)
        assert np.all((B != 0.0).sum(axis=1) <= p + 1)


# ---------------------------------------------------------------- knot insertion (Fig. 1)
def _c1_samples(N=40):
    field = synth.field_c1(1)
    xs = np.arange(N, dtype=np.float64) / (N - 1)
    return field.value_separable(xs, xs, xs), [xs] * 3


def test_span_errors_match_a_scalar_scan():
    rng = np.random.default_rng(80)
    p, n, res = 3, (7, 9, 6), (23, 17, 19)
    knots = [nonuniform_knots(n[a], p, rng) for a in range(3)]
    axis_u = [grid_params(res[a], rng, "random") for a in range(3)]
    err = rng.random(res)
    got = oe.span_errors(err, axis_u, [p] * 3, knots)
    for a in range(3):
        want = np.zeros(n[a] - p)
        for idx in np.ndindex(*res):
            u = axis_u[a][idx[a]]
            s = max(i for i in range(p, n[a]) if knots[a][i] <= u) - p   # the span rule
            want[s] = max(want[s], err[idx])
        np.testing.assert_array_equal(got[a], want)


def test_adaptive_fit_reaches_the_bound_with_nested_knots():
    F, axis_u = _c1_samples()
    e_max = 2e-3
    prev = None
    for it in range(1, 6):
        knots, P, hist = oe.fit_adaptive(F, axis_u, [3] * 3, [6] * 3, e_max, max_iter=it)
        if prev is not None:
            for a in range(3):                               # knot vectors only grow
                assert set(np.round(prev[a], 15)) <= set(np.round(knots[a], 15))
        prev = knots
    assert len(hist) < 5 and hist[-1][1] <= e_max           # stopped because the bound holds
    assert all(h[1] > e_max for h in hist[:-1])
    # the returned control points are the fixed-knot fit on the final knots
    n = [len(knots[a]) - 4 for a in range(3)]
    np.testing.assert_allclose(P, oe.fit_grid(F, axis_u, [3] * 3, knots, n), rtol=0, atol=1e-12)


def test_adaptive_residual_never_grows_and_loose_bound_keeps_initial_knots():
    """Knot insertion nests the spline spaces, so the least-squares residual
    (sum of squares) cannot grow from one fit to the next."""
    x = np.arange(33, dtype=np.float64) / 32
    g = np.meshgrid(x, x, x, indexing="ij")
    F = np.abs(g[0] - 0.3) ** 3 + 0.5 * np.abs(g[1] - 0.71) ** 2 * g[2]
    axis_u = [x] * 3
    rss = []
    for it in range(1, 5):
        knots, P, hist = oe.fit_adaptive(F, axis_u, [3] * 3, [5] * 3, 1e-6, max_iter=it)
        R = oe.reconstruct_grid(P, axis_u, [3] * 3, knots) - F
        rss.append(float((R * R).sum()))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(rss, rss[1:]))
    assert rss[-1] < 0.05 * rss[0]
    knots, P, hist = oe.fit_adaptive(F, axis_u, [3] * 3, [5] * 3, 10.0)
    assert len(hist) == 1 and all(len(k) == 5 + 4 for k in knots)


def test_adaptive_cap_keeps_the_largest_errors():
    """With a cap on the control points, the spans that are halved are the
    ones of largest error; a cap never reached changes nothing."""
    F, axis_u = _c1_samples(32)
    free, Pf, hf = oe.fit_adaptive(F, axis_u, [3] * 3, [5] * 3, 1e-4, max_iter=2)
    big, Pb, hb = oe.fit_adaptive(F, axis_u, [3] * 3, [5] * 3, 1e-4, max_iter=2, max_ctrl=[32] * 3)
    for a in range(3):
        np.testing.assert_array_equal(free[a], big[a])
    k1, _, h1 = oe.fit_adaptive(F, axis_u, [3] * 3, [5] * 3, 1e-4, max_iter=1)
    capped, _, hc = oe.fit_adaptive(F, axis_u, [3] * 3, [5] * 3, 1e-4, max_iter=2, max_ctrl=[6, 7, 5])
    assert [len(capped[a]) - 4 for a in range(3)] == [6, 7, 5]
    # which spans: recompute the span errors of the first fit by a scalar scan
    n1 = [len(k1[a]) - 4 for a in range(3)]
    P1 = oe.fit_grid(F, axis_u, [3] * 3, k1, n1)
    err = np.abs(oe.reconstruct_grid(P1, axis_u, [3] * 3, k1) - F) / (F.max() - F.min())
    for a, extra in ((0, 1), (1, 2)):
        other = tuple(b for b in range(3) if b != a)
        marg = err.max(axis=other)
        span_err = {}
        for i, u in enumerate(axis_u[a]):
            j = min(int(np.searchsorted(k1[a], u, side="right")) - 1, n1[a] - 1) - 3
            span_err[j] = max(span_err.get(j, 0.0), marg[i])
        order = sorted(span_err, key=lambda j: (-span_err[j], j))[:extra]
        want = sorted([0.5 * (k1[a][3 + j] + k1[a][4 + j]) for j in order])
        added = sorted(set(np.round(capped[a], 14)) - set(np.round(k1[a], 14)))
        np.testing.assert_allclose(added, want, atol=1e-14)
