"""Pins of the oracle's model evaluation (CPU only).

Each test checks the oracle against something other than itself: a linear
scan of the span definition, the full (all-index) recursion, scipy's
B-spline routines, exact polynomial reproduction (Marsden's identity via
blossoms), central finite differences, and scalar re-evaluations of the
exact FP64 decisions.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline, NdBSpline

import synth
from oracle import bspline as ob


def nonuniform_knots(n, p, rng, repeat=True):
    inner = np.sort(rng.uniform(0.0, 1.0, size=n - p - 1))
    if repeat and n - p - 1 >= 3:
        inner[1] = inner[2]          # a double interior knot
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def span_by_scan(T, p, n, u):
    """Largest i in [p, n-1] with T[i] <= u (p if none): the definition."""
    s = p
    for i in range(p, n):
        if T[i] <= u:
            s = i
    return s


def adversarial_u(T):
    vals = [0.0, 1.0, np.nextafter(1.0, 0.0), np.nextafter(0.0, 1.0), 0.5]
    for t in np.unique(T):
        vals += [t, np.nextafter(t, -np.inf), np.nextafter(t, np.inf)]
    vals = np.array(vals)
    return vals[(vals >= 0.0) & (vals <= 1.0)]


# ---------------------------------------------------------------- spans
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n", [6, 9, 16])
def test_span_matches_definition_scan(p, n):
    if n < p + 1:
        pytest.skip("n < p+1")
    rng = np.random.default_rng(10 * p + n)
    for T in (synth.clamped_uniform_knots(n, p), nonuniform_knots(n, p, rng)):
        u = np.concatenate([adversarial_u(T), rng.random(200)])
        got = ob.find_span(T, p, n, u)
        want = np.array([span_by_scan(T, p, n, float(x)) for x in u])
        np.testing.assert_array_equal(got, want)
        # the span is non-empty and holds u
        assert np.all(T[got] <= u)
        assert np.all((u < T[got + 1]) | (got == n - 1))
        assert np.all(T[got] < T[got + 1])


# ---------------------------------------------------------------- basis
def full_recursion(T, p, u):
    """All N_{i,p}(u), i = 0..n-1, from the indicator functions (last span
    closed at the right end), by the recursion over every index."""
    n = len(T) - p - 1
    m = len(T) - 1
    last = max(i for i in range(m) if T[i] < T[i + 1])
    N = np.zeros(m)
    for i in range(m):
        if (T[i] <= u < T[i + 1]) or (i == last and u == T[i + 1]):
            N[i] = 1.0
    for q in range(1, p + 1):
        M = np.zeros(m - q)
        for i in range(m - q):
            a = (u - T[i]) / (T[i + q] - T[i]) if T[i + q] != T[i] else 0.0
            b = (T[i + q + 1] - u) / (T[i + q + 1] - T[i + 1]) if T[i + q + 1] != T[i + 1] else 0.0
            M[i] = a * N[i] + b * N[i + 1]
        N = M
    return N[:n]


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_basis_partition_support_and_full_recursion(p):
    rng = np.random.default_rng(p)
    n = 11
    for T in (synth.clamped_uniform_knots(n, p), nonuniform_knots(n, p, rng)):
        u = np.concatenate([adversarial_u(T), rng.random(64)])
        s = ob.find_span(T, p, n, u)
        N, D = ob.basis_and_derivs(T, p, s, u)
        eps = np.finfo(np.float64).eps
        assert np.all(N >= 0.0)
        assert np.max(np.abs(N.sum(axis=1) - 1.0)) <= 4 * eps
        assert np.max(np.abs(D.sum(axis=1))) <= 64 * eps * np.max(np.abs(D))
        for x, sx, row in zip(u, s, N):
            full = full_recursion(T, p, float(x))
            active = np.zeros(n)
            active[sx - p:sx + 1] = row
            np.testing.assert_allclose(active, full, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_basis_and_derivative_match_scipy(p):
    rng = np.random.default_rng(100 + p)
    n = 13
    # a double interior knot only where the derivative stays continuous
    for T in (synth.clamped_uniform_knots(n, p), nonuniform_knots(n, p, rng, repeat=p >= 3)):
        u = np.concatenate([rng.random(300), [0.0, 1.0, np.nextafter(1.0, 0.0)]])
        s = ob.find_span(T, p, n, u)
        N, D = ob.basis_and_derivs(T, p, s, u)
        full_N = np.zeros((len(u), n))
        full_D = np.zeros((len(u), n))
        for r in range(p + 1):
            full_N[np.arange(len(u)), s - p + r] = N[:, r]
            full_D[np.arange(len(u)), s - p + r] = D[:, r]
        ref = BSpline.design_matrix(u, T, p).toarray()
        np.testing.assert_allclose(full_N, ref, rtol=0, atol=1e-14)
        for i in range(n):
            c = np.zeros(n)
            c[i] = 1.0
            d_ref = BSpline(T, c, p).derivative()(u)
            scale = max(1.0, np.max(np.abs(d_ref)))
            np.testing.assert_allclose(full_D[:, i], d_ref, rtol=0, atol=1e-13 * scale)


# ---------------------------------------------------------------- values
def blossom_coeffs(T, p, n, poly):
    """B-spline coefficients of sum_k poly[k] u^k (k <= p) by Marsden's
    identity: P_i = sum_k poly[k] e_k(T[i+1..i+p]) / C(p,k)."""
    out = np.zeros(n)
    for i in range(n):
        ts = T[i + 1:i + p + 1]
        for k, ck in enumerate(poly):
            ek = sum(math.prod(c) for c in itertools.combinations(ts, k)) if k else 1.0
            out[i] += ck * ek / math.comb(p, k)
    return out


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("uniform", [True, False])
def test_polynomial_reproduction(p, uniform):
    rng = np.random.default_rng(7 * p + uniform)
    ns = [p + 3, p + 6, p + 9]
    knots, rows, polys = [], [], []
    for a in range(3):
        T = synth.clamped_uniform_knots(ns[a], p) if uniform else nonuniform_knots(ns[a], p, rng)
        poly = rng.uniform(-1, 1, size=p + 1)
        knots.append(T)
        polys.append(poly)
        rows.append(blossom_coeffs(T, p, ns[a], poly))
    P = rows[0][:, None, None] * rows[1][None, :, None] * rows[2][None, None, :]
    model = synth.single_block_model(P, [p, p, p], knots)
    u = np.concatenate([rng.random((500, 3)), np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0.5]])])
    f, g, _ = ob.block_eval_param(model.blocks[0], u)

    def pv(c, x):
        return sum(ck * x ** k for k, ck in enumerate(c))

    def pd(c, x):
        return sum(k * ck * x ** (k - 1) for k, ck in enumerate(c) if k)

    vals = [pv(polys[a], u[:, a]) for a in range(3)]
    ders = [pd(polys[a], u[:, a]) for a in range(3)]
    f_ref = vals[0] * vals[1] * vals[2]
    g_ref = np.stack([ders[0] * vals[1] * vals[2], vals[0] * ders[1] * vals[2],
                      vals[0] * vals[1] * ders[2]], axis=1)
    scale = max(1.0, np.max(np.abs(P)))
    assert np.max(np.abs(f - f_ref)) <= 1e-13 * scale
    assert np.max(np.abs(g - g_ref)) <= 1e-11 * scale * max(ns)


def test_constant_and_linear_precision():
    p, n = 3, 9
    T = synth.clamped_uniform_knots(n, p)
    rng = np.random.default_rng(3)
    u = rng.random((400, 3))
    const = synth.single_block_model(np.full((n, n, n), 2.5), [p] * 3, [T] * 3)
    f, g, _ = ob.block_eval_param(const.blocks[0], u)
    assert np.max(np.abs(f - 2.5)) <= 1e-14 and np.max(np.abs(g)) <= 1e-12
    P = synth.linear_precision_ctrl([T] * 3, [p] * 3, (0.25, 1.0, -2.0, 0.5))
    lin = synth.single_block_model(P, [p] * 3, [T] * 3)
    f, g, _ = ob.block_eval_param(lin.blocks[0], u)
    np.testing.assert_allclose(f, 0.25 + u[:, 0] - 2 * u[:, 1] + 0.5 * u[:, 2], atol=1e-14)
    np.testing.assert_allclose(g, np.tile([1.0, -2.0, 0.5], (len(u), 1)), atol=1e-12)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_values_and_partials_match_scipy_ndbspline(p):
    rng = np.random.default_rng(50 + p)
    ns = (p + 4, p + 7, p + 5)
    knots = [synth.clamped_uniform_knots(ns[0], p), nonuniform_knots(ns[1], p, rng),
             synth.clamped_uniform_knots(ns[2], p)]
    P = rng.standard_normal(ns)
    model = synth.single_block_model(P, [p] * 3, knots)
    u = rng.random((600, 3))
    f, g, _ = ob.block_eval_param(model.blocks[0], u)
    nd = NdBSpline(tuple(knots), P, p)
    np.testing.assert_allclose(f, nd(u), rtol=0, atol=1e-13)
    for a in range(3):
        nu = [0, 0, 0]
        nu[a] = 1
        ref = nd(u, nu=nu)
        np.testing.assert_allclose(g[:, a], ref, rtol=0, atol=1e-11 * np.max(np.abs(ref)))


def test_world_gradient_vs_central_differences():
    model = synth.model_c1()
    blk = model.blocks[0]
    h = 1.0 / (16 - 3)
    eta = 1e-4 * h
    rng = np.random.default_rng(5)
    x = rng.uniform(0.02, 0.98, size=(400, 3))
    # keep 2*eta away from knots
    frac = (x / h) % 1.0
    ok = np.all((frac > 2 * eta / h) & (frac < 1 - 2 * eta / h), axis=1)
    x = x[ok]
    r = ob.evaluate(model, x)
    fd = np.zeros_like(x)
    for a in range(3):
        e = np.zeros(3)
        e[a] = eta
        fd[:, a] = (ob.evaluate(model, x + e)["f"] - ob.evaluate(model, x - e)["f"]) / (2 * eta)
    G = np.max(np.abs(r["grad"]))
    assert np.max(np.abs(r["grad"] - fd)) <= 1e-7 * G
    assert blk.ctrl.shape == (16, 16, 16)


def test_affine_world_map_gradient_units():
    p, n = 3, 8
    T = synth.clamped_uniform_knots(n, p)
    P = synth.linear_precision_ctrl([T] * 3, [p] * 3, (1.0, 3.0, -1.0, 2.0))
    lo, hi = np.array([-1.0, 0.5, 2.0]), np.array([1.0, 0.75, 6.0])
    model = synth.single_block_model(P, [p] * 3, [T] * 3, lo=lo, hi=hi)
    rng = np.random.default_rng(9)
    x = lo + rng.random((300, 3)) * (hi - lo)
    r = ob.evaluate(model, x)
    u = (x - lo) / (hi - lo)
    np.testing.assert_allclose(r["f"], 1 + 3 * u[:, 0] - u[:, 1] + 2 * u[:, 2], atol=1e-13)
    np.testing.assert_allclose(r["grad"], np.tile(np.array([3.0, -1.0, 2.0]) / (hi - lo), (len(x), 1)),
                               rtol=1e-12)


def scalar_map(model, x):
    """D1 + D3 by plain Python loops over the edge lists."""
    bids, us = [], []
    for a in range(3):
        E = [float(e) for e in model.edges[a]]
        G = model.grid[a]
        xa = float(x[a])
        xc = min(max(xa, E[0]), E[G])
        b = 0
        for i in range(G):
            if E[i] <= xc:
                b = i
        ie = 1.0 / (E[b + 1] - E[b])
        ua = (xc - E[b]) * ie
        us.append(min(max(ua, 0.0), 1.0))
        bids.append(b)
    return bids, us


def test_block_owner_and_map_vs_scalar_loop():
    rng = np.random.default_rng(11)
    edges = [np.array([0.0, 0.3, 1.0]), np.array([-0.5, 0.1, 0.2, 0.9]), np.array([0.0, 0.5, 1.0])]
    blocks = []
    for _ in range(2 * 3 * 2):
        n = rng.integers(5, 9, size=3)
        knots = [synth.clamped_uniform_knots(int(k), 3) for k in n]
        blocks.append(synth.BlockSpec([3, 3, 3], knots, rng.standard_normal(tuple(int(k) for k in n))))
    model = synth.ModelSpec([2, 3, 2], np.array([0.0, -0.5, 0.0]), np.array([1.0, 0.9, 1.0]),
                            edges, blocks, voxel=0.01)
    pts = [rng.uniform(-0.7, 1.2, size=3) for _ in range(300)]
    for a in range(3):
        for e in edges[a]:
            v = rng.uniform(0, 1, size=3)
            v[a] = e
            pts.append(v.copy())
            v[a] = np.nextafter(e, -np.inf)
            pts.append(v.copy())
    pts = np.array(pts)
    bids, u, _ = ob.world_to_param(model, pts)
    for k in range(len(pts)):
        b, us = scalar_map(model, pts[k])
        assert list(bids[k]) == b
        assert list(u[k]) == us
    # evaluation by the owning block only
    r = ob.evaluate(model, pts)
    flat = (bids[:, 0] * 3 + bids[:, 1]) * 2 + bids[:, 2]
    for k in range(0, len(pts), 37):
        f1, _, _ = ob.block_eval_param(model.blocks[int(flat[k])], u[k:k + 1])
        assert r["f"][k] == f1[0]


def test_decode_grid_matches_pointwise_evaluation():
    model = synth.model_c1()
    ax = [synth.grid_axis(9), synth.grid_axis(7), synth.grid_axis(5)]
    out = ob.decode_grid(model, ax)
    g = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
    r = ob.evaluate(model, g)
    np.testing.assert_array_equal(out[..., 0].reshape(-1), r["f"])
    np.testing.assert_array_equal(out[..., 1:].reshape(-1, 3), r["grad"])
    idx = np.array([[0, 0, 0], [8, 6, 4], [3, 2, 1]])
    sub = ob.decode_grid(model, ax, out_index=idx)
    for k, (a, b, c) in enumerate(idx):
        np.testing.assert_array_equal(sub[k], out[a, b, c])
