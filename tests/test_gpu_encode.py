"""GPU parity of the fixed-knot encoder (mfa_encode_grid) against the FP64
oracle (oracle.encode.fit_grid), through the C ABI.

Tolerance: both sides compute in FP64 (the samples are FP32, promoted
exactly), by different routes (SVD pseudo-inverse and tensordot in the
oracle; Cholesky of the Gram matrix, banded solves and matrix-core GEMMs on
the device).
The Gram matrices of these collocation matrices have condition numbers
below ~1e4 and each control point sums at most ~1e6 products, so the two
agree to ~1e-12 of max|F|; the bound is set at 1e-10 of max|F|, normwise.
"""
import numpy as np
import pytest

import synth
from oracle import encode as oe
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu

REL_ENC = 1e-10


@pytest.fixture(scope="module")
def mfa():
    import paper_2312_15073_amd as m
    return m


def spaced_knots(n, p, rng):
    m = n - p
    inner = (np.arange(1, m) + rng.uniform(-0.3, 0.3, size=m - 1)) / m
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def run_case(mfa, dev, F32, axis_u, degree, n_ctrl, knots, work=None):
    import torch
    vals = torch.as_tensor(np.ascontiguousarray(F32, dtype=np.float32)).to(dev)
    P = mfa.encode_grid(vals, axis_u, degree, n_ctrl, knots=knots, work=work)
    torch.cuda.synchronize()
    kn = [synth.clamped_uniform_knots(n_ctrl[a], degree[a]) if knots is None or knots[a] is None
          else knots[a] for a in range(3)]
    ref = oe.fit_grid(F32.astype(np.float64), axis_u, degree, kn, n_ctrl)
    got = P.cpu().numpy()
    err = np.abs(got - ref).max()
    tol = REL_ENC * np.abs(F32).max()
    assert err <= tol, f"control-point error {err:.3e} > {tol:.3e}"
    return got


def test_encode_compressed_model_128_to_48(mfa, dev):
    # the compressed model's workload: 8-Gaussian field sampled on 128^3
    # (+1 % uniform noise) fitted with 48^3 control points, degree 3
    field = synth.field_c1(1)
    xs = np.arange(128, dtype=np.float64) / 127
    F = field.value_separable(xs, xs, xs)
    rng = np.random.default_rng(4)
    F = (F + rng.uniform(-0.01, 0.01, size=F.shape) * float(F.max() - F.min())).astype(np.float32)
    announce("encode 128^3 -> 48^3 p=3")
    run_case(mfa, dev, F, [xs, xs, xs], (3, 3, 3), (48, 48, 48), None)


def test_encode_ragged_sizes_random_parameters_nonuniform_knots(mfa, dev):
    # GEMM edges: M, N not multiples of the 32-wide tiles, K not a multiple
    # of 4; parameters unsorted; a different degree per axis
    rng = np.random.default_rng(5)
    res, degree, n_ctrl = (37, 50, 29), (2, 3, 4), (9, 17, 6)
    axis_u = []
    for a in range(3):
        u = np.linspace(0.0, 1.0, res[a])
        axis_u.append(rng.permutation(u))
    knots = [spaced_knots(n_ctrl[a], degree[a], rng) for a in range(3)]
    F = rng.standard_normal(res).astype(np.float32)
    announce("encode ragged 37x50x29")
    run_case(mfa, dev, F, axis_u, degree, n_ctrl, knots)


@pytest.mark.parametrize("p0", [1, 7])
def test_encode_banded_first_product_many_fibers(mfa, dev, p0):
    """2^17 fibers (512 x 256 samples along axes 1 and 2) and 90 control
    points along axis 0: the first mode product takes the banded route
    (B0^T F and two banded Cholesky solves per fiber) with the samples of
    axis 0 in shuffled order, non-uniform knots and the smallest and
    largest degree accepted; the other two products stay GEMMs."""
    rng = np.random.default_rng(30 + p0)
    res, degree, n_ctrl = (300, 512, 256), (p0, 3, 2), (90, 40, 33)
    axis_u = [rng.permutation(np.linspace(0.0, 1.0, res[0])), np.linspace(0.0, 1.0, res[1]),
              np.linspace(0.0, 1.0, res[2])]
    knots = [spaced_knots(n_ctrl[0], p0, rng), None, None]
    F = rng.standard_normal(res).astype(np.float32)
    announce(f"encode banded first product 300x512x256 p0={p0}")
    run_case(mfa, dev, F, axis_u, degree, n_ctrl, knots)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_encode_degrees(mfa, dev, p):
    rng = np.random.default_rng(10 + p)
    res = (3 * (p + 6), 2 * (p + 8), 40)
    n_ctrl = (p + 6, p + 8, 13)
    axis_u = [np.linspace(0.0, 1.0, r) for r in res]
    F = rng.uniform(-2.0, 3.0, size=res).astype(np.float32)
    announce(f"encode p={p}")
    run_case(mfa, dev, F, axis_u, (p, p, p), n_ctrl, None)


def test_encode_reproduces_spline_and_reuses_workspace(mfa, dev):
    """Samples of a spline of the fitted space come back as its control
    points; the second call reuses the first call's (larger) workspace."""
    import torch
    from oracle import bspline as ob
    rng = np.random.default_rng(20)
    p, n = 3, (10, 12, 8)
    knots = [spaced_knots(n[a], p, rng) for a in range(3)]
    C0 = rng.standard_normal(n)
    model = synth.single_block_model(C0, [p] * 3, knots)
    axis_u = [np.linspace(0.0, 1.0, 3 * n[a]) for a in range(3)]
    F = ob.decode_grid(model, axis_u)[..., 0].astype(np.float32)
    big = mfa.encode_workspace_bytes((64, 64, 64), (20, 20, 20))
    work = torch.zeros((big,), dtype=torch.uint8, device=dev)
    announce("encode spline reproduction, shared workspace")
    run_case(mfa, dev, rng.standard_normal((64, 64, 64)).astype(np.float32),
             [np.linspace(0, 1, 64)] * 3, (3, 3, 3), (20, 20, 20), None, work=work)
    got = run_case(mfa, dev, F, axis_u, (p, p, p), n, knots, work=work)
    # F holds the spline rounded to FP32: the fit reproduces C0 to that rounding
    assert np.abs(got - C0).max() <= 1e-5 * np.abs(C0).max()


def test_encode_plan_serves_several_blocks(mfa, dev):
    """One plan, eight octant blocks of one volume (the partition of
    Sec. IV-A1): each apply equals the oracle fit of its block."""
    import torch
    rng = np.random.default_rng(30)
    res, n_ctrl = (24, 20, 28), (10, 9, 12)
    axis_u = [np.linspace(0.0, 1.0, r) for r in res]
    announce("encode plan, 8 blocks")
    plan = mfa.EncodePlan(res, axis_u, (3, 3, 3), n_ctrl, device=dev)
    blocks = [rng.standard_normal(res).astype(np.float32) for _ in range(8)]
    outs = [plan.apply(torch.as_tensor(b).to(dev)) for b in blocks]
    torch.cuda.synchronize()
    kn = [synth.clamped_uniform_knots(n, 3) for n in n_ctrl]
    for b, o in zip(blocks, outs):
        ref = oe.fit_grid(b.astype(np.float64), axis_u, (3, 3, 3), kn, n_ctrl)
        assert np.abs(o.cpu().numpy() - ref).max() <= REL_ENC * np.abs(b).max()


# ---------------------------------------------------------------- knot insertion (Fig. 1)
def oracle_adaptive_with_margin(F64, axis_u, degree, n_init, e_max, max_iter, max_ctrl, margin=1e-6):
    """The oracle's adaptive fit, checking that no span error of any pass
    lies within a relative margin of e_max (there the two sides' FP64
    rounding could take different split decisions)."""
    ref = oe.fit_adaptive(F64, axis_u, degree, n_init, e_max, max_iter=max_iter, max_ctrl=max_ctrl)
    rng = float(F64.max() - F64.min()) or 1.0
    for k in range(1, len(ref[2]) + 1):
        kn, P, _ = oe.fit_adaptive(F64, axis_u, degree, n_init, e_max, max_iter=k, max_ctrl=max_ctrl)
        err = np.abs(oe.reconstruct_grid(P, axis_u, degree, kn) - F64) / rng
        for e in oe.span_errors(err, axis_u, degree, kn):
            assert np.all(np.abs(e - e_max) > margin * e_max), "span error at the bound"
    return ref


def run_adaptive(mfa, dev, F32, axis_u, degree, n_init, e_max, max_fits, max_ctrl=None):
    import torch
    F64 = F32.astype(np.float64)
    knots, P, hist = mfa.encode_adaptive(torch.as_tensor(F32).to(dev), axis_u, degree, n_init,
                                         e_max, max_ctrl=max_ctrl, max_fits=max_fits)
    rk, rP, rh = oracle_adaptive_with_margin(F64, axis_u, degree, n_init, e_max, max_fits, max_ctrl)
    for a in range(3):
        np.testing.assert_array_equal(knots[a], rk[a])                  # same split decisions
    assert [h[0] for h in hist] == [tuple(h[0]) for h in rh]
    for (_, e), (_, re) in zip(hist, rh):
        assert abs(e - re) <= 1e-9 * max(re, 1e-12)
    got = P.cpu().numpy()
    assert got.shape == rP.shape
    assert np.abs(got - rP).max() <= REL_ENC * np.abs(F32).max()
    return knots, hist


def test_encode_adaptive_gaussian_field_reaches_the_bound(mfa, dev):
    field = synth.field_c1(1)
    xs = np.arange(48, dtype=np.float64) / 47
    F = field.value_separable(xs, xs, xs).astype(np.float32)
    announce("adaptive encode 48^3 e_max=2e-3")
    knots, hist = run_adaptive(mfa, dev, F, [xs] * 3, (3, 3, 3), (6, 6, 6), 2e-3, 10)
    assert len(hist) >= 2 and hist[-1][1] <= 2e-3


def test_encode_adaptive_ragged_unsorted_mixed_degrees_with_cap(mfa, dev):
    rng = np.random.default_rng(90)
    res, degree = (45, 38, 53), (2, 3, 4)
    x = [np.linspace(0.0, 1.0, r) for r in res]
    g = np.meshgrid(*x, indexing="ij")
    F = (np.abs(g[0] - 0.37) ** 2.5 + np.sin(6.0 * g[1]) * g[2] + 0.3 * np.exp(-40 * (g[2] - 0.6) ** 2))
    perm = [rng.permutation(r) for r in res]
    F = F[np.ix_(*perm)].astype(np.float32)                          # samples in shuffled order
    axis_u = [x[a][perm[a]] for a in range(3)]
    announce("adaptive encode ragged 45x38x53, capped")
    knots, hist = run_adaptive(mfa, dev, F, axis_u, degree, (4, 5, 6), 5e-4, 6, max_ctrl=(12, 15, 11))
    assert max(h[0][0] for h in hist) <= 12 and max(h[0][2] for h in hist) <= 11


def test_encode_adaptive_loose_bound_is_one_fixed_knot_fit(mfa, dev):
    rng = np.random.default_rng(91)
    res = (20, 24, 28)
    axis_u = [np.linspace(0.0, 1.0, r) for r in res]
    F = rng.standard_normal(res).astype(np.float32)
    announce("adaptive encode, loose bound")
    knots, hist = run_adaptive(mfa, dev, F, axis_u, (3, 3, 3), (7, 8, 9), 10.0, 4)
    assert len(hist) == 1 and hist[0][0] == (7, 8, 9)


def test_encode_adaptive_long_axes_split_products(mfa, dev):
    """Long axes 1 and 2 with few control points: the fit's second and third
    products have few tiles and run split along K (chunks of 84 and 77, and
    of 68, 68 and 66 values, both with a ragged K tail)."""
    res = (24, 161, 202)
    x = [np.linspace(0.0, 1.0, r) for r in res]
    g = np.meshgrid(*x, indexing="ij")
    F = (np.sin(3.0 * g[0] + 5.0 * g[1]) * np.cos(4.0 * g[2]) + 0.2 * np.exp(-30 * (g[1] - 0.4) ** 2)
         + 0.1 * g[0] * g[2]).astype(np.float32)
    announce("adaptive encode 24x161x202 (split products)")
    knots, hist = run_adaptive(mfa, dev, F, x, (3, 3, 3), (5, 6, 7), 1e-3, 3)
    assert len(hist) >= 2


def test_encode_adaptive_long_axis_y_rows_outside_lds(mfa, dev):
    """1300 control points on axis 2 at degree 3: the inversion's y rows
    (16 x 1300 doubles) exceed the LDS and stay in the output rows; the fit
    still equals the oracle's."""
    rng = np.random.default_rng(92)
    res = (5, 6, 2600)
    x = [np.linspace(0.0, 1.0, r) for r in res]
    g = np.meshgrid(*x, indexing="ij")
    F = (np.sin(40.0 * g[2]) * (1 + g[0]) + 0.5 * g[1] * np.cos(25.0 * g[2])
         + 0.01 * rng.standard_normal(res)).astype(np.float32)
    announce("adaptive encode 5x6x2600, 1300 control points on axis 2")
    knots, hist = run_adaptive(mfa, dev, F, x, (1, 2, 3), (2, 3, 1300), 10.0, 2)
    assert len(hist) == 1 and hist[0][0] == (2, 3, 1300)


def test_encode_adaptive_factor_outside_lds(mfa, dev):
    """5200 control points on axis 2 at degree 3: the factor alone (5200 x 4
    doubles) exceeds the LDS and is read from global memory.  The field is
    constant along axes 0 and 1 (linear there, two control points each), so
    every row of the fit is the 1-D least-squares fit along axis 2, solved
    here from the banded normal equations by scipy."""
    import torch
    from scipy.linalg import solveh_banded
    from scipy.interpolate import BSpline
    res = (3, 3, 10400)
    x = [np.linspace(0.0, 1.0, r) for r in res]
    g2 = np.sin(30.0 * x[2]) + 0.3 * np.cos(170.0 * x[2] ** 2)
    F = np.broadcast_to(g2, res).astype(np.float32).copy()
    n, p = 5200, 3
    announce("adaptive encode 3x3x10400, 5200 control points on axis 2")
    knots, P, hist = mfa.encode_adaptive(torch.as_tensor(F).to(dev), x, (1, 1, p), (2, 2, n), 10.0,
                                         max_ctrl=(2, 2, n), max_fits=1)
    T = synth.clamped_uniform_knots(n, p)
    B = BSpline.design_matrix(x[2], T, p).toarray()
    G = B.T @ B
    ab = np.zeros((p + 1, n))                         # upper banded form of the Gram matrix
    for d in range(p + 1):
        ab[p - d, d:] = np.diagonal(G, d)
    ref = solveh_banded(ab, B.T @ F[0, 0].astype(np.float64))
    got = P.cpu().numpy()
    assert got.shape == (2, 2, n)
    tol = REL_ENC * np.abs(F).max() * 10
    for i in range(2):
        for j in range(2):
            assert np.abs(got[i, j] - ref).max() <= tol
