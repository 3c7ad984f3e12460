"""Pins of the oracle's first-hit isosurface renderer (CPU only).

Each test checks render_iso against something other than its own steps: a
plane (linear field) whose hit sample, depth and shading have closed forms;
a sphere (quadratic field) whose depth must lie within the error bound of
linear interpolation between two samples; a scalar re-evaluation of every
ray on tiny images; and the no-hit cases.
"""
import math

import numpy as np
import pytest

import synth
from oracle import bspline as ob
from oracle import render as orr

RGB = (0.9, 0.6, 0.3)


def params_for(step, max_samples=1024):
    return dict(step=step, max_samples=max_samples, ka=0.3, kd=0.6, ks=0.3, g0=1e-6, shininess=16)


def linear_field(a, b):
    def fn(x):
        return a * x[:, 0] + b, np.tile([a, 0.0, 0.0], (x.shape[0], 1))
    return fn


@pytest.mark.parametrize("a,b,xs", [(2.5, -0.3, 0.437), (-1.5, 0.9, 0.6123), (0.8, 0.0, 0.05)])
def test_plane_hit_sample_depth_and_shading_closed_form(a, b, xs):
    """f = a x0 + b seen along +x: every ray enters the box at t_near = 1.5
    (eye 2 in front of the centre), samples sit at x0 = (k + 1/2) dt, the
    first sample past x0 = xs is the hit, linear interpolation is exact, so
    t* = 1.5 + xs, and the normal is the view axis: diff = 1."""
    W, H, dt = 7, 5, 1.0 / 100
    cam = synth.axis_camera(W, H, axis=0, half_extent=0.45)
    iso = a * xs + b
    out = orr.render_iso(linear_field(a, b), (0, 0, 0), (1, 1, 1), cam, params_for(dt), W, H, iso, RGB)
    k_want = math.ceil(xs / dt - 0.5)
    assert np.all(out["hit"] == k_want)
    np.testing.assert_allclose(out["depth"], 1.5 + xs, rtol=0, atol=1e-12)
    c = [v * (0.3 + 0.6) + 0.3 for v in RGB]
    np.testing.assert_allclose(out["rgba"], np.tile([*c, 1.0], (W * H, 1)), rtol=0, atol=1e-12)


def test_plane_through_a_spline_model_with_linear_precision():
    """The same closed form through the B-spline oracle: control points at
    the Greville abscissae reproduce f = u0 exactly (linear precision)."""
    p, n = 3, (9, 6, 7)
    knots = [synth.clamped_uniform_knots(n[a], p) for a in range(3)]
    xi = synth.greville(knots[0], p, n[0])
    C = np.broadcast_to(xi[:, None, None], n).copy()
    model = synth.single_block_model(C, [p] * 3, knots)
    W, H, dt = 5, 4, 1.0 / 64
    cam = synth.axis_camera(W, H, axis=0, half_extent=0.4)
    out = orr.render_iso(orr.model_field(model), model.lo, model.hi, cam, params_for(dt), W, H,
                         0.3, RGB)
    assert np.all(out["hit"] == math.ceil(0.3 / dt - 0.5))
    np.testing.assert_allclose(out["depth"], 1.8, rtol=0, atol=1e-12)


def sphere_field(c, scale=1.0):
    c = np.asarray(c, np.float64)

    def fn(x):
        r = x - c
        return scale * (r * r).sum(axis=1), 2.0 * scale * r
    return fn


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_sphere_depth_within_linear_interpolation_bound(kind):
    """phi(t) = |o + t d - c|^2 - r^2 is quadratic along a ray; the root t*
    of the linear interpolant between the bracketing samples satisfies
    |t* - t0| <= |d|^2 dt^2 / (4 min |phi'|) over the bracket."""
    W, H, dt = 40, 32, 1.0 / 50
    cam = (synth.ortho_camera(W, H, half_extent=0.5) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=70, el_deg=-15))
    c, r = np.array([0.52, 0.47, 0.5]), 0.3
    out = orr.render_iso(sphere_field(c), (0, 0, 0), (1, 1, 1), cam, params_for(dt), W, H, r * r, RGB)
    o, d = orr.pixel_rays(cam, W, H)
    t_near, t_far, miss = orr.slab(o, d, (0, 0, 0), (1, 1, 1))
    oc = o - c
    A = (d * d).sum(1)
    B = 2 * (d * oc).sum(1)
    Cq = (oc * oc).sum(1) - r * r
    disc = B * B - 4 * A * Cq
    hits = 0
    for q in range(W * H):
        if disc[q] <= 0 or miss[q]:
            assert out["hit"][q] == -1
            continue
        t0 = (-B[q] - math.sqrt(disc[q])) / (2 * A[q])
        t1 = (-B[q] + math.sqrt(disc[q])) / (2 * A[q])
        ks = [k for k in range(out["K"][q]) if t0 < t_near[q] + (k + 0.5) * dt < t1]
        if not ks:                      # the chord falls between two samples
            assert out["hit"][q] == -1
            continue
        k = ks[0]
        if abs(t_near[q] + (k + 0.5) * dt - t0) < 1e-9:
            continue                    # a sample on the surface: either side is right
        assert out["hit"][q] == k
        lo_t, hi_t = t_near[q] + (k - 0.5) * dt, t_near[q] + (k + 0.5) * dt
        dphi = [abs(2 * A[q] * t + B[q]) for t in (lo_t, hi_t)]
        bound = A[q] * dt * dt / (4 * min(dphi))
        assert abs(out["depth"][q] - t0) <= bound * (1 + 1e-9) + 1e-12
        hits += 1
        # shading with the exact normal at the exact hit (a change of order dt^2)
        n = (o[q] + t0 * d[q] - c) / r
        L = -d[q] / math.sqrt(A[q])
        diff = abs(float(n @ L))
        want = np.array(RGB) * (0.3 + 0.6 * diff) + 0.3 * diff ** 16
        np.testing.assert_allclose(out["rgba"][q, :3], want, rtol=0, atol=50 * bound + 1e-9)
    assert hits > 80


def brute_force_iso(model, cam, params, W, H, iso, rgb):
    """Scalar Python re-evaluation of every ray and sample (tiny images)."""
    lo, hi = [float(v) for v in model.lo], [float(v) for v in model.hi]
    eye, fw, rt, up = (list(map(float, cam[k])) for k in ("eye", "forward", "right", "up"))
    dt = float(params["step"])
    img = np.zeros((H * W, 4))
    hits = np.full(H * W, -1)
    depth = np.full(H * W, np.inf)
    for j in range(H):
        for i in range(W):
            px = float(2 * i + 1 - W) * float(cam["sx"])
            py = float(H - 2 * j - 1) * float(cam["sy"])
            if cam["kind"] == synth.ORTHO:
                o = [(eye[a] + px * rt[a]) + py * up[a] for a in range(3)]
                d = list(fw)
            else:
                o = list(eye)
                d = [(fw[a] + px * rt[a]) + py * up[a] for a in range(3)]
            tn, tfar, miss = 0.0, math.inf, False
            for a in range(3):
                if d[a] == 0.0:
                    miss |= o[a] < lo[a] or o[a] > hi[a]
                    continue
                inv = 1.0 / d[a]
                t1, t2 = (lo[a] - o[a]) * inv, (hi[a] - o[a]) * inv
                tn, tfar = max(tn, min(t1, t2)), min(tfar, max(t1, t2))
            miss |= tn >= tfar
            K = 0 if miss else int(min(math.floor((tfar - tn) / dt), params["max_samples"]))
            prev = None
            for k in range(K):
                t = tn + (k + 0.5) * dt
                f = float(ob.evaluate(model, np.array([[o[a] + t * d[a] for a in range(3)]]))["f"][0])
                if prev is not None and (f >= iso) != (prev >= iso):
                    w = (iso - prev) / (f - prev)
                    ts = tn + ((k - 1) + 0.5 + w) * dt
                    g = [float(v) for v in ob.evaluate(
                        model, np.array([[o[a] + ts * d[a] for a in range(3)]]))["grad"][0]]
                    nd = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
                    gn = max(math.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]), float(params["g0"]))
                    dif = abs(sum((g[a] / gn) * (-d[a] / nd) for a in range(3)))
                    sh = float(params["ka"]) + float(params["kd"]) * dif
                    img[j * W + i] = [rgb[c] * sh + float(params["ks"]) * dif ** params["shininess"]
                                      for c in range(3)] + [1.0]
                    hits[j * W + i] = k
                    depth[j * W + i] = ts
                    break
                prev = f
    return img, hits, depth


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_vectorised_iso_matches_scalar_brute_force(kind):
    model = synth.model_c1()
    W, H = 6, 5
    cam = (synth.ortho_camera(W, H, half_extent=0.7) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=130, el_deg=25))
    params = synth.render_params(model, step=1.0 / 40)
    lo, hi = model.ctrl_min_max()
    iso = lo + 0.3 * (hi - lo)
    out = orr.render_iso(orr.model_field(model), model.lo, model.hi, cam, params, W, H, iso, RGB)
    img, hits, depth = brute_force_iso(model, cam, params, W, H, iso, RGB)
    np.testing.assert_array_equal(out["hit"], hits)
    np.testing.assert_allclose(out["depth"], depth, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["rgba"], img, rtol=0, atol=1e-13)
    assert (hits >= 0).sum() >= 5 and (hits < 0).sum() >= 1


def test_no_surface_outside_the_value_range_and_margin_is_the_closest_sample():
    model = synth.model_c1()
    W, H = 9, 7
    cam = synth.perspective_camera(W, H)
    params = synth.render_params(model, step=1.0 / 30)
    lo, hi = model.ctrl_min_max()
    field = orr.model_field(model)
    for iso in (hi + 0.1, lo - 0.1):        # convex hull: f never reaches iso
        out = orr.render_iso(field, model.lo, model.hi, cam, params, W, H, iso, RGB)
        assert np.all(out["hit"] == -1) and np.all(np.isinf(out["depth"]))
        assert np.all(out["rgba"] == 0.0)
    iso = lo + 0.5 * (hi - lo)
    out = orr.render_iso(field, model.lo, model.hi, cam, params, W, H, iso, RGB)
    o, d = orr.pixel_rays(cam, W, H)
    for q in range(W * H):                  # margin: min |f_j - iso| over the samples examined
        n = out["hit"][q] + 1 if out["hit"][q] >= 0 else out["K"][q]
        if n == 0:
            assert np.isinf(out["margin"][q])
            continue
        tn = orr.slab(o[q:q + 1], d[q:q + 1], model.lo, model.hi)[0][0]
        x = o[q] + (tn + (np.arange(n) + 0.5) * params["step"])[:, None] * d[q]
        assert out["margin"][q] == np.abs(field(x)[0] - iso).min()
