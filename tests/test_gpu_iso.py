"""GPU parity of the first-hit isosurface render (mfa_render_iso) against
the FP64 oracle (oracle.render.render_iso), through the C ABI.

Decisions: the schedule K per ray is exact (FP64 on both sides).  The hit
sample is decided by FP32 values on the GPU and FP64 values in the oracle,
so it must be equal on every ray whose examined samples all lie farther
than a band from the level: 2 x the FP32 value tolerance (1e-5 x max|P|,
normwise).  A ray whose GPU hit differs from the oracle's has a sample on
the other side in one of the two, so its oracle margin is within the band:
the rule cannot hide a wrong decision outside it.

Continuous results on the rays outside the band:
* depth: w = (iso - fa) / (fb - fa) moves by at most 2 tol / |fb - fa| when
  fa, fb move by tol, so |t*_gpu - t*_ref| <= step (2 tol / |fb - fa| + 1e-6);
* colour: the GPU's shading at its own hit point against the oracle's
  shading at that same point.  With the gradient within 1e-5 G (G the
  largest oracle gradient component at the hit points), the unit normal
  moves by at most 2 sqrt(3) 1e-5 G / max(|g|, g0) and the colour by
  (kd + ks m) times that (rgb <= 1), plus 1e-5 for FP32 shading.
"""
import numpy as np
import pytest

import synth
from oracle import render as orr
from tests.gpu_common import announce
from tests.test_gpu_parity import small_multiblock

pytestmark = pytest.mark.gpu

RGB = (0.9, 0.7, 0.4)
TOL = 1e-5


@pytest.fixture(scope="module")
def mfa():
    import paper_2312_15073_amd as m
    return m


def iso_level(model, frac):
    lo, hi = model.ctrl_min_max()
    return float(np.float32(lo + frac * (hi - lo)))


def check_iso(model, cam, params, W, H, iso, got, ref, pix_flat=None):
    rgba, depth, ns, ne = got
    rgba, depth = rgba.reshape(-1, 4), depth.reshape(-1)
    ns, ne = ns.reshape(-1, 2), ne.reshape(-1)
    if pix_flat is not None:
        rgba, depth, ns, ne = rgba[pix_flat], depth[pix_flat], ns[pix_flat], ne[pix_flat]
    maxP = max(float(np.abs(b.ctrl).max()) for b in model.blocks)
    tol_f = TOL * maxP
    np.testing.assert_array_equal(ns[:, 0], ref["K"])                       # schedule: exact
    hit = ns[:, 1]
    out = ref["margin"] > 2 * tol_f
    np.testing.assert_array_equal(hit[out], ref["hit"][out])
    assert (~out).sum() <= 0.02 * len(out) + 2, f"{(~out).sum()} rays in the band"
    miss = out & (ref["hit"] < 0)
    assert np.all(rgba[miss] == 0.0) and np.all(np.isinf(depth[miss]))
    h = np.nonzero(out & (ref["hit"] >= 0))[0]
    step = float(params["step"])
    slope = np.abs(ref["fb"][h] - ref["fa"][h])
    dd = np.abs(depth[h] - ref["depth"][h])
    assert np.all(dd <= step * (2 * tol_f / slope + 1e-6)), f"depth error {dd.max():.3e}"
    # shading at the GPU's own hit point, by the oracle
    o, d = orr.pixel_rays(cam, W, H, pixels=None if pix_flat is None else
                          np.stack([pix_flat // W, pix_flat % W], axis=1))
    x = o[h] + depth[h][:, None] * d[h]
    _, g = orr.model_field(model)(x)
    L = -d[h] / np.sqrt((d[h] * d[h]).sum(axis=1))[:, None]
    want = orr.phong(np.tile(RGB, (len(h), 1)), g, L, params["ka"], params["kd"], params["ks"],
                     params["g0"], params["shininess"])
    G = np.abs(g).max()
    gn = np.maximum(np.sqrt((g * g).sum(axis=1)), float(params["g0"]))
    fac = float(params["kd"]) + float(params["ks"]) * params["shininess"]
    tol_c = fac * 2 * np.sqrt(3) * TOL * G / gn + 1e-5
    err = np.abs(rgba[h, :3] - want).max(axis=1)
    assert np.all(err <= tol_c), f"colour error {err.max():.3e}"
    assert np.all(rgba[h, 3] == 1.0)
    return dict(hits=len(h), band=int((~out).sum()), evaluated=int(ne.sum()))


def run(mfa, dev, model, cam, params, W, H, iso, storage="f32"):
    with mfa.Model(model, storage) as M:
        got = mfa.render_iso(M, cam, params, W, H, iso, RGB, debug=True, device=dev)
        got = [t.cpu().numpy() for t in got]
    ref = orr.render_iso(orr.model_field(model), model.lo, model.hi, cam, params, W, H, iso, RGB)
    return got, ref


@pytest.mark.parametrize("kind", ["ortho", "persp"])
@pytest.mark.parametrize("frac", [0.3, 0.55])
def test_iso_c1_matches_oracle(mfa, dev, kind, frac):
    model = synth.model_c1()
    W, H = 64, 48
    cam = (synth.ortho_camera(W, H) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=-35, el_deg=30))
    params = synth.render_params(model)
    iso = iso_level(model, frac)
    announce(f"iso c1 {kind} {W}x{H} level {frac}")
    got, ref = run(mfa, dev, model, cam, params, W, H, iso)
    r = check_iso(model, cam, params, W, H, iso, got, ref)
    assert r["hits"] > 100


@pytest.mark.parametrize("p", [2, 5])
def test_iso_degrees_and_ragged_image(mfa, dev, p):
    model = synth.model_c1(p=p)
    W, H = 37, 29
    cam = synth.perspective_camera(W, H, az_deg=200, el_deg=-20)
    params = synth.render_params(model)
    iso = iso_level(model, 0.4)
    announce(f"iso c1 p={p} {W}x{H}")
    got, ref = run(mfa, dev, model, cam, params, W, H, iso)
    check_iso(model, cam, params, W, H, iso, got, ref)


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_iso_multiblock(mfa, dev, kind):
    model = small_multiblock()
    W, H = 48, 40
    cam = (synth.ortho_camera(W, H, az_deg=50, el_deg=25) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=-40, el_deg=30))
    params = synth.render_params(model)
    iso = iso_level(model, 0.35)
    announce(f"iso multiblock {kind}")
    got, ref = run(mfa, dev, model, cam, params, W, H, iso)
    r = check_iso(model, cam, params, W, H, iso, got, ref)
    assert r["hits"] > 50


def test_iso_strongly_graded_knots(mfa, dev):
    """A single block with strongly graded knots runs the general kernels
    (span guess tables, leaps through the stored knots)."""
    from tests.test_gpu_parity import graded_knots
    p, ns = 3, (33, 27, 30)
    knots = [graded_knots(n, p, 4, phase=a) for a, n in enumerate(ns)]
    F = synth.field_c1()
    g = [synth.greville(T, p, n) for T, n in zip(knots, ns)]
    X = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    model = synth.single_block_model(F.value(X).reshape(ns), [p] * 3, knots, voxel=1.0 / 63)
    W, H = 56, 44
    cam = synth.perspective_camera(W, H, az_deg=150, el_deg=20)
    params = synth.render_params(model)
    iso = iso_level(model, 0.3)
    announce("iso strongly graded knots")
    got, ref = run(mfa, dev, model, cam, params, W, H, iso)
    r = check_iso(model, cam, params, W, H, iso, got, ref)
    assert r["hits"] > 100


def test_iso_outside_the_value_range_evaluates_nothing(mfa, dev):
    """Every macro cell's bounds lie below (above) the level: no sample is
    evaluated, no surface is hit."""
    model = synth.model_c1()
    W, H = 40, 30
    cam = synth.perspective_camera(W, H)
    params = synth.render_params(model)
    lo, hi = model.ctrl_min_max()
    announce("iso outside the value range")
    with mfa.Model(model, "f32") as M:
        for iso in (hi + 0.5 * (hi - lo), lo - 0.5 * (hi - lo)):
            rgba, depth, ns, ne = [t.cpu().numpy() for t in
                                   mfa.render_iso(M, cam, params, W, H, iso, RGB, debug=True,
                                                  device=dev)]
            assert np.all(rgba == 0.0) and np.all(np.isinf(depth))
            assert np.all(ns[..., 1] == -1) and ne.sum() == 0
            assert ns[..., 0].sum() > 10000


def test_iso_arguments(mfa, dev):
    model = synth.model_c1()
    params = synth.render_params(model)
    cam = synth.perspective_camera(8, 8)
    with mfa.Model(model, "f32") as M:
        with pytest.raises(mfa.MFAError):
            mfa.render_iso(M, cam, params, 8, 8, float("nan"), RGB, device=dev)
        with pytest.raises(mfa.MFAError):
            mfa.render_iso(M, cam, params, 8, 8, 0.5, (1.0, float("inf"), 0.0), device=dev)
        with pytest.raises(mfa.MFAError):
            mfa.render_iso(M, cam, params, 0, 8, 0.5, RGB, device=dev)


def test_iso_c2_1024_sampled(mfa, dev):
    """The 128^3 model's 1024^2 perspective frame, checked on sampled pixels."""
    model = synth.model_c2()
    W = H = 1024
    cam = synth.perspective_camera(W, H)
    params = synth.render_params(model)
    iso = iso_level(model, 0.3)
    announce("iso c2 1024x1024 (sampled)")
    with mfa.Model(model, "f32") as M:
        got = [t.cpu().numpy() for t in
               mfa.render_iso(M, cam, params, W, H, iso, RGB, debug=True, device=dev)]
    rng = np.random.default_rng(9)
    pix = np.stack([rng.integers(0, H, 300), rng.integers(0, W, 300)], axis=1)
    pix = np.concatenate([pix, [[0, 0], [H - 1, W - 1], [H // 2, W // 2]]])
    ref = orr.render_iso(orr.model_field(model), model.lo, model.hi, cam, params, W, H, iso, RGB,
                         pixels=pix)
    flat = pix[:, 0] * W + pix[:, 1]
    r = check_iso(model, cam, params, W, H, iso, got, ref, pix_flat=flat)
    assert r["hits"] > 50
    assert (got[2][..., 1] >= 0).sum() > 100000       # a real frame: many hits
