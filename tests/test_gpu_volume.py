"""GPU parity of the local-filter volume renders and of the analytic
Marschner-Lobb render (mfa_render_volume) against the FP64 oracle
(oracle.render.render with oracle.filters fields), through the C ABI.

The acceptance is that of the MFA renders: K per ray exact; samples used
equal to an exact FP32 replay of the kernel's own opacities, and to the
oracle's outside the termination band (in-band rays within one sample);
image RMSE <= 1e-5 and max-abs <= 1e-3 outside the band.  The grid
coordinate of a sample is taken in FP64 on both sides (the oracle divides
by h, the kernel multiplies by the host's 1 / h): at a cell face the two
may pick neighbouring cells, between which the filters are continuous.
"""
import numpy as np
import pytest

import synth
from oracle import filters as of
from oracle import render as orr
from tests.gpu_common import announce, composite_band

pytestmark = pytest.mark.gpu

KINDS = {"trilinear": of.TRILINEAR, "catmull_rom": of.CATMULL_ROM, "cubic_bspline": of.BSPLINE3}


@pytest.fixture(scope="module")
def mfa():
    import paper_2312_15073_amd as m
    return m


def smooth_volume(N, seed):
    field = synth.field_c1(seed)
    ax = [np.linspace(0.0, 1.0, n) for n in N]
    return field.value_separable(*ax).astype(np.float32)


def params_for(vmin, vmax, step, max_samples=512):
    p = dict(tf=synth.tf_table_A(), vmin=np.float32(vmin), vmax=np.float32(vmax), step=float(step),
             max_samples=max_samples, ert_alpha=np.float32(0.99), ka=np.float32(0.3),
             kd=np.float32(0.6), ks=np.float32(0.3), shininess=16)
    p["g0"] = np.float32(0.01 * (float(p["vmax"]) - float(p["vmin"])))
    return p


def check(mfa, dev, samples, kind, lo, hi, cam, params, W, H, field, dims=None, tol_rmse=1e-5,
          tol_max=1e-3):
    import torch
    vol = None if samples is None else torch.as_tensor(samples).to(dev)
    rgba, ns, al = mfa.render_volume(vol, kind, lo, hi, cam, params, W, H, dims=dims, nsamp=True,
                                     alpha=True, device=dev)
    rgba, ns, al = rgba.cpu().numpy().reshape(-1, 4), ns.cpu().numpy().reshape(-1, 2), al.cpu().numpy()
    ref = orr.render(field, lo, hi, cam, params, W, H, record_alpha=True)
    K, used = ns[:, 0], ns[:, 1]
    np.testing.assert_array_equal(K, ref["K"])
    rep = orr.ert_replay_f32(al.reshape(W * H, -1), K, params["ert_alpha"])
    np.testing.assert_array_equal(used, rep)
    band = composite_band(ref["alpha"], ref["used"], float(params["ert_alpha"]))
    out = ~band
    np.testing.assert_array_equal(used[out], ref["used"][out])
    assert np.all(np.abs(used[band] - ref["used"][band]) <= 1)
    diff = np.abs(rgba[out] - ref["rgba"][out])
    rmse = float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0
    assert rmse <= tol_rmse, f"image RMSE {rmse:.3e}"
    assert diff.max(initial=0.0) <= tol_max, f"image max-abs {diff.max():.3e}"
    assert ref["rgba"][:, 3].max() > 0.3                    # a real image
    return dict(band=int(band.sum()), rmse=rmse)


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("cam_kind", ["ortho", "persp"])
def test_filters_match_oracle(mfa, dev, kind, cam_kind):
    N = (21, 17, 24)
    V = smooth_volume(N, seed=3)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    W, H = 48, 40
    cam = (synth.ortho_camera(W, H, az_deg=40, el_deg=25) if cam_kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=-60, el_deg=35))
    params = params_for(V.min(), V.max(), step=1.0 / 80)
    announce(f"volume {kind} {cam_kind}")
    check(mfa, dev, V, kind, lo, hi, cam, params, W, H,
          of.grid_field(V.astype(np.float64), lo, hi, KINDS[kind]))


def test_filters_on_a_non_unit_box_and_axis_aligned_rays(mfa, dev):
    N = (9, 12, 10)
    V = smooth_volume(N, seed=4)
    lo, hi = (-1.0, 2.0, 0.5), (2.0, 3.5, 4.0)
    W, H = 24, 20
    cam = dict(kind=synth.ORTHO, eye=np.array([0.5, 2.75, -5.0]), forward=np.array([0.0, 0.0, 1.0]),
               right=np.array([1.0, 0.0, 0.0]), up=np.array([0.0, 1.0, 0.0]), sx=1.6 / W, sy=0.8 / H)
    params = params_for(V.min(), V.max(), step=0.02)
    announce("volume non-unit box, axis-aligned rays")
    for kind in KINDS:
        check(mfa, dev, V, kind, lo, hi, cam, params, W, H,
              of.grid_field(V.astype(np.float64), lo, hi, KINDS[kind]))


def test_marschner_lobb_field_matches_oracle(mfa, dev):
    """The analytic field in FP32 (sines and cosines of arguments up to
    12 pi): the value is within ~1e-6 of the FP64 oracle, the gradient
    (magnitude up to ~10) within ~1e-5 relative, so the image keeps the
    render tolerances."""
    W, H = 40, 32
    cam = synth.perspective_camera(W, H, az_deg=30, el_deg=20, dist=14.0,
                                   centre=(3.5, 3.5, 3.5))
    params = params_for(0.0, 1.0, step=7.0 / 255 / 2, max_samples=1024)
    announce("volume Marschner-Lobb analytic")
    check(mfa, dev, None, "marschner_lobb", of.ML_LO, of.ML_HI, cam, params, W, H, of.ml_value_grad,
          dims=(256, 256, 256))


def test_marschner_lobb_samples_through_filters(mfa, dev):
    N = 48
    V = of.ml_samples(N).astype(np.float32)
    W, H = 32, 32
    cam = synth.ortho_camera(W, H, half_extent=4.5, dist=14.0, centre=(3.5, 3.5, 3.5))
    params = params_for(0.0, 1.0, step=7.0 / (N - 1) / 2)
    announce("volume Marschner-Lobb 48^3 through the filters")
    for kind in KINDS:
        check(mfa, dev, V, kind, of.ML_LO, of.ML_HI, cam, params, W, H,
              of.grid_field(V.astype(np.float64), of.ML_LO, of.ML_HI, KINDS[kind]))
