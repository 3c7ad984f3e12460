"""GPU parity of the object-space split (partial renders of boxes of blocks,
Sec. IV-A4) and of the depth-ordered "over" compositing (Sec. IV-A5)
against the FP64 oracle, through the C ABI.

Keys (FP64 slab entry parameters) must be equal; images follow the render
tolerance (RMSE <= 1e-5 and max-abs <= 1e-3 outside the early-termination
band); the compositing kernel alone is compared at 1e-6 (FP32 "over" of
values in [0, 1]).
"""
import numpy as np
import pytest

import synth
from oracle import render as orr
from tests.gpu_common import announce, composite_band
from tests.test_gpu_parity import small_multiblock, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfa():
    import paper_2312_15073_amd as m
    return m


def region_arg(model, blo, bhi):
    rlo = [model.edges[a][blo[a]] for a in range(3)]
    rhi = [model.edges[a][bhi[a]] for a in range(3)]
    return (orr.block_owner_fn(model), blo, bhi, rlo, rhi)


def partition(model, cuts):
    out = []
    for a0 in ((0, cuts[0]), (cuts[0], model.grid[0])):
        for a1 in ((0, cuts[1]), (cuts[1], model.grid[1])):
            out.append(((a0[0], a1[0], 0), (a0[1], a1[1], model.grid[2])))
    return out


def image_close(got, ref, mask):
    diff = np.abs(got[mask] - ref[mask])
    rmse = float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0
    assert rmse <= 1e-5, f"image RMSE {rmse:.3e}"
    assert diff.max(initial=0.0) <= 1e-3, f"image max-abs {diff.max():.3e}"


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_partial_renders_and_composite_match_oracle(mfa, dev, kind):
    model = small_multiblock()
    W, H = 48, 40
    cam = (synth.ortho_camera(W, H, az_deg=50, el_deg=25) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=-40, el_deg=30))
    params = synth.render_params(model)
    ert = float(params["ert_alpha"])
    field = orr.model_field(model)
    boxes = partition(model, (1, 1))
    announce(f"partial renders 3x2x2 {kind} {W}x{H}, {len(boxes)} regions")
    with mfa.Model(model, "f32") as M:
        gpu = [mfa.render_partial(M, cam, params, W, H, blo, bhi, device=dev) for blo, bhi in boxes]
        comp = mfa.composite_over([g[0] for g in gpu], [g[1] for g in gpu]).cpu().numpy()
        gpu = [(g[0].cpu().numpy().reshape(-1, 4), g[1].cpu().numpy().reshape(-1)) for g in gpu]
    band_all = np.zeros(W * H, dtype=bool)
    refs = []
    for (blo, bhi), (img, key) in zip(boxes, gpu):
        ref = orr.render(field, model.lo, model.hi, cam, params, W, H, record_alpha=True,
                         region=region_arg(model, blo, bhi))
        np.testing.assert_array_equal(key, ref["key"])               # exact FP64 slab entry
        band = composite_band(ref["alpha"], ref["used"], ert)
        band_all |= band
        image_close(img, ref["rgba"], ~band)
        refs.append(ref)
    ref_comp = orr.composite([r["rgba"] for r in refs], [r["key"] for r in refs])
    image_close(comp.reshape(-1, 4), ref_comp, ~band_all)
    multi = sum(np.isfinite(r["key"]).astype(int) for r in refs)
    assert (multi >= 2).sum() > 100                                   # rays cross regions


def test_composite_equals_full_render_without_termination(mfa, dev):
    """Associativity of "over": partials of a partition composited in key
    order give the full frame (termination off), up to FP32 rounding."""
    model = small_multiblock(seed=24)
    W, H = 64, 48
    cam = synth.perspective_camera(W, H, az_deg=120, el_deg=-20)
    params = synth.render_params(model)
    params["ert_alpha"] = 2.0
    announce("composite vs full frame, termination off")
    with mfa.Model(model, "f32") as M:
        full = mfa.render_frame(M, cam, params, W, H, device=dev).cpu().numpy()
        parts = [mfa.render_partial(M, cam, params, W, H, blo, bhi, device=dev)
                 for blo, bhi in partition(model, (2, 1))]
        comp = mfa.composite_over([p[0] for p in parts], [p[1] for p in parts]).cpu().numpy()
    assert np.abs(comp - full).max() <= 1e-5


@pytest.mark.parametrize("G", [1, 5, 16])
def test_composite_kernel_against_oracle(mfa, dev, G):
    import torch
    rng = np.random.default_rng(G)
    H, W = 37, 61
    imgs = rng.uniform(0.0, 1.0, size=(G, H, W, 4)).astype(np.float32)
    imgs[..., :3] *= imgs[..., 3:4]                                   # premultiplied
    keys = rng.choice([0.25, 0.5, 1.0, 2.0, np.inf], size=(G, H, W))  # many ties
    keys[:, :, :7] = rng.uniform(0.0, 3.0, size=(G, H, 7))
    announce(f"composite kernel G={G}")
    out = mfa.composite_over([to_dev(i, dev) for i in imgs],
                             [to_dev(k, dev) for k in keys]).cpu().numpy()
    ref = orr.composite(imgs.reshape(G, -1, 4).astype(np.float64), keys.reshape(G, -1))
    assert np.abs(out.reshape(-1, 4) - ref).max() <= 1e-6


def test_partial_render_of_a_single_block_model_is_the_full_render(mfa, dev):
    model = synth.model_c1()
    W, H = 50, 37
    cam = synth.perspective_camera(W, H)
    params = synth.render_params(model)
    announce("partial render of a single-block model")
    with mfa.Model(model, "f32") as M:
        full = mfa.render_frame(M, cam, params, W, H, device=dev).cpu().numpy()
        img, key = mfa.render_partial(M, cam, params, W, H, (0, 0, 0), (1, 1, 1), device=dev)
        img, key = img.cpu().numpy(), key.cpu().numpy().reshape(-1)
        with pytest.raises(mfa.MFAError):
            mfa.render_partial(M, cam, params, W, H, (0, 0, 0), (1, 2, 1), device=dev)
    np.testing.assert_array_equal(img, full)
    ref = orr.render(orr.model_field(model), model.lo, model.hi, cam, params, W, H,
                     region=region_arg(model, (0, 0, 0), (1, 1, 1)))
    np.testing.assert_array_equal(key, ref["key"])
