"""Pins of the oracle's ray caster (CPU only): closed forms, geometric
invariants, associativity of "over", and brute-force scalar images."""
import math

import numpy as np
import pytest

import synth
from oracle import bspline as ob
from oracle import render as orr


def linear_model(coeffs=(0.0, 1.0, 0.0, 0.0), n=8, p=3):
    T = synth.clamped_uniform_knots(n, p)
    P = synth.linear_precision_ctrl([T] * 3, [p] * 3, coeffs)
    return synth.single_block_model(P, [p] * 3, [T] * 3, voxel=1.0 / 64)


# ---------------------------------------------------------------- closed form
def test_constant_opacity_closed_form_and_termination():
    """Linear field f = u0, constant TF (alpha 0.1), axis-aligned rays.

    A_k = 1 - 0.9^(k+1); termination at the first k with A_k >= 0.99,
    i.e. 44 samples; C = c' A with c' = rgb (ka + kd) + ks (gradient parallel
    to the view direction, |g| > g0).
    """
    model = linear_model()
    W = H = 6
    cam = synth.axis_camera(W, H, axis=0, half_extent=0.45)
    rgb = np.array([0.2, 0.5, 0.9])
    params = synth.render_params(model, tf=synth.tf_table_constant([*rgb, 0.1]),
                                 step=1.0 / 128, vmin=0.0, vmax=1.0)
    out = orr.render(orr.model_field(model), model.lo, model.hi, cam, params, W, H)
    assert np.all(out["K"] == 128)
    assert np.all(out["used"] == 44)
    a32 = float(np.float32(0.1))                 # the table holds FP32 entries
    A = 1.0 - (1.0 - a32) ** 44
    np.testing.assert_allclose(out["rgba"][:, 3], A, rtol=0, atol=1e-14)
    rgb = rgb.astype(np.float32).astype(np.float64)
    ka, kd, ks = (float(np.float32(v)) for v in (0.3, 0.6, 0.3))
    cprime = rgb * (ka + kd) + ks
    np.testing.assert_allclose(out["rgba"][:, :3], np.tile(cprime * A, (W * H, 1)), atol=1e-14)
    # FP32 replay of the same opacities gives the same count
    out2 = orr.render(orr.model_field(model), model.lo, model.hi, cam, params, W, H,
                      record_alpha=True)
    np.testing.assert_array_equal(orr.ert_replay_f32(out2["alpha"], out2["K"], 0.99), out2["used"])


def test_no_termination_full_length_and_max_samples_cap():
    model = linear_model()
    cam = synth.axis_camera(4, 4, axis=1, half_extent=0.4)
    p = synth.render_params(model, tf=synth.tf_table_constant([1, 1, 1, 0.01]), step=1.0 / 64,
                            vmin=0.0, vmax=1.0, ert_alpha=2.0)
    out = orr.render(orr.model_field(model), model.lo, model.hi, cam, p, 4, 4)
    assert np.all(out["K"] == 64) and np.all(out["used"] == 64)
    a32 = float(np.float32(0.01))
    np.testing.assert_allclose(out["rgba"][:, 3], 1 - (1 - a32) ** 64, atol=1e-14)
    p2 = dict(p, max_samples=10)
    out = orr.render(orr.model_field(model), model.lo, model.hi, cam, p2, 4, 4)
    assert np.all(out["K"] == 10)


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_slab_entry_exit_on_box_faces(kind):
    W, H = 24, 16
    cam = (synth.ortho_camera(W, H, az_deg=37, el_deg=-21) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=200, el_deg=35))
    o, d = orr.pixel_rays(cam, W, H)
    lo, hi = np.zeros(3), np.ones(3)
    tn, tf, miss = orr.slab(o, d, lo, hi)
    hit = ~miss
    assert hit.sum() > 0
    for t in (tn[hit], tf[hit]):
        x = o[hit] + t[:, None] * d[hit]
        assert np.all(x >= -1e-12) and np.all(x <= 1 + 1e-12)
        on_face = np.min(np.minimum(np.abs(x - 0.0), np.abs(x - 1.0)), axis=1)
        assert np.max(on_face) <= 1e-12
    # a missed ray's line really misses the box (dense check along the line)
    ts = np.linspace(0, 6, 4001)
    for k in np.nonzero(miss)[0][:50]:
        x = o[k] + ts[:, None] * d[k]
        inside = np.all((x > 1e-9) & (x < 1 - 1e-9), axis=1)
        assert not inside.any()


def test_camera_rays_symmetric_and_parallel():
    W, H = 8, 6
    cam = synth.ortho_camera(W, H)
    o, d = orr.pixel_rays(cam, W, H)
    assert np.all(d == cam["forward"])
    c = np.asarray(cam["eye"])
    om = o.reshape(H, W, 3)
    np.testing.assert_allclose(om + om[::-1, ::-1], np.broadcast_to(2 * c, om.shape), atol=1e-14)
    pc = synth.perspective_camera(W, H)
    o, d = orr.pixel_rays(pc, W, H)
    assert np.all(o == pc["eye"])
    np.testing.assert_allclose(d @ pc["forward"], 1.0, atol=1e-14)   # depth-parametrised
    # row 0 is the top row: its rays lean along +up
    dm = d.reshape(H, W, 3)
    assert np.all(dm[0] @ pc["up"] > 0) and np.all(dm[-1] @ pc["up"] < 0)


def test_zero_direction_component_and_eye_inside():
    o = np.array([[0.5, 0.5, -1.0], [1.5, 0.5, -1.0], [0.5, 0.5, 0.5]])
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    tn, tf, miss = orr.slab(o, d, np.zeros(3), np.ones(3))
    assert list(miss) == [False, True, False]
    assert tn[0] == 1.0 and tf[0] == 2.0
    assert tn[2] == 0.0 and tf[2] == 0.5


# ---------------------------------------------------------------- TF / Phong
def test_transfer_function_entries_midpoints_and_clamp():
    tf = synth.tf_table_A().astype(np.float64)
    f = np.array([0.0, 255.0, 64.0, 64.5, -3.0, 300.0, 254.5])
    out = orr.transfer(f, tf, 0.0, 255.0)
    np.testing.assert_array_equal(out[0], tf[0])
    np.testing.assert_array_equal(out[1], tf[255])
    np.testing.assert_array_equal(out[2], tf[64])
    np.testing.assert_allclose(out[3], 0.5 * (tf[64] + tf[65]), atol=1e-15)
    np.testing.assert_array_equal(out[4], tf[0])
    np.testing.assert_array_equal(out[5], tf[255])
    np.testing.assert_allclose(out[6], 0.5 * (tf[254] + tf[255]), atol=1e-15)


def test_phong_limits():
    rgb = np.array([[0.5, 0.25, 1.0]] * 3)
    L = np.array([[0.0, 0.0, 1.0]] * 3)
    g = np.array([[0.0, 0.0, -5.0], [3.0, 0.0, 0.0], [0.0, 0.0, 0.5]])
    c = orr.phong(rgb, g, L, 0.3, 0.6, 0.3, g0=1.0, m=16)   # FP64 coefficients here
    np.testing.assert_allclose(c[0], rgb[0] * 0.9 + 0.3, atol=1e-15)     # parallel (two-sided)
    np.testing.assert_allclose(c[1], rgb[1] * 0.3, atol=1e-15)           # perpendicular
    np.testing.assert_allclose(c[2], rgb[2] * (0.3 + 0.6 * 0.5) + 0.3 * 0.5 ** 16, atol=1e-15)


# ---------------------------------------------------------------- associativity
def test_over_is_associative_for_segments():
    model = synth.model_c1()
    W = H = 10
    cam = synth.perspective_camera(W, H, az_deg=60, el_deg=10)
    params = synth.render_params(model, ert_alpha=2.0)
    fld = orr.model_field(model)
    full = orr.render(fld, model.lo, model.hi, cam, params, W, H)
    kmax = int(full["K"].max())
    cuts = [0, kmax // 3, 2 * kmax // 3, kmax]
    segs = [orr.render(fld, model.lo, model.hi, cam, params, W, H, k_range=(a, b))["rgba"]
            for a, b in zip(cuts[:-1], cuts[1:])]
    left = orr.over(orr.over(segs[0], segs[1]), segs[2])
    right = orr.over(segs[0], orr.over(segs[1], segs[2]))
    np.testing.assert_allclose(left, full["rgba"], atol=1e-14)
    np.testing.assert_allclose(right, full["rgba"], atol=1e-14)


# ---------------------------------------------------------------- brute force
def brute_force_image(model, cam, params, W, H):
    """Scalar Python re-evaluation of every ray and sample (tiny images)."""
    tf = np.asarray(params["tf"], dtype=np.float64)
    lo, hi = [float(v) for v in model.lo], [float(v) for v in model.hi]
    img = np.zeros((H * W, 4))
    cnt = np.zeros((H * W, 2), dtype=np.int64)
    eye, fw, rt, up = (list(map(float, cam[k])) for k in ("eye", "forward", "right", "up"))
    vmin, vmax = float(params["vmin"]), float(params["vmax"])
    dt = float(params["step"])
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
            nd = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
            L = [-d[a] / nd for a in range(3)]
            C, A, used = [0.0, 0.0, 0.0], 0.0, 0
            for k in range(K):
                t = tn + (k + 0.5) * dt
                x = np.array([[o[a] + t * d[a] for a in range(3)]])
                r = ob.evaluate(model, x)
                f, g = float(r["f"][0]), [float(v) for v in r["grad"][0]]
                s = min(max((f - vmin) / (vmax - vmin), 0.0), 1.0) * 255.0
                i0 = int(min(math.floor(s), 254.0))
                w = s - i0
                col = [(1.0 - w) * tf[i0][c] + w * tf[i0 + 1][c] for c in range(4)]
                gn = math.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])
                den = max(gn, float(params["g0"]))
                dif = abs((g[0] / den) * L[0] + (g[1] / den) * L[1] + (g[2] / den) * L[2])
                spec = 1.0
                for _ in range(params["shininess"]):
                    spec *= dif
                om = 1.0 - A
                for c in range(3):
                    cc = col[c] * (float(params["ka"]) + float(params["kd"]) * dif) + float(params["ks"]) * spec
                    C[c] = C[c] + (om * col[3]) * cc
                A = A + om * col[3]
                used = k + 1
                if A >= float(params["ert_alpha"]):
                    break
            img[j * W + i] = [*C, A]
            cnt[j * W + i] = [K, used]
    return img, cnt


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_vectorised_render_matches_scalar_brute_force(kind):
    model = synth.model_c1()
    W, H = 6, 5
    cam = (synth.ortho_camera(W, H, half_extent=0.7) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=130, el_deg=25))
    params = synth.render_params(model, step=1.0 / 40)
    out = orr.render(orr.model_field(model), model.lo, model.hi, cam, params, W, H)
    img, cnt = brute_force_image(model, cam, params, W, H)
    np.testing.assert_array_equal(out["K"], cnt[:, 0])
    np.testing.assert_array_equal(out["used"], cnt[:, 1])
    np.testing.assert_allclose(out["rgba"], img, rtol=0, atol=1e-14)
    assert out["rgba"][:, 3].max() > 0.1        # the image is not empty


def test_ert_replay_matches_fp64_decision_outside_band():
    model = synth.model_c1()
    W = H = 16
    cam = synth.ortho_camera(W, H)
    params = synth.render_params(model)
    out = orr.render(orr.model_field(model), model.lo, model.hi, cam, params, W, H, record_alpha=True)
    rep = orr.ert_replay_f32(out["alpha"], out["K"], params["ert_alpha"])
    assert (out["used"] < out["K"]).sum() >= 5           # some rays terminate early
    np.testing.assert_array_equal(rep, out["used"])


# ---------------------------------------------------------------- object-space compositing
def small_multiblock_model(seed=21, p=3):
    """3x2x2 blocks with uneven edges and control-point counts."""
    rng = np.random.default_rng(seed)
    edges = [np.array([0.0, 0.3, 0.55, 1.0]), np.array([0.0, 0.6, 1.0]), np.array([0.0, 0.45, 1.0])]
    blocks = []
    for _ in range(12):
        n = [int(v) for v in rng.integers(p + 2, 9, size=3)]
        knots = [synth.clamped_uniform_knots(n[a], p) for a in range(3)]
        blocks.append(synth.BlockSpec([p] * 3, knots, rng.uniform(0.0, 1.0, size=n)))
    return synth.ModelSpec([3, 2, 2], np.zeros(3), np.ones(3), edges, blocks, voxel=1.0 / 40)


def region_arg(model, blo, bhi):
    rlo = [model.edges[a][blo[a]] for a in range(3)]
    rhi = [model.edges[a][bhi[a]] for a in range(3)]
    return (orr.block_owner_fn(model), blo, bhi, rlo, rhi)


def _partition(model, cuts):
    """Block boxes of the split of the block grid at the given cut per axis."""
    out = []
    for a0 in ((0, cuts[0]), (cuts[0], model.grid[0])):
        for a1 in ((0, cuts[1]), (cuts[1], model.grid[1])):
            out.append(((a0[0], a1[0], 0), (a0[1], a1[1], model.grid[2])))
    return out


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_composite_of_partials_equals_full_render_without_termination(kind):
    """Associativity of "over" (Sec. IV-A5): the key-ordered composite of
    the partial images of a partition of the blocks equals the full render
    when termination is off; every ray crosses several regions."""
    model = small_multiblock_model()
    W, H = 14, 11
    cam = (synth.ortho_camera(W, H, az_deg=35.0, el_deg=25.0) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=35.0, el_deg=25.0))
    lo, hi = model.ctrl_min_max()
    params = synth.render_params(model, tf=synth.tf_table_constant([0.9, 0.4, 0.2, 0.03]),
                                 vmin=lo, vmax=hi)
    params["ert_alpha"] = 2.0
    field = orr.model_field(model)
    full = orr.render(field, model.lo, model.hi, cam, params, W, H)
    parts = [orr.render(field, model.lo, model.hi, cam, params, W, H,
                        region=region_arg(model, blo, bhi))
             for blo, bhi in _partition(model, (1, 1))]
    comp = orr.composite([p["rgba"] for p in parts], [p["key"] for p in parts])
    np.testing.assert_allclose(comp, full["rgba"], rtol=0, atol=1e-12)
    crossing = sum(np.isfinite(p["key"]).astype(int) for p in parts)
    assert (crossing >= 2).sum() >= 10 and crossing.max() >= 3     # rays through several regions


def test_region_keys_order_the_sample_runs():
    """Along each ray the composited samples of a region form one run, and
    the runs come in the order of the region keys."""
    model = small_multiblock_model(seed=22)
    W, H = 9, 7
    cam = synth.perspective_camera(W, H, az_deg=200.0, el_deg=-30.0)
    lo, hi = model.ctrl_min_max()
    params = synth.render_params(model, tf=synth.tf_table_constant([1, 1, 1, 0.02]),
                                 vmin=lo, vmax=hi)
    params["ert_alpha"] = 2.0
    field = orr.model_field(model)
    boxes = _partition(model, (2, 1))
    parts = [orr.render(field, model.lo, model.hi, cam, params, W, H, record_alpha=True,
                        region=region_arg(model, blo, bhi)) for blo, bhi in boxes]
    for pix in range(W * H):
        runs = []
        for g, p in enumerate(parts):
            nz = np.nonzero(p["alpha"][pix] > 0)[0]
            if len(nz):
                assert np.all(np.diff(nz) == 1)          # one contiguous run
                runs.append((p["key"][pix], nz[0], nz[-1]))
        runs.sort()
        for (k1, a1, b1), (k2, a2, b2) in zip(runs, runs[1:]):
            assert b1 < a2                               # key order = sample order


def test_composite_brute_force_and_single_region():
    rng = np.random.default_rng(7)
    G, m = 4, 50
    imgs = rng.uniform(0, 1, size=(G, m, 4))
    keys = rng.permutation(np.concatenate([rng.uniform(0, 5, size=(G - 1) * m), np.full(m, np.inf)]))
    keys = keys.reshape(G, m)
    got = orr.composite(imgs, keys)
    for i in range(m):
        C, A = np.zeros(3), 0.0
        for g in sorted(range(G), key=lambda g: (keys[g, i], g)):
            C = C + (1.0 - A) * imgs[g, i, :3]
            A = A + (1.0 - A) * imgs[g, i, 3]
        np.testing.assert_allclose(got[i], np.append(C, A), rtol=0, atol=1e-14)
    # one region holding every block: the partial render is the full render
    model = small_multiblock_model(seed=23)
    cam = synth.ortho_camera(8, 8)
    lo, hi = model.ctrl_min_max()
    params = synth.render_params(model, vmin=lo, vmax=hi)
    field = orr.model_field(model)
    full = orr.render(field, model.lo, model.hi, cam, params, 8, 8)
    part = orr.render(field, model.lo, model.hi, cam, params, 8, 8,
                      region=region_arg(model, (0, 0, 0), tuple(model.grid)))
    np.testing.assert_array_equal(part["rgba"], full["rgba"])
    np.testing.assert_array_equal(part["used"], full["used"])
