"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Small workloads are compared element by element (several tiles plus ragged
tails); the full-size point / grid / frame workloads are compared on
sampled outputs that the oracle evaluates one by one.
"""
import numpy as np
import pytest

import synth
from oracle import bspline as ob
from oracle import quant
from oracle import render as orr
from tests.gpu_common import announce, assert_values_close, composite_band

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfa():
    import paper_2312_15073_amd as m
    return m


@pytest.fixture(scope="module")
def c1():
    return synth.model_c1()


def to_dev(x, dev, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def adversarial_points(model, rng, n_rand):
    """Random points plus points exactly on knots, on the box faces and
    outside the box (clamped by the map)."""
    pts = [rng.random((n_rand, 3)).astype(np.float32)]
    T = model.blocks[0].knots[0]
    knots = np.unique(T).astype(np.float32)
    k = rng.choice(knots, size=(400, 3))
    pts.append(k)
    pts.append(np.array([[0, 0, 0], [1, 1, 1], [1, 0, 1], [-0.25, 0.5, 1.5], [2, -1, 0.5],
                         [np.nextafter(np.float32(1), np.float32(0))] * 3], dtype=np.float32))
    return np.concatenate(pts).astype(np.float32)


def oracle_points(model, pts32):
    return ob.evaluate(model, pts32.astype(np.float64))


# ------------------------------------------------------------------ points
@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_decode_points_single_block_fp32(mfa, dev, p):
    model = synth.model_c1(p=p)
    rng = np.random.default_rng(100 + p)
    pts = adversarial_points(model, rng, 20000)
    announce(f"decode_points c1 p={p} n={len(pts)}")
    with mfa.Model(model, "f32") as M:
        out, dbg = mfa.decode_points(M, to_dev(pts.T, dev), dbg=True)
        out, dbg = out.cpu().numpy(), dbg.cpu().numpy()
    ref = oracle_points(model, pts)
    np.testing.assert_array_equal(dbg[:, :3], ref["spans"])
    assert np.all(dbg[:, 3] == 0)
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(model.blocks[0].ctrl)))


@pytest.mark.parametrize("n", [1, 63, 255, 257, 1000])
def test_decode_points_ragged_sizes(mfa, dev, c1, n):
    pts = synth.random_points(n, seed=n)
    announce(f"decode_points ragged n={n}")
    with mfa.Model(c1, "f32") as M:
        out = mfa.decode_points(M, to_dev(pts, dev)).cpu().numpy()
    ref = oracle_points(c1, pts.T)
    assert out.shape == (n, 4)
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(c1.blocks[0].ctrl)))


def test_decode_points_empty_is_noop(mfa, dev, c1):
    import torch
    announce("decode_points n=0")
    with mfa.Model(c1, "f32") as M:
        out = mfa.decode_points(M, torch.zeros((3, 0), dtype=torch.float32, device=dev))
    assert out.shape == (0, 4)


def test_decode_points_nonunit_box_and_nonuniform_knots(mfa, dev):
    rng = np.random.default_rng(7)
    p = 3
    ns = (11, 14, 9)
    knots = []
    for a, n in enumerate(ns):
        inner = np.sort(rng.uniform(0, 1, n - p - 1))
        inner[2] = inner[3]
        knots.append(np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]))
    P = rng.standard_normal(ns)
    model = synth.single_block_model(P, [p] * 3, knots, lo=(-2.0, 0.5, 1.0), hi=(3.0, 0.75, 9.0))
    pts = (model.lo + rng.random((30000, 3)) * (model.hi - model.lo)).astype(np.float32)
    announce("decode_points non-uniform knots, non-unit box")
    with mfa.Model(model, "f32") as M:
        out, dbg = mfa.decode_points(M, to_dev(pts.T, dev), dbg=True)
        out, dbg = out.cpu().numpy(), dbg.cpu().numpy()
    ref = oracle_points(model, pts)
    np.testing.assert_array_equal(dbg[:, :3], ref["spans"])
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(P)))


def graded_knots(n, p, ratio_log2, phase=0):
    """Clamped knots whose span widths cycle through 2^0 .. 2^-ratio_log2,
    so that floor(u * nsp) can miss the span by many spans."""
    w = 2.0 ** -((np.arange(n - p) + phase) % (ratio_log2 + 1))
    inner = np.cumsum(w)[:-1] / w.sum()
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_decode_points_strongly_graded_knots(mfa, dev, storage):
    rng = np.random.default_rng(17)
    p, ns = 3, (41, 37, 29)
    knots = [graded_knots(n, p, 5, phase=a) for a, n in enumerate(ns)]
    P = rng.standard_normal(ns)
    model = synth.single_block_model(P, [p] * 3, knots)
    pts = rng.random((3, 50000)).astype(np.float32)
    for a in range(3):                       # points on knots and one ulp off
        T = knots[a][p + 1:ns[a]].astype(np.float32)
        pts[a, :len(T)] = T
        pts[a, len(T):2 * len(T)] = np.nextafter(T, np.float32(0))
    announce(f"decode_points strongly graded knots {storage}")
    with mfa.Model(model, storage) as M:
        out, dbg = mfa.decode_points(M, to_dev(pts, dev), dbg=True)
        srt = mfa.decode_points(M, to_dev(pts, dev), sorted_order=True)
        out, dbg, srt = out.cpu().numpy(), dbg.cpu().numpy(), srt.cpu().numpy()
    qP = quant.stored_values(P, storage) if storage != "f32" else P
    ref = oracle_points(synth.single_block_model(qP, [p] * 3, knots), pts.T)
    np.testing.assert_array_equal(dbg[:, :3], ref["spans"])
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(P)))
    np.testing.assert_array_equal(srt, out)                          # same sums in both orders


# ------------------------------------------------------------------ grid
def test_decode_grid_c1_full(mfa, dev, c1):
    ax = [synth.grid_axis(64)] * 3
    announce("decode_grid c1 64^3")
    with mfa.Model(c1, "f32") as M:
        out, spans = mfa.decode_grid(M, [to_dev(a, dev) for a in ax], spans=True)
        out, spans = out.cpu().numpy(), spans.cpu().numpy()
    ref = ob.decode_grid(c1, ax)
    rs = ob.grid_spans(c1, ax)
    np.testing.assert_array_equal(spans, np.concatenate(rs))
    assert_values_close(out.reshape(-1, 4), ref[..., 0].reshape(-1), ref[..., 1:].reshape(-1, 3),
                        np.max(np.abs(c1.blocks[0].ctrl)))


def test_decode_grid_ragged_unsorted_tables(mfa, dev, c1):
    rng = np.random.default_rng(3)
    ax = [rng.permutation(np.concatenate([synth.grid_axis(30), [-0.2, 1.3]])),
          np.sort(rng.random(5)),
          np.concatenate([synth.grid_axis(70)[::-1], [0.5]])]
    announce("decode_grid ragged 32x5x71 unsorted")
    with mfa.Model(c1, "f32") as M:
        out, spans = mfa.decode_grid(M, [to_dev(a, dev) for a in ax], spans=True)
        out, spans = out.cpu().numpy(), spans.cpu().numpy()
    ref = ob.decode_grid(c1, ax)
    np.testing.assert_array_equal(spans, np.concatenate(ob.grid_spans(c1, ax)))
    assert_values_close(out.reshape(-1, 4), ref[..., 0].reshape(-1), ref[..., 1:].reshape(-1, 3),
                        np.max(np.abs(c1.blocks[0].ctrl)))


# ------------------------------------------------------------------ render
def check_render(mfa, dev, model, cam, params, W, H, storage="f32", ref_model=None):
    ref_model = ref_model or model
    with mfa.Model(model, storage) as M:
        rgba, ns, al, ne = mfa.render_frame(M, cam, params, W, H, nsamp=True, alpha=True,
                                            neval=True, device=dev)
        rgba, ns, al, ne = rgba.cpu().numpy(), ns.cpu().numpy(), al.cpu().numpy(), ne.cpu().numpy()
    ref = orr.render(orr.model_field(ref_model), model.lo, model.hi, cam, params, W, H,
                     record_alpha=True)
    K = ns[..., 0].reshape(-1)
    used = ns[..., 1].reshape(-1)
    ne = ne.reshape(-1)
    assert np.all(ne <= used) and np.all(ne >= 0)
    np.testing.assert_array_equal(K, ref["K"])                      # schedule: exact
    # exact FP32 replay of the kernel's own opacities: identical decisions
    alpha = al.reshape(W * H, -1)
    rep = orr.ert_replay_f32(alpha, K, params["ert_alpha"])
    np.testing.assert_array_equal(used, rep)
    # against the FP64 oracle: equal outside the threshold band
    band = composite_band(ref["alpha"], ref["used"], float(params["ert_alpha"]))
    out = ~band
    np.testing.assert_array_equal(used[out], ref["used"][out])
    assert np.all(np.abs(used[band] - ref["used"][band]) <= 1)
    img = rgba.reshape(-1, 4)
    diff = np.abs(img[out] - ref["rgba"][out])
    rmse = float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0
    assert rmse <= 1e-5, f"image RMSE {rmse:.3e}"
    assert diff.max(initial=0.0) <= 1e-3, f"image max-abs {diff.max():.3e}"
    return dict(band=int(band.sum()), rmse=rmse, samples=int(used.sum()),
                terminated=int((used < K).sum()), evaluated=int(ne.sum()))


def test_render_c1_ortho_128(mfa, dev, c1):
    W = H = 128
    cam = synth.ortho_camera(W, H)
    params = synth.render_params(c1)
    announce("render c1 128x128 ortho")
    r = check_render(mfa, dev, c1, cam, params, W, H)
    assert r["samples"] > 100000 and r["terminated"] > 100
    assert r["evaluated"] < r["samples"]         # transparent cells were skipped


def test_render_c1_perspective_ragged(mfa, dev, c1):
    W, H = 100, 37
    cam = synth.perspective_camera(W, H, az_deg=-70, el_deg=40, dist=1.6)
    params = synth.render_params(c1, max_samples=90)
    announce("render c1 100x37 perspective, max_samples 90")
    check_render(mfa, dev, c1, cam, params, W, H)


def test_render_c1_axis_aligned_rays(mfa, dev, c1):
    W, H = 80, 72
    cam = synth.axis_camera(W, H, axis=2, half_extent=0.55)     # two direction components are 0
    params = synth.render_params(c1)
    announce("render c1 80x72 axis-aligned ortho")
    r = check_render(mfa, dev, c1, cam, params, W, H)
    assert r["evaluated"] < r["samples"]


def test_render_graded_knots(mfa, dev):
    # Knots crowded towards 0: the model runs the general kernels (span
    # guess tables; leap targets through the stored knots of the cell
    # faces); the image, the sample counts and the FP32 replay must match.
    p = 3
    ns = (20, 26, 17)
    knots = [np.concatenate([np.zeros(p + 1), np.linspace(0, 1, n - p + 1)[1:-1] ** 2,
                             np.ones(p + 1)]) for n in ns]
    F = synth.field_c1()
    g = [synth.greville(T, p, n) for T, n in zip(knots, ns)]
    X = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    P = F.value(X).reshape(ns)
    model = synth.single_block_model(P, [p] * 3, knots, voxel=1.0 / 63)
    W, H = 96, 80
    cam = synth.perspective_camera(W, H, az_deg=110, el_deg=-25, dist=1.8)
    params = synth.render_params(model)
    announce("render graded knots 96x80 perspective")
    r = check_render(mfa, dev, model, cam, params, W, H)
    assert r["evaluated"] < r["samples"]


def test_render_graded_128_tables_over_40kb(mfa, dev):
    """128 graded spans per axis: every span has its own basis table, the
    records and tables take about 54 KB of LDS in the graded single-block
    kernel."""
    model = synth.model_c2_graded()
    W, H = 32, 24
    cam = synth.perspective_camera(W, H, az_deg=70, el_deg=15)
    params = synth.render_params(model)
    announce("render graded 128^3 model, tables in LDS")
    r = check_render(mfa, dev, model, cam, params, W, H)
    assert r["evaluated"] > 1000


def test_render_closed_form_constant_opacity(mfa, dev):
    T = synth.clamped_uniform_knots(8, 3)
    P = synth.linear_precision_ctrl([T] * 3, [3] * 3, (0.0, 1.0, 0.0, 0.0))
    model = synth.single_block_model(P, [3] * 3, [T] * 3, voxel=1.0 / 64)
    cam = synth.axis_camera(20, 20, axis=0, half_extent=0.45)
    params = synth.render_params(model, tf=synth.tf_table_constant([0.2, 0.5, 0.9, 0.1]),
                                 step=1.0 / 128, vmin=0.0, vmax=1.0)
    announce("render closed form")
    with mfa.Model(model, "f32") as M:
        rgba, ns = mfa.render_frame(M, cam, params, 20, 20, nsamp=True, device=dev)
        rgba, ns = rgba.cpu().numpy(), ns.cpu().numpy()
    assert np.all(ns[..., 0] == 128) and np.all(ns[..., 1] == 44)
    A = 1 - (1 - float(np.float32(0.1))) ** 44
    np.testing.assert_allclose(rgba[..., 3], A, atol=1e-6)


# ------------------------------------------------------------------ precision forms
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("p", [2, 3, 5])
def test_reduced_precision_storage(mfa, dev, dtype, p):
    model = synth.model_c1(p=p)
    P = model.blocks[0].ctrl
    qP = quant.stored_values(P, dtype)
    qmodel = synth.single_block_model(qP, [p] * 3, model.blocks[0].knots, voxel=model.voxel)
    pts = synth.random_points(20011, seed=40 + p)
    announce(f"decode_points {dtype} p={p}")
    with mfa.Model(model, dtype) as M:
        bits = M.export_ctrl(0)
        out = mfa.decode_points(M, to_dev(pts, dev)).cpu().numpy()
        info = M.info()
    np.testing.assert_array_equal(bits, quant.stored_bits(P, dtype))
    assert info["vmin"] == np.float32(qP.min()) and info["vmax"] == np.float32(qP.max())
    ref_q = oracle_points(qmodel, pts.T)
    assert_values_close(out, ref_q["f"], ref_q["grad"], np.max(np.abs(P)))
    # against the FP64 model: within the storage bound plus arithmetic error
    ref = oracle_points(model, pts.T)
    dP = np.max(np.abs(qP - P))
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(P)), extra_f=dP,
                        extra_g=2 * p * (16 - p) * dP)


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_render_degree_and_storage(mfa, dev, p, storage):
    """Every degree's and storage form's render kernel against the oracle on
    the control points as stored (the kernel's own arithmetic error): sample
    schedule exact, FP32 replay of the termination exact, samples used equal
    outside the threshold band, image within the render tolerance.  The frame
    is ragged (70 x 54: partial 8 x 8 tiles on two sides)."""
    model = synth.model_c1(p=p)
    qP = quant.stored_values(model.blocks[0].ctrl, storage)
    qmodel = synth.single_block_model(qP, [p] * 3, model.blocks[0].knots, voxel=model.voxel)
    W, H = 70, 54
    cam = synth.perspective_camera(W, H, az_deg=25.0 + 40.0 * p, el_deg=15.0 + 5.0 * p, dist=1.9)
    params = synth.render_params(model)
    announce(f"render c1 p={p} {storage} {W}x{H} perspective")
    r = check_render(mfa, dev, model, cam, params, W, H, storage=storage, ref_model=qmodel)
    assert r["samples"] > 20000 and r["evaluated"] < r["samples"]


# ------------------------------------------------------------------ full-size workloads (sampled)
@pytest.fixture(scope="module")
def c2():
    return synth.model_c2()


def test_c2_grid_512_sampled(mfa, dev, c2):
    import torch
    ax = [synth.grid_axis(512)] * 3
    announce("decode_grid c2 512^3 (sampled)")
    with mfa.Model(c2, "f32") as M:
        out, spans = mfa.decode_grid(M, [to_dev(a, dev) for a in ax], spans=True)
        rng = np.random.default_rng(5)
        idx = rng.integers(0, 512, size=(3000, 3))
        idx = np.concatenate([idx, [[0, 0, 0], [511, 511, 511], [0, 511, 255]]])
        sel = out[torch.as_tensor(idx[:, 0]), torch.as_tensor(idx[:, 1]), torch.as_tensor(idx[:, 2])]
        got = sel.cpu().numpy()
        spans = spans.cpu().numpy()
        del out
    np.testing.assert_array_equal(spans, np.concatenate(ob.grid_spans(c2, ax)))
    ref = ob.decode_grid(c2, ax, out_index=idx)
    assert_values_close(got, ref[:, 0], ref[:, 1:], np.max(np.abs(c2.blocks[0].ctrl)))


def test_c2_points_1e7_sampled(mfa, dev, c2):
    pts = synth.random_points(10_000_000, seed=12)
    announce("decode_points c2 1e7 (sampled)")
    with mfa.Model(c2, "f32") as M:
        out, dbg = mfa.decode_points(M, to_dev(pts, dev), dbg=True)
        rng = np.random.default_rng(6)
        k = np.concatenate([rng.integers(0, pts.shape[1], size=20000), [0, pts.shape[1] - 1]])
        import torch
        kt = torch.as_tensor(k, device=dev)
        got = out[kt].cpu().numpy()
        gs = dbg[kt].cpu().numpy()
    ref = oracle_points(c2, pts[:, k].T)
    np.testing.assert_array_equal(gs[:, :3], ref["spans"])
    assert_values_close(got, ref["f"], ref["grad"], np.max(np.abs(c2.blocks[0].ctrl)))


def test_c2_render_1024_sampled(mfa, dev, c2):
    W = H = 1024
    cam = synth.perspective_camera(W, H)
    params = synth.render_params(c2)
    announce("render c2 1024x1024 perspective (sampled)")
    with mfa.Model(c2, "f32") as M:
        rgba, ns, ne = mfa.render_frame(M, cam, params, W, H, nsamp=True, neval=True, device=dev)
        rgba, ns = rgba.cpu().numpy().reshape(-1, 4), ns.cpu().numpy().reshape(-1, 2)
        ne = ne.cpu().numpy().reshape(-1)
    assert np.all(ne <= ns[:, 1]) and ne.sum() < 0.6 * ns[:, 1].sum()
    rng = np.random.default_rng(8)
    pix = np.stack([rng.integers(0, H, 240), rng.integers(0, W, 240)], axis=1)
    pix = np.concatenate([pix, [[0, 0], [H - 1, W - 1], [H // 2, W // 2]]])
    ref = orr.render(orr.model_field(c2), c2.lo, c2.hi, cam, params, W, H, pixels=pix,
                     record_alpha=True)
    flat = pix[:, 0] * W + pix[:, 1]
    np.testing.assert_array_equal(ns[flat, 0], ref["K"])
    band = composite_band(ref["alpha"], ref["used"], float(params["ert_alpha"]))
    np.testing.assert_array_equal(ns[flat, 1][~band], ref["used"][~band])
    diff = np.abs(rgba[flat][~band] - ref["rgba"][~band])
    assert diff.max(initial=0) <= 1e-3 and np.sqrt(np.mean(diff ** 2)) <= 1e-5
    assert ns[:, 1].sum() > 1e7          # a real frame: many samples


# ------------------------------------------------------------------ multi-block models
def small_multiblock(seed=21, p=3, graded=False):
    """3x2x2 blocks with uneven edges and uneven control-point counts, each
    block fitted to one Gaussian-sum field at its Greville abscissae.
    graded: knots crowded towards each block's low face (u^1.5), so that
    every span has its own basis table (hundreds of tables).  The crowding
    is kept moderate: the FP32 rounding error of a gradient grows with the
    chain-rule scale of the narrowest span, which the normwise tolerance
    does not see (quadratic crowding of these small blocks exceeds it by
    7 %, in the unsorted decode as well)."""
    rng = np.random.default_rng(seed)
    field = synth.field_c1(seed)
    edges = [np.array([0.0, 0.3, 0.55, 1.0]), np.array([0.0, 0.6, 1.0]), np.array([0.0, 0.45, 1.0])]
    blocks = []
    for b0 in range(3):
        for b1 in range(2):
            for b2 in range(2):
                n = [int(v) for v in rng.integers(p + 2, 14, size=3)]
                if graded:
                    knots = [np.concatenate([np.zeros(p + 1), np.linspace(0, 1, n[a] - p + 1)[1:-1] ** 1.5,
                                             np.ones(p + 1)]) for a in range(3)]
                else:
                    knots = [synth.clamped_uniform_knots(n[a], p) for a in range(3)]
                lo = np.array([edges[0][b0], edges[1][b1], edges[2][b2]])
                hi = np.array([edges[0][b0 + 1], edges[1][b1 + 1], edges[2][b2 + 1]])
                xs = [lo[a] + synth.greville(knots[a], p, n[a]) * (hi[a] - lo[a]) for a in range(3)]
                blocks.append(synth.BlockSpec([p] * 3, knots, field.value_separable(*xs)))
    return synth.ModelSpec([3, 2, 2], np.zeros(3), np.ones(3), edges, blocks, voxel=1.0 / 63)


def test_decode_points_multiblock(mfa, dev):
    model = small_multiblock()
    rng = np.random.default_rng(4)
    pts = [rng.random((30000, 3)).astype(np.float32)]
    for a in range(3):                      # points exactly on block faces
        for e in model.edges[a]:
            v = rng.random((50, 3)).astype(np.float32)
            v[:, a] = np.float32(e)
            pts.append(v)
    pts.append(np.array([[-0.5, 0.5, 0.5], [1.5, 2.0, -3.0]], dtype=np.float32))
    pts = np.concatenate(pts)
    announce(f"decode_points multi-block 3x2x2 n={len(pts)}")
    with mfa.Model(model, "f32") as M:
        out, dbg = mfa.decode_points(M, to_dev(pts.T, dev), dbg=True)
        out, dbg = out.cpu().numpy(), dbg.cpu().numpy()
    ref = oracle_points(model, pts)
    flat = (ref["blocks"][:, 0] * 2 + ref["blocks"][:, 1]) * 2 + ref["blocks"][:, 2]
    np.testing.assert_array_equal(dbg[:, 3], flat)
    np.testing.assert_array_equal(dbg[:, :3], ref["spans"])
    pmax = max(np.abs(b.ctrl).max() for b in model.blocks)
    assert_values_close(out, ref["f"], ref["grad"], pmax)


@pytest.mark.parametrize("kind", ["ortho", "persp"])
def test_render_multiblock_rays_cross_blocks(mfa, dev, kind):
    model = small_multiblock()
    W, H = 72, 56
    cam = (synth.ortho_camera(W, H, az_deg=50, el_deg=25) if kind == "ortho"
           else synth.perspective_camera(W, H, az_deg=-40, el_deg=30))
    params = synth.render_params(model)
    announce(f"render multi-block {kind} {W}x{H}")
    r = check_render(mfa, dev, model, cam, params, W, H)
    assert r["samples"] > 20000


def test_render_multiblock_more_edges_than_the_lds_copy(mfa, dev):
    """254 x 1 x 1 blocks: 259 block edges, more than the render's LDS copy
    holds, so the frame takes the kernel that reads the edges from global
    memory; rays cross many blocks along axis 0."""
    rng = np.random.default_rng(23)
    p = 3
    field = synth.field_c1(23)
    g0 = 254
    edges = [np.linspace(0.0, 1.0, g0 + 1), np.array([0.0, 1.0]), np.array([0.0, 1.0])]
    blocks = []
    for b0 in range(g0):
        n = [int(v) for v in rng.integers(p + 1, p + 3, size=3)]
        knots = [synth.clamped_uniform_knots(n[a], p) for a in range(3)]
        lo = np.array([edges[0][b0], 0.0, 0.0])
        hi = np.array([edges[0][b0 + 1], 1.0, 1.0])
        xs = [lo[a] + synth.greville(knots[a], p, n[a]) * (hi[a] - lo[a]) for a in range(3)]
        blocks.append(synth.BlockSpec([p] * 3, knots, field.value_separable(*xs)))
    model = synth.ModelSpec([g0, 1, 1], np.zeros(3), np.ones(3), edges, blocks, voxel=1.0 / 63)
    W, H = 48, 40
    cam = synth.perspective_camera(W, H, az_deg=20, el_deg=15)
    params = synth.render_params(model)
    announce(f"render multi-block {g0}x1x1 {W}x{H}")
    r = check_render(mfa, dev, model, cam, params, W, H)
    assert r["samples"] > 10000


def test_render_and_sorted_decode_multiblock_with_many_basis_tables(mfa, dev):
    """Graded knots in every block: the basis tables exceed the kernels' LDS
    copy, so the render reads them from the global pool and the sorted
    decode runs one point per thread."""
    import torch
    model = small_multiblock(seed=23, graded=True)
    n_tables = sum(b.ctrl.shape[a] - 3 for b in model.blocks for a in range(3))
    assert n_tables * 28 > 1024
    W, H = 64, 48
    cam = synth.perspective_camera(W, H, az_deg=20, el_deg=35)
    params = synth.render_params(model)
    announce(f"render multi-block graded {W}x{H} ({n_tables} spans)")
    r = check_render(mfa, dev, model, cam, params, W, H)
    assert r["samples"] > 10000
    rng = np.random.default_rng(6)
    pts = rng.random((40000, 3)).astype(np.float32)
    announce("sorted decode multi-block graded n=40000")
    with mfa.Model(model, "f32") as M:
        x = to_dev(pts.T, dev)
        direct = mfa.decode_points(M, x)
        srt = mfa.decode_points(M, x, sorted_order=True)
        assert torch.equal(direct.view(torch.int32), srt.view(torch.int32))
        out = srt.cpu().numpy()
    ref = oracle_points(model, pts)
    assert_values_close(out, ref["f"], ref["grad"], max(np.abs(blk.ctrl).max() for blk in model.blocks))


@pytest.fixture(scope="module")
def c4():
    return synth.model_c4()


def test_c4_points_sampled(mfa, dev, c4):
    import torch
    n = 20_000_000
    pts = synth.random_points(n, seed=14)
    announce(f"decode_points 8x8x8-block model n={n} (sampled)")
    with mfa.Model(c4, "f32") as M:
        out, dbg = mfa.decode_points(M, to_dev(pts, dev), dbg=True)
        rng = np.random.default_rng(9)
        k = np.concatenate([rng.integers(0, n, size=20000), [0, n - 1]])
        kt = torch.as_tensor(k, device=dev)
        got, gd = out[kt].cpu().numpy(), dbg[kt].cpu().numpy()
    ref = oracle_points(c4, pts[:, k].T)
    flat = (ref["blocks"][:, 0] * 8 + ref["blocks"][:, 1]) * 8 + ref["blocks"][:, 2]
    np.testing.assert_array_equal(gd[:, 3], flat)
    np.testing.assert_array_equal(gd[:, :3], ref["spans"])
    assert_values_close(got, ref["f"], ref["grad"], max(np.abs(b.ctrl).max() for b in c4.blocks))


def test_c4_render_2048_sampled(mfa, dev, c4):
    W = H = 2048
    cam = synth.perspective_camera(W, H, az_deg=35, el_deg=25)
    params = synth.render_params(c4, max_samples=2048)
    announce("render 8x8x8-block model 2048x2048 (sampled)")
    with mfa.Model(c4, "f32") as M:
        rgba, ns, ne = mfa.render_frame(M, cam, params, W, H, nsamp=True, neval=True, device=dev)
        rgba, ns = rgba.cpu().numpy().reshape(-1, 4), ns.cpu().numpy().reshape(-1, 2)
        ne = ne.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(10)
    pix = np.stack([rng.integers(0, H, 120), rng.integers(0, W, 120)], axis=1)
    pix = np.concatenate([pix, [[H // 2, W // 2], [H // 3, W // 2]]])
    ref = orr.render(orr.model_field(c4), c4.lo, c4.hi, cam, params, W, H, pixels=pix,
                     record_alpha=True)
    flat = pix[:, 0] * W + pix[:, 1]
    np.testing.assert_array_equal(ns[flat, 0], ref["K"])
    band = composite_band(ref["alpha"], ref["used"], float(params["ert_alpha"]))
    np.testing.assert_array_equal(ns[flat, 1][~band], ref["used"][~band])
    diff = np.abs(rgba[flat][~band] - ref["rgba"][~band])
    assert diff.max(initial=0) <= 1e-3 and np.sqrt(np.mean(diff ** 2)) <= 1e-5
    assert np.all(ne <= ns[:, 1]) and ns[:, 1].sum() > 1e8


# ------------------------------------------------------------------ sorted decode
def _sorted_matches_unsorted(mfa, dev, model, pts, storage="f32"):
    """Sorted decode against the unsorted one, bit for bit: with debug
    outputs (results written at the input positions directly) and without
    (above 1024 buckets the results then go through the coarse order and
    are gathered back)."""
    with mfa.Model(model, storage) as M:
        x = to_dev(pts, dev)
        a, da = mfa.decode_points(M, x, dbg=True)
        b, db = mfa.decode_points(M, x, dbg=True, sorted_order=True)
        c = mfa.decode_points(M, x, sorted_order=True)
        a, da, b, db, c = (a.cpu().numpy(), da.cpu().numpy(), b.cpu().numpy(), db.cpu().numpy(),
                           c.cpu().numpy())
    np.testing.assert_array_equal(b.view(np.uint32), a.view(np.uint32))   # bit for bit
    np.testing.assert_array_equal(db, da)
    np.testing.assert_array_equal(c.view(np.uint32), a.view(np.uint32))
    return a


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_sorted_decode_single_block(mfa, dev, c1, storage):
    rng = np.random.default_rng(30)
    pts = adversarial_points(c1, rng, 50000).T.copy()
    announce(f"sorted decode c1 {storage} n={pts.shape[1]}")
    out = _sorted_matches_unsorted(mfa, dev, c1, pts, storage)
    if storage == "f32":
        ref = oracle_points(c1, pts.T)
        assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(c1.blocks[0].ctrl)))


def test_sorted_decode_few_buckets(mfa, dev):
    # 2 x 3 x 4 spans: the whole model is one bucket (its window fits the LDS).
    rng = np.random.default_rng(31)
    P = rng.standard_normal((5, 6, 7))
    model = synth.single_block_model(P, [3] * 3)
    pts = synth.random_points(30001, seed=31, lo=(-0.05, -0.05, -0.05), hi=(1.05, 1.05, 1.05))
    announce("sorted decode, 24 buckets")
    out = _sorted_matches_unsorted(mfa, dev, model, pts)
    ref = oracle_points(model, pts.T)
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(P)))


def test_sorted_decode_graded_knots(mfa, dev):
    # Knots crowded towards 0 along every axis: the bucket estimate
    # floor(u * nsp) then lies far from the exact span for most points, whose
    # rows come from global memory instead of the bucket's LDS window.
    rng = np.random.default_rng(41)
    p = 3
    ns = (40, 33, 47)
    knots = []
    for n in ns:
        inner = np.linspace(0, 1, n - p + 1)[1:-1] ** 2
        knots.append(np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]))
    P = rng.standard_normal(ns)
    model = synth.single_block_model(P, [p] * 3, knots, lo=(-1.0, 0.0, 2.0), hi=(1.0, 0.5, 5.0))
    pts = (model.lo + rng.random((200000, 3)) * (model.hi - model.lo)).astype(np.float32).T.copy()
    announce("sorted decode graded knots")
    out = _sorted_matches_unsorted(mfa, dev, model, pts)
    ref = oracle_points(model, pts.T)
    assert_values_close(out, ref["f"], ref["grad"], np.max(np.abs(P)))


def test_sorted_decode_multiblock_and_scratch_regrowth(mfa, dev):
    model = small_multiblock()
    announce("sorted decode multi-block, growing n")
    with mfa.Model(model, "f32") as M:
        for n in (1000, 257, 120001, 5):           # grow, shrink, grow, tiny
            pts = synth.random_points(n, seed=n, lo=(-0.1, -0.1, -0.1), hi=(1.1, 1.1, 1.1))
            x = to_dev(pts, dev)
            a = mfa.decode_points(M, x).cpu().numpy()
            b = mfa.decode_points(M, x, sorted_order=True).cpu().numpy()
            np.testing.assert_array_equal(b.view(np.uint32), a.view(np.uint32))
    ref = oracle_points(model, pts.T)
    assert_values_close(b, ref["f"], ref["grad"], max(np.abs(bl.ctrl).max() for bl in model.blocks))


def test_sorted_decode_multiblock_points_on_faces(mfa, dev):
    """Points at the FP32 roundings of block faces and their FP32
    neighbours: the sort's FP32 block choice can differ from the exact FP64
    owner there, which the decode detects and evaluates in the owner block;
    results equal the unsorted decode bit for bit (spans and blocks too)."""
    model = small_multiblock()
    rng = np.random.default_rng(44)
    pts = [rng.random((20000, 3)).astype(np.float32)]
    for a in range(3):
        for e in model.edges[a]:
            e32 = np.float32(e)
            for v in (np.nextafter(e32, np.float32(-1)), e32, np.nextafter(e32, np.float32(2))):
                q = rng.random((300, 3)).astype(np.float32)
                q[:, a] = v
                pts.append(q)
    pts = np.concatenate(pts).T.copy()
    announce(f"sorted decode multi-block, points on faces n={pts.shape[1]}")
    out = _sorted_matches_unsorted(mfa, dev, model, pts)
    ref = oracle_points(model, pts.T)
    assert_values_close(out, ref["f"], ref["grad"], max(np.abs(b.ctrl).max() for b in model.blocks))


def test_sorted_decode_c2_1e7(mfa, dev, c2):
    pts = synth.random_points(10_000_000, seed=12)
    announce("sorted decode c2 1e7")
    _sorted_matches_unsorted(mfa, dev, c2, pts)


def test_sorted_decode_one_bucket_several_chunks_per_workgroup(mfa, dev, c1):
    """The 16^3 model is one sort bucket.  34e6 points exceed 512 histogram
    workgroups of one 64512-point chunk each, so every workgroup counts two
    chunks and, before the second, moves its (64512-point) bucket counter to
    the global counts: totals and results must come out as in the unsorted
    decode, bit for bit."""
    n = 34_000_000
    assert n > 512 * 1024 * 63
    pts = synth.random_points(n, seed=16, lo=(-0.05,) * 3, hi=(1.05,) * 3)
    announce(f"sorted decode c1 one bucket n={n}")
    _sorted_matches_unsorted(mfa, dev, c1, pts)


@pytest.mark.parametrize("n", [1, 777, 5000, 300001])
def test_sorted_decode_c4_small_inputs(mfa, dev, c4, n):
    """Few points over the 8x8x8-block model's ~18k buckets: the coarse runs
    are short, so chunks of the second scatter pass span many coarse keys
    and records beyond the chunk's key table claim their slots one by one."""
    pts = synth.random_points(n, seed=200 + n, lo=(-0.02,) * 3, hi=(1.02,) * 3)
    announce(f"sorted decode 8x8x8-block model n={n}")
    out = _sorted_matches_unsorted(mfa, dev, c4, pts)
    if n <= 5000:
        ref = oracle_points(c4, pts.T)
        assert_values_close(out, ref["f"], ref["grad"], max(np.abs(b.ctrl).max() for b in c4.blocks))


def test_sorted_decode_c4_2e7(mfa, dev, c4):
    pts = synth.random_points(20_000_000, seed=15)
    announce("sorted decode 8x8x8-block model 2e7")
    _sorted_matches_unsorted(mfa, dev, c4, pts)


# ------------------------------------------------------------------ value-only queries
@pytest.mark.parametrize("which", ["c1", "graded", "multiblock", "c4"])
@pytest.mark.parametrize("sorted_order", [False, True])
def test_decode_points_value_only(mfa, dev, which, sorted_order, request):
    """Value-only queries (Fig. 8a): the value of the value+gradient query,
    bit for bit (the same sums; the gradient terms are dropped), and the
    oracle's value within the FP32 tolerance.  The 8x8x8-block model's
    sorted decode takes the two-level sort and the gather of its results
    from the coarse order."""
    if which == "c4":
        model = request.getfixturevalue("c4")
    elif which == "c1":
        model = synth.model_c1()
    elif which == "graded":
        p, ns = 3, (41, 37, 29)
        knots = [graded_knots(n, p, 5, phase=a) for a, n in enumerate(ns)]
        model = synth.single_block_model(np.random.default_rng(18).standard_normal(ns), [p] * 3, knots)
    else:
        model = small_multiblock()
    rng = np.random.default_rng(60)
    pts = np.concatenate([rng.random((30001, 3)).astype(np.float32),
                          adversarial_points(model, rng, 10)]).T.copy()
    announce(f"value-only decode {which} sorted={sorted_order} n={pts.shape[1]}")
    with mfa.Model(model, "f32") as M:
        x = to_dev(pts, dev)
        full = mfa.decode_points(M, x, sorted_order=sorted_order).cpu().numpy()
        val = mfa.decode_points(M, x, sorted_order=sorted_order, value_only=True).cpu().numpy()
    assert val.shape == (pts.shape[1],)
    np.testing.assert_array_equal(val.view(np.uint32), full[:, 0].copy().view(np.uint32))
    ref = oracle_points(model, pts.T)
    pmax = max(np.abs(b.ctrl).max() for b in model.blocks)
    assert np.max(np.abs(val - ref["f"])) <= 1e-5 * pmax


def test_decode_grid_value_only(mfa, dev, c1):
    rng = np.random.default_rng(61)
    ax = [synth.grid_axis(64), np.sort(rng.random(37)), synth.grid_axis(70)]
    announce("value-only grid 64x37x70")
    with mfa.Model(c1, "f32") as M:
        t = [to_dev(a, dev) for a in ax]
        full = mfa.decode_grid(M, t).cpu().numpy()
        val = mfa.decode_grid(M, t, value_only=True).cpu().numpy()
    assert val.shape == (64, 37, 70)
    np.testing.assert_array_equal(val.view(np.uint32), full[..., 0].copy().view(np.uint32))
    ref = ob.decode_grid(c1, ax)
    assert np.max(np.abs(val - ref[..., 0])) <= 1e-5 * np.max(np.abs(c1.blocks[0].ctrl))


def test_sorted_decode_calls_on_two_streams_are_ordered(mfa, dev, c1):
    """Sorted calls on one model from two streams share the model's scratch:
    the library orders them (a call waits for the previous sorted call's
    kernels), also when a larger n replaces the scratch; every result equals
    the unsorted decode bit for bit."""
    import torch
    sizes = [300001, 1000, 700001, 200000, 5, 900000]
    announce("sorted decode on two streams, growing and shrinking n")
    with mfa.Model(c1, "f32") as M:
        xs = [to_dev(synth.random_points(n, seed=70 + k), dev) for k, n in enumerate(sizes)]
        refs = [mfa.decode_points(M, x) for x in xs]
        outs = [torch.full((x.shape[1], 4), -1.0, device=dev) for x in xs]
        torch.cuda.synchronize()
        streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
        for k, (x, o) in enumerate(zip(xs, outs)):
            s = streams[k % 2]
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                mfa.decode_points(M, x, out=o, sorted_order=True, stream=s)
        torch.cuda.synchronize()
        for r, o in zip(refs, outs):
            np.testing.assert_array_equal(o.cpu().numpy().view(np.uint32), r.cpu().numpy().view(np.uint32))


# ------------------------------------------------------------------ serving
def test_server_results_equal_direct_calls(mfa, dev, c1):
    import torch
    multi = small_multiblock()
    models = [mfa.Model(c1, "f32"), mfa.Model(c1, "bf16"), mfa.Model(multi, "f32")]
    specs = [c1, c1, multi]
    rng = np.random.default_rng(50)
    announce("server: mixed renders and point queries on 3 models")
    with mfa.Server(hbm_budget_bytes=1 << 34, queue_cap=256, max_batch_items=64) as S:
        ids = [S.add_model(M) for M in models]
        jobs = []
        for q in range(24):
            k = q % 3
            if q % 2 == 0:
                W, H = int(rng.integers(20, 90)), int(rng.integers(20, 70))
                cam = synth.perspective_camera(W, H, az_deg=float(rng.uniform(0, 360)),
                                               el_deg=float(rng.uniform(-50, 50)))
                params = synth.render_params(specs[k], max_samples=int(rng.integers(50, 400)))
                tf = to_dev(params["tf"], dev)
                out = torch.full((H, W, 4), -1.0, device=dev)
                t = S.submit_render(ids[k], cam, params, W, H, out, tf_dev=tf)
                jobs.append(("r", k, t, out, (cam, params, W, H, tf)))
            else:
                n = int(rng.integers(1, 5000))
                x = to_dev(synth.random_points(n, seed=q), dev)
                out = torch.full((n, 4), -1.0, device=dev)
                t = S.submit_points(ids[k], x, out)
                jobs.append(("p", k, t, out, x))
        stats = [S.wait(j[2]) for j in jobs]
    # the oracle on the control points as each model stores them
    qc1 = synth.single_block_model(quant.stored_values(c1.blocks[0].ctrl, "bf16"), [3] * 3,
                                   c1.blocks[0].knots, voxel=c1.voxel)
    oracle_specs = [c1, qc1, multi]
    pmax = [np.max(np.abs(c1.blocks[0].ctrl))] * 2 + [max(np.abs(b.ctrl).max() for b in multi.blocks)]
    for (kind, k, t, out, arg), st in zip(jobs, stats):
        assert st["status"] == 0 and st["done"] == 1
        got = out.cpu().numpy()
        if kind == "r":
            cam, params, W, H, tf = arg
            ref = mfa.render_frame(models[k], cam, params, W, H, tf_dev=tf, device=dev)
        else:
            ref = mfa.decode_points(models[k], arg)
        # served results equal the direct calls bit for bit ...
        np.testing.assert_array_equal(got.view(np.uint32), ref.cpu().numpy().view(np.uint32))
        # ... and the oracle at the decode and render tolerances
        spec = oracle_specs[k]
        if kind == "r":
            ro = orr.render(orr.model_field(spec), spec.lo, spec.hi, cam, params, W, H,
                            record_alpha=True)
            band = composite_band(ro["alpha"], ro["used"], float(params["ert_alpha"]))
            diff = np.abs(got.reshape(-1, 4)[~band] - ro["rgba"][~band])
            assert diff.max(initial=0.0) <= 1e-3, f"served frame {t}: max-abs {diff.max():.3e}"
            rmse = float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0
            assert rmse <= 1e-5, f"served frame {t}: RMSE {rmse:.3e}"
        else:
            po = oracle_points(spec, arg.cpu().numpy().T)
            assert_values_close(got, po["f"], po["grad"], pmax[k])
    for M in models:
        M.close()
