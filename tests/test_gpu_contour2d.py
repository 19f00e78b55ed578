"""GPU parity of the 2D method (SN_LINES on images) through the C ABI against
the oracle's 2D extraction and its (unchanged) smoothing.

Bar, as for volumes: points, segments, label pairs and stencil bit-exact;
smoothed in-plane offsets within 1e-5 pixel of the FP64 oracle, the z offset
exactly 0; world points within 1e-5 * spacing + 1 float32 ulp, with z equal to
origin[2].
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def sn(torch):
    import paper_2401_14906_amd as sn

    sn.load_library()
    return sn


@pytest.fixture(scope="module")
def ctx(sn):
    c = sn.Context(0)
    yield c
    c.close()


def announce(msg):
    print(f"[case] {msg}", flush=True)


def check_contour(g, o, img, iters, lam, d, shape, spacing, origin):
    import oracle

    assert g.points.shape[0] == o.n_points
    assert g.polys.shape == (o.n_quads, 2)
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    assert g.label_pairs.dtype == img.dtype
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if not o.n_points:
        return
    pos = o.smooth(iters, lam, d, shape)
    ref = pos - o.centres()
    err = np.max(np.abs(g.offsets[:, :2].astype(np.float64) - ref[:, :2]))
    assert err <= TOL, f"offset error {err}"
    assert np.all(g.offsets[:, 2] == 0.0)
    # world xyz of the index-space positions, the image in the plane z = origin[2]
    w = oracle.world(pos, origin, (spacing[0], spacing[1], 0.0))[:, :2]
    h = np.asarray(spacing[:2], np.float64)
    ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(g.points[:, :2].astype(np.float64) - w) <= TOL * h + ulp)
    assert np.all(g.points[:, 2] == np.float32(origin[2]))


def run_image(ctx, sn, img, selected=(), background=0, iters=0, lam=0.5, d=1.0, shape="box",
              spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    import oracle

    t = sn.to_device(img)
    m = ctx.extract(t, spacing=spacing, origin=origin, selected=selected, background=background)
    ctx.smooth(m, iterations=iters, relaxation=lam, constraint=d, shape=shape)
    g = m.to_host()
    o = oracle.extract2d(img, selected, background)
    check_contour(g, o, img, iters, lam, d, shape, spacing, origin)
    m.free()
    return g, o


def test_single_pixel(ctx, sn):
    announce("2D single pixel")
    img = np.zeros((3, 3), np.uint16)
    img[1, 1] = 5
    g, o = run_image(ctx, sn, img, iters=3, lam=0.5, d=1.0)
    assert g.polys.tolist() == [[0, 1], [2, 0], [3, 1], [2, 3]]
    np.testing.assert_allclose(g.points[:, :2], [[0.9375, 0.9375], [1.0625, 0.9375],
                                                 [0.9375, 1.0625], [1.0625, 1.0625]], atol=1e-6)


def test_random_images(ctx, sn):
    rng = np.random.default_rng(2024)
    dts = [np.uint8, np.uint16, np.uint32]
    for c in range(90):
        M = int(rng.integers(1, 40)) if c % 3 else int(rng.integers(60, 300))
        N = int(rng.integers(1, 40))
        dt = dts[c % 3]
        nv = int(rng.integers(1, 7))
        img = (synth.blocky_tiny if c % 2 else synth.random_tiny)(rng, (M, N, 1), nv, dt).reshape(N, M)
        bg = int(rng.integers(0, 2))
        sel = tuple(int(x) for x in rng.choice(np.arange(nv + 1), size=int(rng.integers(0, 3)),
                                               replace=False) if int(x) != bg)
        iters = int(rng.integers(0, 12))
        lam = float(rng.uniform(0.1, 1.0))
        d = float(rng.choice([0.2, 0.5, 1.0]))
        shape = "sphere" if c % 4 == 1 else "box"
        spacing = (float(rng.uniform(0.5, 2)), float(rng.uniform(0.5, 2)), 3.0)
        origin = (float(rng.uniform(-5, 5)), float(rng.uniform(-5, 5)), float(rng.uniform(-5, 5)))
        announce(f"2D random {c}: {M}x{N} {np.dtype(dt).name} nv={nv} sel={sel} bg={bg} "
                 f"iters={iters} {shape}")
        run_image(ctx, sn, img, sel, bg, iters, lam, d, shape, spacing, origin)


def test_u32_selection_forms_2d(ctx, sn):
    """u32 images with a selection of small labels (bitmap classification, next
    to values of 65536 and more that share their low bits) and of large
    labels (sorted-list classification)."""
    rng = np.random.default_rng(31)
    pool = np.array([0, 1, 2, 65536 + 1, 65536 + 2, 2**32 - 1, 70_000, 70_001], dtype=np.uint64)
    for M, N in ((37, 29), (64, 21)):
        img = pool[rng.integers(0, len(pool), size=(N, M))].astype(np.uint32)
        for sel in ((1,), (2, 65535), (70_000,), (65537, 2**32 - 1)):
            announce(f"2D u32 selection {sel} {M}x{N}")
            run_image(ctx, sn, img, selected=sel, iters=4)


def test_degenerate_images(ctx, sn):
    for shape in [(1, 1), (1, 17), (17, 1), (2, 2), (2, 130)]:
        announce(f"2D degenerate {shape}")
        img = np.arange(np.prod(shape)).reshape(shape).astype(np.uint8)
        run_image(ctx, sn, img, iters=4)


def test_section_image(ctx, sn):
    """A 2048^2 section-like image (both generation forms: the staged form
    runs for images with at least 8 points per cell word on average)."""
    v = synth.section_like(seed=11, n=2048, n_cells=2500)
    announce("2D section 2048^2 u32")
    run_image(ctx, sn, v.labels, iters=v.iterations, lam=v.relaxation, d=v.constraint)
    announce("2D section 2048^2 u32, one label of many selected, sphere")
    run_image(ctx, sn, v.labels, selected=(17, 1000), iters=5, d=0.5, shape="sphere")


def test_section_bench_size(ctx, sn):
    """The benchmark's 2D configuration in full: the 8192^2 section-like u32
    image, extraction and 20 sweeps, every output against the oracle."""
    v = synth.section_like()
    announce(f"2D {v.name}, {v.iterations} sweeps")
    run_image(ctx, sn, v.labels, iters=v.iterations, lam=v.relaxation, d=v.constraint)


def test_batch_of_images_and_volumes(ctx, sn, torch):
    """Images and volumes in one batch: every mesh equals its plain extraction."""
    rng = np.random.default_rng(5)
    vols = []
    for c in range(8):
        if c % 2:
            M, N = (int(x) for x in rng.integers(20, 200, size=2))
            vols.append(synth.blocky_tiny(rng, (M, N, 1), 5, np.uint16).reshape(N, M))
        else:
            vols.append(synth.blocky_tiny(rng, (24, 20, 16), 5, np.uint16))
    params = [(int(rng.integers(3, 15)), 0.5, 1.0) for _ in vols]
    ts = [sn.to_device(v) for v in vols]
    announce("2D/3D mixed batch")
    meshes = ctx.batch_submit([dict(labels=t) for t in ts], params)
    for v, t, m, (it, lam, d) in zip(vols, ts, meshes, params):
        a = m.to_host()
        p = ctx.extract(t)
        ctx.smooth(p, iterations=it, relaxation=lam, constraint=d)
        b = p.to_host()
        for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
            np.testing.assert_array_equal(getattr(a, f), getattr(b, f), err_msg=f)
        m.free()
        p.free()


def test_served_images_equal_plain(ctx, sn, torch):
    """Images and volumes served together (fused into batches on two streams):
    every result equals the plain result of the same request."""
    rng = np.random.default_rng(9)
    items = []
    for c in range(12):
        if c % 3:
            M, N = (int(x) for x in rng.integers(30, 300, size=2))
            lab = synth.blocky_tiny(rng, (M, N, 1), 6, np.uint16).reshape(N, M)
        else:
            lab = synth.blocky_tiny(rng, (20, 18, 14), 6, np.uint16)
        items.append((sn.to_device(lab), int(rng.integers(2, 12))))
    alone = []
    for t, it in items:
        m = ctx.extract(t)
        ctx.smooth(m, iterations=it, relaxation=0.5, constraint=0.8)
        alone.append(m.to_host())
        m.free()
    srv = ctx.serve_start(hbm_budget_bytes=2 << 30, max_inflight=16, n_streams=2, max_batch=6)
    try:
        announce(f"2D/3D served: {len(items)} requests")
        tickets = [srv.submit(t, iterations=it, relaxation=0.5, constraint=0.8) for t, it in items]
        for tk, ref in zip(tickets, alone):
            got = srv.wait(tk, timeout_us=60_000_000)
            g = got.to_host()
            for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
                np.testing.assert_array_equal(getattr(g, f), getattr(ref, f), err_msg=f)
            got.free()
    finally:
        srv.stop()


def test_invalid_image_arguments(ctx, sn, torch):
    t = sn.to_device(np.zeros((5, 6), np.uint16))
    m = ctx.extract(t)
    with pytest.raises(sn.SNError):
        ctx.triangulate(m, "fixed")  # an image's contour has no quads
    m.free()
    v, keep = sn.make_volume(sn.to_device(np.zeros((2, 5, 6), np.uint16)))
    v.prim = sn.SN_LINES  # an image must have dims[2] == 1
    out = ctypes.c_void_p()
    assert sn._lib.sn_extract(ctx._h, ctypes.byref(v), None, ctypes.byref(out)) == sn.SN_EINVAL
