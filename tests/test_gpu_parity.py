"""GPU parity: the HIP path (through the C ABI) against the oracle.

Bar: points, quads, label pairs and stencil bit-exact; smoothed cell-relative
offsets within 1e-5 voxel of the FP64 oracle; world points within
1e-5 * spacing + 1 float32 ulp.  The 1e-5 bound holds by construction: each
sweep is a convex combination followed by a clamp (non-expansive in the max
norm), computed in FP64 and stored in FP32, so the stored error grows by at
most half an FP32 ulp of |offset| <= constraint per sweep: <= 40 * 2^-25 ~ 1.2e-6
for 40 sweeps at constraint 1.
"""
from __future__ import annotations

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


def check_mesh(g, o, labels_dtype, prim=4):
    assert g.points.shape[0] == o.n_points, (g.points.shape, o.n_points)
    assert g.stencil_ids.shape[0] == o.n_stencil
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if prim == 4:
        np.testing.assert_array_equal(g.polys, o.quads)
        np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    else:
        tris, tp = o.triangulate()
        np.testing.assert_array_equal(g.polys, tris)
        np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), tp)
    assert g.label_pairs.dtype == labels_dtype


def check_smooth(g, o, iters, lam, d, spacing=(1, 1, 1), origin=(0, 0, 0)):
    import oracle

    pos = o.smooth(iters, lam, d)
    ref = pos - o.centres()
    if o.n_points:
        err = np.max(np.abs(g.offsets.astype(np.float64) - ref))
        assert err <= TOL, f"offset error {err}"
        w = oracle.world(pos, origin, spacing)
        h = np.asarray(spacing, np.float64)
        ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(g.points.astype(np.float64) - w) <= TOL * h + ulp)
    return ref


def run_case(ctx, sn, vol, selected=(), background=0, iters=0, lam=0.5, d=1.0,
             spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), prim=4):
    import oracle

    t = sn.to_device(vol)
    m = ctx.extract(t, spacing=spacing, origin=origin, selected=selected, background=background,
                    prim=prim)
    ctx.smooth(m, iterations=iters, relaxation=lam, constraint=d)
    g = m.to_host()
    o = oracle.extract(vol, selected, background)
    check_mesh(g, o, vol.dtype, prim)
    check_smooth(g, o, iters, lam, d, spacing, origin)
    m.free()
    return g, o


def test_tiny_random_cases(ctx, sn):
    """Many small volumes: ragged rows (M not a multiple of 64), several words
    per row, all dtypes, selections, non-zero backgrounds, degenerate dims."""
    rng = np.random.default_rng(1234)
    for case in range(160):
        dims = tuple(int(x) for x in rng.integers(1, 20, size=3))
        if case % 10 == 0:
            dims = (int(rng.integers(60, 200)), int(rng.integers(2, 6)), int(rng.integers(2, 6)))
        dt = [np.uint8, np.uint16, np.uint32][case % 3]
        nv = int(rng.integers(1, 8))
        gen = synth.blocky_tiny if case % 2 else synth.random_tiny
        vol = gen(rng, dims, nv, dt)
        bg = int(rng.integers(0, 3))
        sel = ()
        if case % 4 == 1:
            sel = tuple(sorted({int(x) for x in rng.integers(0, nv, size=2)} - {bg}))
        iters = int(rng.integers(0, 12))
        lam = float(rng.choice([0.0, 0.3, 0.5, 1.0]))
        d = float(rng.choice([0.0, 0.25, 0.8, 1.0]))
        sp = tuple(float(x) for x in rng.uniform(0.5, 3.0, size=3))
        org = tuple(float(x) for x in rng.uniform(-50, 50, size=3))
        prim = 3 if case % 7 == 3 else 4
        announce(f"tiny {case}: dims={dims} dtype={np.dtype(dt).name} sel={sel} bg={bg} "
                 f"iters={iters} lam={lam} d={d} prim={prim}")
        run_case(ctx, sn, vol, sel, bg, iters, lam, d, sp, org, prim)


@pytest.mark.parametrize("bpw", [1, 2, 4, 8, 16])
def test_schedule_invariance(ctx, sn, bpw):
    """Every batches-per-wave schedule gives the same bytes (rows of 3, 4, 5
    and 7 words: ragged batches and tiles that straddle rows)."""
    rng = np.random.default_rng(77)
    announce(f"schedule bpw={bpw}")
    ctx.set_batches_per_wave(bpw)
    try:
        for M in (130, 250, 300, 420):
            vol = synth.blocky_tiny(rng, (M, 21, 9), 6, np.uint16)
            run_case(ctx, sn, vol, iters=7)
    finally:
        ctx.set_batches_per_wave(0)


SCHEDULES = [dict(edge_segments=1, count_words=1, gen_groups=1),
             dict(edge_segments=2, count_words=4, gen_groups=3),
             dict(edge_segments=8, count_words=1, gen_groups=8),
             dict(edge_segments=16, count_words=4, gen_groups=16)]


@pytest.mark.parametrize("k", range(len(SCHEDULES)))
def test_schedule_knobs(sn, torch, k):
    """Every value of every schedule knob (k_edges segments per wave, the
    k_count form, k_generate groups per wave) gives the oracle's results:
    rows of ragged lengths (short rows sharing segments, rows of several
    segments), all label types, an image, and a batch of them; the sweep
    chunk of the large-mesh form on the torso and the 2D section."""
    sc = SCHEDULES[k]
    rng = np.random.default_rng(90 + k)
    c = sn.Context(0)
    try:
        vols = [synth.blocky_tiny(rng, (M, 23, 11), 6, dt)
                for M, dt in ((40, np.uint8), (100, np.uint16), (300, np.uint32), (530, np.uint16))]
        for vol in vols:
            announce(f"schedule {sc}: dims={vol.shape[::-1]} {vol.dtype}")
            c.schedule_set(sn.to_device(vol), **sc)
            assert {f: c.schedule_get(sn.to_device(vol))[f] for f in sc} == sc
            run_case(c, sn, vol, iters=5)
        img = synth.blocky_tiny(rng, (333, 97, 1), 5, np.uint16).reshape(97, 333)
        ti = sn.to_device(img)
        c.schedule_set(ti, prim=sn.SN_LINES, **sc)
        m = c.extract(ti)
        g = m.to_host()
        m.free()
        import oracle

        o = oracle.extract2d(img)
        np.testing.assert_array_equal(g.polys, o.quads)
        np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
        # a batch takes the schedule of its largest volume
        ts = [sn.to_device(v) for v in vols]
        plain = []
        for t in ts:
            m = c.extract(t)
            c.smooth(m, iterations=5)
            plain.append(m.to_host())
            m.free()
        ms = c.batch_submit([dict(labels=t) for t in ts], [(5, 0.5, 1.0)] * len(ts))
        for kk, m in enumerate(ms):
            g = m.to_host()
            m.free()
            for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
                assert np.array_equal(getattr(g, f), getattr(plain[kk], f)), (kk, f)
    finally:
        c.close()


def test_sweep_chunk_knob(sn, torch, monkeypatch):
    """The sweep chunk of a schedule sets the slab-chunked block order of the
    large-mesh form (here forced on the torso): offsets equal the oracle's for
    chunks of 1, 7 and 64 blocks."""
    import oracle

    monkeypatch.setenv("SN_TEST_SWEEP_SMALL_POINTS", "0")
    c = sn.Context(0)
    monkeypatch.delenv("SN_TEST_SWEEP_SMALL_POINTS")
    try:
        v = synth.torso_like()
        t = sn.to_device(v.labels)
        o = oracle.extract(v.labels)
        ref = o.smooth(v.iterations, v.relaxation, v.constraint) - o.centres()
        for ch in (1, 7, 64):
            announce(f"sweep chunk {ch} on the torso (large-mesh form)")
            c.schedule_set(t, sweep_chunk=ch)
            m = c.extract(t, spacing=v.spacing)
            c.smooth(m, iterations=v.iterations, relaxation=v.relaxation, constraint=v.constraint)
            g = m.to_host()
            m.free()
            assert np.max(np.abs(g.offsets.astype(np.float64) - ref)) <= TOL
    finally:
        c.close()


def test_autotune_records_a_valid_schedule(sn, torch, tmp_path, monkeypatch):
    """sn_autotune picks a schedule within the knobs' ranges, reports it, keeps
    it in SN_AUTOTUNE_CACHE (read back by a new context), and extraction under
    it gives the oracle's results."""
    import json

    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SN_AUTOTUNE_CACHE", str(cache))
    c = sn.Context(0)
    try:
        rng = np.random.default_rng(95)
        vol = synth.blocky_tiny(rng, (200, 60, 40), 7, np.uint16)
        t = sn.to_device(vol)
        announce("autotune on a 200x60x40 u16 volume")
        g = c.autotune(t)
        sc = c.schedule_get(t)
        assert g == sc["gen_groups"]
        # count_words 0 is the size-based default, kept when neither form beats it
        assert sc["edge_segments"] in (1, 2, 4, 8) and sc["count_words"] in (0, 1, 4)
        assert sc["gen_groups"] in (1, 2, 3, 4, 8)
        run_case(c, sn, vol, iters=4)
        saved = json.loads(cache.read_text())
        assert any(e["edge_segments"] == sc["edge_segments"] for e in saved.values())
    finally:
        c.close()
    c2 = sn.Context(0)
    try:
        assert c2.schedule_get(t) == sc
    finally:
        c2.close()


def test_dtype_edge_values(ctx, sn):
    rng = np.random.default_rng(5)
    for dt, top in ((np.uint8, 255), (np.uint16, 65535), (np.uint32, 2**32 - 1)):
        base = synth.random_tiny(rng, (23, 17, 11), 3, dt)
        vol = np.where(base == 2, top, base).astype(dt)
        announce(f"edge values {np.dtype(dt).name} top={top}")
        run_case(ctx, sn, vol, iters=3)                       # top as a label
        run_case(ctx, sn, vol, background=top, iters=3)       # top as background
        run_case(ctx, sn, vol, selected=(top,), iters=3)      # only top selected
        run_case(ctx, sn, vol, selected=(1, top), background=0, iters=3)


@pytest.mark.parametrize("offset", [0, 70_000])
def test_large_selection_u32(ctx, sn, offset):
    """A u32 selection with many entries: labels below 65536 take the bitmap,
    larger ones the sorted list."""
    rng = np.random.default_rng(6)
    vol = (rng.integers(0, 5000, size=(20, 30, 40)) + offset).astype(np.uint32)
    sel = tuple(int(x) + offset for x in rng.choice(5000, size=1500, replace=False) if x != 0)
    announce(f"u32 selection of 1500 labels from {offset}")
    run_case(ctx, sn, vol, selected=sel, iters=2)


def test_u32_small_selection_ignores_large_values(ctx, sn):
    """A u32 selection of small labels (bitmap classification) next to values
    of 65536 and more, some equal to a selected label modulo 2^16 or 2^5:
    those are never selected."""
    rng = np.random.default_rng(8)
    pool = np.array([0, 1, 2, 3, 65536, 65537, 65538, 65536 + 3, 2**31 + 1, 2**32 - 1,
                     2**32 - 65536 + 2, 33, 35], dtype=np.uint64)
    for shape in ((14, 19, 23), (9, 13, 24)):  # ragged rows, then rows of a multiple of 4
        vol = pool[rng.integers(0, len(pool), size=shape)].astype(np.uint32)
        for sel, bg in (((1, 3), 0), ((2,), 7), ((1, 2, 3, 33), 0), ((65535,), 0)):
            announce(f"u32 small selection {sel} bg={bg} shape={shape}")
            run_case(ctx, sn, vol, selected=sel, background=bg, iters=3)
    vol2 = np.where(vol == 65536, 65535, vol).astype(np.uint32)
    announce("u32 selection of 65535 next to 65536")
    run_case(ctx, sn, vol2, selected=(65535,), iters=2)


def test_degenerate_volumes(ctx, sn):
    for dims in [(1, 1, 1), (1, 7, 7), (7, 1, 7), (7, 7, 1), (2, 2, 2), (2, 30, 2)]:
        M, N, O = dims
        vol = (np.arange(M * N * O) % 3).astype(np.uint16).reshape(O, N, M)
        announce(f"degenerate {dims}")
        run_case(ctx, sn, vol, iters=2)
    announce("uniform volume")
    run_case(ctx, sn, np.full((9, 8, 7), 3, np.uint16), iters=4)
    v = np.zeros((3, 3, 3), np.uint8)
    v[1, 1, 1] = 9
    announce("single voxel")
    g, _ = run_case(ctx, sn, v, iters=16, lam=0.5, d=1.0)
    np.testing.assert_allclose(np.abs(g.offsets), 0.5 - 0.5 * (2 / 3) ** 16, atol=TOL)


def test_spheres_small_config(ctx, sn):
    v = synth.spheres_small()
    announce(v.name)
    run_case(ctx, sn, v.labels, iters=v.iterations, lam=v.relaxation, d=v.constraint)


def test_torso_like_config(ctx, sn):
    v = synth.torso_like()
    announce(v.name)
    run_case(ctx, sn, v.labels, iters=v.iterations, lam=v.relaxation, d=v.constraint,
             spacing=v.spacing)


def test_resmooth_restarts_from_cache(ctx, sn, torch):
    import oracle

    rng = np.random.default_rng(8)
    vol = synth.blocky_tiny(rng, (40, 33, 21), 5, np.uint16)
    t = sn.to_device(vol)
    m = ctx.extract(t)
    o = oracle.extract(vol)
    for iters, lam, d in [(20, 0.5, 1.0), (5, 1.0, 0.3), (20, 0.5, 1.0), (0, 0.5, 1.0),
                          (33, 0.25, 0.6)]:
        announce(f"resmooth {iters} {lam} {d}")
        ctx.smooth(m, iterations=iters, relaxation=lam, constraint=d)
        check_smooth(m.to_host(), o, iters, lam, d)
    m.free()


def test_graph_replays_match_eager(ctx, sn, torch):
    """Batches smooth through a HIP graph of sweep kernels; repeated with other
    device work and synchronisations in between, every batch gives the result
    of the single-mesh path with one profiled launch per sweep."""
    rng = np.random.default_rng(9)
    vols = [synth.blocky_tiny(rng, (70, 50, 30), 7, np.uint16),
            synth.blocky_tiny(rng, (40, 66, 21), 5, np.uint16),
            synth.random_tiny(rng, (33, 20, 17), 4, np.uint16)]
    params = [(17, 0.5, 0.7), (9, 0.25, 1.0), (23, 1.0, 0.4)]
    ts = [sn.to_device(v) for v in vols]
    ctx.profile(2)  # every sweep its own launch and events
    ref = []
    for t, (it, lam, d) in zip(ts, params):
        m = ctx.extract(t)
        ctx.smooth(m, iterations=it, relaxation=lam, constraint=d)
        ref.append(m.to_host())
        m.free()
    ctx.profile(False)
    ctx.profile_reset()
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(6):
        junk.add_(1.0)
        torch.cuda.synchronize()
        announce(f"batch graph replay {rep}")
        ms = ctx.batch_submit([dict(labels=t) for t in ts], params)
        for k, m in enumerate(ms):
            g = m.to_host()
            assert np.array_equal(g.offsets, ref[k].offsets), f"replay {rep} volume {k}"
            assert np.array_equal(g.points, ref[k].points), f"replay {rep} volume {k}"
            m.free()


def test_determinism(ctx, sn):
    rng = np.random.default_rng(10)
    vol = synth.random_tiny(rng, (100, 60, 40), 6, np.uint32)
    t = sn.to_device(vol)
    outs = []
    for _ in range(2):
        m = ctx.extract(t)
        ctx.smooth(m, iterations=9)
        outs.append(m.to_host())
        m.free()
    for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
        assert np.array_equal(getattr(outs[0], f), getattr(outs[1], f)), f


def test_invalid_arguments(ctx, sn, torch):
    t = sn.to_device(np.zeros((4, 4, 4), np.uint16))
    with pytest.raises(sn.SNError) as e:
        ctx.extract(t, spacing=(0.0, 1.0, 1.0))
    assert e.value.status == sn.SN_EINVAL
    with pytest.raises(sn.SNError):
        ctx.extract(t, selected=(0,), background=0)  # background selected
    with pytest.raises(sn.SNError):
        ctx.extract(t, background=70000)  # does not fit u16
    # sizes whose int32 indexing bound would overflow int64 if multiplied
    # unchecked: refused before any device work
    import ctypes
    for dims in [(1 << 30, 1 << 30, 1 << 30), (1 << 30, 1 << 16, 1 << 16), (64, 1 << 30, 1 << 30)]:
        v, keep = sn.make_volume(t)
        v.dims[:] = dims
        out = ctypes.c_void_p()
        st = sn._lib.sn_extract(ctx._h, ctypes.byref(v), None, ctypes.byref(out))
        assert st == sn.SN_ETOOBIG and not out.value, (dims, st)
    m = ctx.extract(t)
    with pytest.raises(sn.SNError):
        ctx.smooth(m, iterations=-1)
    with pytest.raises(sn.SNError):
        ctx.smooth(m, relaxation=1.5)
    m.free()


def test_wide_count_tiles(sn, torch, monkeypatch):
    """The counting pass's wide form (four words per thread, taken for large
    launches) forced on small volumes: same results against the oracle."""
    monkeypatch.setenv("SN_TEST_COUNT_WIDE_WORDS", "0")
    c = sn.Context(0)
    try:
        rng = np.random.default_rng(4321)
        for case in range(24):
            dims = (int(rng.integers(2, 300)), int(rng.integers(2, 40)), int(rng.integers(2, 30)))
            dt = [np.uint8, np.uint16, np.uint32][case % 3]
            vol = (synth.blocky_tiny if case % 2 else synth.random_tiny)(rng, dims, 5, dt)
            announce(f"wide count {case}: dims={dims} {np.dtype(dt).name}")
            run_case(c, sn, vol, iters=int(rng.integers(0, 8)))
        v = synth.torso_like()
        announce("wide count: " + v.name)
        run_case(c, sn, v.labels, iters=v.iterations, lam=v.relaxation, d=v.constraint,
                 spacing=v.spacing)
    finally:
        c.close()


def test_sphere_constraint(ctx, sn, torch):
    """Sphere constraint (radius d around the cell centre): offsets and world
    points against the oracle on tiny cases, spacing included, and the
    spheres configuration; the batched path with mixed shapes gives the
    plain results byte for byte."""
    import oracle

    rng = np.random.default_rng(41)
    cases = [
        (synth.random_tiny(rng, (30, 22, 17), 5, np.uint16), (1.0, 1.0, 1.0), (19, 1.0, 0.4)),
        (synth.blocky_tiny(rng, (41, 33, 25), 6, np.uint8), (0.6, 1.4, 2.5), (25, 0.5, 0.7)),
        (synth.random_tiny(rng, (18, 15, 12), 4, np.uint32), (1.0, 2.0, 1.0), (8, 0.9, 0.05)),
        (synth.spheres_small().labels, (1.0, 1.0, 1.0), (16, 0.5, 1.0)),
    ]
    plain = []
    for k, (lab, sp, (it, lam, d)) in enumerate(cases):
        announce(f"sphere constraint case {k}: dims={lab.shape[::-1]} {lab.dtype} {(it, lam, d)}")
        t = sn.to_device(lab)
        m = ctx.extract(t, spacing=sp)
        ctx.smooth(m, iterations=it, relaxation=lam, constraint=d, shape="sphere")
        g = m.to_host()
        m.free()
        plain.append(g)
        o = oracle.extract(lab)
        pos = o.smooth(it, lam, d, shape="sphere")
        ref = pos - o.centres()
        if o.n_points:
            err = np.max(np.abs(g.offsets.astype(np.float64) - ref))
            assert err <= TOL, f"case {k}: offset error {err}"
            assert np.max(np.linalg.norm(g.offsets.astype(np.float64), axis=1)) <= d + 1e-6
            w = oracle.world(pos, (0.0, 0.0, 0.0), sp)
            h = np.asarray(sp, np.float64)
            ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
            assert np.all(np.abs(g.points.astype(np.float64) - w) <= TOL * h + ulp)
    announce("sphere constraint: batch with mixed shapes")
    ts = [sn.to_device(lab) for lab, _, _ in cases]
    specs = [dict(labels=t, spacing=sp) for t, (_, sp, _) in zip(ts, cases)]
    params = [(it, lam, d, "sphere") for _, _, (it, lam, d) in cases]
    box = (9, 0.5, 0.6, "box")
    for m_, g, k in zip(ctx.batch_submit(specs + specs[:1], params + [box]), plain + [None],
                        range(len(cases) + 1)):
        h_ = m_.to_host()
        m_.free()
        if g is None:  # the same volume under the box constraint, alone
            m = ctx.extract(ts[0], spacing=cases[0][1])
            ctx.smooth(m, iterations=9, relaxation=0.5, constraint=0.6)
            g = m.to_host()
            m.free()
        assert np.array_equal(h_.offsets, g.offsets) and np.array_equal(h_.points, g.points), k


def test_label_subsets_of_many_spheres(ctx, sn, torch):
    """The label-count workload at reduced size (96^3 u16, 32 overlapping
    spheres): the first k labels selected, k = 1, 5, 32, against the oracle
    (topology bit-exact, smoothed offsets and world points to the bar)."""
    vol = synth.synthetic_spheres(seed=7, n=96, count=32)
    for k in (1, 5, 32):
        announce(f"label subset: first {k} of 32 spheres")
        run_case(ctx, sn, vol.labels, selected=tuple(range(1, k + 1)), iters=25, lam=0.5, d=1.0)


def test_extreme_aspect_ratios(ctx, sn, torch):
    """Rows far longer than a group (100 000 samples: 1 563 words per row, the
    x-neighbour distances of the sweeps and the row division of the world
    points at their widest), columns of one-cell rows (a group spans 32 rows),
    and a thin slab, each against the oracle, smoothed with both constraints."""
    rng = np.random.default_rng(51)
    cases = [((100_000, 3, 3), np.uint16, 7), ((3, 4, 70_000), np.uint8, 4),
             ((4, 40_000, 3), np.uint32, 9), ((700, 500, 3), np.uint16, 6)]
    for dims, dt, nv in cases:
        M, N, O = dims
        vol = synth.blocky_tiny(rng, dims, nv, dt)
        announce(f"extreme aspect {dims} {np.dtype(dt).name}")
        run_case(ctx, sn, vol, iters=6, lam=0.7, d=0.8, spacing=(0.5, 1.0, 3.0))
        t = sn.to_device(vol)
        m = ctx.extract(t)
        ctx.smooth(m, iterations=6, relaxation=0.7, constraint=0.8, shape="sphere")
        g = m.to_host()
        m.free()
        import oracle

        o = oracle.extract(vol)
        if o.n_points:
            ref = o.smooth(6, 0.7, 0.8, shape="sphere") - o.centres()
            assert np.max(np.abs(g.offsets.astype(np.float64) - ref)) <= TOL


@pytest.mark.parametrize("form", ["knob", "wide"])
def test_unpacked_neighbour_table(sn, torch, monkeypatch, form):
    """The sweeps keep the 16-byte neighbour table (ids plus the face byte)
    when a mesh's id distances do not fit the packed 8-byte word: forced by
    the context knob SN_TEST_SWEEP_UNPACKED on tiny volumes, the spheres
    configuration and a batch, and reached naturally by a volume whose rows
    (4095 cells) and slices (4095 x 129 cells) need 12 + 20 distance bits.
    Everything against the oracle; the batch equals the plain results."""
    import oracle

    rng = np.random.default_rng(81)
    if form == "knob":
        monkeypatch.setenv("SN_TEST_SWEEP_UNPACKED", "1")
        cases = [(synth.blocky_tiny(rng, (37, 29, 23), 5, np.uint16), (21, 0.5, 1.0)),
                 (synth.random_tiny(rng, (65, 9, 14), 4, np.uint8), (7, 1.0, 0.6)),
                 (synth.spheres_small().labels, (16, 0.5, 1.0))]
    else:
        cases = [(synth.blocky_tiny(rng, (4096, 130, 3), 6, np.uint16), (12, 0.5, 0.8))]
    c = sn.Context(0)
    monkeypatch.delenv("SN_TEST_SWEEP_UNPACKED", raising=False)
    try:
        plain = []
        for k, (lab, (it, lam, d)) in enumerate(cases):
            announce(f"unpacked table ({form}) case {k}: dims={lab.shape[::-1]} {(it, lam, d)}")
            t = sn.to_device(lab)
            m = c.extract(t)
            c.smooth(m, iterations=it, relaxation=lam, constraint=d)
            g = m.to_host()
            m.free()
            o = oracle.extract(lab)
            check_mesh(g, o, lab.dtype)
            check_smooth(g, o, it, lam, d)
            plain.append(g)
        if len(cases) > 1:
            announce(f"unpacked table ({form}): the cases as one batch")
            ts = [sn.to_device(lab) for lab, _ in cases]
            ms = c.batch_submit([dict(labels=t) for t in ts], [p for _, p in cases])
            for k, m in enumerate(ms):
                g = m.to_host()
                m.free()
                for f in ("points", "offsets", "polys", "label_pairs", "stencil_off",
                          "stencil_ids"):
                    assert np.array_equal(getattr(g, f), getattr(plain[k], f)), (k, f)
    finally:
        c.close()


@pytest.mark.gpu
def test_labels_at_unaligned_offsets(ctx, sn, torch):
    """Label volumes that start at every element offset of a larger buffer
    (base addresses not 4- or 16-byte aligned: the narrow row loads), with
    rows of odd and of 4-multiple lengths, equal the oracle."""
    import oracle

    rng = np.random.default_rng(77)
    for dt, offs in ((np.uint8, (1, 2, 3, 5)), (np.uint16, (1, 2, 3)), (np.uint32, (1, 2, 3))):
        for dims in ((37, 11, 7), (64, 9, 6), (200, 5, 4)):
            vol = synth.blocky_tiny(rng, dims, 6, dt)
            n = vol.size
            for off in offs:
                announce(f"unaligned: {np.dtype(dt).name} dims={dims} offset={off}")
                buf = np.zeros(n + 8, dt)
                buf[off:off + n] = vol.ravel()
                tb = sn.to_device(buf)
                t = tb[off:off + n].view(vol.shape)
                m = ctx.extract(t)
                ctx.smooth(m, iterations=3, relaxation=0.5, constraint=1.0)
                g = m.to_host()
                o = oracle.extract(vol)
                check_mesh(g, o, vol.dtype)
                check_smooth(g, o, 3, 0.5, 1.0)
                m.free()
