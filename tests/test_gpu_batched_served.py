"""GPU checks of the batched and served forms: every mesh that comes out of a
batch (one fused extraction over many volumes, one sweep graph for
all of them) or out of the request server (continuous batching on several
streams) is the mesh the plain per-volume path gives for the same volume and
parameters, byte for byte; a sample of them is also checked against the
oracle to the parity bar (topology bit-exact, offsets within 1e-5 voxel)."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
FIELDS = ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids")


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


def same_mesh(a, b, what):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x.dtype == y.dtype and x.shape == y.shape, f"{what}: {f} {x.shape} vs {y.shape}"
        assert np.array_equal(x, y), f"{what}: {f} differs"


def against_oracle(g, labels, selected, background, iters, lam, d):
    import oracle

    o = oracle.extract(labels, selected, background)
    assert g.points.shape[0] == o.n_points
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if o.n_points:
        ref = o.smooth(iters, lam, d) - o.centres()
        assert np.max(np.abs(g.offsets.astype(np.float64) - ref)) <= TOL


def mixed_volumes(seed, count):
    """Uneven sizes (ragged rows, 1..6 words per row), all three label types,
    selections and non-zero backgrounds, per-volume smoothing parameters.
    Volumes 5, 29, ... (u32) have their labels above 65536 (a selection takes the
    sorted-list classification, the other u32 selections the bitmap)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        dims = (int(rng.integers(3, 300)), int(rng.integers(2, 40)), int(rng.integers(2, 30)))
        if k % 9 == 4:
            dims = (1, 5, 5)  # no cells at all
        dt = [np.uint8, np.uint16, np.uint32][k % 3]
        nv = int(rng.integers(2, 9))
        gen = synth.blocky_tiny if k % 2 else synth.random_tiny
        lab = gen(rng, dims, nv, dt)
        bg = int(rng.integers(0, 2))
        sel = ()
        if k % 4 == 1:
            sel = tuple(sorted({int(x) for x in rng.integers(0, nv, size=3)} - {bg}))
        if k % 24 == 5:  # u32
            lab = (lab.astype(np.uint64) + 70_000).astype(np.uint32)
            sel = tuple(x + 70_000 for x in sel)
        params = (int(rng.integers(0, 30)), float(rng.choice([0.25, 0.5, 1.0])),
                  float(rng.choice([0.5, 0.8, 1.0])))
        sp = tuple(float(x) for x in rng.uniform(0.5, 2.5, size=3))
        out.append(dict(labels=lab, selected=sel, background=bg, params=params, spacing=sp))
    return out


def plain_result(ctx, sn, t, v):
    m = ctx.extract(t, spacing=v["spacing"], selected=v["selected"], background=v["background"])
    it, lam, d = v["params"]
    ctx.smooth(m, iterations=it, relaxation=lam, constraint=d)
    g = m.to_host()
    m.free()
    return g


def test_batch_marshalling_matches_single(sn, torch):
    """The batch call's record arrays hold, field for field, what the
    single-volume structures hold (the selected labels by content)."""
    import ctypes

    rng = np.random.default_rng(5)
    specs = [dict(labels=sn.to_device(rng.integers(0, 9, (4, 5, 7)).astype(np.uint8))),
             dict(labels=sn.to_device(rng.integers(0, 9, (3, 6)).astype(np.uint16)),
                  spacing=(0.5, 2, 3), origin=(1, -2, 7.5)),
             dict(labels=sn.to_device(rng.integers(0, 9, (6, 5, 4)).astype(np.uint32)),
                  selected=(3, 1, 3), background=2, prim=sn.SN_TRIS)]
    arr, keep = sn.volume_array(specs)
    for k, d in enumerate(specs):
        v, kp = sn.make_volume(**d)
        for f in ("labels", "dtype", "n_selected", "background", "prim"):
            assert int(arr[f][k]) == int(getattr(v, f) or 0), (k, f)
        for f in ("dims", "spacing", "origin"):
            assert list(arr[f][k]) == list(getattr(v, f)), (k, f)
        if v.n_selected:
            got = np.ctypeslib.as_array(ctypes.cast(int(arr["selected"][k]),
                                                    ctypes.POINTER(ctypes.c_uint32)), (v.n_selected,))
            assert list(got) == list(v.selected[:v.n_selected])
    pa = sn.params_array([(5, 0.25, 0.8), (0, 1.0, 0.0, "sphere"), (7, 0.5, 1.0, 1)])
    for k, p in enumerate([(5, 0.25, 0.8), (0, 1.0, 0.0, "sphere"), (7, 0.5, 1.0, 1)]):
        q = sn.smooth_params(*p)
        assert (int(pa["iterations"][k]), float(pa["relaxation"][k]), float(pa["constraint"][k]),
                int(pa["shape"][k])) == (q.iterations, q.relaxation, q.constraint, q.shape)
    with pytest.raises(TypeError):
        sn.volume_array([dict(labels=specs[0]["labels"], spacng=(1, 1, 1))])


def test_batched_equals_plain(ctx, sn):
    vols = mixed_volumes(21, 40)
    ts = [sn.to_device(v["labels"]) for v in vols]
    alone = []
    for k, (t, v) in enumerate(zip(ts, vols)):
        announce(f"plain {k}: dims={v['labels'].shape[::-1]} {v['labels'].dtype} {v['params']}")
        alone.append(plain_result(ctx, sn, t, v))
    specs = [dict(labels=t, spacing=v["spacing"], selected=v["selected"],
                  background=v["background"]) for t, v in zip(ts, vols)]
    announce(f"batch of {len(vols)}")
    ms = ctx.batch_submit(specs, [v["params"] for v in vols])
    for k, m in enumerate(ms):
        same_mesh(m.to_host(), alone[k], f"batched volume {k}")
        m.free()
    for k in (0, 1, 2, 5, 7):
        v = vols[k]
        announce(f"oracle check of volume {k}")
        against_oracle(alone[k], v["labels"], v["selected"], v["background"], *v["params"])


def test_batched_schedules_and_repeat(ctx, sn):
    """Two batches in a row, the second smaller, under several batches-per-wave
    schedules: same bytes as the plain path every time."""
    vols = mixed_volumes(22, 12)
    ts = [sn.to_device(v["labels"]) for v in vols]
    alone = [plain_result(ctx, sn, t, v) for t, v in zip(ts, vols)]
    try:
        for bpw in (1, 4, 16):
            ctx.set_batches_per_wave(bpw)
            for lo in (0, 7):
                announce(f"batch bpw={bpw} from {lo}")
                specs = [dict(labels=ts[k], spacing=vols[k]["spacing"],
                              selected=vols[k]["selected"], background=vols[k]["background"])
                         for k in range(lo, len(vols))]
                ms = ctx.batch_submit(specs, [vols[k]["params"] for k in range(lo, len(vols))])
                for j, m in enumerate(ms):
                    same_mesh(m.to_host(), alone[lo + j], f"bpw {bpw} volume {lo + j}")
                    m.free()
    finally:
        ctx.set_batches_per_wave(0)


def test_meshes_freed_while_their_batch_runs(ctx, sn):
    """The meshes of one batch call share a completion event, and a freed
    mesh's blocks go back to the pool to be reused once that event has
    completed.  Meshes freed while their batch still runs, a batch mesh
    smoothed again on its own (it then takes an event of its own) whose batch
    mates are freed before it, and later calls that reuse the freed blocks:
    every mesh keeps the plain path's bytes."""
    vols = mixed_volumes(24, 16)
    ts = [sn.to_device(v["labels"]) for v in vols]
    alone = [plain_result(ctx, sn, t, v) for t, v in zip(ts, vols)]
    specs = [dict(labels=t, spacing=v["spacing"], selected=v["selected"],
                  background=v["background"]) for t, v in zip(ts, vols)]
    params = [v["params"] for v in vols]
    for rep in range(3):
        announce(f"free while running, round {rep}")
        ms = ctx.batch_submit(specs, params)
        for m in ms[::2]:
            m.free()  # its batch is most likely still running
        again = ctx.batch_submit(specs, params)
        keep = ms[1]
        it, lam, d = vols[1]["params"]
        ctx.smooth(keep, iterations=it, relaxation=lam, constraint=d)
        for m in ms[3::2]:
            m.free()
        plain = [plain_result(ctx, sn, ts[k], vols[k]) for k in (0, 2, 4)]
        same_mesh(keep.to_host(), alone[1], f"round {rep}: re-smoothed batch mesh")
        keep.free()
        for k, m in enumerate(again):
            same_mesh(m.to_host(), alone[k], f"round {rep}: second batch volume {k}")
            m.free()
        for g, k in zip(plain, (0, 2, 4)):
            same_mesh(g, alone[k], f"round {rep}: plain volume {k}")


def test_served_equals_alone(ctx, sn, torch):
    """Requests submitted in a burst are fused into batches on two streams; every
    result equals the plain result for the same request run alone."""
    vols = mixed_volumes(23, 30)
    ts = [sn.to_device(v["labels"]) for v in vols]
    alone = [plain_result(ctx, sn, t, v) for t, v in zip(ts, vols)]
    srv = ctx.serve_start(hbm_budget_bytes=4 << 30, max_inflight=32, n_streams=2, max_batch=8)
    try:
        order = list(range(len(vols))) * 2  # each volume requested twice
        announce(f"served: {len(order)} requests")
        tickets = []
        for k in order:
            v = vols[k]
            it, lam, d = v["params"]
            tickets.append((k, srv.submit(ts[k], iterations=it, relaxation=lam, constraint=d,
                                          spacing=v["spacing"], selected=v["selected"],
                                          background=v["background"])))
        for k, tk in tickets:
            m = srv.wait(tk, timeout_us=60_000_000)
            same_mesh(m.to_host(), alone[k], f"served request of volume {k}")
            m.free()
        st = srv.stats()
        assert st["n_done"] == len(order) and st["n_rejected"] == 0
        assert st["n_batches"] < len(order), "requests were never fused into batches"
        assert st["p99_us"] >= st["p50_us"] > 0
    finally:
        srv.stop()


def test_served_admission_by_footprint(ctx, sn, torch):
    """A budget below one request's footprint still runs it (alone), and the
    reserved bytes never exceed the budget while more than one request is in
    flight."""
    rng = np.random.default_rng(24)
    labs = [synth.blocky_tiny(rng, (120, 90, 60), 5, np.uint16) for _ in range(6)]
    ts = [sn.to_device(x) for x in labs]
    ref = []
    for t in ts:
        m = ctx.extract(t)
        ctx.smooth(m, iterations=12)
        ref.append(m.to_host())
        m.free()
    budget = 1 << 20  # smaller than any single footprint
    srv = ctx.serve_start(hbm_budget_bytes=budget, max_inflight=8, n_streams=2, max_batch=8)
    try:
        announce("served under a tiny budget")
        tks = [srv.submit(t, iterations=12) for t in ts]
        for k, tk in enumerate(tks):
            m = srv.wait(tk, timeout_us=60_000_000)
            same_mesh(m.to_host(), ref[k], f"tiny-budget request {k}")
            m.free()
        st = srv.stats()
        assert st["n_done"] == len(ts)
        assert st["n_batches"] == len(ts), "over-budget requests must run one at a time"
    finally:
        srv.stop()


def test_served_poll_and_stop(ctx, sn, torch):
    rng = np.random.default_rng(25)
    lab = synth.blocky_tiny(rng, (64, 40, 30), 4, np.uint8)
    t = sn.to_device(lab)
    srv = ctx.serve_start(hbm_budget_bytes=1 << 30, n_streams=1)
    tk = srv.submit(t, iterations=5)
    announce("poll until done")
    m = None
    for _ in range(200000):
        m = srv.poll(tk)
        if m is not None:
            break
    if m is None:
        m = srv.wait(tk, timeout_us=60_000_000)
    ref = plain_result(ctx, sn, t, dict(spacing=(1.0, 1.0, 1.0), selected=(), background=0,
                                        params=(5, 0.5, 1.0)))
    same_mesh(m.to_host(), ref, "polled request")
    m.free()
    with pytest.raises(sn.SNError):
        srv.poll(tk)  # already claimed
    srv.stop()
