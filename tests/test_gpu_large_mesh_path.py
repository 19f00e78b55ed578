"""The large-mesh sweep form against the oracle in full.

Meshes of more than 2^24 points (sweep data far beyond the last-level cache)
take another form of the sweeps: non-temporal loads of the read-once streams
and non-temporal offset stores, and, for a single mesh, the slab-chunked
block order, in which XCD x takes logical blocks x*C .. x*C + C - 1 of every
run of 8*C blocks (the tail that does not fill a run keeps its blocks).  The
benchmark's connectome volume takes it; here the context's test knob
SN_TEST_SWEEP_SMALL_POINTS=0 sends every mesh there, and SN_TEST_SWEEP_CHUNK
sets C, so that element-by-element comparisons with the oracle cover the form
on tiny volumes (ragged runs and tails), the 64^3 spheres, the torso (several
chunk sizes, both constraint shapes), the 2D section image, a batch of 64
volumes, and the paper-scale synthetic volume (512^3, 128 spheres; one and
all labels selected, in both sweep forms).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from slab_oracle import compare_mesh

pytestmark = pytest.mark.gpu

TOL = 1e-5
WORKERS = max(1, min(16, os.cpu_count() or 1))


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


def announce(msg):
    print(f"[case] {msg}", flush=True)


def big_context(sn, monkeypatch, chunk=0):
    """A context whose every mesh takes the large-mesh sweep form (the knobs
    are read when the context is made)."""
    monkeypatch.setenv("SN_TEST_SWEEP_SMALL_POINTS", "0")
    if chunk:
        monkeypatch.setenv("SN_TEST_SWEEP_CHUNK", str(chunk))
    else:
        monkeypatch.delenv("SN_TEST_SWEEP_CHUNK", raising=False)
    c = sn.Context(0)
    monkeypatch.delenv("SN_TEST_SWEEP_SMALL_POINTS")
    monkeypatch.delenv("SN_TEST_SWEEP_CHUNK", raising=False)
    return c


def oracle_check(g, labels, iters, lam, d, shape="box", selected=(), background=0,
                 spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Every output of a volume's mesh against the oracle on the whole volume."""
    import oracle

    o = oracle.extract(labels, selected, background)
    assert g.points.shape[0] == o.n_points
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if o.n_points:
        pos = o.smooth(iters, lam, d, shape) if iters > 0 else o.centres()
        err = float(np.max(np.abs(g.offsets.astype(np.float64) - (pos - o.centres()))))
        assert err <= TOL, f"offsets differ by {err}"
        w = oracle.world(pos, origin, spacing)
        h = np.asarray(spacing, np.float64)
        ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(g.points.astype(np.float64) - w) <= TOL * h + ulp)


def run(ctx, sn, lab, iters, lam, d, shape="box", selected=(), background=0,
        spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    t = sn.to_device(lab)
    m = ctx.extract(t, spacing=spacing, origin=origin, selected=selected, background=background)
    ctx.smooth(m, iterations=iters, relaxation=lam, constraint=d, shape=shape)
    g = m.to_host()
    m.free()
    return g


@pytest.mark.parametrize("chunk", [0, 1, 2, 3, 5])
def test_tiny_volumes(sn, torch, monkeypatch, chunk):
    """Ragged volumes of up to a few thousand points (a few sweep blocks, so
    runs of 8*C blocks are often incomplete), all label types, both shapes."""
    c = big_context(sn, monkeypatch, chunk)
    try:
        rng = np.random.default_rng(900 + chunk)
        for case in range(30):
            dims = (int(rng.integers(2, 90)), int(rng.integers(2, 40)), int(rng.integers(2, 30)))
            dt = [np.uint8, np.uint16, np.uint32][case % 3]
            lab = (synth.blocky_tiny if case % 2 else synth.random_tiny)(rng, dims, 5, dt)
            it = int(rng.integers(0, 9))
            shape = "sphere" if case % 4 == 3 else "box"
            announce(f"large-mesh form, chunk {chunk}, case {case}: dims={dims} "
                     f"{np.dtype(dt).name} {it} sweeps {shape}")
            g = run(c, sn, lab, it, 0.6, 0.7, shape, spacing=(1.0, 2.0, 0.5), origin=(1, 2, 3))
            oracle_check(g, lab, it, 0.6, 0.7, shape, spacing=(1.0, 2.0, 0.5), origin=(1, 2, 3))
    finally:
        c.close()


@pytest.mark.parametrize("chunk", [0, 3, 7])
def test_configurations(sn, torch, monkeypatch, chunk):
    """The 64^3 spheres and the 256^3 torso (box and sphere) in the large-mesh
    form, against the oracle in full."""
    c = big_context(sn, monkeypatch, chunk)
    try:
        v = synth.spheres_small()
        announce(f"large-mesh form, chunk {chunk}: {v.name}")
        g = run(c, sn, v.labels, v.iterations, v.relaxation, v.constraint)
        oracle_check(g, v.labels, v.iterations, v.relaxation, v.constraint)
        v = synth.torso_like()
        for shape in ("box", "sphere"):
            announce(f"large-mesh form, chunk {chunk}: {v.name} {shape}")
            g = run(c, sn, v.labels, v.iterations, v.relaxation, v.constraint, shape,
                    spacing=v.spacing)
            oracle_check(g, v.labels, v.iterations, v.relaxation, v.constraint, shape,
                         spacing=v.spacing)
    finally:
        c.close()


def test_section_image(sn, torch, monkeypatch):
    """The 8192^2 section image (7.1 M points, one cell slice: the slab-chunked
    order spans the whole image, with a tail) in the large-mesh form."""
    import oracle

    c = big_context(sn, monkeypatch)
    try:
        v = synth.section_like()
        announce(f"large-mesh form: 2D {v.name}")
        g = run(c, sn, v.labels, v.iterations, v.relaxation, v.constraint)
    finally:
        c.close()
    o = oracle.extract2d(v.labels)
    assert g.points.shape[0] == o.n_points
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    pos = o.smooth(v.iterations, v.relaxation, v.constraint)
    err = float(np.max(np.abs(g.offsets[:, :2].astype(np.float64) - (pos - o.centres())[:, :2])))
    assert err <= TOL, f"offsets differ by {err}"
    assert np.all(g.offsets[:, 2] == 0.0)


@pytest.mark.timeout(600)
def test_batch_of_64(sn, torch, monkeypatch):
    """The batched workload with every mesh in the large-mesh form: batched
    equals plain byte for byte, and every mesh the oracle."""
    c = big_context(sn, monkeypatch)
    try:
        vols = synth.batch_volumes(count=64)
        ts = [sn.to_device(v.labels) for v in vols]
        announce("large-mesh form: batch of 64 volumes")
        ms = c.batch_submit([dict(labels=t) for t in ts],
                            [(v.iterations, v.relaxation, v.constraint) for v in vols])
        got = [m.to_host() for m in ms]
        for m in ms:
            m.free()
        for k, (t, v) in enumerate(zip(ts, vols)):
            m = c.extract(t)
            c.smooth(m, iterations=v.iterations, relaxation=v.relaxation, constraint=v.constraint)
            p = m.to_host()
            m.free()
            for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
                assert np.array_equal(getattr(got[k], f), getattr(p, f)), f"volume {k}: {f}"
    finally:
        c.close()
    announce(f"oracle check of all 64 volumes, {WORKERS} threads")
    with ThreadPoolExecutor(max_workers=WORKERS) as ex:
        futs = [ex.submit(oracle_check, got[k], v.labels, v.iterations, v.relaxation, v.constraint)
                for k, v in enumerate(vols)]
        for f in futs:
            f.result()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("big", [False, True])
def test_paper_scale_synthetic(sn, torch, monkeypatch, big):
    """The paper-scale synthetic volume (512^3 u16, 128 overlapping spheres,
    25 sweeps) with the first label and with all 128 selected, against the
    oracle (assembled from z-slab crops) in full; in the form its size takes
    (3.4 M points: the cache-resident form) and in the large-mesh form."""
    if big:
        c = big_context(sn, monkeypatch)
    else:
        c = sn.Context(0)
    v = synth.synthetic_spheres()
    try:
        for k in (1, 128):
            sel = tuple(range(1, k + 1))
            announce(f"{v.name}, first {k} labels, large-mesh form {big}")
            g = run(c, sn, v.labels, v.iterations, v.relaxation, v.constraint, selected=sel)
            compare_mesh(g, v.labels, v.iterations, v.relaxation, v.constraint, selected=sel,
                         slab=32, workers=WORKERS)
    finally:
        c.close()


def test_world_points_from_emit(sn, torch, monkeypatch):
    """Volumes of 2^32 cells or more keep no cell index per point, so their
    world points come from k_emit after the sweeps instead of from the last
    sweep.  The knob SN_TEST_NO_PCELL sends small volumes there: plain calls
    (both sweep forms) and a batch give the bytes of the ordinary path, and
    the oracle's offsets and world points."""
    import oracle

    rng = np.random.default_rng(61)
    vols = [synth.blocky_tiny(rng, (45, 23, 17), 6, np.uint16),
            synth.random_tiny(rng, (19, 31, 12), 4, np.uint8),
            synth.blocky_tiny(rng, (130, 9, 7), 5, np.uint32)]
    params = [(9, 0.5, 0.8), (0, 0.5, 1.0), (4, 1.0, 0.3)]
    spacing, origin = (0.7, 1.3, 2.1), (3.0, -4.0, 1.5)
    monkeypatch.delenv("SN_TEST_NO_PCELL", raising=False)
    ref_ctx = sn.Context(0)
    try:
        ref = []
        for v, (it, lam, d) in zip(vols, params):
            m = ref_ctx.extract(sn.to_device(v), spacing=spacing, origin=origin)
            ref_ctx.smooth(m, iterations=it, relaxation=lam, constraint=d)
            ref.append(m.to_host())
            m.free()
    finally:
        ref_ctx.close()
    for small in ("", "0"):
        monkeypatch.setenv("SN_TEST_NO_PCELL", "1")
        if small:
            monkeypatch.setenv("SN_TEST_SWEEP_SMALL_POINTS", small)
        else:
            monkeypatch.delenv("SN_TEST_SWEEP_SMALL_POINTS", raising=False)
        c = sn.Context(0)
        try:
            ts = [sn.to_device(v) for v in vols]
            for k, (t, (it, lam, d)) in enumerate(zip(ts, params)):
                announce(f"no cell index: volume {k}, large-mesh form {bool(small)}")
                m = c.extract(t, spacing=spacing, origin=origin)
                c.smooth(m, iterations=it, relaxation=lam, constraint=d)
                g = m.to_host()
                m.free()
                for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
                    assert np.array_equal(getattr(g, f), getattr(ref[k], f)), (k, f)
                o = oracle.extract(vols[k])
                pos = o.smooth(it, lam, d)
                if o.n_points:
                    assert np.max(np.abs(g.offsets.astype(np.float64) - (pos - o.centres()))) <= TOL
                    w = oracle.world(pos, origin, spacing)
                    ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
                    assert np.all(np.abs(g.points.astype(np.float64) - w) <= TOL * np.asarray(spacing) + ulp)
            announce(f"no cell index: a batch, large-mesh form {bool(small)}")
            ms = c.batch_submit([dict(labels=t, spacing=spacing, origin=origin) for t in ts], params)
            for k, m in enumerate(ms):
                g = m.to_host()
                m.free()
                for f in ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids"):
                    assert np.array_equal(getattr(g, f), getattr(ref[k], f)), (k, f)
        finally:
            c.close()
