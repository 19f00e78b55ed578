"""Parity at the benchmark's full sizes, element by element.

* The connectome-like 1024x1024x512 uint32 volume (50 000 stretched cells, 2 %
  membrane; 20 sweeps, relaxation 0.5, constraint 0.8), extracted and smoothed
  on the GPU exactly as the benchmark runs it, against the serial oracle
  assembled from z-slab crops (tests/slab_oracle.py: every point's offset and
  world point, every stencil offset and id, quad and label pair).  Its 140 M
  points take the large-mesh sweep form (non-temporal accesses, slab-chunked
  block order).
* The batched workload (64 uneven volumes): every batched mesh byte-equal to
  the plain one and every one against the oracle.
* The served workload's pool: every served result byte-equal to the same
  request run alone and every one against the oracle.

Oracle runs go to a pool of host threads (the oracle's C calls release the
GIL).
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


def announce(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.timeout(900)
def test_connectome_full_size(torch):
    import paper_2401_14906_amd as sn

    sn.load_library()
    ctx = sn.Context(0)
    vol = synth.connectome_like()
    lab = vol.labels
    announce(f"{vol.name}: GPU extract + {vol.iterations} sweeps")
    t = sn.to_device(lab)
    m = ctx.extract(t, spacing=vol.spacing, origin=vol.origin)
    ctx.smooth(m, iterations=vol.iterations, relaxation=vol.relaxation, constraint=vol.constraint)
    g = m.to_host()
    m.free()
    del t
    ctx.close()
    P, Q = g.points.shape[0], g.polys.shape[0]
    assert P > (1 << 24), "the connectome mesh must take the large-mesh sweep form"
    announce(f"{P} points, {Q} quads: oracle on z-slab crops, {WORKERS} threads")
    worst = compare_mesh(g, lab, vol.iterations, vol.relaxation, vol.constraint,
                         spacing=vol.spacing, origin=vol.origin, slab=32, workers=WORKERS)
    announce(f"largest offset error {worst:.2e}")


FIELDS = ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids")


def same_mesh(a, b, what):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x.shape == y.shape and np.array_equal(x, y), f"{what}: {f} differs"


def oracle_check(g, labels, iters, lam, d, selected=()):
    """A mesh against the oracle on the whole volume; raises on a mismatch."""
    import oracle

    o = oracle.extract(labels, selected)
    assert g.points.shape[0] == o.n_points
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if o.n_points:
        pos = o.smooth(iters, lam, d)
        err = float(np.max(np.abs(g.offsets.astype(np.float64) - (pos - o.centres()))))
        assert err <= TOL, f"offsets differ by {err}"
        w = oracle.world(pos, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
        ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(g.points.astype(np.float64) - w) <= TOL + ulp)
    return o.n_points


def oracle_check_all(jobs):
    """oracle_check over (name, mesh, labels, iters, lam, d, selected) jobs in
    host threads; every failure is reported."""
    with ThreadPoolExecutor(max_workers=WORKERS) as ex:
        futs = [(j[0], ex.submit(oracle_check, *j[1:])) for j in jobs]
        errs = []
        for name, f in futs:
            try:
                f.result()
            except AssertionError as e:
                errs.append(f"{name}: {e}")
    assert not errs, "\n".join(errs[:8])


@pytest.mark.timeout(600)
def test_batched_configuration(torch):
    """The 64-volume batched workload as the benchmark runs it: every batched
    mesh equals the plain one byte for byte, and every one the oracle."""
    import paper_2401_14906_amd as sn

    sn.load_library()
    ctx = sn.Context(0)
    vols = synth.batch_volumes(count=64)
    ts = [sn.to_device(v.labels) for v in vols]
    announce("batched configuration: 64 volumes")
    ms = ctx.batch_submit([dict(labels=t) for t in ts],
                          [(v.iterations, v.relaxation, v.constraint) for v in vols])
    got = [m.to_host() for m in ms]
    for m in ms:
        m.free()
    for k, (t, v) in enumerate(zip(ts, vols)):
        m = ctx.extract(t)
        ctx.smooth(m, iterations=v.iterations, relaxation=v.relaxation, constraint=v.constraint)
        same_mesh(got[k], m.to_host(), f"batch volume {k}")
        m.free()
    ctx.close()
    announce(f"oracle check of all 64 volumes, {WORKERS} threads")
    oracle_check_all([(f"batch volume {k} {v.labels.shape}", got[k], v.labels, v.iterations,
                       v.relaxation, v.constraint, ()) for k, v in enumerate(vols)])


@pytest.mark.timeout(600)
def test_served_configuration(torch):
    """The served workload's volume pool (cubic edges 32..512, u8/u16/u32,
    label subsets): results served in fused batches equal the plain results
    for the same requests, and every one the oracle."""
    import paper_2401_14906_amd as sn

    sn.load_library()
    ctx = sn.Context(0)
    vols = synth.serve_pool(seed=5, count=16)
    ts = [sn.to_device(v.labels) for v in vols]
    present = [np.flatnonzero(np.bincount(v.labels.ravel())) for v in vols]
    rng = np.random.default_rng(5)
    reqs = []
    for _ in range(48):
        k = int(rng.integers(0, len(vols)))
        labs = present[k][present[k] != 0]
        sel = tuple(int(x) for x in rng.choice(labs, size=int(rng.integers(1, min(20, len(labs)) + 1)),
                                               replace=False))
        reqs.append((k, sel, int(rng.integers(10, 41))))
    srv = ctx.serve_start(hbm_budget_bytes=32 << 30, max_inflight=64, n_streams=2, max_batch=16)
    announce(f"served configuration: {len(reqs)} requests")
    tks = [srv.submit(ts[k], iterations=it, relaxation=0.5, constraint=1.0, selected=sel)
           for k, sel, it in reqs]
    got = []
    for tk in tks:
        m = srv.wait(tk, timeout_us=120_000_000)
        got.append(m.to_host())
        m.free()
    assert srv.stats()["n_batches"] < len(reqs)
    srv.stop()
    for n, (k, sel, it) in enumerate(reqs):
        m = ctx.extract(ts[k], selected=sel)
        ctx.smooth(m, iterations=it, relaxation=0.5, constraint=1.0)
        same_mesh(got[n], m.to_host(), f"request {n}")
        m.free()
    ctx.close()
    announce(f"oracle check of all {len(reqs)} requests, {WORKERS} threads")
    oracle_check_all([(f"request {n} {vols[k].labels.shape} {vols[k].labels.dtype}", got[n],
                       vols[k].labels, it, 0.5, 1.0, sel) for n, (k, sel, it) in enumerate(reqs)])
