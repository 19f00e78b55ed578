"""Failure paths and device-memory accounting, through the C ABI.

* SN_TEST_MEM_LIMIT caps the context's device pool: sn_extract,
  sn_batch_submit and sn_smooth then return SN_ENOMEM, hold no memory
  afterwards and leave the context usable (the next call matches the oracle).
  The paper's own run on its largest volume failed this way, on allocation in
  its generation pass (Sec. 4.2).
* A served batch that hits SN_ENOMEM runs its requests one at a time; the cap
  is set from the pool peaks (sn_ctx_memory) of the same requests run one at
  a time and fused, so that only the fused form fails.
* Two-phase admission: reservations never exceed the budget while requests
  overlap, and a batch whose exact mesh does not fit next to another waiting
  batch steps back to the queue (n_requeued) and still gives the plain result.
* Labels written on the submitter's stream are read only after that write.

Kernels are never made to fault: every failure here is a host-side refusal of
an allocation, and the waits are bounded sleep kernels on a torch stream.
"""
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


def announce(msg):
    print(f"[case] {msg}", flush=True)


def same_mesh(a, b, what):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x.shape == y.shape and np.array_equal(x, y), f"{what}: {f} differs"


def against_oracle(g, lab, iters, lam=0.5, d=1.0):
    import oracle

    o = oracle.extract(lab)
    assert g.points.shape[0] == o.n_points
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if o.n_points:
        ref = (o.smooth(iters, lam, d) if iters else o.centres()) - o.centres()
        assert np.max(np.abs(g.offsets.astype(np.float64) - ref)) <= TOL


def limited_context(sn, monkeypatch, limit):
    monkeypatch.setenv("SN_TEST_MEM_LIMIT", str(int(limit)))
    c = sn.Context(0)
    monkeypatch.delenv("SN_TEST_MEM_LIMIT")
    return c


def plain(ctx, t, it):
    m = ctx.extract(t)
    ctx.smooth(m, iterations=it)
    g = m.to_host()
    m.free()
    return g


def test_extract_and_batch_enomem(sn, torch, monkeypatch):
    """A 4 MiB cap: the torso volume (its cut-edge planes alone take 6 MiB)
    and a batch holding it fail with SN_ENOMEM; no memory stays handed out; a
    small volume (about 0.9 MB of mesh and smoothing buffers) then extracts and
    smooths to the oracle's result, alone and twice in a batch."""
    c = limited_context(sn, monkeypatch, 4 << 20)
    try:
        big = sn.to_device(synth.torso_like().labels)
        rng = np.random.default_rng(61)
        small = synth.blocky_tiny(rng, (30, 20, 16), 5, np.uint16)
        ts = sn.to_device(small)
        announce("ENOMEM: torso under a 4 MiB cap")
        with pytest.raises(sn.SNError) as e:
            c.extract(big)
        assert e.value.status == sn.SN_ENOMEM
        torch.cuda.synchronize()
        assert c.memory()[0] == 0, "a failed extraction still holds memory"
        g = plain(c, ts, 6)
        against_oracle(g, small, 6)
        announce("ENOMEM: a batch holding the torso")
        with pytest.raises(sn.SNError) as e:
            c.batch_submit([dict(labels=ts), dict(labels=big)], [(6, 0.5, 1.0), (6, 0.5, 1.0)])
        assert e.value.status == sn.SN_ENOMEM
        torch.cuda.synchronize()
        assert c.memory()[0] == 0, "a failed batch still holds memory"
        ms = c.batch_submit([dict(labels=ts), dict(labels=ts)], [(6, 0.5, 1.0), (3, 0.5, 1.0)])
        gs = [m.to_host() for m in ms]
        for m in ms:
            m.free()
        against_oracle(gs[0], small, 6)
        against_oracle(gs[1], small, 3)
    finally:
        c.close()


def test_smooth_enomem_keeps_the_mesh(sn, torch, monkeypatch):
    """A cap that admits the extraction but not the smoothing buffers:
    sn_smooth fails with SN_ENOMEM and the unsmoothed mesh stays valid."""
    rng = np.random.default_rng(62)
    lab = synth.blocky_tiny(rng, (80, 60, 40), 6, np.uint16)
    t = sn.to_device(lab)
    probe = sn.Context(0)
    m = probe.extract(t)
    # the extraction's peak (scratch, word metadata, outputs) and what the
    # mesh keeps; the smoothing block (40 bytes per point) is larger than the
    # scratch, so a cap at the peak admits the extraction and refuses it
    held, peak = probe.memory()
    m.free()
    probe.close()
    c = limited_context(sn, monkeypatch, peak)
    try:
        announce("ENOMEM in smoothing")
        m = c.extract(t)
        with pytest.raises(sn.SNError) as e:
            c.smooth(m, iterations=5)
        assert e.value.status == sn.SN_ENOMEM
        g = m.to_host()
        against_oracle(g, lab, 0)
        assert c.memory()[0] == held
        m.free()
        torch.cuda.synchronize()
        assert c.memory()[0] == 0
    finally:
        c.close()


def served_requests(rng, n):
    return [synth.blocky_tiny(rng, (70 + 6 * k, 50, 40), 6, np.uint16) for k in range(n)]


def sparse_requests(n):
    """Volumes whose extraction scratch (cut-edge planes, word bases: about
    0.6 bytes per voxel) dwarfs their mesh: one small sphere each."""
    out = []
    for k in range(n):
        dims = (256 + 16 * k, 192, 160)
        c = np.array([[dims[0] / 2, dims[1] / 2, dims[2] / 2]])
        out.append(synth.spheres(dims, 2, c, [6.0 + k], [k + 1]))
    return out


def gate(torch, cycles=20_000_000):
    """A torch stream held busy by a bounded sleep kernel."""
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(cycles)
    return s


def test_served_enomem_splits_the_batch(sn, torch, monkeypatch):
    """A fused batch that exceeds the pool cap runs its requests one at a
    time, with the plain results.  The requests hold small meshes but large
    extraction scratch, which a fused batch needs for all of them at once: the
    cap is the pool peak of the same sequence run one request at a time
    (results held) plus 4 MiB, far below the fused form's peak."""
    labs = sparse_requests(5)
    blocker = synth.torso_like().labels
    its = [4 + k for k in range(len(labs))]
    ts = [sn.to_device(x) for x in labs]
    tb = sn.to_device(blocker)
    # peaks: the blocker then every request alone (results held), and the
    # blocker then the fused batch
    a = sn.Context(0)
    held = []
    for t, it in [(tb, 3)] + list(zip(ts, its)):
        m = a.extract(t)
        a.smooth(m, iterations=it)
        held.append(m)
    ref = [m.to_host() for m in held[1:]]
    seq_peak = a.memory()[1]
    for m in held:
        m.free()
    a.close()
    b = sn.Context(0)
    mb = b.extract(tb)
    b.smooth(mb, iterations=3)
    ms = b.batch_submit([dict(labels=t) for t in ts], [(it, 0.5, 1.0) for it in its])
    fused_peak = b.memory()[1]
    for m in ms + [mb]:
        m.free()
    b.close()
    cap = seq_peak + (4 << 20)
    assert fused_peak > cap + (8 << 20), (fused_peak, seq_peak)
    c = limited_context(sn, monkeypatch, cap)
    srv = c.serve_start(hbm_budget_bytes=64 << 30, max_inflight=16, n_streams=1, max_batch=16)
    try:
        announce(f"served batch over a pool cap of {cap} bytes (one at a time {seq_peak}, "
                 f"fused {fused_peak})")
        # the blocker's labels wait behind a sleep on its stream, so the other
        # requests queue up meanwhile and the worker takes them as one batch
        s = gate(torch)
        tk_b = srv.submit(tb, iterations=3, stream=s)
        tks = [srv.submit(t, iterations=it) for t, it in zip(ts, its)]
        for k, tk in enumerate(tks):
            try:
                m = srv.wait(tk, timeout_us=60_000_000)
            except sn.SNError:
                announce(f"request {k} failed; pool {c.memory()}, stats {srv.stats()}")
                raise
            same_mesh(m.to_host(), ref[k], f"split request {k}")
            m.free()
        srv.wait(tk_b, timeout_us=60_000_000).free()
        st = srv.stats()
        assert st["n_done"] == len(ts) + 1 and st["n_rejected"] == 0
        assert st["n_split_batches"] >= 1, "the fused batch did not hit the cap"
    finally:
        srv.stop()
        c.close()
    for k in (0, len(labs) - 1):
        against_oracle(ref[k], labs[k], its[k])


def test_totals_of_recycled_host_blocks(sn, torch):
    """Contexts made and closed one after another run the same number of
    extractions on different volumes: the count totals a call reads are its
    own, never a stamp an earlier context left in a recycled pinned block."""
    import oracle

    rng = np.random.default_rng(65)
    vols = [synth.blocky_tiny(rng, (40 + 7 * k, 30 + 3 * k, 20 + 2 * k), 4 + k, np.uint16)
            for k in range(4)]
    want = []
    for lab in vols:
        o = oracle.extract(lab)
        want.append((o.n_points, o.n_quads, o.n_stencil))
    ts = [sn.to_device(x) for x in vols]
    for rot in range(len(vols)):
        announce(f"context {rot}: volumes rotated by {rot}")
        ctx = sn.Context(0)
        try:
            for k in range(len(vols)):
                v = (k + rot) % len(vols)
                m = ctx.extract(ts[v])
                got = (m.n_points, m.n_quads, m.n_stencil)
                m.free()
                assert got == want[v], f"context {rot}, call {k}: {got} against {want[v]}"
        finally:
            ctx.close()


def test_served_phase2_steps_back(sn, torch):
    """Two dense requests admitted together on two streams with the server's
    first estimate (16 bytes per voxel), under a budget that holds one exact
    mesh next to the other's estimate but not two exact meshes: when both are
    counted and waiting, one steps back to the queue, the other runs, and the
    first follows; reservations stay within the budget and results are the
    plain ones."""
    rng = np.random.default_rng(64)
    dims = (60, 50, 40)
    # the same volume twice: equal exact meshes, so neither fits beside the other
    lab = synth.random_tiny(rng, dims, 6, np.uint16)
    labs = [lab, lab]
    ts = [sn.to_device(x) for x in labs]
    ctx = sn.Context(0)
    try:
        ref = []
        mesh_bytes = 0
        for t in ts:
            m = ctx.extract(t)
            ctx.smooth(m, iterations=8)
            mesh_bytes = max(mesh_bytes, ctx.memory()[0])
            ref.append(m.to_host())
            m.free()
            torch.cuda.synchronize()
        vox = int(np.prod(dims))
        est = 16 * vox
        assert mesh_bytes > 4 * est, "the volumes must be dense for this test"
        budget = mesh_bytes + est // 2
        srv = ctx.serve_start(hbm_budget_bytes=budget, max_inflight=8, n_streams=2, max_batch=1)
        try:
            announce(f"phase 2: budget {budget}, exact mesh {mesh_bytes}, estimate {est}")
            s = gate(torch)
            tks = [srv.submit(t, iterations=8, stream=s) for t in ts]
            for k, tk in enumerate(tks):
                m = srv.wait(tk, timeout_us=60_000_000)
                same_mesh(m.to_host(), ref[k], f"request {k}")
                m.free()
            st = srv.stats()
            assert st["n_done"] == 2
            assert st["peak_reserved_bytes"] <= budget
            assert st["n_requeued"] >= 1, "neither batch stepped back"
        finally:
            srv.stop()
    finally:
        ctx.close()
    against_oracle(ref[0], labs[0], 8)


def test_served_reads_labels_after_the_submitters_write(sn, torch):
    """Labels copied into place on a torch stream behind a sleep kernel and
    submitted with that stream: the server reads them after the copy."""
    rng = np.random.default_rng(65)
    lab = synth.blocky_tiny(rng, (90, 70, 50), 7, np.uint32)
    src = sn.to_device(lab)
    ctx = sn.Context(0)
    try:
        ref = plain(ctx, src, 9)
        srv = ctx.serve_start(hbm_budget_bytes=8 << 30, n_streams=2)
        try:
            announce("labels written on the submitter's stream")
            dst = torch.zeros_like(src)
            torch.cuda.synchronize()
            s = gate(torch)
            with torch.cuda.stream(s):
                dst.copy_(src)
                tk = srv.submit(dst, iterations=9)  # torch's current stream: s
            m = srv.wait(tk, timeout_us=60_000_000)
            same_mesh(m.to_host(), ref, "request behind the copy")
            m.free()
        finally:
            srv.stop()
    finally:
        ctx.close()


def test_served_admission_within_budget(sn, torch):
    """A budget of about two and a half requests' exact footprints: requests
    overlap (the peak reservation exceeds one request's) and the reservation
    never exceeds the budget; every result is the plain one."""
    rng = np.random.default_rng(66)
    labs = served_requests(rng, 8)
    ts = [sn.to_device(x) for x in labs]
    ctx = sn.Context(0)
    try:
        ref = []
        single = 0
        for t in ts:
            probe = sn.Context(0)
            m = probe.extract(t)
            probe.smooth(m, iterations=10)
            ref.append(m.to_host())
            m.free()
            single = max(single, probe.memory()[1])
            probe.close()
        budget = int(2.5 * single)
        srv = ctx.serve_start(hbm_budget_bytes=budget, max_inflight=8, n_streams=2, max_batch=4)
        try:
            announce(f"admission within a budget of {budget} bytes")
            s = gate(torch, 5_000_000)
            tks = [srv.submit(t, iterations=10, stream=s) for t in ts]
            for k, tk in enumerate(tks):
                m = srv.wait(tk, timeout_us=60_000_000)
                same_mesh(m.to_host(), ref[k], f"request {k}")
                m.free()
            st = srv.stats()
            assert st["n_done"] == len(ts)
            assert st["peak_reserved_bytes"] <= budget
            assert st["peak_reserved_bytes"] > single, "requests never overlapped"
        finally:
            srv.stop()
    finally:
        ctx.close()
