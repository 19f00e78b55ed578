"""Parity at the largest configuration: the connectome-like 1024x1024x512
uint32 volume (50 000 stretched cells, 2 % membrane; 20 sweeps, relaxation
0.5, constraint 0.8), extracted and smoothed on the GPU exactly as the
benchmark runs it.  The oracle cannot run on the whole volume in test time,
so the check is split:

* totals P, Q, S against closed forms accumulated slab by slab over the whole
  volume (point iff the 8 corners differ, quad iff an interior edge is cut,
  two directed stencil entries per non-uniform interior face);
* for sampled cells, the point id (count of point cells before it in linear
  order), its stencil ids, and for sampled cut edges the quad index, its four
  point ids and label pair - all from those same closed forms;
* for sampled points, the smoothed offset and world point against the FP64
  oracle run on a crop of the volume around the point.  After n sweeps a
  point depends only on points within n stencil steps, and a step moves one
  cell along one axis, so a crop reaching n + 4 cells beyond the point in
  every direction (or to the volume's own faces) gives the same value.
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


class _Dev:
    """A device array as a torch tensor without a copy."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 3, "strides": None}


def dev(torch, ptr, shape, typestr):
    return torch.as_tensor(_Dev(ptr, shape, typestr), device="cuda")


def announce(msg):
    print(f"[case] {msg}", flush=True)


def slab_counts(lab):
    """Per cell row (j, k): point count, quad count (all axes), and the total
    number of directed stencil entries, from the closed forms."""
    O, N, M = lab.shape
    pts_row = np.zeros((O - 1, N - 1), np.int64)
    quad_row = np.zeros((O, N), np.int64)  # quads owned by sample row (j, k)
    S = 0
    for k in range(O - 1):
        a, b = lab[k], lab[k + 1]
        c = [a[:-1, :-1], a[:-1, 1:], a[1:, :-1], a[1:, 1:], b[:-1, :-1], b[:-1, 1:], b[1:, :-1],
             b[1:, 1:]]
        mx = np.maximum.reduce(c)
        mn = np.minimum.reduce(c)
        pts_row[k] = (mx != mn).sum(1)
        # faces between cells: x-faces at sample column i (1 <= i <= M-2) of cell row (j,k)
        fx = [a[:-1, 1:-1], a[1:, 1:-1], b[:-1, 1:-1], b[1:, 1:-1]]
        S += 2 * int((np.maximum.reduce(fx) != np.minimum.reduce(fx)).sum())
        # y-faces at sample row j (1 <= j <= N-2)
        fy = [a[1:-1, :-1], a[1:-1, 1:], b[1:-1, :-1], b[1:-1, 1:]]
        S += 2 * int((np.maximum.reduce(fy) != np.minimum.reduce(fy)).sum())
        # z-faces at sample layer k+1 (1 <= k+1 <= O-2)
        if k + 1 <= O - 2:
            fz = [b[:-1, :-1], b[:-1, 1:], b[1:, :-1], b[1:, 1:]]
            S += 2 * int((np.maximum.reduce(fz) != np.minimum.reduce(fz)).sum())
    for k in range(0, O - 1):
        a = lab[k]
        # x-edges of rows j = 1..N-2 (i <= M-2) and y-edges of rows j <= N-2
        # (1 <= i <= M-2) need 1 <= k <= O-2; z-edges (1 <= i <= M-2,
        # 1 <= j <= N-2) need k <= O-2
        if k >= 1:
            quad_row[k, 1:N - 1] += (a[1:N - 1, :-1] != a[1:N - 1, 1:]).sum(1)
            quad_row[k, :N - 1] += (a[:N - 1, 1:M - 1] != a[1:, 1:M - 1]).sum(1)
        quad_row[k, 1:N - 1] += (a[1:N - 1, 1:M - 1] != lab[k + 1][1:N - 1, 1:M - 1]).sum(1)
    return pts_row, quad_row, S


def host(x):
    """numpy view of a device tensor (or a numpy array itself)."""
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


def check_samples(lab, row_base, qrow_base, mesh, n_it, lam, dist, n_points=120, n_quads=200,
                  seed=99):
    """Sampled checks of a mesh of `lab` (unit spacing, zero origin, every
    label selected, background 0); `mesh` maps points, offsets, stencil_off,
    stencil_ids, quads, label_pairs to host or device arrays."""
    import oracle

    O, N, M = lab.shape
    points, offsets = mesh["points"], mesh["offsets"]
    st_off, st_ids = mesh["stencil_off"], mesh["stencil_ids"]
    quads, pairs = mesh["quads"], mesh["label_pairs"]

    def has_point(i, j, k):
        c = lab[k:k + 2, j:j + 2, i:i + 2]
        return c.max() != c.min()

    def pid(i, j, k):
        row = lab[k:k + 2, j:j + 2, :]
        c = [row[0, 0, :-1], row[0, 0, 1:], row[0, 1, :-1], row[0, 1, 1:], row[1, 0, :-1],
             row[1, 0, 1:], row[1, 1, :-1], row[1, 1, 1:]]
        pm = np.maximum.reduce(c) != np.minimum.reduce(c)
        return int(row_base[j + (N - 1) * k] + pm[:i].sum())

    rng = np.random.default_rng(seed)
    h = n_it + 4
    checked = 0
    while checked < n_points:
        i, j, k = int(rng.integers(0, M - 1)), int(rng.integers(0, N - 1)), int(rng.integers(0, O - 1))
        if not has_point(i, j, k):
            continue
        p = pid(i, j, k)
        # stencil ids in face order -x, +x, -y, +y, -z, +z
        exp = []
        for (di, dj, dk, a) in ((-1, 0, 0, 0), (1, 0, 0, 0), (0, -1, 0, 1), (0, 1, 0, 1),
                                (0, 0, -1, 2), (0, 0, 1, 2)):
            ni, nj, nk = i + di, j + dj, k + dk
            if not (0 <= ni < M - 1 and 0 <= nj < N - 1 and 0 <= nk < O - 1):
                continue
            # shared face: the sample plane between the two cells
            s = [slice(k, k + 2), slice(j, j + 2), slice(i, i + 2)]
            s[2 - a] = slice(max(i, ni) if a == 0 else (max(j, nj) if a == 1 else max(k, nk)),
                             (max(i, ni) if a == 0 else (max(j, nj) if a == 1 else max(k, nk))) + 1)
            f = lab[tuple(s)]
            if f.max() != f.min():
                exp.append(pid(ni, nj, nk))
        b0, b1 = int(host(st_off[p:p + 2])[0]), int(host(st_off[p:p + 2])[1])
        assert host(st_ids[b0:b1]).tolist() == exp, (i, j, k)
        # smoothing on a crop around the cell
        lo = [max(x - h, 0) for x in (i, j, k)]
        hi = [min(x + h + 2, n) for x, n in zip((i, j, k), (M, N, O))]
        crop = np.ascontiguousarray(lab[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
        o = oracle.extract(crop)
        cells = o.cells_ijk()
        q = int(np.flatnonzero((cells[:, 0] == i - lo[0]) & (cells[:, 1] == j - lo[1]) &
                               (cells[:, 2] == k - lo[2]))[0])
        ref = o.smooth(n_it, lam, dist)[q] - o.centres()[q]
        got = host(offsets[p]).astype(np.float64)
        assert np.max(np.abs(got - ref)) <= TOL, (i, j, k, got, ref)
        w = np.array([i, j, k], np.float64) + 0.5 + ref  # unit spacing, zero origin
        gw = host(points[p]).astype(np.float64)
        ulp = np.spacing(np.abs(w).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(gw - w) <= TOL + ulp), (i, j, k)
        checked += 1

    checked = 0
    while checked < n_quads:
        a = int(rng.integers(0, 3))
        i, j, k = int(rng.integers(1, M - 1)), int(rng.integers(1, N - 1)), int(rng.integers(1, O - 1))
        s0 = lab[k, j, i]
        s1 = lab[k + (a == 2), j + (a == 1), i + (a == 0)] if (i + (a == 0) < M and
                                                              j + (a == 1) < N and
                                                              k + (a == 2) < O) else s0
        if s0 == s1 or (a == 0 and i > M - 2) or (a == 1 and j > N - 2) or (a == 2 and k > O - 2):
            continue
        # quad index: quads of earlier sample rows, then of this row at smaller i or axis
        row = k * N + j
        before = 0
        ra = lab[k, j]
        for ax in range(3):
            if ax == 0:
                if not (1 <= j <= N - 2 and 1 <= k <= O - 2):
                    continue
                cut = ra[:-1] != ra[1:]
                lo_i, hi_i = 0, M - 1
            elif ax == 1:
                if not (j <= N - 2 and 1 <= k <= O - 2):
                    continue
                cut = ra[1:M - 1] != lab[k, j + 1, 1:M - 1]
                lo_i, hi_i = 1, M - 1
            else:
                if not (1 <= j <= N - 2 and k <= O - 2):
                    continue
                cut = ra[1:M - 1] != lab[k + 1, j, 1:M - 1]
                lo_i, hi_i = 1, M - 1
            upto = i + 1 if ax < a else i  # same i: earlier axes come first
            before += int(cut[:max(0, min(upto, hi_i) - lo_i)].sum())
        qi = int(qrow_base[row] + before)
        if a == 0:
            cs = [(i, j - 1, k - 1), (i, j - 1, k), (i, j, k), (i, j, k - 1)]
        elif a == 1:
            cs = [(i - 1, j, k - 1), (i, j, k - 1), (i, j, k), (i - 1, j, k)]
        else:
            cs = [(i - 1, j - 1, k), (i - 1, j, k), (i, j, k), (i, j - 1, k)]
        assert host(quads[qi]).tolist() == [pid(*c) for c in cs], (a, i, j, k)
        assert host(pairs[qi]).astype(np.uint32).tolist() == [int(s0), int(s1)]
        checked += 1


def test_connectome_full_size(torch):
    import paper_2401_14906_amd as sn

    sn.load_library()
    ctx = sn.Context(0)
    vol = synth.connectome_like()
    lab = vol.labels
    O, N, M = lab.shape
    announce(f"{vol.name}: GPU extract + {vol.iterations} sweeps")
    t = sn.to_device(lab)
    m = ctx.extract(t, spacing=vol.spacing)
    ctx.smooth(m, iterations=vol.iterations, relaxation=vol.relaxation, constraint=vol.constraint)
    torch.cuda.synchronize()
    v = m.view()
    P, Q, S = int(v.n_points), int(v.n_quads), int(v.n_stencil)

    announce("closed-form totals, slab by slab")
    pts_row, quad_row, S_ref = slab_counts(lab)
    assert P == int(pts_row.sum())
    assert Q == int(quad_row.sum())
    assert S == S_ref
    row_base = np.concatenate([[0], np.cumsum(pts_row.ravel())])  # by row r = j + (N-1) k
    qrow_base = np.concatenate([[0], np.cumsum(quad_row.ravel())])  # by sample row j + N k

    mesh = {"points": dev(torch, v.points, (P, 3), "<f4"),
            "offsets": dev(torch, v.offsets, (P, 3), "<f4"),
            "stencil_off": dev(torch, v.stencil_off, (P + 1,), "<i4"),
            "stencil_ids": dev(torch, v.stencil_ids, (S,), "<i4"),
            "quads": dev(torch, v.quads, (Q, 4), "<i4"),
            "label_pairs": dev(torch, v.label_pairs, (Q, 2), "<i4")}
    announce("sampled points and quads")
    check_samples(lab, row_base, qrow_base, mesh, vol.iterations, vol.relaxation, vol.constraint,
                  n_points=400, n_quads=1000)
    m.free()
    ctx.close()


FIELDS = ("points", "offsets", "polys", "label_pairs", "stencil_off", "stencil_ids")


def same_mesh(a, b, what):
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x.shape == y.shape and np.array_equal(x, y), f"{what}: {f} differs"


def oracle_check(g, labels, iters, lam, d, selected=()):
    import oracle

    o = oracle.extract(labels, selected)
    assert g.points.shape[0] == o.n_points
    np.testing.assert_array_equal(g.polys, o.quads)
    np.testing.assert_array_equal(g.label_pairs.astype(np.uint32), o.pairs)
    np.testing.assert_array_equal(g.stencil_off.astype(np.int64), o.st_off)
    np.testing.assert_array_equal(g.stencil_ids, o.st_ids)
    if o.n_points:
        ref = o.smooth(iters, lam, d) - o.centres()
        assert np.max(np.abs(g.offsets.astype(np.float64) - ref)) <= TOL


def test_batched_configuration(torch):
    """The 64-volume batched workload as the benchmark runs it: every batched
    mesh equals the plain one byte for byte; four of them against the oracle."""
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
    sizes = np.array([v.labels.size for v in vols])
    for k in np.argsort(sizes)[[0, 1, 31, 63]]:
        v = vols[int(k)]
        announce(f"oracle check of batch volume {int(k)} {v.labels.shape}")
        oracle_check(got[int(k)], v.labels, v.iterations, v.relaxation, v.constraint)
    ctx.close()


def test_served_configuration(torch):
    """The served workload's volume pool (cubic edges 32..512, u8/u16/u32,
    label subsets): results served in fused batches equal the plain results
    for the same requests; two small ones against the oracle."""
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
    small = sorted(range(len(reqs)), key=lambda n: vols[reqs[n][0]].labels.size)[:2]
    for n in small:
        k, sel, it = reqs[n]
        announce(f"oracle check of request {n} {vols[k].labels.shape} {vols[k].labels.dtype}")
        oracle_check(got[n], vols[k].labels, it, 0.5, 1.0, sel)
    ctx.close()
