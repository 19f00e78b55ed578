"""The oracle of a large volume, assembled from z-slab crops (test helper).

The serial oracle (``oracle/``) takes minutes on the largest volumes, and its
memory grows with the whole mesh.  Its result is local, though:

* extraction: a cell's point, a face-neighbour link and a quad depend only on
  the samples of the cells involved (Sec. 2.2), so the cells of slices
  k0 .. k1-1 are extracted identically from any crop that holds sample slices
  k0 - 1 .. k1 + 1;
* smoothing: one Jacobi sweep of Eq. (1) moves a point by its face neighbours
  only, so after n sweeps a point depends on the points within n stencil
  steps, at most n cell slices away.  In a crop, only the first and last cell
  slice have stencils cut short by the crop, and their error reaches one more
  slice inward per sweep: points n or more slices inside the crop are exact
  after n sweeps.

So the volume is cut into slabs of cell slices; slab [k0, k1) is extracted and
smoothed by the serial oracle on the crop of sample slices
[k0 - h, k1 + 1 + h) (clipped to the volume) with h = n + 1, and its points,
quads and stencil entries are kept.  Point ids are contiguous in cell order
and a crop holds whole slices, so a crop's point id maps to the global one by
a shift; quads are ordered by their origin sample, whose cell is the third
vertex of every quad, so a slab's quads are a contiguous run as well.  Bases
are the oracle's own counts summed over earlier slabs.

Crops run in a thread pool: the oracle's C calls release the GIL (ctypes) and
keep no global state.  ``tests/test_slab_oracle.py`` checks on the CPU that
the assembled result equals the oracle on the whole volume, bit for bit.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

import oracle


@dataclass
class SlabRef:
    k0: int              # first cell slice of the slab
    k1: int              # one past the last
    p0: int              # global id of the slab's first point
    q0: int              # global index of its first quad
    s0: int              # global index of its first stencil entry
    cells: np.ndarray    # int64 [p] global linear cell index of each point
    delta: np.ndarray    # float64 [p, 3] offsets from the cell centre after smoothing
    world: np.ndarray    # float64 [p, 3] world points
    st_off: np.ndarray   # int64 [p + 1] global CSR offsets
    st_ids: np.ndarray   # int64 [s] global neighbour ids
    quads: np.ndarray    # int64 [q, 4] global point ids
    pairs: np.ndarray    # uint32 [q, 2]


def _crop_reference(lab, k0, k1, halo, iterations, relaxation, constraint, shape, selected,
                    background, spacing, origin):
    """Oracle results of cell slices [k0, k1) from a crop reaching `halo`
    slices beyond them; ids relative to the slab's first point."""
    O, N, M = lab.shape
    c0 = max(0, k0 - halo)
    c1 = min(O, k1 + 1 + halo)
    crop = np.ascontiguousarray(lab[c0:c1])
    o = oracle.extract(crop, selected, background)
    per_slice = (M - 1) * (N - 1)
    kc = o.cell_of // per_slice + c0
    pa, pb = int(np.searchsorted(kc, k0)), int(np.searchsorted(kc, k1))
    qk = kc[o.quads[:, 2]] if o.n_quads else np.zeros(0, np.int64)
    qa, qb = int(np.searchsorted(qk, k0)), int(np.searchsorted(qk, k1))
    sa, sb = int(o.st_off[pa]), int(o.st_off[pb])
    cen = o.centres()
    pos = o.smooth(iterations, relaxation, constraint, shape) if iterations > 0 else cen
    delta = (pos - cen)[pa:pb]
    glob = pos[pa:pb].copy()
    glob[:, 2] += c0  # the crop's index space starts at sample slice c0
    world = oracle.world(glob, origin, spacing) if pb > pa else np.zeros((0, 3))
    return dict(P=pb - pa, Q=qb - qa, S=sb - sa,
                cells=o.cell_of[pa:pb] + c0 * per_slice,
                delta=delta, world=world,
                st_off=o.st_off[pa:pb + 1] - sa,
                st_ids=o.st_ids[sa:sb].astype(np.int64) - pa,
                quads=o.quads[qa:qb].astype(np.int64) - pa,
                pairs=o.pairs[qa:qb].copy())


def slab_reference(labels, iterations, relaxation, constraint, shape="box", selected=(),
                   background=0, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), slab=32,
                   workers=None, halo=None):
    """Yield SlabRef for consecutive slabs of `slab` cell slices, in order.

    `halo` (default iterations + 1 cell slices) exists so that a test can show
    that too small a halo is caught."""
    lab = np.asarray(labels)
    if lab.ndim != 3:
        raise ValueError("slab_reference takes a volume (O, N, M)")
    O, N, M = lab.shape
    CO = max(O - 1, 0) if min(O, N, M) >= 2 else 0
    h = iterations + 1 if halo is None else halo
    if workers is None:
        workers = max(1, min(16, os.cpu_count() or 1))
    bounds = [(k, min(k + slab, CO)) for k in range(0, CO, slab)]
    args = (h, iterations, relaxation, constraint, shape, selected, background, spacing, origin)
    p0 = q0 = s0 = 0
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {}
        nxt = 0
        # at most 2 * workers crops in flight or waiting: bounded memory
        for i, (k0, k1) in enumerate(bounds):
            while nxt < len(bounds) and nxt < i + 2 * workers:
                a, b = bounds[nxt]
                futs[nxt] = ex.submit(_crop_reference, lab, a, b, *args)
                nxt += 1
            r = futs.pop(i).result()
            yield SlabRef(k0=k0, k1=k1, p0=p0, q0=q0, s0=s0, cells=r["cells"],
                          delta=r["delta"], world=r["world"], st_off=r["st_off"] + s0,
                          st_ids=r["st_ids"] + p0, quads=r["quads"] + p0, pairs=r["pairs"])
            p0 += r["P"]
            q0 += r["Q"]
            s0 += r["S"]


def compare_mesh(g, labels, iterations, relaxation, constraint, shape="box", selected=(),
                 background=0, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), slab=32,
                 workers=None, tol=1e-5, progress=None):
    """Compare a host mesh `g` (points, offsets, polys, label_pairs, stencil_off,
    stencil_ids; quads) with the slab-assembled oracle, element by element:
    integer outputs exactly, offsets within `tol` voxels, world points within
    tol * spacing + one float32 ulp.  Returns the largest offset error."""
    P = g.points.shape[0]
    Q = g.polys.shape[0]
    S = g.stencil_ids.shape[0]
    h = np.asarray(spacing, np.float64)
    worst = 0.0
    last = None
    for r in slab_reference(labels, iterations, relaxation, constraint, shape, selected,
                            background, spacing, origin, slab, workers):
        n, nq = r.delta.shape[0], r.quads.shape[0]
        ns = int(r.st_off[-1] - r.st_off[0])
        where = f"cell slices {r.k0}..{r.k1 - 1}"
        assert r.p0 + n <= P and r.q0 + nq <= Q and r.s0 + ns <= S, f"{where}: mesh too small"
        np.testing.assert_array_equal(g.stencil_off[r.p0:r.p0 + n + 1].astype(np.int64), r.st_off,
                                      err_msg=f"{where}: stencil offsets")
        np.testing.assert_array_equal(g.stencil_ids[r.s0:r.s0 + ns].astype(np.int64), r.st_ids,
                                      err_msg=f"{where}: stencil ids")
        np.testing.assert_array_equal(g.polys[r.q0:r.q0 + nq].astype(np.int64), r.quads,
                                      err_msg=f"{where}: quads")
        np.testing.assert_array_equal(g.label_pairs[r.q0:r.q0 + nq].astype(np.uint32), r.pairs,
                                      err_msg=f"{where}: label pairs")
        if n:
            off = g.offsets[r.p0:r.p0 + n].astype(np.float64)
            err = float(np.max(np.abs(off - r.delta)))
            assert err <= tol, f"{where}: offsets differ by {err}"
            worst = max(worst, err)
            w = g.points[r.p0:r.p0 + n].astype(np.float64)
            ulp = np.spacing(np.abs(r.world).astype(np.float32)).astype(np.float64)
            bad = np.abs(w - r.world) > tol * h + ulp
            assert not bad.any(), f"{where}: world points differ at {np.argwhere(bad)[:4].tolist()}"
        last = r
        if progress:
            progress(r)
    tot = (0, 0, 0) if last is None else (last.p0 + last.delta.shape[0],
                                          last.q0 + last.quads.shape[0],
                                          int(last.st_off[-1]))
    assert (P, Q, S) == tot, f"mesh totals {(P, Q, S)} against the oracle's {tot}"
    return worst
