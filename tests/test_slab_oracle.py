"""The slab-assembled oracle equals the oracle on the whole volume (CPU).

The full-size GPU parity test compares the largest volume with the serial
oracle run on z-slab crops (tests/slab_oracle.py).  This checks, on volumes
the oracle finishes in well under a second, that the assembly changes
nothing: point cells, stencil, quads, label pairs, offsets and world points
equal those of one oracle run on the whole volume (integers bit for bit,
offsets and points to FP64 rounding, since a crop's index space is shifted
along z), for slabs of
one cell slice up to the whole volume, with selections, a non-zero
background, both constraint shapes, spacing and origin.  A halo one slice
short of the n + 1 the locality argument needs is caught.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from slab_oracle import compare_mesh, slab_reference


def whole(lab, it, lam, d, shape="box", selected=(), bg=0, spacing=(1, 1, 1), origin=(0, 0, 0)):
    o = oracle.extract(lab, selected, bg)
    cen = o.centres()
    pos = o.smooth(it, lam, d, shape) if it > 0 else cen
    return o, pos - cen, oracle.world(pos, origin, spacing) if o.n_points else np.zeros((0, 3))


def assembled(lab, it, lam, d, slab, **kw):
    refs = list(slab_reference(lab, it, lam, d, slab=slab, workers=4, **kw))
    cat = lambda f: np.concatenate([getattr(r, f) for r in refs]) if refs else None
    st_off = np.concatenate([refs[0].st_off[:1]] + [r.st_off[1:] for r in refs])
    return SimpleNamespace(cells=cat("cells"), delta=cat("delta"), world=cat("world"),
                           st_off=st_off, st_ids=cat("st_ids"), quads=cat("quads"),
                           pairs=cat("pairs"))


CASES = [
    # dims (M, N, O), labels, sweeps, relaxation, constraint, shape, selection, background
    ((23, 19, 31), 6, 0, 0.5, 1.0, "box", (), 0),
    ((23, 19, 31), 6, 1, 0.5, 1.0, "box", (), 0),
    ((30, 17, 40), 9, 5, 0.5, 0.8, "box", (), 0),
    ((30, 17, 40), 9, 7, 0.7, 0.6, "sphere", (), 0),
    ((26, 22, 35), 12, 4, 0.5, 1.0, "box", (2, 5, 7, 9), 3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("slab", [1, 3, 8, 64])
def test_slabs_equal_whole_volume(case, slab):
    dims, nl, it, lam, d, shape, sel, bg = CASES[case]
    rng = np.random.default_rng(100 + case)
    lab = synth.blocky_tiny(rng, dims, nl, np.uint16)
    spacing, origin = (1.0, 1.5, 2.5), (3.0, -2.0, 0.5)
    o, delta, world = whole(lab, it, lam, d, shape, sel, bg, spacing, origin)
    a = assembled(lab, it, lam, d, slab, shape=shape, selected=sel, background=bg,
                  spacing=spacing, origin=origin)
    assert o.n_points > 100 and o.n_quads > 100
    np.testing.assert_array_equal(a.cells, o.cell_of)
    np.testing.assert_array_equal(a.st_off, o.st_off)
    np.testing.assert_array_equal(a.st_ids, o.st_ids)
    np.testing.assert_array_equal(a.quads, o.quads)
    np.testing.assert_array_equal(a.pairs, o.pairs)
    # the oracle smooths absolute index-space positions, and a crop's z starts
    # at its first sample slice: the same arithmetic up to FP64 rounding
    assert np.max(np.abs(a.delta - delta), initial=0.0) <= 1e-12
    assert np.max(np.abs(a.world - world), initial=0.0) <= 1e-12 * 1e3


def test_short_halo_is_caught():
    """With a halo of n slices instead of n + 1 a slab's own edge slices still
    come out right, but a halo of n - 1 leaves the error of the crop's cut
    stencil inside the slab: the comparison must see it."""
    rng = np.random.default_rng(7)
    lab = synth.random_tiny(rng, (20, 18, 40), 3, np.uint8)
    it = 6
    _, delta, _ = whole(lab, it, 0.5, 1.0)
    short = np.concatenate([r.delta for r in slab_reference(lab, it, 0.5, 1.0, slab=4, workers=4,
                                                            halo=it - 1)])
    # the error entering from the cut stencil shrinks with every step inward,
    # but stays far above FP64 rounding
    assert np.max(np.abs(short - delta)) > 1e-9
    ok = np.concatenate([r.delta for r in slab_reference(lab, it, 0.5, 1.0, slab=4, workers=4)])
    assert np.max(np.abs(ok - delta)) <= 1e-12


def test_compare_mesh_accepts_oracle_and_rejects_a_slip():
    """compare_mesh on a host mesh built from the whole-volume oracle passes;
    one quad id, one stencil id or one offset off by more than the tolerance
    fails it."""
    rng = np.random.default_rng(11)
    lab = synth.blocky_tiny(rng, (28, 24, 30), 8, np.uint16)
    it, lam, d = 5, 0.5, 1.0
    o, delta, world = whole(lab, it, lam, d)
    g = SimpleNamespace(points=world.astype(np.float32), offsets=delta.astype(np.float32),
                        polys=o.quads.copy(), label_pairs=o.pairs.astype(np.uint16),
                        stencil_off=o.st_off.astype(np.int32), stencil_ids=o.st_ids.copy())
    assert compare_mesh(g, lab, it, lam, d, slab=5, workers=4) <= 1e-7
    for field, idx, bump in (("polys", (o.n_quads // 2, 1), 1), ("stencil_ids", o.n_stencil - 3, 1),
                             ("offsets", (o.n_points // 3, 2), 3e-5)):
        arr = getattr(g, field)
        arr[idx] += bump
        with pytest.raises(AssertionError):
            compare_mesh(g, lab, it, lam, d, slab=5, workers=4)
        arr[idx] -= bump
