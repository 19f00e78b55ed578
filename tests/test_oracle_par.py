"""The all-cores oracle (the serial oracle's loops over z-slices with OpenMP,
used only as the benchmark's all-cores CPU baseline) equals the serial oracle
bit for bit: point cells, quads, label pairs, stencil, and smoothed positions
under both constraint shapes, at several thread counts, on ragged volumes whose
slice counts do not divide evenly among the threads."""
from __future__ import annotations

import numpy as np
import pytest

import synth


def _same(a, b):
    np.testing.assert_array_equal(a.cell_of, b.cell_of)
    np.testing.assert_array_equal(a.quads, b.quads)
    np.testing.assert_array_equal(a.pairs, b.pairs)
    np.testing.assert_array_equal(a.st_off, b.st_off)
    np.testing.assert_array_equal(a.st_ids, b.st_ids)


CASES = [
    ("blocky u16", (37, 23, 19), 6, np.uint16, ()),
    ("random u8", (17, 31, 13), 3, np.uint8, ()),
    ("random u32 selection", (29, 11, 21), 9, np.uint32, (2, 5, 7)),
    ("one slice of cells", (40, 30, 2), 4, np.uint16, ()),
    ("thin", (2, 2, 50), 3, np.uint8, ()),
]


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_extract_and_smooth_equal_serial(orc, case, threads):
    name, dims, nv, dt, sel = CASES[case]
    rng = np.random.default_rng(100 + case)
    gen = synth.blocky_tiny if "blocky" in name else synth.random_tiny
    lab = gen(rng, dims, nv, dt)
    a = orc.extract(lab, sel)
    b = orc.extract_par(lab, sel, threads=threads)
    _same(a, b)
    for shape in ("box", "sphere"):
        pa = a.smooth(7, 0.5, 0.8, shape)
        pb = b.smooth_par(7, 0.5, 0.8, shape, threads=threads)
        assert np.array_equal(pa, pb), f"{name}: {shape} smoothing differs"


def test_background_and_degenerate(orc):
    rng = np.random.default_rng(7)
    lab = synth.random_tiny(rng, (9, 8, 7), 4, np.uint16)
    _same(orc.extract(lab, (), 2), orc.extract_par(lab, (), 2, threads=4))
    for dims in ((1, 5, 5), (5, 1, 5), (5, 5, 1), (1, 1, 1)):
        lab = synth.random_tiny(rng, dims, 3, np.uint8)
        a, b = orc.extract(lab), orc.extract_par(lab, threads=2)
        assert b.n_points == a.n_points == 0 and b.n_quads == a.n_quads == 0


def test_spheres_small_config(orc):
    """The 64^3 spheres configuration with its 16 sweeps, all threads."""
    vol = synth.spheres_small()
    a = orc.extract(vol.labels)
    b = orc.extract_par(vol.labels)
    _same(a, b)
    assert np.array_equal(a.smooth(vol.iterations, vol.relaxation, vol.constraint),
                          b.smooth_par(vol.iterations, vol.relaxation, vol.constraint))
