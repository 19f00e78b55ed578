"""Pins of the oracle's diagonal rules for the triangulation step (Sec. 2.5
lists shortest diagonal, minimum area and most co-planar; the measures are
the readings stated in oracle/sn_oracle.c and include/sn.h).  Each expected
choice below is worked out by hand in its comment, so a swapped diagonal, a
wrong triangle, a reversed comparison or a lost tie-break fails a case."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

FIXED, SHORTEST, MIN_AREA, PLANAR = 0, 1, 2, 3


def P(*x):
    return np.array(x, dtype=np.float64)


def test_planar_square_ties_go_to_ac():
    # unit square: both diagonals have length^2 2, both splits area 1, all
    # normals (0,0,1): every rule ties and takes A-C
    a, b, c, d = P(0, 0, 0), P(1, 0, 0), P(1, 1, 0), P(0, 1, 0)
    assert all(oracle.split_ac(a, b, c, d, r) for r in (FIXED, SHORTEST, MIN_AREA, PLANAR))


def test_planar_rhombus_separates_shortest_from_area_and_planarity():
    # a=(-2,0,0) b=(0,-1,0) c=(2,0,0) d=(0,1,0): |AC|^2 = 16 > |BD|^2 = 4, so the
    # shortest diagonal is B-D; the quad is planar, so both splits have area
    # 2 + 2 = 4 and normals (0,0,4): area and planarity tie and take A-C
    a, b, c, d = P(-2, 0, 0), P(0, -1, 0), P(2, 0, 0), P(0, 1, 0)
    assert not oracle.split_ac(a, b, c, d, SHORTEST)
    assert oracle.split_ac(a, b, c, d, MIN_AREA)
    assert oracle.split_ac(a, b, c, d, PLANAR)
    # the other way round: |AC|^2 = 4 < |BD|^2 = 16
    a, b, c, d = P(-1, 0, 0), P(0, -2, 0), P(1, 0, 0), P(0, 2, 0)
    assert oracle.split_ac(a, b, c, d, SHORTEST)


def test_folded_square():
    # c lifted by 1: a=(0,0,0) b=(1,0,0) c=(1,1,1) d=(0,1,0)
    #   A-C: normals ABC (0,-1,1), ACD (-1,0,1): areas sqrt2/2 each, sum 1.414,
    #        cosine 1/2
    #   B-D: normals ABD (0,0,1), BCD (-1,-1,1): areas 1/2 + sqrt3/2 = 1.366,
    #        cosine 1/sqrt3 = 0.577
    #   -> minimum area B-D, most planar B-D; shortest: |AC|^2 3 > |BD|^2 2, B-D
    a, b, c, d = P(0, 0, 0), P(1, 0, 0), P(1, 1, 1), P(0, 1, 0)
    assert not oracle.split_ac(a, b, c, d, MIN_AREA)
    assert not oracle.split_ac(a, b, c, d, PLANAR)
    assert not oracle.split_ac(a, b, c, d, SHORTEST)
    # d lifted instead: the mirror image, A-C for all three
    a, b, c, d = P(0, 0, 0), P(1, 0, 0), P(1, 1, 0), P(0, 1, 1)
    assert oracle.split_ac(a, b, c, d, MIN_AREA)
    assert oracle.split_ac(a, b, c, d, PLANAR)
    assert oracle.split_ac(a, b, c, d, SHORTEST)


def test_area_and_planarity_disagree():
    # a=(0,0,0) b=(1,0,0) c=(1,1,2) d=(0,1,-1)
    #   A-C: ABC normal (0,-2,1) area sqrt5/2, ACD normal (-3,1,1) area sqrt11/2,
    #        sum 2.776; cosine -1/sqrt55 = -0.135
    #   B-D: ABD normal (0,1,1) area sqrt2/2, BCD normal (-3,-2,1) area
    #        sqrt14/2, sum 2.578; cosine -1/sqrt28 = -0.189
    #   -> minimum area B-D, most planar A-C; shortest: 6 > 3, B-D
    a, b, c, d = P(0, 0, 0), P(1, 0, 0), P(1, 1, 2), P(0, 1, -1)
    assert not oracle.split_ac(a, b, c, d, MIN_AREA)
    assert oracle.split_ac(a, b, c, d, PLANAR)
    assert not oracle.split_ac(a, b, c, d, SHORTEST)


def test_area_sums_use_the_split_triangles():
    # a=(0,0,0) b=(1,0,0) c=(0,1,-1) d=(0,0,1)
    #   A-C: ABC normal (0,1,1) area sqrt2/2, ACD normal (1,0,0) area 1/2, sum 1.207
    #   B-D: ABD normal (0,-1,0) area 1/2, BCD normal (1,2,1) area sqrt6/2, sum 1.725
    #   -> minimum area A-C; a sum that took ACD in place of BCD (1/2 + 1/2 = 1)
    #   would pick B-D.  Shortest: |AC|^2 = |BD|^2 = 2, a tie -> A-C.  Most
    #   planar: cosine 0 for A-C against -2/sqrt6 for B-D -> A-C
    a, b, c, d = P(0, 0, 0), P(1, 0, 0), P(0, 1, -1), P(0, 0, 1)
    assert oracle.split_ac(a, b, c, d, MIN_AREA)
    assert oracle.split_ac(a, b, c, d, SHORTEST)
    assert oracle.split_ac(a, b, c, d, PLANAR)


def test_degenerate_split_is_not_preferred_by_planarity():
    # b = c: the A-C split has the degenerate triangle ABC (cosine -2), the B-D
    # split has ABD (0,0,1) and BCD degenerate too (b = c): both -2, tie -> A-C;
    # with b on the A-C diagonal only A-C's triangle ABC is degenerate: a=(0,0,0)
    # b=(1,1,0) c=(2,2,0) d=(0,2,0): ABC degenerate -> A-C cosine -2; B-D:
    # ABD normal (0,0,2), BCD normal (0,0,2) -> cosine 1: B-D
    a, b, c, d = P(0, 0, 0), P(1, 1, 0), P(2, 2, 0), P(0, 2, 0)
    assert not oracle.split_ac(a, b, c, d, PLANAR)
    a, b, c, d = P(0, 0, 0), P(1, 0, 0), P(1, 0, 0), P(0, 1, 0)
    assert oracle.split_ac(a, b, c, d, PLANAR)


def test_triangles_of_each_split():
    # two quads over six points; the first is the folded square of
    # test_folded_square (B-D under minimum area)
    pts = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 1], [0, 1, 0], [2, 0, 0], [2, 1, 0]], np.float64)
    quads = np.array([[0, 1, 2, 3], [1, 4, 5, 2]], np.int32)
    t = oracle.triangulate_rule(quads, pts, MIN_AREA)
    # quad 0 (folded, c lifted): B-D -> (A,B,D), (B,C,D)
    assert t[0].tolist() == [0, 1, 3] and t[1].tolist() == [1, 2, 3]
    t0 = oracle.triangulate_rule(quads, pts, FIXED)
    assert t0[0].tolist() == [0, 1, 2] and t0[1].tolist() == [0, 2, 3]
    assert t0[2].tolist() == [1, 4, 5] and t0[3].tolist() == [1, 5, 2]


@pytest.mark.parametrize("rule", [FIXED, SHORTEST, MIN_AREA, PLANAR])
def test_splits_on_an_extracted_mesh_are_valid(rule):
    """On a smoothed oracle mesh every quad becomes one of its two splits, with
    the quad's orientation; the fixed rule is the plain two-triangle split."""
    import synth

    rng = np.random.default_rng(3)
    lab = synth.blocky_tiny(rng, (14, 12, 10), 4, np.uint16)
    o = oracle.extract(lab, (), 0)
    pts = o.smooth(6, 0.5, 1.0)
    tris = oracle.triangulate_rule(o.quads, pts, rule)
    for q, (A, B, C, D) in enumerate(o.quads):
        t = [tris[2 * q].tolist(), tris[2 * q + 1].tolist()]
        assert t in ([[A, B, C], [A, C, D]], [[A, B, D], [B, C, D]]), (q, t)
    if rule == FIXED:
        plain, _ = o.triangulate()
        assert np.array_equal(tris, plain)
