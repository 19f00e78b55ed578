"""Pins of the oracle's 2D SurfaceNets (the method in the plane, Sec. 5):
closed forms, a hand-worked single pixel, half-plane sheets, smoothing closed
forms, and a cross-check against the (separately pinned) 3D oracle on images
extruded to three identical slices."""
from __future__ import annotations

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle


def closed_forms_2d(C):
    """Points, segments, pairs and stencil of a classified image C [N, M],
    written from other characterisations than the oracle's: a cell has a point
    iff its four corners are not all equal; a segment is a cut edge with a cell
    on each side; the stencil is the segment graph, in face order."""
    N, M = C.shape
    CM, CN = M - 1, N - 1
    corners = [C[:-1, :-1], C[:-1, 1:], C[1:, :-1], C[1:, 1:]]
    has = np.maximum.reduce(corners) != np.minimum.reduce(corners)  # [CN, CM]
    pid = -np.ones((max(CN, 0), max(CM, 0)), np.int64)
    pid[has] = np.arange(int(has.sum()))
    segs, pairs, keys = [], [], []
    for j in range(N):
        for i in range(M):
            # x-edge (i,j)-(i+1,j) between cells (i,j-1) and (i,j)
            if i + 1 < M and C[j, i] != C[j, i + 1] and 1 <= j <= N - 2:
                segs.append((pid[j, i], pid[j - 1, i]))
                pairs.append((C[j, i], C[j, i + 1]))
                keys.append((j * M + i, 0))
            # y-edge (i,j)-(i,j+1) between cells (i-1,j) and (i,j)
            if j + 1 < N and C[j, i] != C[j + 1, i] and 1 <= i <= M - 2:
                segs.append((pid[j, i - 1], pid[j, i]))
                pairs.append((C[j, i], C[j + 1, i]))
                keys.append((j * M + i, 1))
    order = sorted(range(len(keys)), key=lambda q: keys[q])
    segs = [segs[q] for q in order]
    pairs = [pairs[q] for q in order]
    P = int(has.sum())
    ij = np.argwhere(has)  # (j, i) in id order
    nbrs = [[] for _ in range(P)]
    for a, b in segs:
        nbrs[a].append(b)
        nbrs[b].append(a)

    def face(p, q):
        (jp, ip), (jq, iq) = ij[p], ij[q]
        return {(-1, 0): 0, (1, 0): 1, (0, -1): 2, (0, 1): 3}[(iq - ip, jq - jp)]

    stencil = [sorted(n, key=lambda q, p=p: face(p, q)) for p, n in enumerate(nbrs)]
    cells = ij[:, 1] + CM * ij[:, 0] if P else np.zeros(0, np.int64)
    return cells, segs, pairs, stencil


def check_2d(img, selected=(), background=0):
    m = oracle.extract2d(img, selected, background)
    C = img.astype(np.int64)
    if selected:
        keep = np.isin(C, np.asarray(selected)) & (C != background)
    else:
        keep = C != background
    C = np.where(keep, C, background)
    cells, segs, pairs, stencil = closed_forms_2d(C)
    assert np.array_equal(m.cell_of, cells)
    assert [tuple(s) for s in m.quads.tolist()] == [tuple(map(int, s)) for s in segs]
    assert [tuple(p) for p in m.pairs.tolist()] == [tuple(map(int, p)) for p in pairs]
    got = [m.st_ids[m.st_off[p]:m.st_off[p + 1]].tolist() for p in range(m.n_points)]
    assert got == [[int(x) for x in s] for s in stencil]
    return m


def test_single_pixel_closed_loop():
    img = np.zeros((3, 3), np.uint16)
    img[1, 1] = 7
    m = check_2d(img)
    assert m.n_points == 4 and m.n_quads == 4
    c = m.centres()[:, :2]
    assert np.array_equal(c, [[0.5, 0.5], [1.5, 0.5], [0.5, 1.5], [1.5, 1.5]])
    # orient every segment with the pixel's region on its left (back as given,
    # front reversed): a single counter-clockwise loop around (1, 1)
    nxt = {}
    for (a, b), (f, bk) in zip(m.quads.tolist(), m.pairs.tolist()):
        if bk == 7:
            nxt[a] = b
        else:
            assert f == 7
            nxt[b] = a
    assert sorted(nxt) == [0, 1, 2, 3] and sorted(nxt.values()) == [0, 1, 2, 3]
    loop, p = [0], nxt[0]
    while p != 0:
        loop.append(p)
        p = nxt[p]
    assert len(loop) == 4
    xy = c[loop]
    area = 0.5 * sum(xy[k, 0] * xy[(k + 1) % 4, 1] - xy[(k + 1) % 4, 0] * xy[k, 1] for k in range(4))
    assert area == 1.0  # counter-clockwise, the unit square of the four centres
    assert all(m.st_off[p + 1] - m.st_off[p] == 2 for p in range(4))


@pytest.mark.parametrize("axis", [0, 1])
def test_half_plane(axis):
    M, N, h = 9, 7, 4
    img = np.zeros((N, M), np.uint8)
    if axis == 0:
        img[:, h:] = 3
    else:
        img[h:, :] = 3
    m = check_2d(img)
    other = N if axis == 0 else M
    assert m.n_points == other - 1 and m.n_quads == other - 2
    c = m.centres()
    assert np.all(c[:, axis] == h - 0.5)
    # a straight contour stays straight under smoothing
    s = m.smooth(10, 0.5, 1.0)
    assert np.all(s[:, axis] == h - 0.5)


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(M=st.integers(1, 12), N=st.integers(1, 12), nv=st.integers(1, 6),
       dt=st.sampled_from([np.uint8, np.uint16, np.uint32]), seed=st.integers(0, 2**31),
       nsel=st.integers(0, 3), bg=st.integers(0, 2))
def test_closed_forms_random(M, N, nv, dt, seed, nsel, bg):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, nv + 1, size=(N, M)).astype(dt)
    sel = tuple(int(x) for x in rng.choice(np.arange(nv + 1), size=min(nsel, nv + 1), replace=False)
                if int(x) != bg)
    check_2d(img, sel, bg)


@pytest.mark.parametrize("lam,d,n", [(0.5, 1.0, 16), (0.5, 0.2, 16), (0.3, 0.45, 40), (1.0, 1.0, 3)])
def test_single_pixel_smoothing_closed_form(lam, d, n):
    # each corner point moves along its diagonal: with two neighbours the
    # half-size s shrinks by (1 - lambda) per sweep until the constraint
    # holds it (box: per axis at 1/2 - d; circle: at 1/2 - d/sqrt2)
    img = np.zeros((3, 3), np.uint16)
    img[1, 1] = 1
    m = oracle.extract2d(img)
    for shape, lim in (("box", 0.5 - d), ("sphere", 0.5 - d / np.sqrt(2))):
        s = m.smooth(n, lam, d, shape)
        half = abs(s[:, :2] - 1.0)
        want = max(lim, 0.5 * (1 - lam) ** n)
        assert np.allclose(half, want, rtol=0, atol=1e-12), (shape, half, want)
        assert np.all(s[:, 2] == 0.5)  # no motion out of the plane


@pytest.mark.parametrize("seed", range(5))
def test_extruded_image_matches_the_3d_oracle(seed):
    """An image stacked into three identical slices: the 3D mesh has two
    points per 2D point (layers k = 0, 1), and its quads are exactly the 2D
    segments, in the same order, on the same pair of cell columns, with the
    same label pairs (every cut edge lies in the middle slice's plane; the
    quads of the outer slices touch the cell-grid boundary and are open)."""
    rng = np.random.default_rng(seed)
    M, N = rng.integers(3, 12, size=2)
    img = rng.integers(0, 4, size=(N, M)).astype(np.uint16)
    m2 = oracle.extract2d(img)
    m3 = oracle.extract(np.stack([img, img, img]))
    assert m3.n_points == 2 * m2.n_points and m3.n_quads == m2.n_quads
    ijk = m3.cells_ijk()
    c2 = m2.cell_of
    CM = M - 1
    for q in range(m2.n_quads):
        cells2 = {int(c2[v]) for v in m2.quads[q]}
        cols3 = {int(ijk[v, 0] + CM * ijk[v, 1]) for v in m3.quads[q]}
        assert cells2 == cols3
    assert np.array_equal(m2.pairs, m3.pairs)
    # in-layer stencil of layer 0 = the 2D stencil (plus the twin above)
    layer0 = np.flatnonzero(ijk[:, 2] == 0)
    for p2, p3 in enumerate(layer0):
        n3 = [int(ijk[q, 0] + CM * ijk[q, 1]) for q in m3.st_ids[m3.st_off[p3]:m3.st_off[p3 + 1]]
              if ijk[q, 2] == 0]
        n2 = [int(c2[q]) for q in m2.st_ids[m2.st_off[p2]:m2.st_off[p2 + 1]]]
        assert n3 == n2


def test_degenerate_images():
    for shape in [(1, 1), (1, 9), (9, 1), (2, 2)]:
        img = np.arange(np.prod(shape)).reshape(shape).astype(np.uint8)
        m = check_2d(img)
        if min(shape) < 2:
            assert m.n_points == 0 and m.n_quads == 0
