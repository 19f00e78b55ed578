"""Pins for the oracle: checks against what the paper and mathematics fix.

Each test compares the oracle (plain serial C) with something that is not the
oracle: closed forms written differently (tests/closed_forms.py), worked cases
whose answer is known by hand or printed in the paper (tests/golden/),
invariants of the method, textbook linear algebra (scipy.sparse) and brute
force.  No GPU is touched.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def check_against_closed_forms(orc, labels, selected=(), background=0):
    m = orc.extract(labels, selected, background)
    c = cf.classify(labels, selected, background)
    pm = cf.point_mask(c)
    # P1: point set and order
    np.testing.assert_array_equal(m.cell_of, np.flatnonzero(pm.ravel()))
    # P2: quads (count, vertex ids, order) and label pairs
    q, pr, _ = cf.quads(c)
    np.testing.assert_array_equal(m.quads.astype(np.int64), q)
    np.testing.assert_array_equal(m.pairs.astype(np.int64), pr)
    # stencil (face rule)
    off, ids = cf.stencil(c)
    np.testing.assert_array_equal(m.st_off, off)
    np.testing.assert_array_equal(m.st_ids.astype(np.int64), ids)
    return m


def mesh_edges(quads):
    e = np.concatenate([quads[:, [0, 1]], quads[:, [1, 2]], quads[:, [2, 3]], quads[:, [3, 0]]])
    return np.sort(e, axis=1)


def quad_normal(pts, quad):
    a, b, c, d = (pts[v] for v in quad)
    return np.cross(c - a, d - b)  # the (doubled) vector area of a planar quad


# --------------------------------------------------------------------------
# P3: a single labelled voxel gives a closed cube
# --------------------------------------------------------------------------

def test_single_voxel_closed_cube(orc):
    v = np.zeros((3, 3, 3), np.uint16)
    v[1, 1, 1] = 7
    m = orc.extract(v)
    assert (m.n_points, m.n_quads) == (8, 6)
    ctr = m.centres()
    assert sorted(map(tuple, ctr)) == sorted(itertools.product((0.5, 1.5), repeat=3))
    # closed 2-manifold: every undirected edge in exactly two quads, chi = 2
    e, cnt = np.unique(mesh_edges(m.quads), axis=0, return_counts=True)
    assert np.all(cnt == 2) and len(e) == 12
    assert m.n_points - len(e) + m.n_quads == 2
    # every point has its three cube neighbours
    assert np.all(np.diff(m.st_off) == 3)
    # orientation: flip the quads whose back region is not the voxel, then the
    # directed edges pair up and every normal points away from the voxel centre
    oriented = [q if pr[1] == 7 else q[::-1] for q, pr in zip(m.quads, m.pairs)]
    directed = set()
    for q in oriented:
        for a, b in zip(q, np.roll(q, -1)):
            assert (a, b) not in directed
            directed.add((a, b))
    assert all((b, a) in directed for a, b in directed)
    for q in oriented:
        n = quad_normal(ctr, q)
        assert np.dot(n, ctr[q].mean(0) - 1.0) > 0


# --------------------------------------------------------------------------
# P4: half-space sheets (including the pathological y/z-only case of Sec. 3.4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_halfspace_sheet(orc, axis):
    M, N, O = 5, 7, 9
    dims = (M, N, O)
    h = 2
    k, j, i = np.meshgrid(np.arange(O), np.arange(N), np.arange(M), indexing="ij")
    coord = (i, j, k)[axis]
    v = np.where(coord < h, 3, 0).astype(np.uint8)
    m = orc.extract(v)
    others = [dims[a] for a in range(3) if a != axis]
    assert m.n_points == (others[0] - 1) * (others[1] - 1)
    assert m.n_quads == (others[0] - 2) * (others[1] - 2)
    ctr = m.centres()
    assert np.all(ctr[:, axis] == h - 0.5)
    # each quad separates the labelled half (x < h, the s0 side) from background
    assert np.all(m.pairs[:, 0] == 3) and np.all(m.pairs[:, 1] == 0)
    for q in m.quads:
        n = quad_normal(ctr, q)
        assert n[axis] < 0 and np.count_nonzero(n) == 1  # normal along -axis, towards s0


# --------------------------------------------------------------------------
# P5: Fig. 10 -- eight different labels around one cell
# --------------------------------------------------------------------------

def test_fig10_eight_labels_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "fig10_eight_labels.json")))
    v = np.array(g["volume_kji"], dtype=np.uint16)
    m = orc.extract(v)
    ctr = m.centres()
    centre_cell = np.flatnonzero(np.all(ctr == np.array(g["centre_cell"]) + 0.5, axis=1))
    assert len(centre_cell) == g["expect"]["points_in_centre_cell"]
    p = int(centre_cell[0])
    assert int(np.sum(np.any(m.quads == p, axis=1))) == g["expect"]["quads_at_centre_point"]
    assert int(m.st_off[p + 1] - m.st_off[p]) == g["expect"]["stencil_neighbours"]


# --------------------------------------------------------------------------
# P1/P2/stencil: closed forms on random and exhaustive tiny volumes
# --------------------------------------------------------------------------

@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(M=st.integers(1, 9), N=st.integers(1, 9), O=st.integers(1, 9), nv=st.integers(1, 9),
       dt=st.sampled_from([np.uint8, np.uint16, np.uint32]), seed=st.integers(0, 2**31),
       blocky=st.booleans(), nsel=st.integers(0, 4), bg=st.integers(0, 9))
def test_closed_forms_random(orc, M, N, O, nv, dt, seed, blocky, nsel, bg):
    import synth

    rng = np.random.default_rng(seed)
    gen = synth.blocky_tiny if blocky else synth.random_tiny
    v = gen(rng, (M, N, O), nv, dt)
    sel = tuple(int(x) for x in rng.choice(10, size=nsel, replace=True) if int(x) != bg)
    check_against_closed_forms(orc, v, sel, bg)


def test_closed_forms_exhaustive_2x2x2(orc):
    """All 2^8 binary and 3^8 ternary corner patterns, embedded in a 4^3 volume."""
    for base in (2, 3):
        for pat in itertools.product(range(base), repeat=8):
            v = np.zeros((4, 4, 4), np.uint8)
            v[1:3, 1:3, 1:3] = np.array(pat, np.uint8).reshape(2, 2, 2) + 1
            v[1:3, 1:3, 1:3] -= 1  # the pattern value 0 is the background
            m = check_against_closed_forms(orc, v)
            # P6: no quad repeats a vertex, no duplicate quads
            assert np.all(np.array([len(set(q)) for q in m.quads]) == 4) if m.n_quads else True


def test_degenerate_dims(orc):
    for dims in [(1, 1, 1), (1, 5, 5), (5, 1, 5), (5, 5, 1), (2, 2, 2), (2, 9, 2)]:
        M, N, O = dims
        v = np.arange(M * N * O, dtype=np.uint16).reshape(O, N, M) % 3
        m = check_against_closed_forms(orc, v)
        if min(dims) < 2:
            assert m.n_points == 0 and m.n_quads == 0
        if min(dims) == 2:
            assert m.n_quads == 0  # no edge has four cells around it


# --------------------------------------------------------------------------
# P6/P7: sharing of interior mesh edges, stencil structure
# --------------------------------------------------------------------------

def _interior_pairs(m, quads):
    """Mesh edges between cells whose shared face lies strictly inside the grid."""
    M, N, O = m.dims
    ijk = m.cells_ijk()
    e = mesh_edges(quads)
    a, b = ijk[e[:, 0]], ijk[e[:, 1]]
    lo = np.minimum(a, b)
    d = np.abs(a - b)
    assert np.all(d.sum(1) == 1)  # quad sides join face neighbours only
    ext = np.array([M - 1, N - 1, O - 1])
    inside = np.all((lo >= 1) | (d == 1), axis=1) & np.all((lo <= ext - 2) | (d == 1), axis=1)
    return e, inside


@pytest.mark.parametrize("seed", range(6))
def test_sharing_and_stencil(orc, seed):
    import synth

    rng = np.random.default_rng(100 + seed)
    dims = tuple(int(x) for x in rng.integers(4, 12, size=3))
    v = (synth.blocky_tiny if seed % 2 else synth.random_tiny)(rng, dims, 2 + seed, np.uint16)
    m = orc.extract(v)
    if m.n_quads == 0:
        return
    assert np.all([len(set(q)) == 4 for q in m.quads])
    assert len(np.unique(np.sort(m.quads, 1), axis=0)) == m.n_quads
    e, inside = _interior_pairs(m, m.quads)
    ue, cnt = np.unique(e[inside], axis=0, return_counts=True)
    assert not np.any(cnt == 1)  # a face never has exactly one label change
    # stencil: symmetric, at most 6, and every quad side is a stencil link
    links = set()
    for p in range(m.n_points):
        nb = m.st_ids[m.st_off[p]:m.st_off[p + 1]]
        assert len(nb) <= 6 and len(set(nb)) == len(nb)
        links.update((p, int(q)) for q in nb)
    assert all((b, a) in links for a, b in links)
    for a, b in np.unique(e, axis=0):
        assert (int(a), int(b)) in links


# --------------------------------------------------------------------------
# P8-P12: smoothing
# --------------------------------------------------------------------------

def _sample_mesh(orc, seed=7, dims=(9, 8, 7), nv=4):
    import synth

    rng = np.random.default_rng(seed)
    return orc.extract(synth.blocky_tiny(rng, dims, nv, np.uint16))


def test_smoothing_identity_cases(orc):
    m = _sample_mesh(orc)
    c = m.centres()
    assert np.array_equal(m.smooth(25, 0.0, 1.0), c)  # lambda = 0
    assert np.array_equal(m.smooth(25, 0.7, 0.0), c)  # d = 0
    assert np.array_equal(m.smooth(0, 0.7, 1.0), c)   # no sweeps


@pytest.mark.parametrize("lam,d", [(0.5, 1.0), (1.0, 0.3), (0.9, 0.05)])
def test_smoothing_constraint_box(orc, lam, d):
    m = _sample_mesh(orc, seed=11)
    p = m.smooth(30, lam, d)
    assert np.max(np.abs(p - m.centres())) <= d + 1e-12


@pytest.mark.parametrize("lam,d,n", [(0.5, 1.0, 16), (0.5, 0.2, 16), (1.0, 1.0, 7), (0.3, 0.45, 40),
                                     (1.5, 1.0, 5)])
def test_smoothing_cube_closed_form(orc, lam, d, n):
    """Single voxel: the 8 points stay on a cube whose half-size obeys
    s_{t+1} = max(1/2 - d, s_t (1 - 2 lambda / 3)), s_0 = 1/2."""
    v = np.zeros((3, 3, 3), np.uint8)
    v[1, 1, 1] = 1
    m = orc.extract(v)
    p = m.smooth(n, lam, d)
    s = max(0.5 - d, 0.5 * (1 - 2 * lam / 3) ** n) if lam <= 1.5 else None
    np.testing.assert_allclose(np.abs(p - 1.0), s, rtol=0, atol=1e-14)


@pytest.mark.parametrize("lam,d,n", [(0.5, 1.0, 16), (0.5, 0.2, 16), (1.0, 1.0, 7), (0.3, 0.45, 40),
                                     (1.5, 1.0, 5)])
def test_smoothing_cube_closed_form_sphere(orc, lam, d, n):
    """Single voxel, sphere constraint: the points move along the cube's
    diagonals, so a displacement of u per axis has length sqrt(3) u and the
    sphere of radius d binds at u = d / sqrt(3):
    s_{t+1} = max(1/2 - d / sqrt(3), s_t (1 - 2 lambda / 3))."""
    v = np.zeros((3, 3, 3), np.uint8)
    v[1, 1, 1] = 1
    m = orc.extract(v)
    p = m.smooth(n, lam, d, shape="sphere")
    s = max(0.5 - d / np.sqrt(3.0), 0.5 * (1 - 2 * lam / 3) ** n)
    np.testing.assert_allclose(np.abs(p - 1.0), s, rtol=0, atol=1e-14)


def test_smoothing_sphere_off_diagonal(orc):
    """Two labelled samples (1,1,1), (2,1,1): one sweep with lambda = 1 from
    the centres.  The middle cell (1,0,0) has neighbours -x, +x, +y, +z, so
    it moves by (0, 1/4, 1/4) (length 0.354); the corner cell (0,0,0) has
    +x, +y, +z and moves by (1/3, 1/3, 1/3) (length 0.577).  The sphere of
    radius 0.3 scales both back to length 0.3 along the same directions; the
    box of half-width 0.3 leaves the first and clamps the second per axis."""
    v = np.zeros((3, 3, 4), np.uint16)  # [O][N][M]
    v[1, 1, 1] = v[1, 1, 2] = 5
    m = orc.extract(v)
    c = m.centres()
    mid = int(np.flatnonzero(np.all(c == (1.5, 0.5, 0.5), axis=1))[0])
    cor = int(np.flatnonzero(np.all(c == (0.5, 0.5, 0.5), axis=1))[0])
    ps = m.smooth(1, 1.0, 0.3, shape="sphere") - c
    pb = m.smooth(1, 1.0, 0.3) - c
    r = 0.3 / np.sqrt(2.0)
    np.testing.assert_allclose(ps[mid], (0.0, r, r), atol=1e-15)
    np.testing.assert_allclose(ps[cor], (0.3 / np.sqrt(3.0),) * 3, atol=1e-15)
    np.testing.assert_allclose(pb[mid], (0.0, 0.25, 0.25), atol=1e-15)
    np.testing.assert_allclose(pb[cor], (0.3, 0.3, 0.3), atol=1e-15)


@pytest.mark.parametrize("lam,d", [(0.5, 1.0), (1.0, 0.3), (0.9, 0.05)])
def test_smoothing_constraint_sphere(orc, lam, d):
    m = _sample_mesh(orc, seed=12)
    p = m.smooth(30, lam, d, shape="sphere")
    assert np.max(np.linalg.norm(p - m.centres(), axis=1)) <= d + 1e-12
    # a radius no point reaches constrains nothing: the same as a box that large
    np.testing.assert_array_equal(m.smooth(9, lam, 50.0, shape="sphere"), m.smooth(9, lam, 50.0))


def test_smoothing_linear_part_scipy(orc):
    """With an inactive constraint the n sweeps are the linear map
    (I - lambda (I - D^-1 A))^n applied to the centres; A is built here from
    the closed-form face rule, not from the oracle's stencil."""
    import scipy.sparse as sp
    import synth

    rng = np.random.default_rng(5)
    v = synth.blocky_tiny(rng, (10, 9, 8), 4, np.uint16)
    c = cf.classify(v)
    off, ids = cf.stencil(c)
    P = len(off) - 1
    rows = np.repeat(np.arange(P), np.diff(off))
    A = sp.csr_matrix((np.ones(len(ids)), (rows, ids)), shape=(P, P))
    deg = np.asarray(A.sum(1)).ravel()
    Dinv = sp.diags(np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0))
    I = sp.identity(P)
    lam, n = 0.6, 12
    T = I - lam * (I - Dinv @ A)
    T = T + sp.diags(np.where(deg == 0, lam, 0.0))  # isolated points do not move
    x = cf.centres(cf.point_mask(c))
    for _ in range(n):
        x = T @ x
    m = orc.extract(v)
    np.testing.assert_allclose(m.smooth(n, lam, 1e6), x, rtol=0, atol=1e-12)


def test_plane_stays_flat(orc):
    M, N, O = 6, 9, 11
    k, j, i = np.meshgrid(np.arange(O), np.arange(N), np.arange(M), indexing="ij")
    v = np.where(i < 3, 1, 2).astype(np.uint16)
    m = orc.extract(v)
    for n in (1, 5, 25):
        p = m.smooth(n, 0.5, 1.0)
        assert np.all(p[:, 0] == 2.5)  # bit-constant
        ijk = m.cells_ijk()
        # mirror symmetry of the sheet in y and in z
        for ax, ext in ((1, N - 1), (2, O - 1)):
            mir = ijk.copy()
            mir[:, ax] = ext - 1 - ijk[:, ax]
            idx = {tuple(t): r for r, t in enumerate(ijk)}
            perm = np.array([idx[tuple(t)] for t in mir])
            np.testing.assert_allclose(p[perm, ax], ext - p[:, ax], rtol=0, atol=1e-12)


def test_spacing_commutes_with_box(orc):
    """Smoothing in index space then scaling by the spacing equals smoothing in
    world space with a box of half-width d*h (the constraint per axis)."""
    m = _sample_mesh(orc, seed=3)
    h = np.array([0.7, 1.3, 2.5])
    o = np.array([-4.0, 10.0, 0.25])
    lam, d, n = 0.5, 0.35, 9
    w = orc.world(m.smooth(n, lam, d), o, h)
    x = o + h * m.centres()
    x0 = x.copy()
    for _ in range(n):
        y = x.copy()
        for p in range(m.n_points):
            nb = m.st_ids[m.st_off[p]:m.st_off[p + 1]]
            if len(nb):
                y[p] = x[p] + lam * (x[nb] - x[p]).mean(0)
            y[p] = np.clip(y[p], x0[p] - d * h, x0[p] + d * h)
        x = y
    np.testing.assert_allclose(w, x, rtol=0, atol=1e-11)


def test_world_rejects_other_shapes(orc):
    """The world map reads three coordinates per point: 2D arrays of another
    width, or origin/spacing of another length, are refused before the call."""
    p = np.zeros((4, 3))
    with pytest.raises(ValueError):
        orc.world(np.zeros((4, 2)), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    with pytest.raises(ValueError):
        orc.world(p, (0.0, 0.0), (1.0, 1.0, 1.0))
    with pytest.raises(ValueError):
        orc.world(p, (0.0, 0.0, 0.0), (1.0, 1.0))
    np.testing.assert_array_equal(orc.world(p + 1.0, (1.0, 2.0, 3.0), (2.0, 2.0, 2.0)),
                                  np.tile([3.0, 4.0, 5.0], (4, 1)))


# --------------------------------------------------------------------------
# P14/P15: classification
# --------------------------------------------------------------------------

def test_relabel_bijection(orc):
    import synth

    rng = np.random.default_rng(9)
    v = synth.random_tiny(rng, (7, 6, 8), 5, np.uint16)
    perm = np.array([0, 40000, 7, 65535, 12], np.uint16)  # background 0 kept
    m1, m2 = orc.extract(v), orc.extract(perm[v])
    np.testing.assert_array_equal(m1.cell_of, m2.cell_of)
    np.testing.assert_array_equal(m1.quads, m2.quads)
    np.testing.assert_array_equal(perm[m1.pairs], m2.pairs)
    np.testing.assert_array_equal(m1.st_ids, m2.st_ids)


def test_selection_equals_masking(orc):
    import synth

    rng = np.random.default_rng(10)
    v = synth.random_tiny(rng, (8, 7, 6), 6, np.uint32)
    sel = (2, 5)
    masked = np.where(np.isin(v, sel), v, 0).astype(np.uint32)
    m1, m2 = orc.extract(v, sel, 0), orc.extract(masked)
    for a, b in ((m1.cell_of, m2.cell_of), (m1.quads, m2.quads), (m1.pairs, m2.pairs),
                 (m1.st_off, m2.st_off), (m1.st_ids, m2.st_ids)):
        np.testing.assert_array_equal(a, b)
    # a non-zero background value is written on the background side of pairs
    m3 = orc.extract(v, sel, 4)
    assert set(np.unique(m3.pairs)) <= {2, 4, 5}


# --------------------------------------------------------------------------
# P16: triangulation
# --------------------------------------------------------------------------

def test_triangulation(orc):
    m = _sample_mesh(orc, seed=12)
    tris, tp = m.triangulate()
    assert len(tris) == 2 * m.n_quads
    np.testing.assert_array_equal(tris[0::2], m.quads[:, [0, 1, 2]])
    np.testing.assert_array_equal(tris[1::2], m.quads[:, [0, 2, 3]])
    np.testing.assert_array_equal(tp[0::2], m.pairs)
    np.testing.assert_array_equal(tp[1::2], m.pairs)
    # the paper's triangle counts are twice its quad counts, hence even
    g = json.load(open(os.path.join(GOLDEN, "table1_counts.json")))
    assert all(r["triangles"] % 2 == 0 for r in g["rows"])
