"""Closed forms that pin the oracle from outside (numpy, vectorised).

These restate the *consequences* of the paper's definitions in a different
form from the oracle's cell-by-cell, edge-by-edge loops:

* a cell has a point iff its eight classified corner values are not all equal
  (the 12 edges of a cube connect all eight corners, so "some edge is cut"
  and "not all corners equal" coincide; Sec. 2.2);
* quads are the cut lattice edges whose four surrounding cells exist, in
  lattice order then axis (Sec. 2.2, open boundary of Sec. 4.2);
* a face carries a stencil link iff its four corner values are not all equal
  (Sec. 3.3: a face with a cut edge; the four edges of a square connect its
  four corners).
"""
from __future__ import annotations

import numpy as np


def classify(labels: np.ndarray, selected=(), background: int = 0) -> np.ndarray:
    v = labels.astype(np.int64)
    if len(selected) == 0:
        keep = v != background
    else:
        keep = np.isin(v, np.asarray(list(selected), dtype=np.int64)) & (v != background)
    return np.where(keep, v, background)


def _corners(c):
    """The eight corner views of the cell grid, keyed by (di, dj, dk)."""
    out = {}
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                out[(di, dj, dk)] = c[dk:c.shape[0] - 1 + dk, dj:c.shape[1] - 1 + dj,
                                      di:c.shape[2] - 1 + di]
    return out


def point_mask(c: np.ndarray) -> np.ndarray:
    """bool[O-1, N-1, M-1]: the cell has a point."""
    O, N, M = c.shape
    if min(O, N, M) < 2:
        return np.zeros((max(O - 1, 0), max(N - 1, 0), max(M - 1, 0)), dtype=bool)
    cs = np.stack(list(_corners(c).values()), 0)
    return cs.max(0) != cs.min(0)


def point_ids(pm: np.ndarray) -> np.ndarray:
    """int64 grid of point ids (-1 where no point), ids in cell linear order."""
    flat = pm.ravel()
    ids = np.cumsum(flat) - 1
    return np.where(flat, ids, -1).reshape(pm.shape)


def quads(c: np.ndarray):
    """(quads int64[Q,4], pairs int64[Q,2], key int64[Q]) in canonical order."""
    O, N, M = c.shape
    pm = point_mask(c)
    if pm.size == 0:
        return np.zeros((0, 4), np.int64), np.zeros((0, 2), np.int64), np.zeros(0, np.int64)
    pid = point_ids(pm)
    recs = []
    kk, jj, ii = np.meshgrid(np.arange(O), np.arange(N), np.arange(M), indexing="ij")
    lin = ii + M * (jj + N * kk)
    # x-edges: (i,j,k)-(i+1,j,k), cells (i, j-1..j, k-1..k): 1<=j<=N-2, 1<=k<=O-2, i<=M-2
    s0 = c[1:O - 1, 1:N - 1, 0:M - 1]
    s1 = c[1:O - 1, 1:N - 1, 1:M]
    sel = s0 != s1
    k, j, i = [a[1:O - 1, 1:N - 1, 0:M - 1][sel] for a in (kk, jj, ii)]
    v = np.stack([pid[k - 1, j - 1, i], pid[k, j - 1, i], pid[k, j, i], pid[k - 1, j, i]], 1)
    recs.append((lin[1:O - 1, 1:N - 1, 0:M - 1][sel] * 3 + 0, v, s0[sel], s1[sel]))
    # y-edges: (i,j,k)-(i,j+1,k), cells (i-1..i, j, k-1..k): 1<=i<=M-2, 1<=k<=O-2, j<=N-2
    s0 = c[1:O - 1, 0:N - 1, 1:M - 1]
    s1 = c[1:O - 1, 1:N, 1:M - 1]
    sel = s0 != s1
    k, j, i = [a[1:O - 1, 0:N - 1, 1:M - 1][sel] for a in (kk, jj, ii)]
    v = np.stack([pid[k - 1, j, i - 1], pid[k - 1, j, i], pid[k, j, i], pid[k, j, i - 1]], 1)
    recs.append((lin[1:O - 1, 0:N - 1, 1:M - 1][sel] * 3 + 1, v, s0[sel], s1[sel]))
    # z-edges: (i,j,k)-(i,j,k+1), cells (i-1..i, j-1..j, k): 1<=i<=M-2, 1<=j<=N-2, k<=O-2
    s0 = c[0:O - 1, 1:N - 1, 1:M - 1]
    s1 = c[1:O, 1:N - 1, 1:M - 1]
    sel = s0 != s1
    k, j, i = [a[0:O - 1, 1:N - 1, 1:M - 1][sel] for a in (kk, jj, ii)]
    v = np.stack([pid[k, j - 1, i - 1], pid[k, j, i - 1], pid[k, j, i], pid[k, j - 1, i]], 1)
    recs.append((lin[0:O - 1, 1:N - 1, 1:M - 1][sel] * 3 + 2, v, s0[sel], s1[sel]))
    key = np.concatenate([r[0] for r in recs])
    q = np.concatenate([r[1] for r in recs]).reshape(-1, 4)
    pr = np.stack([np.concatenate([r[2] for r in recs]), np.concatenate([r[3] for r in recs])], 1)
    order = np.argsort(key, kind="stable")
    return q[order], pr[order], key[order]


def stencil(c: np.ndarray):
    """(offsets int64[P+1], ids int64[S]) with faces in order -x,+x,-y,+y,-z,+z."""
    O, N, M = c.shape
    pm = point_mask(c)
    if pm.size == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int64)
    pid = point_ids(pm)
    CO, CN, CM = pm.shape

    def nonuni(a, b, d, e):
        return ~((a == b) & (a == d) & (a == e))

    # faces normal to x at lattice x-plane i: corners c[k..k+1, j..j+1, i]
    fx = nonuni(c[:-1, :-1, :], c[:-1, 1:, :], c[1:, :-1, :], c[1:, 1:, :])  # [CO, CN, M]
    fy = nonuni(c[:-1, :, :-1], c[:-1, :, 1:], c[1:, :, :-1], c[1:, :, 1:])  # [CO, N, CM]
    fz = nonuni(c[:, :-1, :-1], c[:, :-1, 1:], c[:, 1:, :-1], c[:, 1:, 1:])  # [O, CN, CM]
    nb = np.full((CO, CN, CM, 6), -1, dtype=np.int64)
    pad = np.full((CO + 2, CN + 2, CM + 2), -1, dtype=np.int64)
    pad[1:-1, 1:-1, 1:-1] = pid
    face = [fx[:, :, 0:CM], fx[:, :, 1:CM + 1], fy[:, 0:CN, :], fy[:, 1:CN + 1, :],
            fz[0:CO, :, :], fz[1:CO + 1, :, :]]
    nid = [pad[1:-1, 1:-1, 0:CM], pad[1:-1, 1:-1, 2:CM + 2], pad[1:-1, 0:CN, 1:-1],
           pad[1:-1, 2:CN + 2, 1:-1], pad[0:CO, 1:-1, 1:-1], pad[2:CO + 2, 1:-1, 1:-1]]
    exists = np.zeros((CO + 2, CN + 2, CM + 2), dtype=bool)
    exists[1:-1, 1:-1, 1:-1] = True
    nex = [exists[1:-1, 1:-1, 0:CM], exists[1:-1, 1:-1, 2:CM + 2], exists[1:-1, 0:CN, 1:-1],
           exists[1:-1, 2:CN + 2, 1:-1], exists[0:CO, 1:-1, 1:-1], exists[2:CO + 2, 1:-1, 1:-1]]
    for f in range(6):
        link = face[f] & nex[f]
        # a face with a cut edge is shared, so the neighbour cell must have a point
        assert np.all(nid[f][link] >= 0)
        nb[..., f] = np.where(link, nid[f], -1)
    rows = nb.reshape(-1, 6)[pm.ravel()]
    cnt = (rows >= 0).sum(1)
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    ids = rows[rows >= 0]  # row-major: per point, faces in order
    return off, ids.astype(np.int64)


def centres(pm: np.ndarray) -> np.ndarray:
    k, j, i = np.nonzero(pm)  # C order == cell linear order
    return np.stack([i + 0.5, j + 0.5, k + 0.5], 1).astype(np.float64)
