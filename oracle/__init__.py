"""SurfaceNets oracle (test infrastructure only).

Thin ctypes wrapper around ``sn_oracle.c``, the plain serial FP64 statement of
the method (Sections 2.1-2.5 and Eq. (1) of Schroeder et al., "A
High-Performance SurfaceNets Discrete Isocontouring Algorithm").  Only the
tests, the package smoke check and the benchmark's CPU-baseline leg import
this module; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SN_ORACLE_LIB names another build of sn_oracle.c (the mutation test loads
# builds with planted mistakes this way)
_LIB_PATH = os.environ.get("SN_ORACLE_LIB") or os.path.join(_HERE, "libsn_oracle.so")
_lib = None


_PAR_PATH = os.path.join(_HERE, "libsn_oracle_par.so")
_par = None


def build() -> str:
    """Compile libsn_oracle.so with gcc (serial, no fast-math), and
    libsn_oracle_par.so, the same loops over z-slices with OpenMP (the
    benchmark's all-cores CPU baseline)."""
    import subprocess

    src = os.path.join(_HERE, "sn_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, src,
                           "-lm"])
    os.replace(tmp, _LIB_PATH)
    src = os.path.join(_HERE, "sn_oracle_par.c")
    tmp = _PAR_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, _PAR_PATH)
    return _LIB_PATH


def _load_par():
    global _par
    if _par is None:
        if not os.path.exists(_PAR_PATH):
            build()
        lib = ctypes.CDLL(_PAR_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_extract_par.restype = P
        lib.orc_extract_par.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.c_int32,
                                        ctypes.c_uint32, ctypes.c_int32]
        lib.orc_smooth_par.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int32, P]
        lib.orc_smooth_par.restype = ctypes.c_int
        lib.orc_mesh_free.argtypes = [P]
        lib.orc_mesh_free.restype = None
        lib.orc_mesh_sizes.argtypes = [P, P]
        lib.orc_mesh_sizes.restype = None
        lib.orc_mesh_copy.argtypes = [P, P, P, P, P, P]
        lib.orc_mesh_copy.restype = None
        lib.orc_par_max_threads.argtypes = []
        lib.orc_par_max_threads.restype = ctypes.c_int32
        _par = lib
    return _par


def par_threads() -> int:
    """Threads the all-cores oracle uses by default (OpenMP's default)."""
    return int(_load_par().orc_par_max_threads())


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_extract.restype = P
        lib.orc_extract.argtypes = [P, ctypes.c_int, I64, I64, I64, P, ctypes.c_int32,
                                    ctypes.c_uint32]
        lib.orc_extract2d.restype = P
        lib.orc_extract2d.argtypes = [P, ctypes.c_int, I64, I64, P, ctypes.c_int32, ctypes.c_uint32]
        lib.orc_mesh_free.argtypes = [P]
        lib.orc_mesh_free.restype = None
        lib.orc_mesh_sizes.argtypes = [P, P]
        lib.orc_mesh_sizes.restype = None
        lib.orc_mesh_copy.argtypes = [P, P, P, P, P, P]
        lib.orc_mesh_copy.restype = None
        lib.orc_smooth.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P]
        lib.orc_smooth.restype = ctypes.c_int
        lib.orc_smooth_shape.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, P]
        lib.orc_smooth_shape.restype = ctypes.c_int
        lib.orc_centres.argtypes = [P, P]
        lib.orc_centres.restype = None
        lib.orc_world.argtypes = [I64, P, P, P, P]
        lib.orc_world.restype = None
        lib.orc_triangulate.argtypes = [P, P, P]
        lib.orc_triangulate.restype = None
        lib.orc_split_ac.argtypes = [P, P, P, P, ctypes.c_int]
        lib.orc_split_ac.restype = ctypes.c_int
        lib.orc_triangulate_rule.argtypes = [I64, P, P, ctypes.c_int, P]
        lib.orc_triangulate_rule.restype = None
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class OracleMesh:
    dims: tuple            # (M, N, O)
    cell_of: np.ndarray    # int64 [P] linear cell index i + (M-1)(j + (N-1)k)
    quads: np.ndarray      # int32 [Q, 4], or [Q, 2] segments for an image
    pairs: np.ndarray      # uint32 [Q, 2] (front, back)
    st_off: np.ndarray     # int64 [P+1]
    st_ids: np.ndarray     # int32 [S]
    _handle: int = 0
    _par: bool = False     # made by the all-cores library (freed by it)

    @property
    def n_points(self):
        return int(self.cell_of.shape[0])

    @property
    def n_quads(self):
        return int(self.quads.shape[0])

    @property
    def n_stencil(self):
        return int(self.st_ids.shape[0])

    def cells_ijk(self) -> np.ndarray:
        M, N, _ = self.dims
        c = self.cell_of
        return np.stack([c % (M - 1), (c // (M - 1)) % (N - 1), c // ((M - 1) * (N - 1))], 1)

    def centres(self) -> np.ndarray:
        out = np.empty((self.n_points, 3), dtype=np.float64)
        _load().orc_centres(self._handle, _p(out))
        return out

    def smooth(self, iterations: int, relaxation: float, constraint: float,
               shape: str = "box") -> np.ndarray:
        """Index-space positions after `iterations` Jacobi sweeps (FP64), each
        point held in the box of half-width `constraint` per axis or the sphere
        of that radius around its cell centre."""
        out = np.empty((self.n_points, 3), dtype=np.float64)
        rc = _load().orc_smooth_shape(self._handle, int(iterations), float(relaxation),
                                      float(constraint), {"box": 0, "sphere": 1}[shape], _p(out))
        if rc != 0:
            raise MemoryError("oracle smoothing allocation failed")
        return out

    def smooth_par(self, iterations: int, relaxation: float, constraint: float,
                   shape: str = "box", threads: int = 0) -> np.ndarray:
        """smooth() with the points of each sweep spread over `threads` host
        threads (0: all); equal to smooth() bit for bit."""
        out = np.empty((self.n_points, 3), dtype=np.float64)
        rc = _load_par().orc_smooth_par(self._handle, int(iterations), float(relaxation),
                                        float(constraint), {"box": 0, "sphere": 1}[shape],
                                        int(threads), _p(out))
        if rc != 0:
            raise MemoryError("oracle smoothing allocation failed")
        return out

    def triangulate(self):
        tris = np.empty((2 * self.n_quads, 3), dtype=np.int32)
        tp = np.empty((2 * self.n_quads, 2), dtype=np.uint32)
        _load().orc_triangulate(self._handle, _p(tris), _p(tp))
        return tris, tp

    def __del__(self):
        lib = _par if self._par else _lib
        if self._handle and lib is not None:
            lib.orc_mesh_free(self._handle)
            self._handle = 0


def extract(labels: np.ndarray, selected=(), background: int = 0) -> OracleMesh:
    """Extract the SurfaceNets mesh of a label volume of shape (O, N, M)."""
    lib = _load()
    labels = np.ascontiguousarray(labels)
    if labels.dtype not in (np.uint8, np.uint16, np.uint32):
        raise TypeError("labels must be uint8, uint16 or uint32")
    O, N, M = labels.shape
    sel = np.ascontiguousarray(np.asarray(selected, dtype=np.uint32).reshape(-1))
    h = lib.orc_extract(_p(labels), labels.dtype.itemsize, M, N, O,
                        _p(sel) if sel.size else None, int(sel.size), int(background))
    if not h:
        raise MemoryError("oracle extraction failed")
    sizes = np.zeros(4, dtype=np.int64)
    lib.orc_mesh_sizes(h, _p(sizes))
    P, Q, S = (int(x) for x in sizes[:3])
    cell_of = np.empty(P, dtype=np.int64)
    quads = np.empty((Q, 4), dtype=np.int32)
    pairs = np.empty((Q, 2), dtype=np.uint32)
    st_off = np.empty(P + 1, dtype=np.int64)
    st_ids = np.empty(S, dtype=np.int32)
    lib.orc_mesh_copy(h, _p(cell_of), _p(quads), _p(pairs), _p(st_off), _p(st_ids))
    return OracleMesh((M, N, O), cell_of, quads, pairs, st_off, st_ids, h)


def extract_par(labels: np.ndarray, selected=(), background: int = 0,
                threads: int = 0) -> OracleMesh:
    """extract() with the oracle's loops spread over z-slices on `threads`
    host threads (0: all); equal to extract() bit for bit."""
    lib = _load_par()
    labels = np.ascontiguousarray(labels)
    if labels.dtype not in (np.uint8, np.uint16, np.uint32):
        raise TypeError("labels must be uint8, uint16 or uint32")
    if labels.ndim != 3:
        raise ValueError("extract_par takes a volume (O, N, M)")
    O, N, M = labels.shape
    sel = np.ascontiguousarray(np.asarray(selected, dtype=np.uint32).reshape(-1))
    h = lib.orc_extract_par(_p(labels), labels.dtype.itemsize, M, N, O,
                            _p(sel) if sel.size else None, int(sel.size), int(background),
                            int(threads))
    if not h:
        raise MemoryError("oracle extraction failed")
    sizes = np.zeros(4, dtype=np.int64)
    lib.orc_mesh_sizes(h, _p(sizes))
    P, Q, S = (int(x) for x in sizes[:3])
    cell_of = np.empty(P, dtype=np.int64)
    quads = np.empty((Q, 4), dtype=np.int32)
    pairs = np.empty((Q, 2), dtype=np.uint32)
    st_off = np.empty(P + 1, dtype=np.int64)
    st_ids = np.empty(S, dtype=np.int32)
    lib.orc_mesh_copy(h, _p(cell_of), _p(quads), _p(pairs), _p(st_off), _p(st_ids))
    _load()  # centres() and smooth() of the mesh use the serial library
    return OracleMesh((M, N, O), cell_of, quads, pairs, st_off, st_ids, h, True)


def extract2d(labels: np.ndarray, selected=(), background: int = 0) -> OracleMesh:
    """Extract the 2D SurfaceNets contour of a label image of shape (N, M):
    points, segments [Q, 2], label pairs and the stencil; dims are (M, N, 1)."""
    lib = _load()
    labels = np.ascontiguousarray(labels)
    if labels.dtype not in (np.uint8, np.uint16, np.uint32):
        raise TypeError("labels must be uint8, uint16 or uint32")
    N, M = labels.shape
    sel = np.ascontiguousarray(np.asarray(selected, dtype=np.uint32).reshape(-1))
    h = lib.orc_extract2d(_p(labels), labels.dtype.itemsize, M, N,
                          _p(sel) if sel.size else None, int(sel.size), int(background))
    if not h:
        raise MemoryError("oracle extraction failed")
    sizes = np.zeros(4, dtype=np.int64)
    lib.orc_mesh_sizes(h, _p(sizes))
    P, Q, S = (int(x) for x in sizes[:3])
    cell_of = np.empty(P, dtype=np.int64)
    segs = np.empty((Q, 2), dtype=np.int32)
    pairs = np.empty((Q, 2), dtype=np.uint32)
    st_off = np.empty(P + 1, dtype=np.int64)
    st_ids = np.empty(S, dtype=np.int32)
    lib.orc_mesh_copy(h, _p(cell_of), _p(segs), _p(pairs), _p(st_off), _p(st_ids))
    return OracleMesh((M, N, 1), cell_of, segs, pairs, st_off, st_ids, h)


def world(idx_pos: np.ndarray, origin, spacing) -> np.ndarray:
    """World points origin + spacing * p of index-space points p [P, 3]."""
    lib = _load()
    idx_pos = np.ascontiguousarray(idx_pos, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    h = np.ascontiguousarray(spacing, dtype=np.float64)
    # the C loop reads three coordinates per point and three of each vector
    if idx_pos.ndim != 2 or idx_pos.shape[1] != 3 or o.shape != (3,) or h.shape != (3,):
        raise ValueError("world() takes points [P, 3] and 3-vectors origin and spacing")
    out = np.empty_like(idx_pos)
    lib.orc_world(idx_pos.shape[0], _p(idx_pos), _p(o), _p(h), _p(out))
    return out


# Diagonal rules of Sec. 2.5 (readings in sn_oracle.c): 0 fixed (A-C),
# 1 shortest diagonal, 2 minimum area, 3 most planar.
DIAG_RULES = {"fixed": 0, "shortest": 1, "min_area": 2, "planar": 3}


def split_ac(a, b, c, d, rule: int) -> bool:
    """True if quad (a, b, c, d) (world points) is split along A-C under `rule`."""
    pts = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c, d)]
    return bool(_load().orc_split_ac(*(_p(x) for x in pts), int(rule)))


def triangulate_rule(quads: np.ndarray, points: np.ndarray, rule: int) -> np.ndarray:
    """Triangles [2Q, 3] of quads [Q, 4] over world points [P, 3] (FP64) under
    a diagonal rule: (A,B,C), (A,C,D) for the A-C split, (A,B,D), (B,C,D) for B-D."""
    q = np.ascontiguousarray(quads, dtype=np.int32)
    pts = np.ascontiguousarray(points, dtype=np.float64)
    tris = np.empty((2 * q.shape[0], 3), dtype=np.int32)
    _load().orc_triangulate_rule(q.shape[0], _p(q), _p(pts), int(rule), _p(tris))
    return tris
