"""MI355X SurfaceNets: Python binding of libsn.so.

Argument marshalling only: every step of extraction and smoothing runs in the
HIP kernels of ``libsn.so`` (built from ``csrc/`` for gfx950).  PyTorch is used
for device memory and streams.  There is no fallback: if the library is
missing, importing the binding raises.

The functions mirror the C ABI in ``include/sn.h``:

    ctx = Context(0)
    mesh = ctx.extract(labels_cuda_tensor, spacing=(1, 1, 2.5), selected=(), background=0)
    ctx.smooth(mesh, iterations=25, relaxation=0.5, constraint=1.0)
    host = mesh.to_host()        # numpy arrays
    meshes = ctx.batch_submit([...], [...])
    srv = ctx.serve_start(...); t = srv.submit(...); mesh = srv.wait(t)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsn.so")

SN_OK, SN_EINVAL, SN_ENOMEM, SN_EDEVICE, SN_ETOOBIG = 0, -1, -2, -3, -4
SN_EAGAIN, SN_ENOTFOUND, SN_ESHUTDOWN, SN_ETIMEDOUT = -5, -6, -7, -8
SN_LINES, SN_TRIS, SN_QUADS = 2, 3, 4
_NP_DT = {1: np.uint8, 2: np.uint16, 4: np.uint32}
# tessellating-diagonal rules of sn_triangulate
DIAG_RULES = {"fixed": 0, "shortest": 1, "min_area": 2, "planar": 3}


class SNError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsn status {status}: {msg}")
        self.status = status


class sn_volume(ctypes.Structure):
    _fields_ = [("labels", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 3), ("spacing", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3), ("selected", ctypes.POINTER(ctypes.c_uint32)),
                ("n_selected", ctypes.c_int32), ("background", ctypes.c_uint32),
                ("prim", ctypes.c_int32)]


class sn_smooth_params(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("relaxation", ctypes.c_float),
                ("constraint", ctypes.c_float), ("shape", ctypes.c_int32)]


class sn_mesh_view(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_quads", ctypes.c_int64),
                ("n_stencil", ctypes.c_int64), ("n_polys", ctypes.c_int64),
                ("prim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("points", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("polys", ctypes.c_void_p), ("label_pairs", ctypes.c_void_p),
                ("stencil_off", ctypes.c_void_p), ("stencil_ids", ctypes.c_void_p),
                ("quads", ctypes.c_void_p)]


class sn_serve_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32)]


class sn_serve_stats(ctypes.Structure):
    _fields_ = [("n_submitted", ctypes.c_int64), ("n_done", ctypes.c_int64),
                ("n_rejected", ctypes.c_int64), ("n_batches", ctypes.c_int64),
                ("voxels_done", ctypes.c_int64), ("point_iters_done", ctypes.c_int64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("peak_reserved_bytes", ctypes.c_int64), ("n_split_batches", ctypes.c_int64),
                ("n_requeued", ctypes.c_int64)]


class sn_extract_arrays(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("polys", ctypes.c_void_p),
                ("label_pairs", ctypes.c_void_p), ("stencil_off", ctypes.c_void_p),
                ("stencil_ids", ctypes.c_void_p), ("cap_points", ctypes.c_int64),
                ("cap_polys", ctypes.c_int64), ("cap_stencil", ctypes.c_int64)]


class sn_schedule(ctypes.Structure):
    _fields_ = [("gen_groups", ctypes.c_int32), ("count_words", ctypes.c_int32),
                ("edge_segments", ctypes.c_int32), ("sweep_chunk", ctypes.c_int32)]


class sn_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


# every entry point declared in include/sn.h: (name, restype, argtypes)
_P = ctypes.c_void_p
_S = ctypes.c_int
_API = [
    ("sn_ctx_create", _S, [ctypes.c_int, ctypes.POINTER(_P)]),
    ("sn_ctx_destroy", None, [_P]),
    ("sn_ctx_memory", _S, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    ("sn_strerror", ctypes.c_char_p, [_S]),
    ("sn_last_error", ctypes.c_char_p, []),
    ("sn_version", ctypes.c_char_p, []),
    ("sn_extract", _S, [_P, ctypes.POINTER(sn_volume), _P, ctypes.POINTER(_P)]),
    ("sn_smooth", _S, [_P, _P, ctypes.POINTER(sn_smooth_params), _P]),
    ("sn_triangulate", _S, [_P, _P, ctypes.c_int, _P, _P, _P]),
    ("sn_mesh_view_get", _S, [_P, ctypes.POINTER(sn_mesh_view)]),
    ("sn_mesh_copy_to_host", _S, [_P, _P, _P, _P, _P, _P, _P]),
    ("sn_mesh_free", None, [_P]),
    ("sn_extract_noalloc", _S, [_P, ctypes.POINTER(sn_volume), _P,
                                ctypes.POINTER(sn_extract_arrays), ctypes.POINTER(ctypes.c_int64)]),
    ("sn_noalloc_scratch_bytes", ctypes.c_int64, [ctypes.POINTER(sn_volume)]),
    ("sn_batch_submit", _S, [_P, ctypes.POINTER(sn_volume), ctypes.POINTER(sn_smooth_params),
                             ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    ("sn_serve_start", _S, [_P, ctypes.POINTER(sn_serve_config), ctypes.POINTER(_P)]),
    ("sn_serve_submit", _S, [_P, ctypes.POINTER(sn_volume), ctypes.POINTER(sn_smooth_params), _P,
                             ctypes.POINTER(ctypes.c_uint64)]),
    ("sn_serve_poll", _S, [_P, ctypes.c_uint64, ctypes.POINTER(_P)]),
    ("sn_serve_wait", _S, [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(_P)]),
    ("sn_serve_stats_get", _S, [_P, ctypes.POINTER(sn_serve_stats)]),
    ("sn_serve_stop", _S, [_P]),
    ("sn_autotune", _S, [_P, ctypes.POINTER(sn_volume), _P, ctypes.POINTER(ctypes.c_int32)]),
    ("sn_set_batches_per_wave", _S, [_P, ctypes.c_int32]),
    ("sn_schedule_get", _S, [_P, ctypes.POINTER(sn_volume), ctypes.POINTER(sn_schedule)]),
    ("sn_schedule_set", _S, [_P, ctypes.POINTER(sn_volume), ctypes.POINTER(sn_schedule)]),
    ("sn_profile_enable", _S, [_P, ctypes.c_int]),
    ("sn_profile_reset", _S, [_P]),
    ("sn_profile_read", _S, [_P, ctypes.POINTER(sn_kernel_stat), ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32)]),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsn.so and bind every declared entry point.  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, res, args in _API:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int):
    if st != SN_OK:
        msg = _lib.sn_last_error().decode(errors="replace")
        raise SNError(st, msg or _lib.sn_strerror(st).decode())


def _stream_handle(stream) -> Optional[int]:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


@dataclass
class HostMesh:
    points: np.ndarray        # float32 [P,3] world
    offsets: np.ndarray       # float32 [P,3] cell-relative
    polys: np.ndarray         # int32 [n_polys, prim]
    label_pairs: np.ndarray   # dtype [n_polys, 2]
    stencil_off: np.ndarray   # int32 [P+1]
    stencil_ids: np.ndarray   # int32 [S]


class Mesh:
    """A device-resident mesh owned by libsn (freed by .free() or GC)."""

    def __init__(self, handle: int, keepalive=None):
        self._h = ctypes.c_void_p(handle)
        self._keep = keepalive

    @property
    def handle(self):
        return self._h

    def view(self) -> sn_mesh_view:
        v = sn_mesh_view()
        _check(_lib.sn_mesh_view_get(self._h, ctypes.byref(v)))
        return v

    @property
    def n_points(self):
        return int(self.view().n_points)

    @property
    def n_quads(self):
        return int(self.view().n_quads)

    @property
    def n_stencil(self):
        return int(self.view().n_stencil)

    def to_host(self) -> HostMesh:
        v = self.view()
        P, n, prim, b = int(v.n_points), int(v.n_polys), int(v.prim), int(v.dtype)
        pts = np.empty((P, 3), np.float32)
        off = np.empty((P, 3), np.float32)
        polys = np.empty((n, prim), np.int32)
        lab = np.empty((n, 2), _NP_DT[b])
        so = np.empty(P + 1, np.int32)
        si = np.empty(int(v.n_stencil), np.int32)
        p = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
        _check(_lib.sn_mesh_copy_to_host(self._h, p(pts), p(polys), p(lab), p(so), p(si), p(off)))
        return HostMesh(pts, off, polys, lab, so, si)

    def free(self):
        if self._h and self._h.value:
            if _lib is not None:
                _lib.sn_mesh_free(self._h)
            self._h = ctypes.c_void_p(0)
        self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def to_device(a: np.ndarray, device="cuda"):
    """Copy a host label volume (uint8/16/32) to the GPU, bit-exact (int views)."""
    import torch

    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint8): np.uint8, np.dtype(np.uint16): np.int16,
            np.dtype(np.uint32): np.int32}[a.dtype]
    return torch.from_numpy(a.view(view)).to(device)


def make_volume(labels, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), selected=(),
                background=0, prim=SN_QUADS):
    """Build an sn_volume for a CUDA tensor of shape (O, N, M), or for an image
    of shape (N, M) (2D contours: SN_LINES, dims (M, N, 1)); returns (vol, keepalive)."""
    import torch

    if not isinstance(labels, torch.Tensor) or not labels.is_cuda:
        raise TypeError("labels must be a CUDA (HIP) torch tensor")
    if labels.dim() not in (2, 3) or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous 3-D tensor (O, N, M) or image (N, M)")
    if labels.dim() == 2:
        if prim not in (SN_QUADS, SN_LINES):
            raise ValueError("an image is contoured with segments (SN_LINES)")
        prim = SN_LINES
    b = labels.element_size()
    if b not in (1, 2, 4) or labels.is_floating_point():
        raise TypeError("labels must hold 8-, 16- or 32-bit integers")
    O, N, M = (1, *labels.shape) if labels.dim() == 2 else labels.shape
    v = sn_volume()
    v.labels = labels.data_ptr()
    v.dtype = b
    v.dims[:] = (M, N, O)
    sx, sy, sz = spacing
    v.spacing[0], v.spacing[1], v.spacing[2] = float(sx), float(sy), float(sz)
    ox, oy, oz = origin
    v.origin[0], v.origin[1], v.origin[2] = float(ox), float(oy), float(oz)
    sel = None
    if len(selected):
        sel = np.ascontiguousarray(np.asarray(list(selected), dtype=np.uint32))
        v.selected = sel.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        v.n_selected = int(sel.size)
    v.background = int(background)
    v.prim = int(prim)
    return v, (labels, sel)


def _np_layout(cls, formats):
    """A numpy record type laid out as the ctypes structure `cls`."""
    names = [n for n, _ in cls._fields_]
    return np.dtype({"names": names, "formats": formats,
                     "offsets": [getattr(cls, n).offset for n in names],
                     "itemsize": ctypes.sizeof(cls)})


_VOL_NP = _np_layout(sn_volume, [np.uint64, np.int32, (np.int64, 3), (np.float64, 3),
                                 (np.float64, 3), np.uint64, np.int32, np.uint32, np.int32])
_PAR_NP = _np_layout(sn_smooth_params, [np.int32, np.float32, np.float32, np.int32])
_VOLUME_KEYS = frozenset(("labels", "spacing", "origin", "selected", "background", "prim"))


def volume_array(volumes):
    """sn_volume[n] for dicts of make_volume's keyword arguments, as one numpy
    record array (the same checks and values as make_volume, without a ctypes
    structure per volume); returns (array, keepalive)."""
    import torch

    n = len(volumes)
    a = np.zeros(n, _VOL_NP)
    ptr, size, dims, prim = [0] * n, [0] * n, [None] * n, [SN_QUADS] * n
    keep = []
    a["spacing"] = 1.0
    for k, d in enumerate(volumes):
        if not _VOLUME_KEYS.issuperset(d):
            raise TypeError(f"unknown volume fields {sorted(set(d) - _VOLUME_KEYS)}")
        labels = d["labels"]
        if not isinstance(labels, torch.Tensor) or not labels.is_cuda:
            raise TypeError("labels must be a CUDA (HIP) torch tensor")
        nd = labels.dim()
        if nd not in (2, 3) or not labels.is_contiguous():
            raise ValueError("labels must be a contiguous 3-D tensor (O, N, M) or image (N, M)")
        pk = int(d.get("prim", SN_QUADS))
        if nd == 2:
            if pk not in (SN_QUADS, SN_LINES):
                raise ValueError("an image is contoured with segments (SN_LINES)")
            pk = SN_LINES
        b = labels.element_size()
        if b not in (1, 2, 4) or labels.is_floating_point():
            raise TypeError("labels must hold 8-, 16- or 32-bit integers")
        O, N, M = (1, *labels.shape) if nd == 2 else labels.shape
        ptr[k], size[k], dims[k], prim[k] = labels.data_ptr(), b, (M, N, O), pk
        sel = None
        if "spacing" in d:
            a["spacing"][k] = [float(x) for x in d["spacing"]]
        if "origin" in d:
            a["origin"][k] = [float(x) for x in d["origin"]]
        if len(d.get("selected", ())):
            sel = np.ascontiguousarray(np.asarray(list(d["selected"]), dtype=np.uint32))
            a["selected"][k] = sel.ctypes.data
            a["n_selected"][k] = sel.size
        if "background" in d:
            a["background"][k] = int(d["background"])
        keep.append((labels, sel))
    if n:
        a["labels"], a["dtype"], a["dims"], a["prim"] = ptr, size, dims, prim
    return a, keep


def params_array(params):
    """sn_smooth_params[n] for (iterations, relaxation, constraint[, shape])
    tuples, as one numpy record array."""
    n = len(params)
    a = np.zeros(n, _PAR_NP)
    it, lam, d, sh = [0] * n, [0.0] * n, [0.0] * n, [0] * n
    for k, p in enumerate(params):
        it[k], lam[k], d[k] = int(p[0]), float(p[1]), float(p[2])
        if len(p) > 3:
            sh[k] = SHAPES[p[3]] if isinstance(p[3], str) else int(p[3])
    if n:
        a["iterations"], a["relaxation"], a["constraint"], a["shape"] = it, lam, d, sh
    return a


# constraint regions of the smoothing (sn_constraint_shape)
SHAPES = {"box": 0, "sphere": 1}


def smooth_params(iterations, relaxation, constraint, shape="box") -> sn_smooth_params:
    p = sn_smooth_params()
    p.iterations, p.relaxation, p.constraint = int(iterations), float(relaxation), float(constraint)
    p.shape = SHAPES[shape] if isinstance(shape, str) else int(shape)
    return p


class Context:
    def __init__(self, device: int = 0):
        load_library()
        h = ctypes.c_void_p()
        _check(_lib.sn_ctx_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        if self._h and self._h.value:
            _lib.sn_ctx_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def extract(self, labels, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), selected=(),
                background=0, prim=SN_QUADS, stream=None) -> Mesh:
        v, keep = make_volume(labels, spacing, origin, selected, background, prim)
        out = ctypes.c_void_p()
        _check(_lib.sn_extract(self._h, ctypes.byref(v), _stream_handle(stream), ctypes.byref(out)))
        return Mesh(out.value, keep)

    def smooth(self, mesh: Mesh, iterations=25, relaxation=0.5, constraint=1.0, shape="box",
               stream=None):
        p = smooth_params(iterations, relaxation, constraint, shape)
        _check(_lib.sn_smooth(self._h, mesh.handle, ctypes.byref(p), _stream_handle(stream)))

    def triangulate(self, mesh: Mesh, rule="fixed", labels=True, stream=None):
        """Triangles of the mesh's quads under a diagonal rule ("fixed",
        "shortest", "min_area", "planar"), from its current world points:
        device tensors (tris [2Q, 3] int32, labels [2Q, 2] or None)."""
        import torch

        r = DIAG_RULES[rule] if isinstance(rule, str) else int(rule)
        v = mesh.view()
        nq, b = int(v.n_quads), int(v.dtype)
        tris = torch.empty((2 * nq, 3), dtype=torch.int32, device="cuda")
        lab = None
        if labels:
            lab = torch.empty((2 * nq, 2), dtype={1: torch.uint8, 2: torch.int16, 4: torch.int32}[b],
                              device="cuda")
        _check(_lib.sn_triangulate(self._h, mesh.handle, r, ctypes.c_void_p(tris.data_ptr()),
                                   ctypes.c_void_p(lab.data_ptr()) if lab is not None else None,
                                   _stream_handle(stream)))
        return tris, lab

    def extract_noalloc(self, labels, points, polys, label_pairs, stencil_off, stencil_ids,
                        spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0), selected=(),
                        background=0, prim=SN_QUADS, stream=None) -> tuple:
        """sn_extract_noalloc into caller-owned device tensors: points [cp, 3]
        float32, polys [cq, prim] int32, label_pairs [cq, 2] of the label type,
        stencil_off [cp + 1] int32, stencil_ids [cs] int32 (capacities from the
        shapes).  Returns (points, polys, stencil entries); raises SNError
        (status SN_ENOMEM with .counts when the arrays are too small)."""
        v, keep = make_volume(labels, spacing, origin, selected, background, prim)
        a = sn_extract_arrays()
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
        a.points, a.polys, a.label_pairs = ptr(points), ptr(polys), ptr(label_pairs)
        a.stencil_off, a.stencil_ids = ptr(stencil_off), ptr(stencil_ids)
        a.cap_points = points.shape[0] if points is not None else 0
        a.cap_polys = polys.shape[0] if polys is not None else 0
        a.cap_stencil = stencil_ids.shape[0] if stencil_ids is not None else 0
        if stencil_off is None or stencil_off.shape[0] < a.cap_points + 1:
            raise ValueError("stencil_off needs cap_points + 1 entries")
        counts = (ctypes.c_int64 * 3)()
        st = _lib.sn_extract_noalloc(self._h, ctypes.byref(v), _stream_handle(stream),
                                     ctypes.byref(a), counts)
        if st != SN_OK:
            err = SNError(st, _lib.sn_last_error().decode(errors="replace"))
            err.counts = tuple(int(x) for x in counts)
            raise err
        return tuple(int(x) for x in counts)

    def batch_submit(self, volumes: Sequence[dict], params: Optional[Sequence] = None,
                     stream=None) -> list:
        """volumes: dicts of make_volume keyword arguments; params: (iters, relax, constr[,
        shape])."""
        n = len(volumes)
        arr, keep = volume_array(volumes)
        parr = None
        if params is not None:
            if len(params) != n:
                raise ValueError("one smoothing parameter tuple per volume")
            pa = params_array(params)
            parr = pa.ctypes.data_as(ctypes.POINTER(sn_smooth_params))
        outs = (ctypes.c_void_p * n)()
        _check(_lib.sn_batch_submit(self._h, arr.ctypes.data_as(ctypes.POINTER(sn_volume)), parr, n,
                                    _stream_handle(stream), outs))
        return [Mesh(outs[k], keep[k]) for k in range(n)]

    def autotune(self, labels, spacing=(1.0, 1.0, 1.0), selected=(), background=0,
                 stream=None) -> int:
        v, keep = make_volume(labels, spacing, (0, 0, 0), selected, background)
        ch = ctypes.c_int32()
        _check(_lib.sn_autotune(self._h, ctypes.byref(v), _stream_handle(stream), ctypes.byref(ch)))
        return int(ch.value)

    def memory(self) -> tuple:
        """(bytes handed out by the context's device pool now, most at once)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.sn_ctx_memory(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def set_batches_per_wave(self, bpw: int):
        _check(_lib.sn_set_batches_per_wave(self._h, int(bpw)))

    def schedule_get(self, labels, prim=SN_QUADS) -> dict:
        """The kernel schedule used for volumes of this one's size class."""
        v, keep = make_volume(labels, prim=prim)
        sc = sn_schedule()
        _check(_lib.sn_schedule_get(self._h, ctypes.byref(v), ctypes.byref(sc)))
        return {f: int(getattr(sc, f)) for f, _ in sn_schedule._fields_}

    def schedule_set(self, labels, prim=SN_QUADS, **fields):
        """Set the kernel schedule of this volume's size class (the fields of
        sn_schedule; those not given keep their current values)."""
        cur = self.schedule_get(labels, prim)
        cur.update({k: int(x) for k, x in fields.items()})
        v, keep = make_volume(labels, prim=prim)
        sc = sn_schedule(**cur)
        _check(_lib.sn_schedule_set(self._h, ctypes.byref(v), ctypes.byref(sc)))

    def profile(self, on=True):
        """on: False/0 off, True/1 events per launch (a smoothing call's sweeps as a
        whole), 2 events per sweep, 3 the sweeps only (as with 1)."""
        _check(_lib.sn_profile_enable(self._h, int(on)))

    def profile_reset(self):
        _check(_lib.sn_profile_reset(self._h))

    def profile_read(self) -> dict:
        cap = 64
        arr = (sn_kernel_stat * cap)()
        n = ctypes.c_int32()
        _check(_lib.sn_profile_read(self._h, arr, cap, ctypes.byref(n)))
        return {arr[k].name.decode(): (int(arr[k].launches), float(arr[k].total_ms))
                for k in range(min(n.value, cap))}

    def serve_start(self, hbm_budget_bytes=8 << 30, max_inflight=64, n_streams=2, max_batch=16,
                    queue_capacity=4096) -> "Server":
        cfg = sn_serve_config()
        cfg.hbm_budget_bytes, cfg.max_inflight, cfg.n_streams = hbm_budget_bytes, max_inflight, n_streams
        cfg.max_batch, cfg.queue_capacity = max_batch, queue_capacity
        h = ctypes.c_void_p()
        _check(_lib.sn_serve_start(self._h, ctypes.byref(cfg), ctypes.byref(h)))
        return Server(h, self)


class Server:
    def __init__(self, handle, ctx):
        self._h = handle
        self._ctx = ctx
        self._keep = {}

    def submit(self, labels, iterations=20, relaxation=0.5, constraint=1.0, shape="box",
               stream=None, **vol_kw) -> int:
        """Queue a request; the labels are read after the work enqueued so far on
        `stream` (default: torch's current stream)."""
        v, keep = make_volume(labels, **vol_kw)
        p = smooth_params(iterations, relaxation, constraint, shape)
        t = ctypes.c_uint64()
        _check(_lib.sn_serve_submit(self._h, ctypes.byref(v), ctypes.byref(p),
                                    _stream_handle(stream), ctypes.byref(t)))
        self._keep[int(t.value)] = keep
        return int(t.value)

    def poll(self, ticket: int) -> Optional[Mesh]:
        out = ctypes.c_void_p()
        st = _lib.sn_serve_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(out))
        if st == SN_EAGAIN:
            return None
        keep = self._keep.pop(ticket, None)
        _check(st)
        return Mesh(out.value, keep)

    def wait(self, ticket: int, timeout_us: int = -1) -> Mesh:
        out = ctypes.c_void_p()
        st = _lib.sn_serve_wait(self._h, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(out))
        if st == SN_ETIMEDOUT:
            _check(st)
        keep = self._keep.pop(ticket, None)
        _check(st)
        return Mesh(out.value, keep)

    def stats(self) -> dict:
        s = sn_serve_stats()
        _check(_lib.sn_serve_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def stop(self):
        if self._h and self._h.value:
            _check(_lib.sn_serve_stop(self._h))
            self._h = ctypes.c_void_p(0)
            self._keep.clear()
