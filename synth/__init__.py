"""Seeded synthetic label maps shaped like the paper's evaluation volumes.

The paper evaluates on a random-sphere volume, two anatomical atlases and an
electron-microscopy connectome (Section 4.1, "Methods").  None of those data
are available, so every input here is drawn from a seeded generator that keeps
the shapes, label counts and structure of the workloads:

* ``spheres_small``   - 64^3 uint16, three overlapping balls (the random-sphere
                        volume of Section 4.1, scaled down).
* ``torso_like``      - 256^3 uint16, spacing (1, 1, 2.5): 100 Voronoi cells
                        clipped to an ellipsoidal body, background outside
                        (stands in for the segmented CT torso).
* ``connectome_like`` - 1024x1024x512 uint32, 50,000 needle-shaped cells
                        (Voronoi cells stretched 8x along a random direction per
                        seed) separated by a 2 % membrane of label 0 (stands in
                        for the segmented connectome).
* ``batch_volumes``   - 64 uneven volumes (edges 48..320) of spheres or Voronoi.
* ``serve_pool``      - volumes 32^3..512^3 (log-uniform) in uint8/16/32.

This module holds no SurfaceNets arithmetic; it only writes label volumes.
Random parameters come from ``numpy.random.default_rng(seed)`` and the heavy
rasterisation runs in ``libsynth.so`` (plain C, OpenMP), a deterministic
function of those parameters.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

_DT = {1: np.uint8, 2: np.uint16, 4: np.uint32}


def build() -> str:
    """Compile libsynth.so (gcc, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "synth.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        U32 = ctypes.c_uint32
        D = ctypes.c_double
        lib.synth_fill.argtypes = [P, ctypes.c_int, I64, I64, I64, U32]
        lib.synth_spheres.argtypes = [P, ctypes.c_int, I64, I64, I64, I32, P, P, P, U32]
        lib.synth_voronoi.argtypes = [P, ctypes.c_int, I64, I64, I64, P, I32, P, P, P, U32]
        lib.synth_stretched.argtypes = [P, ctypes.c_int, I64, I64, I64, I32, P, P, P, D, D, D,
                                        U32, P, I64]
        lib.synth_remap_lut.argtypes = [P, ctypes.c_int, I64, P]
        for f in (lib.synth_fill, lib.synth_spheres, lib.synth_voronoi, lib.synth_stretched,
                  lib.synth_remap_lut):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _empty(dims, b):
    M, N, O = dims
    return np.empty((O, N, M), dtype=_DT[b])


@dataclass
class Volume:
    """A label volume plus the extraction/smoothing parameters of its workload."""

    labels: np.ndarray  # shape (O, N, M), x fastest
    spacing: tuple = (1.0, 1.0, 1.0)
    origin: tuple = (0.0, 0.0, 0.0)
    selected: tuple = ()  # empty: every non-background value
    background: int = 0
    iterations: int = 16
    relaxation: float = 0.5
    constraint: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def dims(self):
        if self.labels.ndim == 2:  # an image (N, M)
            N, M = self.labels.shape
            return (M, N, 1)
        O, N, M = self.labels.shape
        return (M, N, O)

    @property
    def nbytes(self):
        return int(self.labels.nbytes)


def spheres(dims, b, centres, radii, labels, background=0) -> np.ndarray:
    lib = _load()
    out = _empty(dims, b)
    c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    lab = np.ascontiguousarray(labels, dtype=np.uint32).reshape(-1)
    lib.synth_spheres(_ptr(out), b, dims[0], dims[1], dims[2], len(r), _ptr(c), _ptr(r),
                      _ptr(lab), background)
    return out


def voronoi(dims, b, spacing, seeds_world, labels, ellipsoid=None, background=0) -> np.ndarray:
    lib = _load()
    out = _empty(dims, b)
    s = np.ascontiguousarray(seeds_world, dtype=np.float64).reshape(-1, 3)
    lab = np.ascontiguousarray(labels, dtype=np.uint32).reshape(-1)
    h = np.ascontiguousarray(spacing, dtype=np.float64)
    ell = None if ellipsoid is None else np.ascontiguousarray(ellipsoid, dtype=np.float64)
    lib.synth_voronoi(_ptr(out), b, dims[0], dims[1], dims[2], _ptr(h), len(lab), _ptr(s),
                      _ptr(lab), None if ell is None else _ptr(ell), background)
    return out


def stretched(dims, b, seeds, dirs, labels, alpha, radius, membrane_frac, background=0,
              sample_stride=101) -> np.ndarray:
    lib = _load()
    M, N, O = dims
    s = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    u = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    lab = np.ascontiguousarray(labels, dtype=np.uint32).reshape(-1)
    tau = 0.0
    if membrane_frac > 0:
        V = M * N * O
        gaps = np.empty((V + sample_stride - 1) // sample_stride, dtype=np.float64)
        lib.synth_stretched(None, b, M, N, O, len(lab), _ptr(s), _ptr(u), _ptr(lab), alpha, radius,
                            0.0, background, _ptr(gaps), sample_stride)
        tau = float(np.quantile(gaps[np.isfinite(gaps)], membrane_frac))
    out = _empty(dims, b)
    lib.synth_stretched(_ptr(out), b, M, N, O, len(lab), _ptr(s), _ptr(u), _ptr(lab), alpha,
                        radius, tau, background, None, 1)
    return out


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def spheres_small(seed: int = 1) -> Volume:
    """64^3 uint16; labels 1, 2, 3 as balls with centre ~ U[16,48]^3 and
    radius ~ U[10,20]; a later label overwrites an earlier one; background 0.
    Quads, all labels, 16 iterations, relaxation 0.5, constraint 1.0."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(16, 48, size=(3, 3))
    r = rng.uniform(10, 20, size=3)
    lab = spheres((64, 64, 64), 2, c, r, [1, 2, 3])
    return Volume(lab, iterations=16, relaxation=0.5, constraint=1.0, name="spheres_small_64^3_u16",
                  meta={"seed": seed})


def synthetic_spheres(seed: int = 6, n: int = 512, count: int = 128) -> Volume:
    """n^3 uint16 with `count` overlapping balls labelled 1..count (a later
    label overwrites an earlier one), background 0: the shape of the paper's
    Synthetic dataset (512^3, 128 spheres, 129 labels with the background).
    Radii ~ U[n/32, n/8], centres uniform inside the volume.  25 iterations,
    relaxation 0.5, constraint 1.0."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(n / 32, n / 8, size=count)
    c = rng.uniform(0, n, size=(count, 3))
    lab = spheres((n, n, n), 2, c, r, np.arange(1, count + 1))
    return Volume(lab, iterations=25, relaxation=0.5, constraint=1.0,
                  name=f"synthetic_spheres_{n}^3_u16_{count}", meta={"seed": seed})


def torso_like(seed: int = 2, n: int = 256) -> Volume:
    """n^3 uint16, spacing (1, 1, 2.5); 100 Voronoi cells (seeds uniform over
    the world box, label = nearest seed + 1, ties to the lower index) clipped
    to an index-space ellipsoid with semi-axes (0.45, 0.35, 0.48) * n centred
    in the volume; 0 outside.  Quads, 25 iterations, relaxation 0.5,
    constraint 1.0."""
    rng = np.random.default_rng(seed)
    h = (1.0, 1.0, 2.5)
    ext = np.array([(n - 1) * h[0], (n - 1) * h[1], (n - 1) * h[2]])
    seeds = rng.uniform(0, 1, size=(100, 3)) * ext
    c = (n - 1) / 2.0
    ell = [c, c, c, 0.45 * n, 0.35 * n, 0.48 * n]
    lab = voronoi((n, n, n), 2, h, seeds, np.arange(1, 101), ellipsoid=ell)
    return Volume(lab, spacing=h, iterations=25, relaxation=0.5, constraint=1.0,
                  name=f"torso_like_{n}^3_u16", meta={"seed": seed})


def connectome_like(seed: int = 3, dims=(1024, 1024, 512), n_cells: int = 50_000,
                    alpha: float = 8.0, radius: float = 32.0, membrane: float = 0.02) -> Volume:
    """uint32; n_cells seeds uniform in the box, each with a random unit
    direction; cell = argmin of |x-s|^2 - (1 - 1/alpha^2)((x-s).u)^2 among
    seeds within `radius` voxels (label = seed index + 1); the `membrane`
    fraction of voxels with the smallest gap between the two best distances
    becomes 0.  Quads, 20 iterations, relaxation 0.5, constraint 0.8."""
    rng = np.random.default_rng(seed)
    M, N, O = dims
    seeds = rng.uniform(0, 1, size=(n_cells, 3)) * np.array([M - 1, N - 1, O - 1])
    d = rng.normal(size=(n_cells, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lab = stretched(dims, 4, seeds, d, np.arange(1, n_cells + 1), alpha, radius, membrane)
    return Volume(lab, iterations=20, relaxation=0.5, constraint=0.8,
                  name=f"connectome_like_{M}x{N}x{O}_u32", meta={"seed": seed})


def section_like(seed: int = 7, n: int = 8192, n_cells: int = 40_000, alpha: float = 4.0,
                 radius: float = 64.0, membrane: float = 0.02) -> Volume:
    """An n x n uint32 image shaped like one section of the connectome-like
    volume (the 2D method, SN_LINES): n_cells seeds uniform in the plane, each
    with a random in-plane direction, cells stretched alpha-fold along it,
    and the `membrane` fraction of pixels with the smallest gap between the two
    best distances set to 0.  20 iterations, relaxation 0.5, constraint 0.8."""
    rng = np.random.default_rng(seed)
    seeds = np.zeros((n_cells, 3))
    seeds[:, :2] = rng.uniform(0, 1, size=(n_cells, 2)) * (n - 1)
    d = np.zeros((n_cells, 3))
    ang = rng.uniform(0, 2 * np.pi, size=n_cells)
    d[:, 0], d[:, 1] = np.cos(ang), np.sin(ang)
    lab = stretched((n, n, 1), 4, seeds, d, np.arange(1, n_cells + 1), alpha, radius, membrane)
    return Volume(lab.reshape(n, n), iterations=20, relaxation=0.5, constraint=0.8,
                  name=f"section_like_{n}^2_u32", meta={"seed": seed})


def mixed_volume(rng: np.random.Generator, dims, b: int, n_labels: int) -> np.ndarray:
    """Either Voronoi cells (no mask) or overlapping balls, chosen by a coin flip."""
    M, N, O = dims
    if rng.uniform() < 0.5:
        seeds = rng.uniform(0, 1, size=(n_labels, 3)) * np.array([M - 1, N - 1, O - 1])
        return voronoi(dims, b, (1.0, 1.0, 1.0), seeds, np.arange(1, n_labels + 1))
    m = float(min(dims))
    c = rng.uniform(0.15, 0.85, size=(n_labels, 3)) * np.array([M, N, O])
    r = rng.uniform(0.08, 0.3, size=n_labels) * m
    return spheres(dims, b, c, r, np.arange(1, n_labels + 1))


def batch_volumes(seed: int = 4, count: int = 64, lo: int = 48, hi: int = 320) -> list:
    """`count` uint16 volumes, each axis ~ U{lo..hi}, 5..80 labels of Voronoi
    or balls, iterations ~ U{15..40}, relaxation 0.5, constraint 1.0."""
    out = []
    for v in range(count):
        rng = np.random.default_rng(seed * 100_003 + v)
        dims = tuple(int(x) for x in rng.integers(lo, hi + 1, size=3))
        nl = int(rng.integers(5, 81))
        lab = mixed_volume(rng, dims, 2, nl)
        out.append(Volume(lab, iterations=int(rng.integers(15, 41)), relaxation=0.5,
                          constraint=1.0, name=f"batch{v}", meta={"seed": seed, "index": v}))
    return out


def serve_pool(seed: int = 5, count: int = 24, lo: int = 32, hi: int = 512) -> list:
    """`count` distinct volumes: cubic edge round(lo * (hi/lo)^U), dtype
    uniform over {u8, u16, u32}, Voronoi or balls with up to 80 labels
    (u8 keeps labels below 256)."""
    out = []
    for v in range(count):
        rng = np.random.default_rng(seed * 100_003 + v)
        L = int(round(lo * (hi / lo) ** rng.uniform()))
        b = int(rng.choice([1, 2, 4]))
        nl = int(rng.integers(5, 81))
        lab = mixed_volume(rng, (L, L, L), b, nl)
        out.append(Volume(lab, name=f"pool{v}", meta={"seed": seed, "index": v, "edge": L}))
    return out


def random_tiny(rng: np.random.Generator, dims, n_values: int, dtype=np.uint16) -> np.ndarray:
    """Uniform i.i.d. labels in [0, n_values) - the harshest case for topology."""
    M, N, O = dims
    return rng.integers(0, n_values, size=(O, N, M)).astype(dtype)


def blocky_tiny(rng: np.random.Generator, dims, n_values: int, dtype=np.uint16) -> np.ndarray:
    """Random labels on a 2x-coarsened grid (larger regions, flatter sheets)."""
    M, N, O = dims
    coarse = rng.integers(0, n_values, size=((O + 1) // 2, (N + 1) // 2, (M + 1) // 2))
    v = coarse.repeat(2, 0).repeat(2, 1).repeat(2, 2)[:O, :N, :M]
    return np.ascontiguousarray(v.astype(dtype))
