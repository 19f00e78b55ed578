"""Planted mistakes in the oracle must fail its pins.

Each mutant below is one plausible slip in ``oracle/sn_oracle.c``: a dropped
term, a wrong sign or index, a transposed operand, a swapped order.  The test
builds every mutant into a temporary library and runs the oracle's pin tests
(``test_oracle_pins.py``, ``test_oracle_pins2d.py``, ``test_oracle_diagonals.py``) against it through
``SN_ORACLE_LIB``; each mutant must make at least one pin fail.  A mutant that
passes every pin would be a mistake the pins cannot see.  Mistakes are planted
only in temporary copies of the oracle, on the CPU.

Some slips change nothing and are left out, because they are equivalent by
the mathematics, not missed by the pins.  A cell has a point iff its eight
corners are not all equal, so dropping any edges that still connect the
eight corners (one edge, or two of one axis) gives the same point set.  The
four edges of a face form a cycle, which never holds exactly one cut, so
dropping one face edge gives the same stencil.  Negating one component of
the cross product is a reflection, which keeps every area and every
angle between normals.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sn_oracle.c")
PINS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
        os.path.join(ROOT, "tests", "test_oracle_pins2d.py"),
        os.path.join(ROOT, "tests", "test_oracle_diagonals.py")]

# (name, original text, mutated text); the original occurs exactly once
MUTANTS = [
    # classification (Sec. 2.1)
    ("selection inverted",
     "cmp_u32) ? v : bg;", "cmp_u32) ? bg : v;"),
    ("selection ignored",
     "cmp_u32) ? v : bg;", "cmp_u32) ? v : v;"),
    ("unselected values become 0, not the background",
     "cmp_u32) ? v : bg;", "cmp_u32) ? v : 0u;"),
    ("empty selection selects nothing",
     "    if (n_sel == 0)\n        return v;", "    if (n_sel == 0)\n        return bg;"),
    # cut edges and points (Sec. 2.2)
    ("cut means equal",
     "return C(v, i, j, k) != C(v, i1, j1, k1);", "return C(v, i, j, k) == C(v, i1, j1, k1);"),
    ("point test ignores the x-edges",
     "if (cut(v, i, j + p, k + q, 0)) return 1; /* x-edges */", "/* x-edges dropped */"),
    ("point test looks one row too far in y",
     "if (cut(v, i + p, j, k + q, 1)) return 1;", "if (cut(v, i + p, j + 1, k + q, 1)) return 1;"),
    # stencil faces (Sec. 3.3)
    ("x-face checks only its y-edges",
     "cut(v, x, j, k + 1, 1) || cut(v, x, j, k, 2) ||\n               cut(v, x, j + 1, k, 2);",
     "cut(v, x, j, k + 1, 1);"),
    ("z-face checks only its y-edges",
     "return cut(v, i, j, z, 0) || cut(v, i, j + 1, z, 0) || cut(v, i, j, z, 1) ||",
     "return cut(v, i, j, z, 1) ||"),
    ("x-faces swapped",
     "int64_t x = i + plus;", "int64_t x = i + 1 - plus;"),
    ("stencil neighbour direction swapped",
     "int64_t d = (f % 2) ? 1 : -1;", "int64_t d = (f % 2) ? -1 : 1;"),
    ("stencil faces in reverse order",
     "for (int f = 0; f < 6; ++f) {\n            int64_t d", "for (int f = 5; f >= 0; --f) {\n            int64_t d"),
    # quads and label pairs (Sec. 2.2-2.3)
    ("stencil ignores the cut edges of a face",
     "if (!cell_exists(&v, ni, nj, nk) || !face_has_cut(&v, i, j, k, f))",
     "if (!cell_exists(&v, ni, nj, nk))"),
    ("2D stencil ignores the shared edge",
     "if (!cell2_exists(M, N, ni[f], nj[f]) || !shared[f])",
     "if (!cell2_exists(M, N, ni[f], nj[f]))"),
    ("x-quad winding reversed",
     "{{i, j - 1, k - 1}, {i, j - 1, k}, {i, j, k}, {i, j, k - 1}}",
     "{{i, j - 1, k - 1}, {i, j, k - 1}, {i, j, k}, {i, j - 1, k}}"),
    ("y-quad winding reversed",
     "{{i - 1, j, k - 1}, {i, j, k - 1}, {i, j, k}, {i - 1, j, k}}",
     "{{i - 1, j, k - 1}, {i - 1, j, k}, {i, j, k}, {i, j, k - 1}}"),
    ("x-quad starting at another corner",
     "{{i, j - 1, k - 1}, {i, j - 1, k}, {i, j, k}, {i, j, k - 1}}",
     "{{i, j - 1, k}, {i, j, k}, {i, j, k - 1}, {i, j - 1, k - 1}}"),
    ("z-quad winding reversed",
     "{{i - 1, j - 1, k}, {i - 1, j, k}, {i, j, k}, {i, j - 1, k}}",
     "{{i - 1, j - 1, k}, {i, j - 1, k}, {i, j, k}, {i - 1, j, k}}"),
    ("back label on the wrong axis",
     "pr[2 * Q + 1] = C(&v, i + (a == 0), j + (a == 1), k + (a == 2));",
     "pr[2 * Q + 1] = C(&v, i + (a == 0), j + (a == 0), k + (a == 2));"),
    ("front and back swapped",
     "pr[2 * Q + 0] = C(&v, i, j, k);", "pr[2 * Q + 0] = C(&v, i + (a == 0), j + (a == 1), k + (a == 2));"),
    # cell centres (Sec. 2.2)
    ("centre with transposed row dims",
     "x[1] = (double)((c / CM) % CN) + 0.5;", "x[1] = (double)((c / CN) % CM) + 0.5;"),
    ("centre without the half-cell offset",
     "x[2] = (double)(c / (CM * CN)) + 0.5;", "x[2] = (double)(c / (CM * CN));"),
    # Eq. (1) and the constraint (Sec. 2.4)
    ("mean over n + 1",
     "lambda * (sum / (double)n);", "lambda * (sum / (double)(n + 1));"),
    ("difference sign flipped",
     "sum += a[3 * (int64_t)m->st_ids[e] + ax] - a[3 * p + ax];",
     "sum += a[3 * p + ax] - a[3 * (int64_t)m->st_ids[e] + ax];"),
    ("in-place (Gauss-Seidel) updates",
     "memcpy(b + 3 * p, q, sizeof q);", "memcpy(b + 3 * p, q, sizeof q);\n            memcpy(a + 3 * p, q, sizeof q);"),
    ("box clamp to the wrong side",
     "if (q[ax] < c[ax] - d) q[ax] = c[ax] - d;", "if (q[ax] < c[ax] - d) q[ax] = c[ax] + d;"),
    ("box around the moving point, not the centre",
     "if (q[ax] < c[ax] - d) q[ax] = c[ax] - d;",
     "if (q[ax] < a[3 * p + ax] - d) q[ax] = a[3 * p + ax] - d;"),
    ("sphere test on the squared length",
     "if (len > d) {",
     "if (len * len > d) {"),
    ("one sweep too few",
     "for (int32_t it = 0; it < iterations; ++it) {",
     "for (int32_t it = 1; it < iterations; ++it) {"),
    ("relaxation times the sum, not the mean",
     "q[ax] = a[3 * p + ax] + lambda * (sum / (double)n);",
     "q[ax] = a[3 * p + ax] + lambda * sum;"),
    ("sphere radius doubled",
     "if (len > d) {", "if (len > 2 * d) {"),
    ("sphere projection transposed",
     "q[1] = c[1] + dy * (d / len);", "q[1] = c[1] + dx * (d / len);"),
    # the method in the plane
    ("2D point test without its y-edges",
     "|| cut(&v, i, j, 0, 1) ||\n                           cut(&v, i + 1, j, 0, 1);", ";"),
    ("2D y-segment on the wrong side",
     "const int64_t ai = a == 0 ? i : i - 1,", "const int64_t ai = a == 0 ? i : i + 1,"),
    ("2D +y face checks the wrong edge",
     "cut(&v, i, j, 0, 0),\n                               cut(&v, i, j + 1, 0, 0)};",
     "cut(&v, i, j, 0, 0),\n                               cut(&v, i, j, 0, 0)};"),
    ("2D back label on the wrong axis",
     "pr[2 * Q + 1] = C(&v, i + (a == 0), j + (a == 1), 0);",
     "pr[2 * Q + 1] = C(&v, i + (a == 1), j + (a == 0), 0);"),
    ("2D segment ends swapped",
     "sg[2 * Q + 0] = (int32_t)pid[ai + CM * aj];\n                sg[2 * Q + 1] = (int32_t)pid[bi + CM * bj];",
     "sg[2 * Q + 0] = (int32_t)pid[bi + CM * bj];\n                sg[2 * Q + 1] = (int32_t)pid[ai + CM * aj];"),
    ("2D stencil faces in reverse order",
     "        for (int f = 0; f < 4; ++f) {\n            if (!cell2_exists(M, N, ni[f], nj[f]) || !shared[f])",
     "        for (int f = 3; f >= 0; --f) {\n            if (!cell2_exists(M, N, ni[f], nj[f]) || !shared[f])"),
    ("2D -x face checks the +x edge",
     "const int shared[4] = {cut(&v, i, j, 0, 1), cut(&v, i + 1, j, 0, 1),",
     "const int shared[4] = {cut(&v, i + 1, j, 0, 1), cut(&v, i + 1, j, 0, 1),"),
    # world coordinates and triangles (Sec. 2.5)
    ("world origin scaled",
     "out[3 * p + ax] = origin[ax] + spacing[ax] * idx_pos[3 * p + ax];",
     "out[3 * p + ax] = spacing[ax] * (origin[ax] + idx_pos[3 * p + ax]);"),
    ("second triangle wound backwards",
     "        t1[0] = v[0], t1[1] = v[2], t1[2] = v[3];\n        if (tri_pairs)",
     "        t1[0] = v[0], t1[1] = v[3], t1[2] = v[2];\n        if (tri_pairs)"),
    ("shortest diagonal picks the longer",
     "return vdot(ac, ac) <= vdot(bd, bd);", "return vdot(ac, ac) >= vdot(bd, bd);"),
    ("minimum area with a wrong triangle",
     "<= tri_area(a, b, d) + tri_area(b, c, d);", "<= tri_area(a, b, d) + tri_area(a, c, d);"),
    ("planarity with a flipped normal",
     "tri_normal(b, c, d, n4);", "tri_normal(b, d, c, n4);"),
    ("cross product with a wrong index",
     "r[1] = x[2] * y[0] - x[0] * y[2];", "r[1] = x[2] * y[0] - x[0] * y[1];"),
]


def _build(src: str, name: str, old: str, new: str, out_dir: str) -> str:
    assert src.count(old) == 1, f"mutant '{name}': its original text must occur exactly once"
    tag = re.sub(r"[^a-z0-9]+", "_", name.lower())
    c_path = os.path.join(out_dir, f"{tag}.c")
    so_path = os.path.join(out_dir, f"{tag}.so")
    with open(c_path, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", so_path,
                           c_path, "-lm"])
    return so_path


def _run_pins(so_path: str, work: str):
    env = dict(os.environ, SN_ORACLE_LIB=so_path)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "--hypothesis-seed=0", *PINS], cwd=work, env=env,
                       capture_output=True, text=True, timeout=600)
    failed = re.findall(r"FAILED \S+::(\S+)", r.stdout)
    return r.returncode, failed


def test_every_mutant_fails_a_pin(tmp_path):
    src = open(SRC).read()
    libs = [_build(src, name, old, new, str(tmp_path)) for name, old, new in MUTANTS]
    works = []
    for k in range(len(MUTANTS)):
        w = tmp_path / f"run{k}"
        w.mkdir()
        works.append(str(w))
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_run_pins, libs, works))
    report = [f"{name}: {'caught by ' + ', '.join(f) if rc != 0 else 'NOT CAUGHT'}"
              for (name, _, _), (rc, f) in zip(MUTANTS, results)]
    print("\n".join(report))
    survivors = [name for (name, _, _), (rc, _) in zip(MUTANTS, results) if rc == 0]
    assert not survivors, "mutants no pin rejects: " + "; ".join(survivors)
