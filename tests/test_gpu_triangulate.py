"""GPU checks of sn_triangulate (the final triangulation of Sec. 2.5 with a
choice of tessellating diagonal) against the oracle's rules.

Both sides decide in FP64 on FP32 world points: the GPU on its own, the
oracle on its FP64 points rounded to FP32.  Those differ within the smoothing
tolerance, so a quad may legitimately be split differently only where the two
splits' measures nearly tie.  Every quad must
be split into one of its two splits with the quad's orientation, label
pairs are the quad's repeated, and the fixed rule equals the split that
SN_TRIS makes at extraction, bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RULES = ("fixed", "shortest", "min_area", "planar")


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def sn(torch):
    import paper_2401_14906_amd as sn

    sn.load_library()
    return sn


@pytest.fixture(scope="module")
def ctx(sn):
    c = sn.Context(0)
    yield c
    c.close()


def announce(msg):
    print(f"[case] {msg}", flush=True)


def measures(quads, pts, rule):
    """(A-C, B-D) measures of every quad (numpy, FP64), for near-tie checks."""
    a, b, c, d = (pts[quads[:, k]] for k in range(4))
    if rule == "shortest":
        return np.sum((c - a) ** 2, 1), np.sum((d - b) ** 2, 1)
    n = lambda x, y, z: np.cross(y - x, z - x)  # noqa: E731
    if rule == "min_area":
        ar = lambda v: 0.5 * np.linalg.norm(v, axis=1)  # noqa: E731
        return ar(n(a, b, c)) + ar(n(a, c, d)), ar(n(a, b, d)) + ar(n(b, c, d))

    def cos(n1, n2):
        l = np.sqrt(np.sum(n1 * n1, 1) * np.sum(n2 * n2, 1))
        return np.where(l > 0, np.sum(n1 * n2, 1) / np.where(l > 0, l, 1), -2.0)
    # planar: larger is preferred; negate so that "smaller wins" like the others
    return -cos(n(a, b, c), n(a, c, d)), -cos(n(a, b, d), n(b, c, d))


def cases():
    rng = np.random.default_rng(31)
    sp = synth.spheres_small()
    yield "spheres 64^3 u16", sp.labels, (), 0, (1.0, 1.0, 1.0), (16, 0.5, 1.0)
    yield "blocky u8 spacing", synth.blocky_tiny(rng, (40, 30, 20), 6, np.uint8), (), 0, \
        (1.0, 1.0, 2.5), (12, 0.5, 1.0)
    yield "random u32 selection", synth.random_tiny(rng, (23, 19, 17), 5, np.uint32), (1, 3), 0, \
        (0.7, 1.3, 1.0), (7, 1.0, 0.6)


@pytest.mark.parametrize("rule", RULES)
def test_triangulate_matches_oracle(ctx, sn, torch, rule):
    import oracle

    r = sn.DIAG_RULES[rule]
    for name, lab, sel, bg, spacing, (it, lam, dd) in cases():
        announce(f"triangulate {rule}: {name}")
        t = sn.to_device(lab)
        m = ctx.extract(t, spacing=spacing, selected=sel, background=bg)
        ctx.smooth(m, iterations=it, relaxation=lam, constraint=dd)
        tris, tl = ctx.triangulate(m, rule)
        g = m.to_host()
        gt = tris.cpu().numpy()
        gl = tl.cpu().numpy().view(g.label_pairs.dtype)
        m.free()
        o = oracle.extract(lab, sel, bg)
        np.testing.assert_array_equal(g.polys, o.quads)
        # the oracle's own world points, rounded to the FP32 the kernel decides on
        w = oracle.world(o.smooth(it, lam, dd), (0.0, 0.0, 0.0), spacing)
        w = w.astype(np.float32).astype(np.float64)
        ot = oracle.triangulate_rule(o.quads, w, r)
        Q = o.quads.shape[0]
        assert gt.shape == (2 * Q, 3)
        # label pairs: each quad's pair, repeated
        np.testing.assert_array_equal(gl[0::2], g.label_pairs)
        np.testing.assert_array_equal(gl[1::2], g.label_pairs)
        q = o.quads
        ac = np.concatenate([q[:, [0, 1, 2]], q[:, [0, 2, 3]]], 1).reshape(-1, 3)
        bd = np.concatenate([q[:, [0, 1, 3]], q[:, [1, 2, 3]]], 1).reshape(-1, 3)
        g_ac = np.all((gt == ac).reshape(Q, 6), 1)
        g_bd = np.all((gt == bd).reshape(Q, 6), 1)
        assert np.all(g_ac | g_bd), "a quad was not split into one of its two splits"
        o_ac = np.all((ot == ac).reshape(Q, 6), 1)
        diff = np.flatnonzero(g_ac != o_ac)
        if rule == "fixed":
            assert diff.size == 0 and np.all(g_ac)
            continue
        if diff.size:
            mac, mbd = measures(q[diff], w, rule)
            tol = 1e-4 * (np.abs(mac) + np.abs(mbd)) + 1e-9
            assert np.all(np.abs(mac - mbd) <= tol), \
                f"{name}: {diff.size} quads split differently away from a tie"
        # symmetric configurations give exact ties that FP32 and FP64 points
        # break differently; they stay rare
        assert diff.size <= max(2, Q // 100), f"{name}: {diff.size} of {Q} quads differ"


def test_fixed_rule_equals_extraction_split(ctx, sn, torch):
    rng = np.random.default_rng(32)
    lab = synth.blocky_tiny(rng, (50, 40, 30), 7, np.uint16)
    t = sn.to_device(lab)
    announce("fixed rule vs SN_TRIS")
    mt = ctx.extract(t, prim=sn.SN_TRIS)
    ref = mt.to_host()
    mt.free()
    m = ctx.extract(t)
    ctx.smooth(m, iterations=9)
    tris, tl = ctx.triangulate(m, "fixed")
    np.testing.assert_array_equal(tris.cpu().numpy(), ref.polys)
    np.testing.assert_array_equal(tl.cpu().numpy().view(ref.label_pairs.dtype), ref.label_pairs)
    # no labels requested: triangles only
    tris2, none = ctx.triangulate(m, "planar", labels=False)
    assert none is None and tris2.shape == tris.shape
    m.free()


@pytest.mark.parametrize("rule", RULES)
def test_triangulate_on_gpu_points_exact(ctx, sn, torch, rule):
    """The oracle's rule run on the GPU's own FP32 world points (widened to
    FP64, as the kernel does) splits every quad exactly as the kernel does: no
    near-tie allowance.  Both evaluate the measures in FP64 in the order
    written, without contraction, so even exact ties (symmetric quads) break
    the same way.  The torso mesh adds 659 K quads with anisotropic spacing."""
    import oracle

    r = sn.DIAG_RULES[rule]
    tv = synth.torso_like()
    extra = [("torso 256^3 u16", tv.labels, (), 0, tv.spacing,
              (tv.iterations, tv.relaxation, tv.constraint))]
    for name, lab, sel, bg, spacing, (it, lam, dd) in list(cases()) + extra:
        announce(f"triangulate {rule} on GPU points: {name}")
        t = sn.to_device(lab)
        m = ctx.extract(t, spacing=spacing, selected=sel, background=bg)
        ctx.smooth(m, iterations=it, relaxation=lam, constraint=dd)
        tris, _ = ctx.triangulate(m, rule, labels=False)
        g = m.to_host()
        gt = tris.cpu().numpy()
        m.free()
        ot = oracle.triangulate_rule(g.polys, g.points.astype(np.float64), r)
        bad = np.flatnonzero(np.any((gt != ot).reshape(-1, 6), 1))
        assert bad.size == 0, f"{name}: {bad.size} of {g.polys.shape[0]} quads split differently " \
                              f"(first {bad[:5].tolist()})"
