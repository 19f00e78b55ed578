"""Benchmark: SurfaceNets extraction + constrained smoothing on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload connectome|torso|spheres|section]
    python bench.py --only batched|served    (that path alone, e.g. under a profiler)

A step is one pass of the whole hot path over one synthetic label volume that
is already resident in HBM: extraction (classification, counting, scan,
generation of points / quads / label pairs / stencil) followed by the
smoothing sweeps and the world-coordinate emit.  The default workload is the
largest single-GPU one, the connectomics-like 1024x1024x512 uint32 volume
(50 000 stretched Voronoi cells, 2 % membrane; 20 sweeps, relaxation 0.5,
constraint 0.8).

One JSON line is printed on stdout; progress goes to stderr.  `value` is
whole-step throughput in Gvoxels/s (voxels / wall time of a full step).
Kernel durations come from HIP events recorded by the library on the stream
each kernel runs on.  In the timed steps only the sweeps (the kernel with the
largest total time, which the roofline object uses) are bracketed; the
extraction kernels are timed with events around every launch in a second,
untimed run of the same number of steps.  Extra objects report the other
volumes (the torso-like atlas, the 64^3 spheres, the 2D method on a
section-like image), the batched path against sequential plain calls, the
served path against a plain FIFO loop, the triangulation rules, a label-count
sweep, and the oracle timed on the host: one core (`cpu_baseline`) and all
cores (`cpu_baseline_all_cores`), on a z-slab sample of the headline volume.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# algorithmic bytes: what the method itself must move.  Input labels, the
# output mesh and, per sweep, the offsets and the stencil.  Metadata of this
# design (cut-edge bit planes, point masks, word bases, the per-point face
# byte) is overhead and is not counted; `design_bytes` adds it back as the
# bytes each kernel reads or writes once in this implementation.
# --------------------------------------------------------------------------

def words_of(dims):
    M, N, O = dims
    # an image (O = 1) has one slice of cell rows
    R = max(N - 1, 0) * (1 if O == 1 else max(O - 1, 0))
    W = (max(M - 1, 0) + 63) // 64
    WS = (M + 63) // 64
    return R * W, 3 * N * O * WS * 8  # cell words, plane bytes


def bytes_extract(V, b, P, Q, S, qb=16):
    """Whole extraction: read the labels once; write points (12 B) and CSR
    offsets (4 B) per point, quads (qb = 16 B; an image's segments 8 B) and
    label pairs (2b B) per quad, 4 B per stencil id."""
    return V * b + 16 * P + 4 + Q * (qb + 2 * b) + 4 * S


def alg_bytes(dims, b, P, Q, S, n, qb=16):
    V = dims[0] * dims[1] * dims[2]
    words, planes = words_of(dims)
    out_gen = 16 * P + 4 + Q * (qb + 2 * b) + 4 * S
    return {
        # kernel: (algorithmic, design)
        "k_edges": (V * b, V * b + planes),
        "k_count": (0, planes + 20 * words),
        "k_generate": (out_gen, out_gen + P + planes + 20 * words + V * b),
        # per sweep: read own offset and CSR offset, stencil ids, write offset;
        # neighbour offsets are re-reads of the array being read (not counted)
        "k_jacobi": (P * (12 + 12 + 4) + 4 * S, P * (12 + 12 + 4 + 1) + 4 * S),
        # read the final offsets, write world points
        "k_emit": (24 * P, 24 * P),
    }


# --------------------------------------------------------------------------


def run_plain_steps(ctx, sn, torch, t, vol, steps):
    """`steps` full plain steps; returns (wall seconds, last mesh sizes)."""
    sizes = None
    for _ in range(steps):
        m = ctx.extract(t, spacing=vol.spacing)
        ctx.smooth(m, iterations=vol.iterations, relaxation=vol.relaxation,
                   constraint=vol.constraint)
        v = m.view()
        sizes = (int(v.n_points), int(v.n_quads), int(v.n_stencil))
        m.free()  # does not wait: the blocks are reused once this step's work is done
    return sizes


def measure_workload(ctx, sn, torch, vol, steps, warmup):
    t = sn.to_device(vol.labels)
    b = vol.labels.dtype.itemsize
    V = int(vol.labels.size)
    # the kernels' schedule is picked by the library's autotuner for this
    # size class (untimed, like the warm-up steps)
    bpw = ctx.autotune(t, spacing=vol.spacing)
    sched = ctx.schedule_get(t)
    log(f"[bench] {vol.name}: autotuned schedule {sched}; warmup {warmup}")
    run_plain_steps(ctx, sn, torch, t, vol, warmup)
    # timed steps: HIP events bracket the sweeps (the dominant kernel, whose
    # launch time the roofline uses) and nothing else
    ctx.profile(3)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, Q, S = run_plain_steps(ctx, sn, torch, t, vol, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = ctx.profile_read()
    # the same number of steps again, untimed, with events around every launch:
    # the per-kernel breakdown of the extraction
    ctx.profile(True)
    ctx.profile_reset()
    run_plain_steps(ctx, sn, torch, t, vol, steps)
    prof = ctx.profile_read()
    ctx.profile(False)
    prof.update(timed)
    n = vol.iterations
    per = {}
    for name, (launches, ms) in prof.items():
        per[name] = {"launches": launches, "avg_us": 1e3 * ms / max(launches, 1),
                     "total_ms": ms, "events": "timed steps" if name in timed else "profiled steps"}
    qb = 8 if vol.labels.ndim == 2 else 16  # an image's segments: two ids
    alg = alg_bytes(vol.dims, b, P, Q, S, n, qb)
    for name, d in per.items():
        if name in alg:
            a, dsg = alg[name]
            d["alg_bytes"] = a
            d["design_bytes"] = dsg
            d["achieved_GBs"] = a / (d["avg_us"] * 1e-6) / 1e9
            d["frac_hbm"] = d["achieved_GBs"] / HBM_PEAK_GBS
            d["design_GBs"] = dsg / (d["avg_us"] * 1e-6) / 1e9
    ext_ms = sum(per.get(k, {}).get("total_ms", 0.0)
                 for k in ("k_edges", "k_count", "k_generate")) / steps
    smo_ms = sum(per.get(k, {}).get("total_ms", 0.0) for k in ("k_jacobi", "k_emit")) / steps
    bx = bytes_extract(V, b, P, Q, S, qb)
    res = {
        "voxels": V, "points": P, "quads": Q, "stencil": S, "iterations": n,
        "batches_per_wave": bpw,
        "schedule": sched,
        "ms_per_step": 1e3 * wall / steps,
        "gvox_per_s": V * steps / wall / 1e9,
        "extract_kernel_ms": ext_ms,
        "smooth_kernel_ms": smo_ms,
        "extract_gvox_per_s": V / (ext_ms * 1e-3) / 1e9 if ext_ms > 0 else None,
        "smooth_gptit_per_s": P * n / (smo_ms * 1e-3) / 1e9 if smo_ms > 0 else None,
        "extract_alg_bytes": bx,
        "extract_alg_GBs": bx / (ext_ms * 1e-3) / 1e9 if ext_ms > 0 else None,
        "extract_frac_hbm": bx / (ext_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if ext_ms > 0 else None,
        "kernels": per,
    }
    del t
    return res


def roofline_of(res, traffic=None):
    per = res["kernels"]
    dom = max((k for k in per if per[k].get("alg_bytes")), key=lambda k: per[k]["total_ms"])
    d = per[dom]
    return {"kernel": dom, "bound": "hbm", "achieved": round(d["achieved_GBs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["frac_hbm"], 4),
            "traffic": traffic, "avg_us": round(d["avg_us"], 2),
            "alg_bytes_per_launch": int(d["alg_bytes"]),
            # counted L2-miss bytes per algorithmic byte: above 1 means re-reads
            "traffic_over_alg": round(traffic / d["alg_bytes"], 3) if traffic else None}


# bounded CPU samples: volumes above this many voxels are timed on a z-slab
# crop of the middle slices (whole x-y slices, so the crop has the volume's
# structure), sized to about CPU_SAMPLE_VOXELS
CPU_SAMPLE_VOXELS = 48 << 20


def cpu_sample(vol):
    """(labels, description) of the oracle's timing sample of `vol`."""
    lab = vol.labels
    if lab.ndim != 3 or lab.size <= CPU_SAMPLE_VOXELS:
        return lab, f"whole {vol.name} volume"
    O, N, M = lab.shape
    s = max(2, min(O, CPU_SAMPLE_VOXELS // (M * N) + 1))
    k0 = (O - s) // 2
    crop = np.ascontiguousarray(lab[k0:k0 + s])
    return crop, f"z-slab crop of {vol.name}: sample slices {k0}..{k0 + s - 1} ({M}x{N}x{s})"


def cpu_baseline(vol, min_seconds=10.0):
    """The oracle (serial C, FP64), timed on one host core (extract +
    smoothing) on a bounded sample of the volume, repeated until at least
    `min_seconds` have passed."""
    import oracle

    lab, what = cpu_sample(vol)
    V = int(lab.size)
    reps, t_all = 0, 0.0
    while t_all < min_seconds and reps < 50:
        t0 = time.perf_counter()
        m = oracle.extract(lab, vol.selected, vol.background)
        m.smooth(vol.iterations, vol.relaxation, vol.constraint)
        t_all += time.perf_counter() - t0
        reps += 1
        del m
    return {"value": round(V * reps / t_all / 1e9, 5), "unit": "Gvoxels/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{what} (extract + {vol.iterations} sweeps) x{reps}, "
                      f"{t_all:.1f} s on 1 core",
            "host": host_cpu()}


def cpu_baseline_all_cores(vol, min_seconds=5.0):
    """The oracle's loops spread over z-slices with OpenMP on every usable host
    core (bit-identical to the serial oracle), on the same sample."""
    import oracle

    lab, what = cpu_sample(vol)
    V = int(lab.size)
    threads = oracle.par_threads()
    reps, t_all, t_ext = 0, 0.0, 0.0
    while t_all < min_seconds and reps < 50:
        t0 = time.perf_counter()
        m = oracle.extract_par(lab, vol.selected, vol.background)
        t1 = time.perf_counter()
        m.smooth_par(vol.iterations, vol.relaxation, vol.constraint)
        t_all += time.perf_counter() - t0
        t_ext += t1 - t0
        reps += 1
        P = m.n_points
        del m
    return {"value": round(V * reps / t_all / 1e9, 5), "unit": "Gvoxels/s", "cores": threads,
            "kind": "oracle, OpenMP over z-slices",
            "extract_gvox_per_s": round(V * reps / t_ext / 1e9, 5),
            "smooth_gptit_per_s": round(P * vol.iterations * reps / (t_all - t_ext) / 1e9, 5)
            if t_all > t_ext else None,
            "sample": f"{what} (extract + {vol.iterations} sweeps) x{reps}, "
                      f"{t_all:.1f} s on {threads} threads",
            "host": host_cpu()}


def host_cpu():
    """The host's CPU model and CPU counts (the oracle's timing runs on one)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def mesh_alg_bytes(V, b, P, Q, S, n):
    """Algorithmic bytes of one volume's extraction and n smoothing sweeps
    (the extraction and per-sweep figures of alg_bytes())."""
    return bytes_extract(V, b, P, Q, S) + n * (P * (12 + 12 + 4) + 4 * S)


def bench_batched(ctx, sn, torch, count=64, reps=3):
    import synth

    log(f"[bench] batched: generating {count} volumes")
    vols = synth.batch_volumes(count=count)
    V = sum(int(v.labels.size) for v in vols)
    ts = [sn.to_device(v.labels) for v in vols]
    specs = [dict(labels=t) for t in ts]
    params = [(v.iterations, v.relaxation, v.constraint) for v in vols]

    def plain():
        for t, v in zip(ts, vols):
            m = ctx.extract(t)
            ctx.smooth(m, iterations=v.iterations, relaxation=v.relaxation, constraint=v.constraint)
            m.free()

    def batched():
        ms = ctx.batch_submit(specs, params)
        for m in ms:
            m.free()

    # mesh sizes (untimed) for the algorithmic bytes of the whole batch
    alg = 0
    for m, v in zip(ctx.batch_submit(specs, params), vols):
        mv = m.view()
        alg += mesh_alg_bytes(int(v.labels.size), v.labels.dtype.itemsize, int(mv.n_points),
                              int(mv.n_quads), int(mv.n_stencil), v.iterations)
        m.free()
    out = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        out[name] = best
        log(f"[bench] batched: {name} {best * 1e3:.1f} ms")
    return {"volumes": count, "voxels": V,
            "plain_ms": round(out["plain"] * 1e3, 2), "batched_ms": round(out["batched"] * 1e3, 2),
            "plain_gvox_per_s": round(V / out["plain"] / 1e9, 3),
            "batched_gvox_per_s": round(V / out["batched"] / 1e9, 3),
            "speedup": round(out["plain"] / out["batched"], 3),
            "alg_bytes": int(alg),
            "plain_alg_GBs": round(alg / out["plain"] / 1e9, 1),
            "batched_alg_GBs": round(alg / out["batched"] / 1e9, 1),
            "plain_frac_hbm": round(alg / out["plain"] / 1e9 / HBM_PEAK_GBS, 4),
            "batched_frac_hbm": round(alg / out["batched"] / 1e9 / HBM_PEAK_GBS, 4)}


def bench_served(ctx, sn, torch, n_requests=2000, pool=24, seed=5):
    import synth

    log(f"[bench] served: generating a pool of {pool} volumes")
    vols = synth.serve_pool(seed=seed, count=pool)
    ts = [sn.to_device(v.labels) for v in vols]
    # labels present in each volume (the generator uses small label values)
    present = [np.flatnonzero(np.bincount(v.labels.ravel())) for v in vols]
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_requests):
        k = int(rng.integers(0, pool))
        labs = present[k][present[k] != 0]
        nsel = int(rng.integers(1, min(20, len(labs)) + 1))
        sel = tuple(int(x) for x in rng.choice(labs, size=nsel, replace=False))
        reqs.append((k, sel, int(rng.integers(10, 41))))

    def plain_one(k, sel, it, wait=False):
        m = ctx.extract(ts[k], selected=sel)
        ctx.smooth(m, iterations=it, relaxation=0.5, constraint=1.0)
        m.free()
        if wait:  # the result is complete on the device
            torch.cuda.current_stream().synchronize()

    vox = [int(vols[k].labels.size) for k, _, _ in reqs]
    # algorithmic bytes of every request (untimed plain runs for the mesh sizes)
    alg = 0
    for k, sel, it in reqs:
        m = ctx.extract(ts[k], selected=sel)
        mv = m.view()
        alg += mesh_alg_bytes(int(vols[k].labels.size), vols[k].labels.dtype.itemsize,
                              int(mv.n_points), int(mv.n_quads), int(mv.n_stencil), it)
        m.free()

    # saturation: every request at once; the plain path runs them one by one
    for r in reqs[:8]:
        plain_one(*r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        plain_one(*r)
    torch.cuda.synchronize()
    sat_plain = time.perf_counter() - t0
    srv = ctx.serve_start(hbm_budget_bytes=32 << 30, max_inflight=64, n_streams=2, max_batch=16)
    t0 = time.perf_counter()
    tks = [srv.submit(ts[k], iterations=it, relaxation=0.5, constraint=1.0, selected=sel)
           for k, sel, it in reqs]
    for tk in tks:
        srv.wait(tk).free()
    sat_served = time.perf_counter() - t0
    sat_batches = srv.stats()["n_batches"]
    srv.stop()
    saturation = {"plain_gvox_per_s": round(sum(vox) / sat_plain / 1e9, 3),
                  "served_gvox_per_s": round(sum(vox) / sat_served / 1e9, 3),
                  "speedup": round(sat_plain / sat_served, 3), "served_batches": sat_batches,
                  "alg_bytes": int(alg),
                  "plain_frac_hbm": round(alg / sat_plain / 1e9 / HBM_PEAK_GBS, 4),
                  "served_frac_hbm": round(alg / sat_served / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"[bench] served: saturation plain {sat_plain * 1e3:.1f} ms, served {sat_served * 1e3:.1f} ms")

    # latency: Poisson streams at 80 % and at 150 % of the plain path's
    # capacity (service time measured first, then frozen)
    t0 = time.perf_counter()
    for r in reqs[:40]:
        plain_one(*r, wait=True)
    svc = (time.perf_counter() - t0) / 40
    log(f"[bench] served: plain service {svc * 1e3:.2f} ms")

    def plain_fifo(arrivals):
        """One request at a time, in arrival order, in real time."""
        lat = []
        start = time.perf_counter()
        for (k, sel, it), a in zip(reqs, arrivals):
            now = time.perf_counter() - start
            if now < a:
                time.sleep(a - now)
            plain_one(k, sel, it, wait=True)
            lat.append(time.perf_counter() - start - a)
        wall = time.perf_counter() - start
        return {"p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                "gvox_per_s": round(sum(vox) / wall / 1e9, 3)}

    def served_stream(arrivals):
        """The server fed at the arrival times; a collector thread waits on
        the tickets in order and frees the meshes."""
        srv = ctx.serve_start(hbm_budget_bytes=32 << 30, max_inflight=64, n_streams=2,
                              max_batch=16)
        tickets = []
        done = []

        def collect():
            for tk in iter(lambda: tickets.pop(0) if tickets else None, "stop"):
                if tk is None:
                    time.sleep(0.0002)
                    continue
                if tk == -1:
                    return
                m = srv.wait(tk)
                done.append(time.perf_counter())
                m.free()

        th = threading.Thread(target=collect)
        th.start()
        start = time.perf_counter()
        for (k, sel, it), a in zip(reqs, arrivals):
            now = time.perf_counter() - start
            if now < a:
                time.sleep(a - now)
            tickets.append(srv.submit(ts[k], iterations=it, relaxation=0.5, constraint=1.0,
                                      selected=sel))
        tickets.append(-1)
        th.join()
        wall = max(done) - start
        st = srv.stats()
        srv.stop()
        return {"p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
                "gvox_per_s": round(sum(vox) / wall / 1e9, 3), "batches": st["n_batches"],
                "done": st["n_done"], "requeued": st.get("n_requeued")}

    loads = {}
    for load in (0.8, 1.5):
        qps = load / svc
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n_requests))
        log(f"[bench] served: Poisson stream at {load:.1f} x plain capacity, {qps:.1f} QPS")
        pl = plain_fifo(arrivals)
        sv = served_stream(arrivals)
        loads[f"{load:.1f}x"] = {"qps": round(qps, 2), "plain_fifo": pl, "served": sv,
                                 "p99_speedup": round(pl["p99_ms"] / max(sv["p99_ms"], 1e-9), 3),
                                 "throughput_ratio": round(sv["gvox_per_s"] /
                                                           max(pl["gvox_per_s"], 1e-12), 3)}
        log(f"[bench] served: p99 plain {pl['p99_ms']:.2f} ms, served {sv['p99_ms']:.2f} ms; "
            f"Gvox/s plain {pl['gvox_per_s']:.2f}, served {sv['gvox_per_s']:.2f}")
    return {"requests": n_requests, "pool_volumes": pool, "saturation": saturation,
            "plain_service_ms": round(svc * 1e3, 4), "poisson": loads}


def bench_triangulate(ctx, sn, torch, vol, reps=10):
    """The final triangulation (Sec. 2.5) of the smoothed mesh of `vol` under
    each diagonal rule, timed with HIP events around the library's launches.
    Algorithmic bytes per launch: quads (16 B) and label pairs (2b B) read,
    points (12 B) read once, triangles (24 B) and their pairs (4b B) written."""
    t = sn.to_device(vol.labels)
    m = ctx.extract(t, spacing=vol.spacing)
    ctx.smooth(m, iterations=vol.iterations, relaxation=vol.relaxation, constraint=vol.constraint)
    v = m.view()
    P, Q, b = int(v.n_points), int(v.n_quads), int(v.dtype)
    alg = Q * (16 + 2 * b + 24 + 4 * b) + 12 * P
    out = {"quads": Q, "alg_bytes_per_launch": alg}
    for rule in ("fixed", "shortest", "min_area", "planar"):
        ctx.triangulate(m, rule)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_reset()
        for _ in range(reps):
            ctx.triangulate(m, rule)
        prof = ctx.profile_read()
        ctx.profile(False)
        n, ms = prof["k_tri_rule"]
        us = 1e3 * ms / n
        out[rule] = {"avg_us": round(us, 2), "alg_GBs": round(alg / (us * 1e-6) / 1e9, 1),
                     "frac_hbm": round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    m.free()
    return out


def bench_label_sweep(ctx, sn, torch, counts=(1, 2, 4, 8, 16, 32, 64, 128), steps=3):
    """Extraction + 25 sweeps of the paper-scale synthetic volume (512^3 u16,
    128 spheres) with the first k labels selected, k = 1 .. 128: the effect of
    the number of extracted objects on the run time.  Kernel times from HIP
    events around every launch; whole steps from the wall clock."""
    import synth

    vol = synth.synthetic_spheres()
    t = sn.to_device(vol.labels)
    V = int(vol.labels.size)
    rows = []
    for k in counts:
        sel = tuple(range(1, k + 1))

        def step():
            m = ctx.extract(t, selected=sel)
            ctx.smooth(m, iterations=vol.iterations, relaxation=vol.relaxation,
                       constraint=vol.constraint)
            v = m.view()
            n = (int(v.n_points), int(v.n_quads))
            m.free()
            return n

        step()
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            P, Q = step()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        prof = ctx.profile_read()
        ctx.profile(False)
        ext = sum(prof.get(n_, (0, 0.0))[1] for n_ in ("k_edges", "k_count", "k_generate")) / steps
        smo = prof.get("k_jacobi", (0, 0.0))[1] / steps
        rows.append({"labels": k, "points": P, "quads": Q, "ms_per_step": round(1e3 * wall, 3),
                     "extract_kernel_ms": round(ext, 3), "smooth_kernel_ms": round(smo, 3),
                     "extract_gvox_per_s": round(V / (ext * 1e-3) / 1e9, 2) if ext > 0 else None})
        log(f"[bench] label sweep: {k} labels, {1e3 * wall:.2f} ms/step, P {P}")
    base = rows[0]["ms_per_step"]
    for r in rows:
        r["relative_time"] = round(r["ms_per_step"] / base, 3)
    del t
    return {"volume": vol.name, "steps": steps, "rows": rows}


COPY_PROBE_BYTES = 256 << 20


def copy_probe(torch, reps=5):
    """A plain streaming kernel of known size (int32 bitwise_not: reads and
    writes COPY_PROBE_BYTES each), timed with events; under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE calibrate the counters of the library's kernels."""
    n = COPY_PROBE_BYTES // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.bitwise_not(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    assert int(dst[12345]) == ~12345
    return {"bytes_read": COPY_PROBE_BYTES, "bytes_written": COPY_PROBE_BYTES,
            "avg_us": round(us, 2), "GBs": round(2 * COPY_PROBE_BYTES / (us * 1e-6) / 1e9, 1)}


def pmc_summary(pmc_dir, out_path, workload):
    """Reduce rocprofv3 --pmc runs (FETCH_SIZE in one, WRITE_SIZE in another,
    CSV output) of `bench.py --copy-probe` to HBM bytes per dispatch of each
    library kernel, each counter scaled by what it reads for the copy probe
    (known bytes / counted bytes).  Merged into the JSON file under
    `workload`."""
    import csv
    import glob

    acc = {}
    for f in sorted(glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"),
                              recursive=True)):
        for row in csv.DictReader(open(f)):
            name = row["Kernel_Name"]
            if "bitwise_not" in name:
                key = "copy_probe"
            else:
                key = name.split("(")[0].split("<")[0].replace("void ", "").replace("sn::", "")
                key = key.strip()
                # one entry per kernel as the library's timing names it: the
                # single-volume forms (_one), the first sweep (k_jacobi_first),
                # the row-width forms of k_edges and the store forms of
                # k_generate (and its image form) count with their kernel
                for suf in ("_one", "_wide", "_narrow", "_staged", "2d"):
                    key = key.replace(suf, "")
                if key.startswith("k_jacobi"):
                    key = "k_jacobi"
            c = row["Counter_Name"]
            d = acc.setdefault(key, {}).setdefault(c, {})
            disp = row.get("Dispatch_Id") or row.get("Correlation_Id") or str(len(d))
            d[disp] = d.get(disp, 0.0) + float(row["Counter_Value"])
    # mean per dispatch over every dispatch of the kernel (all its forms)
    mean = {k: {c: sum(v.values()) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    if "copy_probe" not in mean:
        raise SystemExit("pmc summary: no copy probe dispatches found")
    cp = mean["copy_probe"]
    f_rd = COPY_PROBE_BYTES / (cp["FETCH_SIZE"] * 1024.0)
    f_wr = COPY_PROBE_BYTES / (cp["WRITE_SIZE"] * 1024.0)
    res = {"calibration": {"copy_bytes": COPY_PROBE_BYTES, "fetch_kib": cp["FETCH_SIZE"],
                           "write_kib": cp["WRITE_SIZE"], "read_factor": round(f_rd, 4),
                           "write_factor": round(f_wr, 4)}}
    for k, cs in mean.items():
        if k == "copy_probe" or "FETCH_SIZE" not in cs or "WRITE_SIZE" not in cs:
            continue
        res[k] = {"fetch_kib": round(cs["FETCH_SIZE"], 1), "write_kib": round(cs["WRITE_SIZE"], 1),
                  "bytes": int(cs["FETCH_SIZE"] * 1024 * f_rd + cs["WRITE_SIZE"] * 1024 * f_wr)}
    allj = {}
    if os.path.exists(out_path):
        allj = json.load(open(out_path))
    allj[workload] = res
    with open(out_path, "w") as fh:
        json.dump(allj, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(res, indent=1))


def workload_summary(vol, r, roof):
    """The figures of one more volume for the `extra` object."""
    img = vol.labels.ndim == 2
    unit = "gpix" if img else "gvox"
    return {"name": vol.name, "ms_per_step": round(r["ms_per_step"], 3),
            f"{unit}_per_s": round(r["gvox_per_s"], 3),
            f"extract_{unit}_per_s": round(r["extract_gvox_per_s"], 3),
            "extract_alg_GBs": round(r["extract_alg_GBs"], 1),
            "extract_frac_hbm": round(r["extract_frac_hbm"], 4),
            "smooth_gptit_per_s": round(r["smooth_gptit_per_s"], 3),
            "points": r["points"], ("segments" if img else "quads"): r["quads"],
            "iterations": r["iterations"], "schedule": r["schedule"], "roofline": roof,
            "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                            for kk, vv in d.items()} for k, d in r["kernels"].items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="connectome",
                    choices=["connectome", "torso", "spheres", "section"])
    ap.add_argument("--no-extra", action="store_true", help="skip connectome/batched/served")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM traffic per launch from rocprofv3 counters, if measured")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain streaming kernel of known size (counter calibration)")
    ap.add_argument("--only", choices=["batched", "served"],
                    help="run one of the extra measurements alone and print its figures as the "
                         "JSON line (for a profile of that path); no headline workload")
    ap.add_argument("--pmc-summary", metavar="DIR",
                    help="no GPU work: reduce rocprofv3 --pmc output in DIR into --traffic-json")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.traffic_json, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this implementation runs on a single GPU "
              f"(how the path would shard over z-slabs is a design, not code); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2401_14906_amd as sn

    if not os.path.exists(sn.LIB_PATH):
        from paper_2401_14906_amd import _build

        _build.build()
    ctx = sn.Context(0)
    if args.only:
        log(f"[bench] device {torch.cuda.get_device_name(0)}; {args.only} path alone")
        fn = {"batched": bench_batched, "served": bench_served}[args.only]
        print(json.dumps({"only": args.only, args.only: fn(ctx, sn, torch)}), flush=True)
        ctx.close()
        return
    log(f"[bench] device {torch.cuda.get_device_name(0)}; workload {args.workload}")
    gen = {"torso": synth.torso_like, "connectome": synth.connectome_like,
           "section": synth.section_like,
           "spheres": synth.spheres_small}[args.workload]
    vol = gen()
    res = measure_workload(ctx, sn, torch, vol, args.steps, args.warmup)
    log(f"[bench] {vol.name}: {res['ms_per_step']:.3f} ms/step, {res['gvox_per_s']:.2f} Gvox/s")

    probe = copy_probe(torch) if args.copy_probe else None
    tj_all = json.load(open(args.traffic_json)) if os.path.exists(args.traffic_json) else {}

    def traffic_for(workload, r):
        """Counter-measured HBM bytes per launch of r's dominant kernel, if
        recorded.  The counters give a mean per dispatch; the first two sweeps
        of a mesh share one dispatch, so n sweeps make n - 1 dispatches and the
        per-sweep figure is the dispatch mean times (n - 1) / n."""
        kernel = roofline_of(r)["kernel"]
        entry = tj_all.get(workload, {}).get(kernel)
        if not entry:
            return None
        n = r["iterations"]
        scale = (n - 1) / n if kernel == "k_jacobi" and n >= 2 else 1.0
        return int(round(entry["bytes"] * scale))

    roof = roofline_of(res, traffic_for(args.workload, res))

    extra = {}
    if not args.no_extra:
        # the other volumes: config name -> (generator, --workload key, key of extra)
        others = [("connectome", synth.connectome_like, "connectome_like"),
                  ("torso", synth.torso_like, "torso_like"),
                  ("spheres", synth.spheres_small, "spheres_small"),
                  ("section", synth.section_like, "section_like_2d")]
        for key, gen_o, name in others:
            if key == args.workload:
                continue
            ovol = gen_o()
            ro = measure_workload(ctx, sn, torch, ovol, max(5, args.steps // 2), 2)
            extra[name] = workload_summary(ovol, ro, roofline_of(ro, traffic_for(key, ro)))
            log(f"[bench] {ovol.name}: {ro['ms_per_step']:.3f} ms/step, "
                f"{ro['gvox_per_s']:.2f} Gvox/s")
            del ovol
        extra["batched"] = bench_batched(ctx, sn, torch)
        extra["served"] = bench_served(ctx, sn, torch)
        tvol = vol if args.workload == "torso" else synth.torso_like()
        extra["triangulate"] = bench_triangulate(ctx, sn, torch, tvol)
        extra["label_sweep"] = bench_label_sweep(ctx, sn, torch)

    cpu = cpu_all = None
    if not args.no_cpu:
        log("[bench] oracle on one core")
        cpu = cpu_baseline(vol)
        log("[bench] oracle on all cores")
        cpu_all = cpu_baseline_all_cores(vol)
    line = {
        "metric": "Gvoxels/s extract + Gpoint-iters/s smooth, 1 GPU; batched/served vs plain",
        "value": round(res["gvox_per_s"], 4),
        "unit": "Gvoxels/s (whole step: extract + smooth)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{'u' + str(8 * vol.labels.dtype.itemsize)} labels; f64 math / f32 storage for smoothing",
        "data": "synthetic (seeded generator, resident in HBM)",
        "config": {"workload": vol.name, "dims": list(vol.dims), "spacing": list(vol.spacing),
                   "labels": "all", "prim": "lines" if vol.labels.ndim == 2 else "quads",
                   "iterations": vol.iterations,
                   "relaxation": vol.relaxation, "constraint": vol.constraint,
                   "schedule": res["schedule"]},
        "extract_gvox_per_s": round(res["extract_gvox_per_s"], 3),
        "smooth_gptit_per_s": round(res["smooth_gptit_per_s"], 3),
        "mesh": {"points": res["points"], "quads": res["quads"], "stencil": res["stencil"]},
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in d.items()}
                    for k, d in res["kernels"].items()},
        "roofline": roof,
        "extract_alg_GBs": round(res["extract_alg_GBs"], 1),
        "extract_frac_hbm": round(res["extract_frac_hbm"], 4),
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "extra": extra,
    }
    if probe:
        line["copy_probe"] = probe
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
