"""Benchmark: SurfaceNets extraction + constrained smoothing on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload torso|connectome|spheres]

A step is one pass of the whole hot path over one synthetic label volume that
is already resident in HBM: extraction (classification, counting, scan,
generation of points / quads / label pairs / stencil) followed by the
smoothing sweeps and the world-coordinate emit.  The default workload is the
torso-like 256^3 uint16 volume (100 Voronoi cells in an ellipsoidal body,
spacing 1x1x2.5, 25 sweeps, relaxation 0.5, constraint 1.0).

One JSON line is printed on stdout; progress goes to stderr.  `value` is
whole-step throughput in Gvoxels/s (voxels / wall time of a full step).
Per-kernel durations come from HIP events recorded by the library on the
stream each kernel runs on, during the timed steps; the roofline object uses
the kernel with the largest total time.  Extra objects report the
connectome-like volume, the batched path against sequential plain calls and
the served path against a plain FIFO loop, and the oracle timed on one host
core.
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
# algorithmic bytes (what the method must move; metadata is overhead)
# --------------------------------------------------------------------------

def bytes_count(V, b):
    """k_count: read the label volume once."""
    return V * b


def bytes_generate(V, b, P, Q, S):
    """k_generate: read the volume, write points (12 B), stencil offsets (4 B),
    quads (16 B), label pairs (2b B) and stencil ids (4 B)."""
    return V * b + 12 * P + 4 * (P + 1) + Q * (16 + 2 * b) + 4 * S


def bytes_jacobi_avg(P, S, n):
    """k_jacobi, averaged over n sweeps: read own offset (all but the first
    sweep), faces byte, CSR offset, stencil ids; write the new offset.
    Neighbour offsets are re-reads of the same array (reuse, not counted)."""
    return P * (12.0 * (n - 1) / n + 12 + 1 + 4) + 4 * S


def bytes_emit(P):
    """k_emit: read the final offsets, write world points."""
    return 24 * P


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
        m.free()  # waits for this step's device work
    return sizes


def measure_workload(ctx, sn, torch, vol, steps, warmup):
    t = sn.to_device(vol.labels)
    b = vol.labels.dtype.itemsize
    V = int(vol.labels.size)
    log(f"[bench] {vol.name}: warmup {warmup}")
    run_plain_steps(ctx, sn, torch, t, vol, warmup)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, Q, S = run_plain_steps(ctx, sn, torch, t, vol, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    n = vol.iterations
    per = {}
    for name, (launches, ms) in prof.items():
        per[name] = {"launches": launches, "avg_us": 1e3 * ms / max(launches, 1),
                     "total_ms": ms}
    alg = {"k_count": bytes_count(V, b), "k_generate": bytes_generate(V, b, P, Q, S),
           "k_jacobi": bytes_jacobi_avg(P, S, n), "k_emit": bytes_emit(P)}
    for name, d in per.items():
        if name in alg:
            d["alg_bytes"] = alg[name]
            d["achieved_GBs"] = alg[name] / (d["avg_us"] * 1e-6) / 1e9
            d["frac_hbm"] = d["achieved_GBs"] / HBM_PEAK_GBS
    ext_ms = sum(per.get(k, {}).get("total_ms", 0.0) for k in ("k_count", "k_generate")) / steps
    smo_ms = sum(per.get(k, {}).get("total_ms", 0.0) for k in ("k_jacobi", "k_emit")) / steps
    res = {
        "voxels": V, "points": P, "quads": Q, "stencil": S, "iterations": n,
        "ms_per_step": 1e3 * wall / steps,
        "gvox_per_s": V * steps / wall / 1e9,
        "extract_kernel_ms": ext_ms,
        "smooth_kernel_ms": smo_ms,
        "extract_gvox_per_s": V / (ext_ms * 1e-3) / 1e9 if ext_ms > 0 else None,
        "smooth_gptit_per_s": P * n / (smo_ms * 1e-3) / 1e9 if smo_ms > 0 else None,
        "extract_alg_GBs": (bytes_generate(V, b, P, Q, S)) / (ext_ms * 1e-3) / 1e9 if ext_ms > 0 else None,
        "kernels": per,
    }
    del t
    return res


def roofline_of(res, traffic=None):
    per = res["kernels"]
    dom = max((k for k in per if "alg_bytes" in per[k]), key=lambda k: per[k]["total_ms"])
    d = per[dom]
    return {"kernel": dom, "bound": "hbm", "achieved": round(d["achieved_GBs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["frac_hbm"], 4),
            "traffic": traffic, "avg_us": round(d["avg_us"], 2),
            "alg_bytes_per_launch": int(d["alg_bytes"])}


def cpu_baseline(vol, min_seconds=10.0):
    """The oracle (serial C, FP64), timed on one host core on the whole volume
    (extract + smoothing), repeated until at least `min_seconds` have passed."""
    import oracle

    V = int(vol.labels.size)
    reps, t_all = 0, 0.0
    while t_all < min_seconds and reps < 50:
        t0 = time.perf_counter()
        m = oracle.extract(vol.labels, vol.selected, vol.background)
        m.smooth(vol.iterations, vol.relaxation, vol.constraint)
        t_all += time.perf_counter() - t0
        reps += 1
        del m
    return {"value": round(V * reps / t_all / 1e9, 5), "unit": "Gvoxels/s", "cores": 1,
            "kind": "oracle",
            "sample": f"whole {vol.name} volume (extract + {vol.iterations} sweeps) x{reps}, "
                      f"{t_all:.1f} s on 1 core"}


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
            "speedup": round(out["plain"] / out["batched"], 3)}


def bench_served(ctx, sn, torch, n_requests=240, pool=16, seed=5):
    import synth

    log(f"[bench] served: generating a pool of {pool} volumes")
    vols = synth.serve_pool(seed=seed, count=pool, hi=384)
    ts = [sn.to_device(v.labels) for v in vols]
    present = [np.unique(v.labels) for v in vols]
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_requests):
        k = int(rng.integers(0, pool))
        labs = present[k][present[k] != 0]
        nsel = int(rng.integers(1, min(20, len(labs)) + 1))
        sel = tuple(int(x) for x in rng.choice(labs, size=nsel, replace=False))
        reqs.append((k, sel, int(rng.integers(10, 41))))

    def plain_one(k, sel, it):
        m = ctx.extract(ts[k], selected=sel)
        ctx.smooth(m, iterations=it, relaxation=0.5, constraint=1.0)
        m.free()

    # service time of the plain path, then a Poisson stream at 80 % of its capacity
    for r in reqs[:8]:
        plain_one(*r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs[:40]:
        plain_one(*r)
    torch.cuda.synchronize()
    svc = (time.perf_counter() - t0) / 40
    qps = 0.8 / svc
    arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n_requests))
    vox = [int(vols[k].labels.size) for k, _, _ in reqs]
    log(f"[bench] served: plain service {svc * 1e3:.2f} ms -> {qps:.1f} QPS")

    # plain FIFO: one request at a time, in arrival order, in real time
    lat = []
    start = time.perf_counter()
    for (k, sel, it), a in zip(reqs, arrivals):
        now = time.perf_counter() - start
        if now < a:
            time.sleep(a - now)
        plain_one(k, sel, it)
        lat.append(time.perf_counter() - start - a)
    plain_wall = time.perf_counter() - start
    plain = {"p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
             "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
             "gvox_per_s": round(sum(vox) / plain_wall / 1e9, 3)}

    srv = ctx.serve_start(hbm_budget_bytes=32 << 30, max_inflight=64, n_streams=2, max_batch=16)
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
    served_wall = max(done) - start
    st = srv.stats()
    srv.stop()
    served = {"p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
              "gvox_per_s": round(sum(vox) / served_wall / 1e9, 3), "batches": st["n_batches"],
              "done": st["n_done"]}
    return {"requests": n_requests, "qps": round(qps, 2), "pool_volumes": pool,
            "plain_fifo": plain, "served": served,
            "p99_speedup": round(plain["p99_ms"] / max(served["p99_ms"], 1e-9), 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="torso", choices=["torso", "connectome", "spheres"])
    ap.add_argument("--no-extra", action="store_true", help="skip connectome/batched/served")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM traffic per launch from rocprofv3 counters, if measured")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the method here has no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2401_14906_amd as sn

    if not os.path.exists(sn.LIB_PATH):
        from paper_2401_14906_amd import _build

        _build.build()
    ctx = sn.Context(0)
    log(f"[bench] device {torch.cuda.get_device_name(0)}; workload {args.workload}")
    gen = {"torso": synth.torso_like, "connectome": synth.connectome_like,
           "spheres": synth.spheres_small}[args.workload]
    vol = gen()
    res = measure_workload(ctx, sn, torch, vol, args.steps, args.warmup)
    log(f"[bench] {vol.name}: {res['ms_per_step']:.3f} ms/step, {res['gvox_per_s']:.2f} Gvox/s")

    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            traffic = tj.get(vol.name)
        except Exception:
            traffic = None
    roof = roofline_of(res, (traffic or {}).get(roofline_of(res)["kernel"]) if traffic else None)

    extra = {}
    if not args.no_extra:
        if args.workload != "connectome":
            cvol = synth.connectome_like()
            r3 = measure_workload(ctx, sn, torch, cvol, max(3, args.steps // 4), 1)
            extra["connectome_like"] = {
                "name": cvol.name, "ms_per_step": round(r3["ms_per_step"], 3),
                "gvox_per_s": round(r3["gvox_per_s"], 3),
                "extract_gvox_per_s": round(r3["extract_gvox_per_s"], 3),
                "smooth_gptit_per_s": round(r3["smooth_gptit_per_s"], 3),
                "points": r3["points"], "quads": r3["quads"],
                "roofline": roofline_of(r3),
                "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                                for kk, vv in d.items()} for k, d in r3["kernels"].items()}}
            del cvol
        extra["batched"] = bench_batched(ctx, sn, torch)
        extra["served"] = bench_served(ctx, sn, torch)

    cpu = None if args.no_cpu else cpu_baseline(vol)
    line = {
        "metric": "Gvoxels/s extract + Gpoint-iters/s smooth, 1 GPU; batched/served vs plain",
        "value": round(res["gvox_per_s"], 4),
        "unit": "Gvoxels/s (whole step: extract + smooth)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u16 labels; f64 math / f32 storage for smoothing",
        "data": "synthetic (seeded generator, resident in HBM)",
        "config": {"workload": vol.name, "dims": list(vol.dims), "spacing": list(vol.spacing),
                   "labels": "all", "prim": "quads", "iterations": vol.iterations,
                   "relaxation": vol.relaxation, "constraint": vol.constraint},
        "extract_gvox_per_s": round(res["extract_gvox_per_s"], 3),
        "smooth_gptit_per_s": round(res["smooth_gptit_per_s"], 3),
        "mesh": {"points": res["points"], "quads": res["quads"], "stencil": res["stencil"]},
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in d.items()}
                    for k, d in res["kernels"].items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
