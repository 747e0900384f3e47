#!/usr/bin/env python3
"""Barnes-Hut hot-path benchmark on one MI355X.

Workload (default): Plummer sphere, N = 2^20, seed 2, eps = 0.005, theta = 0.5,
leaf_cap = 1, kick-drift-kick steps with dt = 1e-4 and a full tree rebuild
every step.  A step is one pass of the whole hot path: bbox, Morton keys,
radix sort, octree, upward pass, force walk, kicks and drift.

Prints ONE JSON line.  `value` is force evaluations per second in Mparticles/s
for the FP32 mode, counted over whole steps (N / step time: every step is one
complete force evaluation from positions, tree included); the FP64 mode is
reported beside it.  The walk kernel's own time, measured with events on the
stream it runs on, gives the roofline entry; the oracle timed on the host gives
the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "BH force-evals Mparticles/s at theta=0.5, N=1M (FP32 vs FP64); served p99 latency"
FP32_PEAK = 157.3e12     # MI355X vector FP32 (packed issue)
FP64_PEAK = 78.6e12      # MI355X vector FP64
FLOPS_PER_INTERACTION = 20
FP32_NONPACKED_PEAK = 78.6e12   # the same VALU without packed FP32 issue (how the library is compiled)
HBM_PEAK = 8.0e12               # MI355X HBM3E
# algorithmic bytes per particle of one rebuild with its upward pass (8-bit digits): bbox 24,
# keys 36, sort 8 x 24, permute ~128, node build ~8 + ~48 per node, upward ~32 + ~56 per node,
# with ~1.45 nodes per particle: about 450
BUILD_BYTES_PER_PARTICLE = 450
TRAFFIC_SUMMARY = ROOT / "profiles" / "hbm_traffic_plummer_1M.md"
VALU_SUMMARY = ROOT / "profiles" / "walk_instruction_mix_plummer_1M.md"
WALK_SOURCES = [ROOT / "paper_1109_5190_amd" / "csrc" / f for f in ("bh_walk32.hip", "bh_walk_common.h", "bh_common.h")]


def walk_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        h.update(f.read_bytes())
    return h.hexdigest()


def profile_figure(path, tag, n):
    """A per-launch figure of the FP32 walk from a committed counter summary (its line
    `<tag>: kernel=k_walk32 n=<n> value=<v> source-sha256=<sha>`), or None when the
    summary was taken on another workload size or on a different walk source."""
    import re
    try:
        text = path.read_text()
        sha = walk_source_sha()
    except OSError:
        return None
    m = re.search(tag + r": kernel=k_walk32 n=(\d+) value=(\d+) source-sha256=([0-9a-f]+)", text)
    if not m or int(m.group(1)) != n or m.group(3) != sha:
        return None
    return int(m.group(2))


def walk_traffic(n):
    """HBM bytes per FP32 walk launch (FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated)."""
    return profile_figure(TRAFFIC_SUMMARY, "bench-traffic", n)


def walk_valu(n):
    """VALU instructions (SQ_INSTS_VALU, wavefront instructions) per FP32 walk launch."""
    return profile_figure(VALU_SUMMARY, "bench-valu", n)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--eps", type=float, default=0.005)
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--leaf-cap", type=int, default=1)
    ap.add_argument("--walk-reps", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=524288, help="oracle walk targets for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--shards", type=int, default=8, help="targets split for one GPU's share (0: skip)")
    ap.add_argument("--precisions", default="fp32,fp64")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests per serving run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-precisions", default="fp32,fp64",
                    help="serving runs at --serve-rate; the first is repeated near its measured capacity")
    ap.add_argument("--no-leaf16", action="store_true", help="skip the leaf_cap 16 leg")
    ap.add_argument("--no-sweep", action="store_true", help="skip the two-sphere theta leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-simulation batch leg")
    ap.add_argument("--workload", choices=("plummer1m", "sweep", "batch", "serving"), default="plummer1m",
                    help="plummer1m: the headline line; sweep: the two-sphere and cube systems of 2^22 over "
                         "theta; batch: 512 simulations as one forest; serving: the request stream with "
                         "2000 requests in FP32 and FP64 and an arrival-rate sweep (each prints its own JSON line)")
    ap.add_argument("--sample", type=int, default=2048, help="oracle targets per error check (sweep, batch)")
    return ap.parse_args()


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _errors(acc, ref):
    import numpy as np
    rms = float(np.sqrt(((acc - ref) ** 2).sum() / (ref ** 2).sum()))
    den = np.linalg.norm(ref, axis=1)
    ok = den > 0
    mx = float((np.linalg.norm(acc - ref, axis=1)[ok] / den[ok]).max()) if ok.any() else 0.0
    return rms, mx


def sweep(a, bh, torch):
    """Theta sweep on the two-sphere system (2 x 2^21) and the uniform cube (2^22), eps = 0.005:
    one force evaluation (build + upward + walk) per theta and precision, timed with events on the
    library's stream, and its error against the oracle on sampled targets."""
    import numpy as np

    import icgen
    import oracle
    dev = torch.device("cuda:0")
    ctx = bh.Context(0)
    stream = torch.cuda.current_stream(dev)
    cores = len(os.sched_getaffinity(0))
    rows = []
    systems = {"two_spheres": lambda: icgen.two_plummer(1 << 21, 3, 4), "cube": lambda: icgen.uniform_cube(1 << 22, 5)}
    for name, make in systems.items():
        s = make()
        pos, mass = torch.tensor(s.pos, device=dev), torch.tensor(s.mass, device=dev)
        T = oracle.Tree(s.pos, s.mass, a.leaf_cap)
        rng = np.random.default_rng(21)
        tg = np.sort(rng.choice(s.n, min(a.sample, s.n), replace=False)).astype(np.int64)
        tgd = torch.tensor(tg, device=dev)
        exact = oracle.direct(s.pos, s.mass, eps=0.005, targets=tg, nthreads=cores)["acc"]
        runs = ([(th, "monopole") for th in (0.3, 0.5, 0.7, 1.0)]
                + [(th, v) for v in ("quadrupole", "bmax", "offset", "group") for th in (0.5, 0.7, 1.0)])
        for theta, variant in runs:
            quad, group = variant == "quadrupole", variant == "group"
            open_ = variant if variant in ("bmax", "offset") else "side"
            if group:
                ref = T.walk_group(theta, 0.005, 1.0, 64, tg, nthreads=cores, starts=T.group_cubes(64))
            else:
                ref = T.walk(theta, 0.005, 1.0, tg, nthreads=cores, quad=quad, open=open_)
            inter = None
            for prec in ("fp32", "fp64"):
                p = bh.params(theta, 0.005, 1.0, a.leaf_cap, prec, quad=quad, group=group, open=open_)
                t = bh.Tree(ctx, pos, mass, p).upward()
                acc = t.forces()
                if inter is None:
                    tot = t.forces_stats()["totals"]
                    inter = tot["n_mono"] + tot["n_p2p"]
                torch.cuda.synchronize()
                e0, e1 = _events(torch)
                w0, w1 = _events(torch)
                reps = 3
                e0.record(stream)
                for _ in range(reps):
                    t2 = bh.Tree(ctx, pos, mass, p).upward()
                    t2.forces(acc)
                e1.record(stream)
                torch.cuda.synchronize()
                w0.record(stream)
                for _ in range(reps):
                    t.forces(acc)
                w1.record(stream)
                torch.cuda.synchronize()
                ms_eval = e0.elapsed_time(e1) / reps
                ms_walk = w0.elapsed_time(w1) / reps
                rms, mx = _errors(acc[tgd].cpu().numpy(), ref["acc"])
                rms_exact, _ = _errors(acc[tgd].cpu().numpy(), exact)
                peak = 157.3e12 if prec == "fp32" else 78.6e12
                rows.append({"system": name, "n": s.n, "theta": theta, "precision": prec,
                             "variant": variant,
                             "rms_rel_vs_direct_sum": rms_exact,
                             "ms_force_eval": ms_eval, "mparticles_per_s": s.n / (ms_eval * 1e-3) / 1e6,
                             "ms_walk": ms_walk, "interactions_per_particle": inter / s.n,
                             "walk_tflops": 20 * inter / (ms_walk * 1e-3) / 1e12,
                             "walk_frac_of_peak": 20 * inter / (ms_walk * 1e-3) / peak,
                             "rms_rel_vs_oracle": rms, "max_rel_vs_oracle": mx})
                print(f"# {name} theta={theta} {prec} {variant}: eval {ms_eval:.3f} ms "
                      f"walk {ms_walk:.3f} ms rms {rms:.2e} max {mx:.2e} vs direct {rms_exact:.2e}",
                      file=sys.stderr, flush=True)
                del t, t2
        del T
    return {"metric": "theta sweep: force evaluations Mparticles/s and error vs the FP64 oracle",
            "unit": "Mparticles/s", "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "two unit-mass Plummer spheres of 2^21 at +-(5,0,0), seeds 3/4; uniform cube "
                                   "2^22 in [-1,1]^3, masses U[0.5,1.5]/N, seed 5; eps 0.005; leaf_cap "
                                   f"{a.leaf_cap}; per-body monopole at theta 0.3-1.0; at 0.5-1.0 the quadrupole, "
                                   "the b_max and centre-offset opening radii, and the group criterion "
                                   "(groups: largest cubes of at most 64 bodies)",
                       "error_sample": f"{a.sample} random targets per system (against the oracle at the same "
                                       "settings, and against direct summation)"},
            "results": rows}


def batch(a, bh, torch):
    """512 Plummer simulations (N log-uniform in [1024, 262144], theta from {0.4, 0.5, 0.7},
    eps 0.01, dt 1e-3) as one forest in FP32: launch shape autotuned, then 20 KDK steps replayed
    from one recorded HIP graph; throughput in particle-steps per second."""
    import numpy as np

    import icgen
    import oracle
    dev = torch.device("cuda:0")
    ctx = bh.Context(0)
    stream = torch.cuda.current_stream(dev)
    t0 = time.time()
    inst = icgen.batch_instances(512, 6)
    systems = [icgen.plummer(n, seed) for n, _, seed in inst]
    cat = icgen.concat(*systems)
    print(f"# generated {cat.n} particles in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ns = [n for n, _, _ in inst]
    plist = [bh.params(th, 0.01, 1.0, a.leaf_cap, "fp32") for _, th, _ in inst]
    pos = torch.tensor(cat.pos, device=dev)
    vel = torch.tensor(cat.vel, device=dev)
    mass = torch.tensor(cat.mass, device=dev)
    forest = bh.Forest(ctx, ns, plist, pos, vel, mass)
    shape, tune_ms = forest.autotune()
    acc0 = forest.acc.cpu().numpy()
    dts = [1e-3] * len(ns)
    forest.step_graph(1, dts)      # records the graph and warms up
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    steps = 20
    e0.record(stream)
    forest.step_graph(steps, dts)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    total = int(sum(ns))
    # error at the initial positions on stratified instances
    cores = len(os.sched_getaffinity(0))
    offs = np.concatenate([[0], np.cumsum(ns)])
    order = np.argsort(ns)
    pick = order[np.linspace(0, len(ns) - 1, 8).astype(int)]
    rng = np.random.default_rng(22)
    a_all, r_all = [], []
    for k in pick:
        sk = systems[k]
        tg = np.sort(rng.choice(sk.n, min(256, sk.n), replace=False)).astype(np.int64)
        ref = oracle.forces(sk.pos, sk.mass, theta=inst[k][1], eps=0.01, targets=tg, nthreads=cores)
        a_all.append(acc0[offs[k]:offs[k + 1]][tg])
        r_all.append(ref["acc"])
    rms, mx = _errors(np.concatenate(a_all), np.concatenate(r_all))
    return {"metric": "batch: particle-steps/s of 512 simulations in one forest (FP32, HIP graph)",
            "value": total * steps / (ms * 1e-3), "unit": "particle-steps/s", "n_gpus": 1, "steps": steps,
            "ms_per_step": ms / steps, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "512 Plummer instances, N log-uniform in [1024, 262144] (seed 6), theta from "
                                   "{0.4, 0.5, 0.7}, eps 0.01, dt 1e-3, KDK with a rebuild every step",
                       "total_particles": total, "leaf_cap": a.leaf_cap},
            "autotune": {"walk_shape": bh.shape_name(shape),
                         "walk_ms_by_shape": {bh.shape_name(k): v for k, v in tune_ms.items()},
                         "shapes": "wavefronts per workgroup; p: persistent form (work queue)"},
            "force_error_vs_oracle": {"rms_rel": rms, "max_rel": mx,
                                      "sample": "256 targets on each of 8 instances stratified by N, initial positions"}}


def one_gpu_share(a, tree, stream, torch, ms_walk, acc_full):
    """The walk of one GPU's share when the targets are split G ways (each GPU holding the whole
    tree): ranges on 64-body group boundaries balanced by each group's wavefront work from a
    counting walk, each range walked alone on the whole GPU.  The ranges together reproduce the
    full walk's bits."""
    G = a.shards
    out = {"G": G, "split": "group zones (wavefront work of each 64-body walk group)"}
    acc = torch.empty_like(acc_full)
    gwork = torch.empty((tree.n + 63) // 64, dtype=torch.int64, device=acc.device)
    tree.forces_range(0, tree.n, acc, None, None, None, None, gwork)   # counting walk: wavefront work
    torch.cuda.synchronize()
    b0, b1 = _events(torch)
    b0.record(stream)
    for _ in range(a.walk_reps):
        bounds = tree.shard_bounds_groups(G, gwork)
    b1.record(stream)
    torch.cuda.synchronize()
    out["bounds_ms"] = b0.elapsed_time(b1) / a.walk_reps
    bl = bounds.cpu().tolist()
    ms = []
    for j in range(G):
        tree.forces_range(bl[j], bl[j + 1] - bl[j], acc)
        e0, e1 = _events(torch)
        e0.record(stream)
        for _ in range(a.walk_reps):
            tree.forces_range(bl[j], bl[j + 1] - bl[j], acc)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1) / a.walk_reps)
    out.update(ms=ms, max_ms=max(ms), sum_ms=sum(ms), imbalance=max(ms) * G / sum(ms),
               full_walk_over_G_vs_max=ms_walk / G / max(ms), bitwise_equal_to_walk=bool(torch.equal(acc, acc_full)))
    print(f"# one GPU's share of {G}: slowest range {out['max_ms']:.3f} ms, imbalance {out['imbalance']:.3f}",
          file=sys.stderr, flush=True)
    return out


def copy_bandwidth(torch):
    """Device-to-device copy of 2 GiB (read + write bytes / time), the HBM rate a plain streaming
    kernel reaches on this GPU."""
    x = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    reps = 5
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    bw = 2 * x.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del x, y
    torch.cuda.empty_cache()
    return bw


def serve(a, bh, ctx, torch, precision, rate, nreq):
    """Serving run: Poisson arrivals of simulation requests through the continuous-batching
    server; latency is done - submit per request."""
    import numpy as np

    import icgen
    reqs = icgen.request_stream(nreq, rate, master_seed=7)
    free = torch.cuda.mem_get_info()[0]
    arena = int(min(48 << 30, free * 0.6))
    sv = bh.Server(ctx, arena, max_slots=64, max_resident=1 << 24)
    p = bh.params(0.5, 0.01, 1.0, 1, precision)
    t0 = sv.now()
    ids = []
    for r in reqs:
        while sv.now() - t0 < r["t"]:
            time.sleep(min(0.001, max(0.0, r["t"] - (sv.now() - t0))))
        ids.append(sv.submit(r["n"], r["steps"], r["kind"], r["seed"], p, 1e-3, release=True))
    done = []
    t_note = time.time()
    for k, rid in enumerate(ids):
        while True:
            st = sv.poll(rid)
            if st["state"] in ("done", "failed", "cancelled"):
                break
            time.sleep(0.002)
            if time.time() - t_note > 20.0:   # progress of a long run
                print(f"# serving {precision}: {k} of {len(ids)} requests finished", file=sys.stderr, flush=True)
                t_note = time.time()
        done.append(st)
    sv.close()
    ok = [d for d in done if d["state"] == "done"]
    lat = np.array([d["t_done"] - d["t_submit"] for d in ok])
    wait = np.array([d["t_admit"] - d["t_submit"] for d in ok])
    service = np.array([d["t_done"] - d["t_admit"] for d in ok])
    work = sum(r["n"] * r["steps"] for r, d in zip(reqs, done) if d["state"] == "done")
    span = max(d["t_done"] for d in ok) - min(d["t_submit"] for d in ok)
    offered = rate * float(np.mean([r["n"] * r["steps"] for r in reqs]))
    out = {"requests": len(reqs), "completed": len(ok), "rate_req_per_s": rate, "precision": precision,
           "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
           "max_latency_s": float(lat.max()), "mean_queue_wait_s": float(wait.mean()),
           "mean_service_s": float(service.mean()),
           "throughput_particle_steps_per_s": work / span, "offered_particle_steps_per_s": offered,
           "makespan_s": span, "arena_bytes": arena, "max_slots": 64, "max_resident": 1 << 24,
           "workload": "Poisson arrivals, N log-uniform in [4096, 4194304], steps uniform 1..100, "
                       "Plummer or cube 50/50, theta=0.5, eps=0.01, dt=1e-3, seed 7"}
    print(f"# serving {precision} at {rate:.1f} req/s, R={len(reqs)}: p50 {out['p50_latency_s']:.3f}s "
          f"p99 {out['p99_latency_s']:.3f}s, {out['throughput_particle_steps_per_s']:.3e} particle-steps/s",
          file=sys.stderr, flush=True)
    return out


def serving_c5(a, bh, torch):
    """Serving as specified for the request stream: R = 2000 requests at 200 req/s (exponential
    gaps, seed 7), one FP32 run and one FP64 run; then arrival rates below and around the FP32
    capacity (R = 400 each) for the highest rate whose latency stays bounded: the server keeps up
    (completed work per second >= 95 % of the offered load) and the mean queue wait stays below a
    quarter of the mean service time."""
    import numpy as np

    import icgen
    ctx = ctx_of(bh, torch)
    runs = {prec: serve(a, bh, ctx, torch, prec, 200.0, 2000) for prec in ("fp32", "fp64")}
    # rates in units of the capacity for the sweep's own (smaller) request set
    mean_work = float(np.mean([r["n"] * r["steps"] for r in icgen.request_stream(400, 200.0, master_seed=7)]))
    lam_cap = runs["fp32"]["throughput_particle_steps_per_s"] / mean_work
    sweep = []
    for frac in (0.75, 0.9, 1.0, 1.1, 1.25):
        r = serve(a, bh, ctx, torch, "fp32", frac * lam_cap, 400)
        r["bounded"] = bool(r["throughput_particle_steps_per_s"] >= 0.95 * r["offered_particle_steps_per_s"] and
                            r["mean_queue_wait_s"] <= 0.25 * r["mean_service_s"])
        sweep.append(r)
    ok = [r["rate_req_per_s"] for r in sweep if r["bounded"]]
    return {"metric": "served p99 latency, 2000 requests at 200 req/s (FP32)",
            "value": runs["fp32"]["p99_latency_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "request stream: Poisson arrivals at 200 req/s, R=2000, N log-uniform in "
                                   "[4096, 4194304], steps uniform 1..100, Plummer or cube 50/50, theta 0.5, "
                                   "eps 0.01, dt 1e-3, seed 7"},
            "runs": runs, "capacity_req_per_s": lam_cap, "rate_sweep": sweep,
            "highest_bounded_rate_req_per_s": max(ok) if ok else None}


def theta_two_spheres(a, bh, torch, stream):
    """The theta sweep's two-sphere system (2 x 2^21 at +-(5,0,0), eps 0.005, per-body monopole) in
    both precisions: force evaluations per second (build + upward + walk) and walk TFLOP/s at theta
    0.3 / 0.5 / 0.7 / 1.0, with the error against the oracle on 256 sampled targets per theta (the
    full sweep over both systems and every variant is `--workload sweep`)."""
    import numpy as np

    import icgen
    import oracle
    dev = torch.device("cuda:0")
    ctx = ctx_of(bh, torch)
    s = icgen.two_plummer(1 << 21, 3, 4)
    pos, mass = torch.tensor(s.pos, device=dev), torch.tensor(s.mass, device=dev)
    T = oracle.Tree(s.pos, s.mass, a.leaf_cap)
    rng = np.random.default_rng(21)
    tg = np.sort(rng.choice(s.n, 256, replace=False)).astype(np.int64)
    tgd = torch.tensor(tg, device=dev)
    cores = len(os.sched_getaffinity(0))
    rows = []
    for theta in (0.3, 0.5, 0.7, 1.0):
        ref = T.walk(theta, 0.005, 1.0, tg, nthreads=cores)
        for prec in ("fp32", "fp64"):
            p = bh.params(theta, 0.005, 1.0, a.leaf_cap, prec)
            t = bh.Tree(ctx, pos, mass, p).upward()
            tot = t.forces_stats()["totals"]
            inter = tot["n_mono"] + tot["n_p2p"]
            acc = t.forces()
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            w0, w1 = _events(torch)
            reps = 3
            e0.record(stream)
            for _ in range(reps):
                t.rebuild(pos, mass).upward()
                t.forces(acc)
            e1.record(stream)
            w0.record(stream)
            for _ in range(reps):
                t.forces(acc)
            w1.record(stream)
            torch.cuda.synchronize()
            ms_eval, ms_walk = e0.elapsed_time(e1) / reps, w0.elapsed_time(w1) / reps
            rms, mx = _errors(acc[tgd].cpu().numpy(), ref["acc"])
            peak = 157.3e12 if prec == "fp32" else 78.6e12
            rows.append({"theta": theta, "precision": prec, "ms_force_eval": ms_eval,
                         "mparticles_per_s": s.n / (ms_eval * 1e-3) / 1e6, "ms_walk": ms_walk,
                         "interactions_per_particle": inter / s.n,
                         "walk_tflops": FLOPS_PER_INTERACTION * inter / (ms_walk * 1e-3) / 1e12,
                         "walk_frac_of_peak": FLOPS_PER_INTERACTION * inter / (ms_walk * 1e-3) / peak,
                         "rms_rel_vs_oracle": rms, "max_rel_vs_oracle": mx})
            print(f"# two spheres theta={theta} {prec}: eval {ms_eval:.3f} ms walk {ms_walk:.3f} ms rms {rms:.2e}",
                  file=sys.stderr, flush=True)
            del t
    return {"system": "two unit-mass Plummer spheres of 2^21 at +-(5,0,0), seeds 3/4, eps 0.005, monopole, "
                      f"leaf_cap {a.leaf_cap}", "n": s.n, "results": rows,
            "error_sample": "256 random targets per theta against the oracle at the same settings"}


def leaf16(a, bh, torch, stream, pos0, vel0, mass, s):
    """The headline configuration with leaves of up to 16 particles, FP32 (top level) and FP64
    (`fp64`): step and walk times, interactions per particle and the error against the oracle's
    leaf_cap-16 walk on sampled targets (one oracle reference for both precisions)."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(1)
    ns = min(16384, a.n)
    tg = np.sort(rng.choice(a.n, ns, replace=False)).astype(np.int64)
    ref = oracle.Tree(s.pos, s.mass, 16).walk(a.theta, a.eps, 1.0, tg, nthreads=len(os.sched_getaffinity(0)))

    def leg(prec):
        p = bh.params(a.theta, a.eps, 1.0, 16, prec)
        sim = bh.Sim(ctx_of(bh, torch), pos0.clone(), vel0.clone(), mass, p)
        sim.step(1, a.dt)
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        steps = max(2, min(a.steps, 5))
        e0.record(stream)
        sim.step(steps, a.dt)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / steps
        tree = bh.Tree(sim.ctx, pos0, mass, p).upward()
        st = tree.forces_stats()
        w0, w1 = _events(torch)
        w0.record(stream)
        for _ in range(a.walk_reps):
            tree.forces()
        w1.record(stream)
        torch.cuda.synchronize()
        ms_walk = w0.elapsed_time(w1) / a.walk_reps
        tot = st["totals"]
        inter = tot["n_mono"] + tot["n_p2p"]
        rms, mx = _errors(st["acc"].cpu().numpy()[tg], ref["acc"])
        sets_equal = bool(np.array_equal(st["n_mono"].cpu().numpy()[tg], ref["n_mono"]) and
                          np.array_equal(st["hash"].cpu().numpy().view(np.uint64)[tg], ref["hash"]))
        print(f"# leaf_cap 16 {prec}: step {ms_step:.3f} ms, walk {ms_walk:.3f} ms, {inter / a.n:.1f} "
              f"interactions/particle, rms {rms:.2e}", file=sys.stderr, flush=True)
        return {"ms_per_step": ms_step, "value": a.n / (ms_step * 1e-3) / 1e6,
                "walk_ms": ms_walk, "interactions_per_particle": inter / a.n,
                "walk_tflops": FLOPS_PER_INTERACTION * inter / (ms_walk * 1e-3) / 1e12,
                "force_error_vs_oracle": {"rms_rel": rms, "max_rel": mx, "interaction_sets_equal": sets_equal,
                                          "sample": f"{ns} random targets at the initial positions"}}

    out = {"leaf_cap": 16, "precision": "fp32"}
    out.update(leg("fp32"))
    out["fp64"] = dict(precision="fp64", **leg("fp64"))
    return out


_CTX = None


def ctx_of(bh, torch):
    global _CTX
    if _CTX is None:
        _CTX = bh.Context(0)
    return _CTX


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (no collectives are "
                                   "built; the one_gpu_share leg times one GPU's share of a split)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import icgen
    import paper_1109_5190_amd as bh

    if a.workload == "sweep":
        print(json.dumps(sweep(a, bh, torch)))
        return
    if a.workload == "batch":
        print(json.dumps(batch(a, bh, torch)))
        return
    if a.workload == "serving":
        print(json.dumps(serving_c5(a, bh, torch)))
        return
    dev = torch.device("cuda:0")
    t0 = time.time()
    s = icgen.plummer(a.n, a.seed)
    print(f"# generated {a.n} Plummer particles in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    pos0 = torch.tensor(s.pos, device=dev)
    vel0 = torch.tensor(s.vel, device=dev)
    mass = torch.tensor(s.mass, device=dev)
    ctx = ctx_of(bh, torch)
    stream = torch.cuda.current_stream(dev)

    results = {}
    for prec in a.precisions.split(","):
        p = bh.params(a.theta, a.eps, 1.0, a.leaf_cap, prec)
        # ---- full steps (the headline) ----
        pos = pos0.clone()
        vel = vel0.clone()
        sim = bh.Sim(ctx, pos, vel, mass, p)
        sim.step(a.warmup, a.dt)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(a.steps, a.dt)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / max(a.steps, 1)
        # ---- the walk kernel alone, on a tree at the initial positions ----
        tree = bh.Tree(ctx, pos0, mass, p).upward()
        tree.forces()
        torch.cuda.synchronize()
        w0 = torch.cuda.Event(enable_timing=True)
        w1 = torch.cuda.Event(enable_timing=True)
        w0.record(stream)
        for _ in range(a.walk_reps):
            acc = tree.forces()
        w1.record(stream)
        torch.cuda.synchronize()
        ms_walk = w0.elapsed_time(w1) / a.walk_reps
        # ---- build + upward alone: rebuilt in the tree's workspace, as inside a step ----
        tree.rebuild(pos, mass).upward()
        torch.cuda.synchronize()
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        b0.record(stream)
        for _ in range(a.walk_reps):
            tree.rebuild(pos0, mass).upward()
        b1.record(stream)
        torch.cuda.synchronize()
        ms_build = b0.elapsed_time(b1) / a.walk_reps
        # the two-phase form of the same walk: interaction lists written, then evaluated
        buf = tree.lists_build()
        tree.lists_forces(acc)
        torch.cuda.synchronize()
        l0, l1 = _events(torch)
        l2, l3 = _events(torch)
        l0.record(stream)
        for _ in range(a.walk_reps):
            tree.lists_build(reuse=True)
        l1.record(stream)
        torch.cuda.synchronize()
        l2.record(stream)
        for _ in range(a.walk_reps):
            tree.lists_forces(acc)
        l3.record(stream)
        torch.cuda.synchronize()
        nbytes = int(buf[:256 * 256].cpu().numpy().view(np.uint64)[::32].sum()) * 64 * 16
        lists = {"build_ms": l0.elapsed_time(l1) / a.walk_reps, "eval_ms": l2.elapsed_time(l3) / a.walk_reps,
                 "list_entry_bytes": nbytes, "bitwise_equal_to_walk": bool(torch.equal(acc, tree.forces()))}
        del buf
        st = tree.forces_stats()
        torch.cuda.synchronize()
        shards = one_gpu_share(a, tree, stream, torch, ms_walk, st["acc"]) if a.shards > 1 else None
        tot = st["totals"]
        inter = int(tot["n_mono"] + tot["n_p2p"])
        results[prec] = dict(ms_per_step=ms_step, ms_walk=ms_walk, ms_build_upward=ms_build,
                             interactions=inter, visits=int(tot["n_visits"]), fallbacks=int(tot["n_fallback"]),
                             wave_visits=int(tot["wave_visits"]), wave_entries=int(tot["wave_entries"]),
                             wave_accepts=int(tot["wave_accepts"]), wave_leaves=int(tot["wave_leaves"]),
                             acc=st["acc"].cpu().numpy(), lists=lists, shards=shards)
        print(f"# {prec}: step {ms_step:.3f} ms, walk {ms_walk:.3f} ms, build+upward {ms_build:.3f} ms, "
              f"{inter / a.n:.1f} interactions/particle", file=sys.stderr, flush=True)
        del sim, tree

    head = "fp32" if "fp32" in results else next(iter(results))
    r = results[head]
    peak = FP32_PEAK if head == "fp32" else FP64_PEAK
    achieved = FLOPS_PER_INTERACTION * r["interactions"] / (r["ms_walk"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": a.n / (r["ms_per_step"] * 1e-3) / 1e6,
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"Plummer sphere N={a.n} seed={a.seed} eps={a.eps} theta={a.theta} "
                               f"leaf_cap={a.leaf_cap}, KDK dt={a.dt} with tree rebuild every step",
                   "n": a.n, "theta": a.theta, "eps": a.eps, "leaf_cap": a.leaf_cap, "dt": a.dt},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": walk_traffic(a.n) if head == "fp32" else None,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by their reading for "
                                     "k_keys, whose bytes per dispatch are known)",
                     "kernel": f"k_walk32 ({FLOPS_PER_INTERACTION} flops x {r['interactions']} interactions "
                               f"per launch / {r['ms_walk']:.3f} ms)"},
        "walk_only": {"ms": r["ms_walk"], "mparticles_per_s": a.n / (r["ms_walk"] * 1e-3) / 1e6,
                      "interactions_per_particle": r["interactions"] / a.n,
                      "fp64_fallback_tests": r["fallbacks"], "opening_tests": r["visits"],
                      "wave_visits": r["wave_visits"], "wave_entries": r["wave_entries"],
                      "wave_accepts": r["wave_accepts"], "wave_leaves": r["wave_leaves"],
                      "lane_utilisation": r["interactions"] / max(1, 64 * r["wave_visits"]),
                      "frac_of_nonpacked_fp32_peak": (achieved / FP32_NONPACKED_PEAK if head == "fp32" else None),
                      "valu_insts_per_launch": walk_valu(a.n) if head == "fp32" else None,
                      "valu_lane_slots_per_interaction": (64 * walk_valu(a.n) / r["interactions"]
                                                          if head == "fp32" and walk_valu(a.n) else None),
                      "valu_source": "SQ_INSTS_VALU of the committed counter summary, when taken on this walk "
                                     "source (else null)"},
        "build_upward_ms": r["ms_build_upward"],
        "build_roofline": {"bound": "hbm", "bytes_per_particle_model": BUILD_BYTES_PER_PARTICLE,
                           "achieved": BUILD_BYTES_PER_PARTICLE * a.n / (r["ms_build_upward"] * 1e-3) / 1e12,
                           "peak": HBM_PEAK / 1e12, "unit": "TB/s",
                           "frac": BUILD_BYTES_PER_PARTICLE * a.n / (r["ms_build_upward"] * 1e-3) / HBM_PEAK,
                           "measured_copy_TBps": copy_bandwidth(torch)},
    }
    if r.get("lists"):
        out["two_phase_lists"] = r["lists"]
    if r.get("shards"):
        out["one_gpu_share"] = r["shards"]
    for prec, rr in results.items():
        if prec == head:
            continue
        pk = FP64_PEAK if prec == "fp64" else FP32_PEAK
        ach = FLOPS_PER_INTERACTION * rr["interactions"] / (rr["ms_walk"] * 1e-3)
        out[prec] = {"value": a.n / (rr["ms_per_step"] * 1e-3) / 1e6, "unit": "Mparticles/s",
                     "ms_per_step": rr["ms_per_step"], "walk_ms": rr["ms_walk"],
                     "build_upward_ms": rr["ms_build_upward"],
                     "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": pk / 1e12, "unit": "TFLOP/s",
                                  "frac": ach / pk}}
        if rr.get("lists"):
            out[prec]["two_phase_lists"] = rr["lists"]
        if rr.get("shards"):
            out[prec]["one_gpu_share"] = rr["shards"]

    if not a.no_leaf16:
        out["leaf_cap_16"] = leaf16(a, bh, torch, stream, pos0, vel0, mass, s)
    if not a.no_sweep:
        out["theta_sweep_two_spheres"] = theta_two_spheres(a, bh, torch, stream)
    if not a.no_batch:
        b = batch(a, bh, torch)
        out["batch"] = {k: b[k] for k in ("metric", "value", "unit", "steps", "ms_per_step", "config", "autotune",
                                          "force_error_vs_oracle")}

    if a.serve_requests > 0:
        runs = {}
        precs = [x for x in a.serve_precisions.split(",") if x]
        for prec in precs:
            runs[prec] = serve(a, bh, ctx, torch, prec, a.serve_rate, a.serve_requests)
        # near capacity: the first precision again at 90 % of the request rate its overloaded run sustained
        first = runs[precs[0]]
        mean_work = first["offered_particle_steps_per_s"] / first["rate_req_per_s"]
        lam = 0.9 * first["throughput_particle_steps_per_s"] / mean_work
        runs[precs[0] + "_near_capacity"] = serve(a, bh, ctx, torch, precs[0], lam, a.serve_requests)
        out["serving"] = runs

    if not a.no_cpu:
        import oracle
        ns = min(a.cpu_sample, a.n)
        rng = np.random.default_rng(0)
        targets = np.sort(rng.choice(a.n, size=ns, replace=False)).astype(np.int64)
        cores = len(os.sched_getaffinity(0))
        c0 = time.time()
        T = oracle.Tree(s.pos, s.mass, a.leaf_cap)
        c1 = time.time()
        ref = T.walk(a.theta, a.eps, 1.0, targets, nthreads=cores)
        c2 = time.time()
        t_full = (c1 - c0) + (c2 - c1) * a.n / ns
        out["cpu_baseline"] = {"value": a.n / t_full / 1e6, "unit": "Mparticles/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"full FP64 tree build (1 thread, {c1 - c0:.2f}s) + walk of {ns} random "
                                         f"targets on {cores} threads ({c2 - c1:.2f}s), walk time scaled to N"}
        errs = {}
        for prec, rr in results.items():
            acc = rr["acc"][targets]
            num = np.sqrt(((acc - ref["acc"]) ** 2).sum() / (ref["acc"] ** 2).sum())
            mx = (np.linalg.norm(acc - ref["acc"], axis=1) / np.linalg.norm(ref["acc"], axis=1)).max()
            errs[prec] = {"rms_rel": float(num), "max_rel": float(mx)}
        out["force_error_vs_oracle"] = dict(errs, sample=f"{ns} random targets at the initial positions")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
