"""Benchmark: DSES candidate sweep on one MI355X.

Default (the headline): one step = one full registration (vote, mode, score every
candidate, select) of the scene-scale workload: a 16,384-point six-primitive
reference, a 4,096-point partial source (sigma 0.005 clipped at 0.05, 20%
outliers) and the 294,912-rotation uniform SO(3) grid, eps = 0.02, truncated-L2
error, exact cell-grid scoring; the vote in 32-bit fixed point, the scoring in
float32.  Inputs are synthetic and already
resident in device memory when timing starts.

Prints one JSON line with whole-job throughput (candidate poses scored per
second), per-registration latency percentiles, the dominant kernel's roofline
position (timed with HIP events on its launch stream), the CPU oracle's rate on a
bounded sample of the same workload, and, in the same line, the serving workload
(Poisson requests against resident references: p50/p99 latency served versus one
launch per request, open loop at 0.8 load and closed loop at saturation) and the
object-scale registration (1,024-point reference, 717-point source, 36,864
rotations).  --workload picks another workload alone.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3          # MI355X published FP32 vector peak
WORKLOADS = ("c2", "c1", "c5", "c3", "c4", "local", "fig2", "exhaustive")


# sources that decide what the plain-path sweep launch reads and writes
SWEEP_SOURCES = ("api.hip", "internal.h", "kernels.hip")


def _code_only(text):
    """Source text without comments and with whitespace collapsed (string literals
    in these files hold no comment markers), so that editing a comment does not
    invalidate counters taken on the same code."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_sha():
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_00115_amd", "csrc", name), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload):
    """HBM bytes per sweep launch measured by rocprofv3 counters, if they were taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_k_sweep_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def write_traffic(workload, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """Write profiles/traffic_k_sweep_<workload>.json from four rocprofv3 --pmc
    counter_collection.csv files: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the
    plain sweep launches of `bench.py --workload <workload> --alone --steps 1
    --warmup 0 --cpu-sample 0`, and the same counters of `bench.py --calibrate-copy`,
    whose known byte counts scale them to HBM bytes."""
    import csv

    def per_dispatch(path, counter, pick):
        vals = {}
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] == counter and pick(row["Kernel_Name"]):
                    key = row["Dispatch_Id"]
                    vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
        if not vals:
            raise SystemExit(f"bench.py: no {counter} rows in {path}")
        return sum(vals.values()) / len(vals), len(vals)

    is_sweep = lambda n: n.startswith("void dses::k_sweep<")  # noqa: E731
    is_copy = lambda n: "_add<" in n  # noqa: E731  (the calibration's adds, not its fill)
    fetch, nf = per_dispatch(fetch_csv, "FETCH_SIZE", is_sweep)
    write, nw = per_dispatch(write_csv, "WRITE_SIZE", is_sweep)
    cfetch, _ = per_dispatch(copy_fetch_csv, "FETCH_SIZE", is_copy)
    cwrite, _ = per_dispatch(copy_write_csv, "WRITE_SIZE", is_copy)
    nbytes = 4 * (64 << 20)
    fs, ws = nbytes / (cfetch * 1024.0), nbytes / (cwrite * 1024.0)
    rec = {"workload": workload, "kernel_source_sha": kernel_source_sha(),
           "sweep_dispatches": [nf, nw],
           "fetch_size_kib_per_launch": fetch, "write_size_kib_per_launch": write,
           "calibration": {"kernel": "torch.add(a, 1.0, out=b) on 64 Mi float32",
                           "bytes_read": nbytes, "bytes_written": nbytes,
                           "fetch_size_kib": cfetch, "write_size_kib": cwrite,
                           "fetch_scale": fs, "write_scale": ws},
           "hbm_bytes_per_launch": fetch * 1024.0 * fs + write * 1024.0 * ws,
           "commands": [
               f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python3 "
               f"bench.py --workload {workload} --alone --steps 1 --warmup 0 --cpu-sample 0",
               f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python3 "
               f"bench.py --workload {workload} --alone --steps 1 --warmup 0 --cpu-sample 0",
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python3 "
               "bench.py --calibrate-copy",
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python3 "
               "bench.py --calibrate-copy",
               "python3 bench.py --workload <w> --write-traffic <four counter_collection.csv>"],
           "kernel_sources": list(SWEEP_SOURCES),
           "kernel_source_hash": "sha256 over " + ", ".join(SWEEP_SOURCES) + " without comments "
                                 "and with whitespace collapsed (bench.py kernel_source_sha)"}
    path = os.path.join(ROOT, "profiles", f"traffic_k_sweep_{workload}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps({"wrote": path, "hbm_bytes_per_launch": rec["hbm_bytes_per_launch"]}))


def make_workload(name, grid_level=4):
    from paper_2502_00115_amd import synth
    if name == "c1":
        return synth.make_c1(0), "plain DSES, 256-pt ellipsoid, 64-pt source, 577 rotations"
    if name == "c5":
        p = synth.make_c5(0, grid_level=grid_level)
        return p, (f"scene-scale, 16,384-pt reference, 4,096-pt source, "
                   f"{len(p.rotations):,}-rotation Hopf grid")
    if name == "local":
        return synth.make_local(0), ("local registration with an initial guess: 0.1 m object, "
                                     "2,048-pt reference, 1,434-pt partial source, Euler grid "
                                     "+-5 deg in 0.5 deg steps (9,261 rotations), translation "
                                     "box +-1.6 cm, eps = delta = 2 mm")
    return synth.make_c2(0), ("single registration at object scale: 1,024-pt reference, "
                              "717-pt source, 36,864-rotation Hopf grid")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, sample, threads):
    """The oracle (plain C, FP64, one thread per core over rotations) on a seeded
    sample of the workload's rotations, plus a single-thread run on a few of them."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    which = np.sort(rng.choice(len(p.rotations), min(sample, len(p.rotations)), replace=False))
    box = p.meta.get("t_box")
    kw = {"t_min": -box, "t_max": box} if box is not None else {}
    pairs = float(len(p.src)) * len(p.tgt)
    t0 = time.perf_counter()
    oracle.records(p.src, p.tgt, p.rotations, p.eps, which=which, threads=threads, **kw)
    dt = time.perf_counter() - t0
    one = which[: max(1, min(len(which), int(2.0e8 / pairs) + 1))]
    t1 = time.perf_counter()
    oracle.records(p.src, p.tgt, p.rotations, p.eps, which=one, threads=1, **kw)
    dt1 = time.perf_counter() - t1
    return {"value": len(which) / dt, "unit": "candidates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread_pairs_per_s": len(one) * pairs / dt1,
            "single_thread_candidates_per_s": len(one) / dt1,
            "sample": f"{len(which)} of {len(p.rotations)} rotations of the same registration "
                      f"(seeded), full FP64 vote by the definition + brute-force FP64 scoring, "
                      f"{dt:.1f} s wall on {threads} threads; single thread: {len(one)} "
                      f"rotations in {dt1:.1f} s (a pair is voted and scored)"}


def bench_batch(args):
    """64 registrations of uneven sizes: one batched persistent launch (HIP graph)
    versus 64 plain single-registration launches, same device-resident inputs."""
    import numpy as np
    import torch
    from paper_2502_00115_amd import dses, synth

    probs = synth.make_c3(0, count=64)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    items = [{"src": dev(p.src), "tgt": dev(p.tgt), "rotations": dev(p.rotations), "eps": p.eps}
             for p in probs]
    cands = sum(len(p.rotations) for p in probs)
    # default layout, then one tuning call (its layout is kept for this batch class)
    dses.register_batch(items, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dses.register_batch(items, use_graph=True)
    torch.cuda.synchronize()
    default_s = time.perf_counter() - t0
    default_cfg = dses.batch_last_config()
    t0 = time.perf_counter()
    dses.register_batch(items, use_graph=True, autotune=True)
    tune_s = time.perf_counter() - t0
    tuned_cfg = dses.batch_last_config()
    for _ in range(max(0, args.warmup - 1)):
        dses.register_batch(items, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, st = dses.register_batch(items, use_graph=True)
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) / args.steps
    layout = dses.batch_last_config()
    assert all(v == 0 for v in st)
    t0 = time.perf_counter()
    plain = [dses.register(it["src"], it["tgt"], it["rotations"], it["eps"]) for it in items]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    same = all(a.rot_index == b.rot_index and a.error == b.error for a, b in zip(plain, res))
    # algorithmic work with the exact cell-grid scorer, summed over the batch
    flop = sum((11.0 * len(p.src) * len(p.tgt) + 18.0 * len(p.src)) * len(p.rotations)
               for p in probs)
    achieved = flop / batched / 1e12
    return {"metric": "candidate poses {R,t} scored/sec (1 GPU), batched",
            "value": cands / batched, "unit": "candidates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": batched * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "i32 vote, f32 score", "data": "synthetic",
            "config": {"workload": "64 registrations, M 512-4096 log-uniform, N 30-80% cut, "
                                   "K 4,608-36,864 rotations, one persistent launch replayed "
                                   "from a HIP graph", "candidates": cands},
            "roofline": {"bound": "alu", "kernel": "k_sweep_batch (whole batched call timed)",
                         "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                         "work": "algorithmic (11*N*M + 18*N) FLOP per candidate, summed "
                                 "over the 64 registrations"},
            "plain": {"value": cands / plain_s, "ms_total": plain_s * 1e3,
                      "frac": flop / plain_s / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                      "path": "64 sequential dses_register calls"},
            "layout": layout, "untuned": {"ms": default_s * 1e3, "layout": default_cfg},
            "tuning": {"s": tune_s, "candidates": tuned_cfg["candidates"],
                       "sweep_ms_best": tuned_cfg["sweep_ms"]},
            "identical_to_plain": bool(same)}


def bench_fig2(args):
    """Time per registration against the search range (the shape of the paper's Fig. 2):
    Euler grids in 2.5-degree steps around the identity on the object-scale workload,
    rotation range swept at a +-0.2 translation box, translation range swept at +-45 deg."""
    import numpy as np
    import torch
    from paper_2502_00115_amd import dses, synth

    p = synth.make_c2(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    src, tgt = dev(p.src), dev(p.tgt)
    step = np.deg2rad(2.5)

    def time_one(K, box):
        rot = dev(synth.euler_grid(K, step).reshape(-1, 9).astype(np.float32))
        kw = dict(t_min=-box, t_max=box)
        dses.register(src, tgt, rot, p.eps, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dses.register(src, tgt, rot, p.eps, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        return {"rotations": int(rot.shape[0]), "ms": ms}

    rot_sweep = [dict(range_deg=2.5 * K, t_box=0.2, **time_one(K, 0.2)) for K in (2, 4, 8, 12, 18)]
    t_sweep = [dict(range_deg=45.0, t_box=b, **time_one(18, b)) for b in (0.05, 0.1, 0.2, 0.35, 0.5)]
    total = sum(r["rotations"] for r in rot_sweep + t_sweep)
    secs = sum(r["ms"] for r in rot_sweep + t_sweep) / 1e3
    return {"metric": "registration time vs search range (1 GPU)", "value": total / secs,
            "unit": "candidates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": secs * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "i32 vote, f32 score", "data": "synthetic",
            "config": {"workload": "object-scale registration (717-pt source, 1,024-pt "
                                   "reference, eps = delta = 0.03) over Euler grids of 2.5 deg "
                                   "steps; rotation range at +-0.2 translation, translation "
                                   "range at +-45 deg"},
            "rotation_range": rot_sweep, "translation_range": t_sweep}


def bench_exhaustive(args):
    """Alg. 1 (every rotation x every lattice translation) against DSES on the same
    small registration: the time DSES's vote saves on the same GPU."""
    import numpy as np
    import torch
    from paper_2502_00115_amd import dses, synth

    p = synth.make_c1(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    src, tgt, rot = dev(p.src), dev(p.tgt), dev(p.rotations)
    box = dict(t_min=-0.5, t_max=0.5)

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, r

    t_dses, a = timed(lambda: dses.register(src, tgt, rot, p.eps, **box))
    t_exh, b = timed(lambda: dses.register_exhaustive(src, tgt, rot, p.eps, **box))
    bins = int(round(0.5 / p.eps)) * 2 + 1           # lattice points per axis of +-0.5
    k = len(p.rotations)
    return {"metric": "candidate poses {R,t} scored/sec (1 GPU), exhaustive Alg. 1 vs DSES",
            "value": k * bins ** 3 / t_exh, "unit": "candidates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": t_exh * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32 vote, f32 score",
            "data": "synthetic",
            "config": {"workload": f"64-pt source, 256-pt reference, {k} rotations, translation "
                                   f"box +-0.5 at delta 0.05 ({bins}^3 lattice points); exact "
                                   "cell-grid scoring"},
            "exhaustive": {"ms": t_exh * 1e3, "candidates": k * bins ** 3,
                           "rot_index": b.rot_index, "error": b.error},
            "dses": {"ms": t_dses * 1e3, "candidates": k, "rot_index": a.rot_index,
                     "error": a.error},
            "speedup_dses": t_exh / t_dses}


def bench_serve(args, n_req=None, quiet=False):
    """Poisson arrivals against 8 resident references (with 128^3 distance fields):
    served (continuous batching) versus one launch per request in FIFO order, at 0.8
    of the plain path's capacity; then closed loop (every request outstanding at
    once) for the saturation throughput of both paths."""
    import threading

    import numpy as np
    import torch
    from paper_2502_00115_amd import dses, synth

    n_req = args.requests if n_req is None else n_req
    targets = synth.make_c4_targets(0, count=8)
    T = [dses.Target(t, df_trunc=0.03, df_res=128) for t, _ in targets]
    R = dses.RotationSet(synth.hopf_grid(3).reshape(-1, 9).astype(np.float32))
    reqs = [synth.make_c4_request(i, targets) for i in range(n_req + 8)]
    for tid, src in reqs[:8]:                       # warm-up (staging caches, code objects)
        dses.register_resident(T[tid], R, src, 0.03)
    reqs = reqs[8:]
    # capacity of the plain path fixes the arrival rate
    t0 = time.perf_counter()
    for tid, src in reqs[:16]:
        dses.register_resident(T[tid], R, src, 0.03)
    mean_service = (time.perf_counter() - t0) / 16
    rate = 0.8 / mean_service
    rng = np.random.default_rng(0)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    if not quiet:
        print(f"bench.py: serving, {n_req} requests at {rate:.1f}/s", file=sys.stderr,
              flush=True)

    # plain: one launch per request, FIFO, same arrival times
    lat_plain, svc_plain = [], []
    start = time.perf_counter()
    for (tid, src), at in zip(reqs, arrivals):
        now = time.perf_counter() - start
        if now < at:
            time.sleep(at - now)
        t1 = time.perf_counter()
        dses.register_resident(T[tid], R, src, 0.03)
        svc_plain.append(time.perf_counter() - t1)
        lat_plain.append(time.perf_counter() - start - at)
    plain_wall = time.perf_counter() - start

    # served
    srv = dses.Server(aging=args.aging, slice_mpairs=args.slice_mpairs)
    ids = [None] * n_req
    start = time.perf_counter()

    def producer():
        for i, ((tid, src), at) in enumerate(zip(reqs, arrivals)):
            now = time.perf_counter() - start
            if now < at:
                time.sleep(at - now)
            ids[i] = srv.submit(T[tid], R, src, 0.03)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    done = [srv.wait(rid, timeout_ms=600000) for rid in ids]
    served_wall = time.perf_counter() - start
    lat_served = [g.total_s for g in done]
    queue_served = [g.queue_s for g in done]

    # closed loop: all requests outstanding at once
    t0 = time.perf_counter()
    for tid, src in reqs:
        dses.register_resident(T[tid], R, src, 0.03)
    torch.cuda.synchronize()
    sat_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    ids = [srv.submit(T[tid], R, src, 0.03) for tid, src in reqs]
    for rid in ids:
        srv.wait(rid, timeout_ms=600000)
    sat_served = time.perf_counter() - t0
    srv.close()
    cands = 36864 * n_req
    # algorithmic work with distance-field scoring: 3 FLOP per vote pair, 18 per
    # transformed point, per candidate
    flop = sum((3.0 * len(src) * T[tid].m + 18.0 * len(src)) * 36864 for tid, src in reqs)
    if args.latency_dump:
        with open(args.latency_dump, "w") as f:
            json.dump({"arrival_s": [float(a) for a in arrivals], "plain_s": lat_plain,
                       "served_s": lat_served, "plain_service_s": svc_plain,
                       "n": [len(s) for _, s in reqs[:n_req]],
                       "m": [T[t].m for t, _ in reqs[:n_req]]}, f)
    pct = lambda a, q: float(np.percentile(np.array(a) * 1e3, q))  # noqa: E731
    return {"metric": "registration latency p50/p99, served vs plain (1 GPU)",
            "value": cands / served_wall, "unit": "candidates/s", "n_gpus": 1,
            "steps": n_req, "warmup": 8, "ms_per_step": served_wall / n_req * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32 vote, f32 score",
            "data": "synthetic",
            "config": {"workload": f"{n_req} Poisson requests (rate 0.8x plain capacity = "
                                   f"{rate:.2f}/s) vs 8 resident references with 128^3 "
                                   "distance fields, 36,864 rotations each, DF scoring",
                       "aging": args.aging, "slice_mpairs": args.slice_mpairs},
            "served": {"p50_ms": pct(lat_served, 50), "p99_ms": pct(lat_served, 99),
                       "mean_ms": float(np.mean(lat_served)) * 1e3,
                       "mean_admission_wait_ms": float(np.mean(queue_served)) * 1e3,
                       "throughput": cands / served_wall},
            "plain": {"p50_ms": pct(lat_plain, 50), "p99_ms": pct(lat_plain, 99),
                      "mean_ms": float(np.mean(lat_plain)) * 1e3,
                      "mean_service_ms": float(np.mean(svc_plain)) * 1e3,
                      "throughput": cands / plain_wall, "path": "one launch per request, FIFO"},
            "saturation": {"served": cands / sat_served, "plain": cands / sat_plain,
                           "unit": "candidates/s",
                           "served_frac_of_fp32_peak": flop / sat_served / 1e12
                           / PEAK_FP32_VECTOR_TFLOPS,
                           "plain_frac_of_fp32_peak": flop / sat_plain / 1e12
                           / PEAK_FP32_VECTOR_TFLOPS,
                           "work": "algorithmic (3*N*M + 18*N) FLOP per candidate (DF "
                                   "scoring), whole run",
                           "path": "closed loop: every request outstanding at once"}}


def bench_plain(args, workload, steps, warmup, cpu_sample, scorer="auto", q=0.0):
    """Timed single-registration steps of one workload (inputs resident on the
    device), with the sweep kernel's HIP-event time and the roofline position."""
    import numpy as np
    import torch
    from paper_2502_00115_amd import dses

    p, desc = make_workload(workload, getattr(args, "grid_level", 4))
    dev = torch.device("cuda:0")
    src = torch.from_numpy(p.src).to(dev)
    tgt = torch.from_numpy(p.tgt).to(dev)
    rot = torch.from_numpy(p.rotations).to(dev)
    n, m, k = len(p.src), len(p.tgt), len(p.rotations)

    box = p.meta.get("t_box")
    if box is not None:                  # a local search: the box of the initial guess
        box_kw = {"t_min": -box, "t_max": box}
    else:
        box_kw = {}
    if scorer == "df":
        # distance-field scoring needs the reference resident with its 128^3 field
        target = dses.Target(tgt, df_trunc=p.eps, df_res=128)
        rotset = dses.RotationSet(rot)

        def run(**kw):
            return dses.register_resident(target, rotset, src, p.eps, scorer="df", q=q,
                                          **box_kw, **kw)
    else:
        def run(**kw):
            return dses.register(src, tgt, rot, p.eps, scorer=scorer, q=q, **box_kw, **kw)
    for w in range(warmup):
        ts = time.perf_counter()
        run()
        torch.cuda.synchronize()
        if time.perf_counter() - ts > 2.0:
            print(f"bench.py: {workload} warm-up {w + 1}/{warmup} "
                  f"{time.perf_counter() - ts:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dses.kernel_stats(reset=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        ts = time.perf_counter()
        r = run(timing=True)
        lat.append(time.perf_counter() - ts)
        if lat[-1] > 2.0:
            print(f"bench.py: {workload} step {step + 1}/{steps} {lat[-1]:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = dses.kernel_stats()

    sweep_ms = st["vote_score_ms"] / max(1, st["vote_score_launches"])
    # algorithmic work per candidate: 3 FLOP per vote pair, 8 per brute-force score pair,
    # 18 per transformed point; distance-field scoring replaces the score pairs by
    # one lookup per point
    score_pairs = 0.0 if scorer == "df" else 8.0 * n * m
    scored = k
    if q > 0.0:                          # pruning: every rotation voted, the kept ones scored
        scored = int(np.isfinite(run(records=True).records["error"]).sum())
    flop_per_launch = (3.0 * n * m + 18.0 * n) * k + score_pairs * scored
    achieved = flop_per_launch / (sweep_ms * 1e-3) / 1e12
    # the counters were taken on the default configuration of the workload (every
    # rotation scored, automatic scorer); other configurations run other kernels
    full = workload != "c5" or getattr(args, "grid_level", 4) == 4
    traffic = load_traffic(workload) if q == 0.0 and scorer == "auto" and full else None
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "candidate poses {R,t} scored/sec (1 GPU) + p50/p99 registration latency, "
                  "served vs plain",
        "value": k * steps / elapsed,
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32 vote, f32 score",
        "data": "synthetic",
        "config": {"workload": desc, "n_src": n, "n_ref": m, "rotations": k, "eps": p.eps,
                   "metric": "trunc_l2", "scorer": scorer, "q": q,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)), "path": "plain, one call"},
        "roofline": {"bound": "alu", "kernel": "k_sweep (vote + mode + score)",
                     "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "work": ("algorithmic (3*N*M + 18*N) FLOP per candidate (DF scoring)"
                              if scorer == "df" else
                              "algorithmic (11*N*M + 18*N) FLOP per candidate"),
                     "kernel_ms": sweep_ms},
        "result": {"rot_index": r.rot_index, "inliers": r.inliers, "error": r.error,
                   "rot_err_deg": float(np.rad2deg(np.arccos(np.clip(
                       (np.trace(r.R.astype(np.float64).T @ p.R_true) - 1.0) / 2.0, -1.0, 1.0)))),
                   "t_err": float(np.linalg.norm(r.t.astype(np.float64) - p.t_true))},
    }
    if q > 0.0:
        out["result"]["scored"] = scored
        out["roofline"]["work"] += " (q > 0: score pairs only for the scored rotations)"
    if cpu_sample != 0:
        threads = min(16, len(os.sched_getaffinity(0)))
        sample = cpu_sample if cpu_sample > 0 else max(16, int(2.2e10 / (n * m)))
        print(f"bench.py: oracle CPU baseline on {min(sample, k)} rotations", file=sys.stderr,
              flush=True)
        out["cpu_baseline"] = cpu_baseline(p, sample, threads)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=WORKLOADS, default="c5")
    ap.add_argument("--scorer", default="auto")
    ap.add_argument("--grid-level", type=int, default=4, choices=(0, 1, 2, 3, 4),
                    help="c5: Hopf grid level of the rotation list (4: 294,912 rotations, the "
                         "workload; lower levels are samples for profiling)")
    ap.add_argument("--q", type=float, default=0.0,
                    help="pruning of Alg. 2: score only rotations with M_k >= q M* (0: all)")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="rotations of the oracle CPU baseline (-1: as many as about "
                         "2.2e10 point pairs, some 10-30 s on 16 cores; 0: skip)")
    ap.add_argument("--requests", type=int, default=200, help="c4: measured requests")
    ap.add_argument("--aging", type=float, default=0.0,
                    help="c4: server priority aging (0: library default)")
    ap.add_argument("--latency-dump", default=None,
                    help="c4: write per-request arrival, plain and served latency (JSON)")
    ap.add_argument("--slice-mpairs", type=int, default=0,
                    help="c4: server work per slice, millions of pairs (0: library default)")
    ap.add_argument("--alone", action="store_true",
                    help="the headline workload only (no serving or object-scale figures)")
    ap.add_argument("--lds-probe", action="store_true",
                    help="print the device's LDS atomic throughput (vote ceiling) and exit")
    ap.add_argument("--write-traffic", nargs=4, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic_k_sweep_<workload>.json from rocprofv3 "
                         "counter CSVs (no GPU work)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain elementwise copy of 256 MiB (counter calibration)")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.workload, *args.write_traffic)
        return
    if args.calibrate_copy:
        import torch
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch.add(a, 1.0, out=b)", "bytes_read": 4 * a.numel(),
                          "bytes_written": 4 * b.numel()}), flush=True)
        return
    if args.lds_probe:
        from paper_2502_00115_amd import dses
        print(json.dumps({"lds_atomics": {pat: dses.measure_lds_atomics(pat)
                                          for pat in ("conflict_free", "random")}}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the sweep "
              "would shard by rotation, one slice of the rotation list per GPU, which is "
              "not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c3":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "fig2":
        print(json.dumps(bench_fig2(args)), flush=True)
        return
    if args.workload == "exhaustive":
        print(json.dumps(bench_exhaustive(args)), flush=True)
        return
    out = bench_plain(args, args.workload, args.steps, args.warmup, args.cpu_sample,
                      args.scorer, args.q)
    if (args.workload == "c5" and not args.alone and args.scorer == "auto" and args.q == 0.0
            and args.grid_level == 4):
        # the metric's second half: served vs plain latency on the serving workload
        sv = bench_serve(args, n_req=min(args.requests, 100))
        out["served_vs_plain"] = {"workload": sv["config"]["workload"],
                                  "served": sv["served"], "plain": sv["plain"],
                                  "saturation": sv["saturation"]}
        # the object-scale registration (its own line with --workload c2)
        c2 = bench_plain(args, "c2", 10, 2, 0)
        out["object_scale"] = {"workload": c2["config"]["workload"], "value": c2["value"],
                               "unit": c2["unit"], "ms_per_step": c2["ms_per_step"],
                               "latency_ms": c2["latency_ms"], "roofline": c2["roofline"],
                               "result": c2["result"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
