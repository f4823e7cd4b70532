#!/usr/bin/env python3
"""Throughput benchmark of Coherent Fusion pose scoring on one MI355X.

Workload: 4096 synthetic docked poses (ligands of 20-60 atoms, pockets of
400-900 atoms), 48^3 grids at 1 A, the full-size model (3D-CNN with k=7 convs,
64/128 channels and two residual blocks; SG-CNN with H=64, 3 + 3 gated rounds;
74 -> 64 -> 1 SELU fusion head).  One step = one cf_score_poses call over the
whole batch: centres, voxelisation, conv stack, pooling, neighbour lists,
SG-CNN and fusion head, with inputs already resident in HBM.

Reported: poses/s of the precision form (bfloat16 MFMA, float32 accumulation,
batched 512 poses per launch), the plain float32 path on the same poses, score
error of both against stored FP64 oracle scores, the roofline position of the
dominant kernel (conv3d, timed with HIP events on its own stream) and the FP64
CPU oracle timed on a bounded sample on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2516.6   # MI355X dense bf16 MFMA
PEAK_FP32_TFLOPS = 157.3    # MI355X fp32 (matrix and vector)
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_golden(cfg, G, tag=""):
    path = os.path.join(ROOT, "tests", "golden", f"{cfg}_G{G}{tag}_oracle.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path))


def load_scores(cfg, G, tag=""):
    """Stored oracle scores of poses [0, n): every pose of the scores file when the
    generator wrote one, else the poses stored with their latents."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{cfg}_G{G}{tag}_scores.json")
    if os.path.exists(path):
        return np.array(json.load(open(path))["score"], np.float64)
    gd = load_golden(cfg, G, tag)
    return None if gd is None else np.array([p["score"] for p in gd["poses"]], np.float64)


def provenance(batch, arch, w, seed_poses=0):
    """What the run read: SHA-256 of the pose arrays and of the model blob, the
    seeds, the library file and the host, so that a line can be matched to its inputs."""
    import hashlib
    import platform
    from paper_2104_04547_amd import cfabi
    h = hashlib.sha256()
    for arr in (batch.atom_off, batch.xyz, batch.feat, batch.is_lig):
        h.update(memoryview(arr).cast("B"))
    lib = cfabi.LIB_PATH
    return {"inputs_sha256": h.hexdigest(),
            "weights_sha256": hashlib.sha256(cfabi.pack_model(arch, w)).hexdigest(),
            "library_sha256": hashlib.sha256(open(lib, "rb").read()).hexdigest() if os.path.exists(lib) else None,
            "seed_poses": seed_poses, "seed_weights": 1, "host": platform.node(), "host_cpus": os.cpu_count(),
            "time_utc": time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime())}


ROCTX = False  # --roctx: stage ranges for a tracer around every scoring call


def time_steps(scorer, db, G, steps, warmup, out, timing=False):
    import torch
    from paper_2104_04547_amd import cfabi
    cfabi.cf_timing_enable(scorer.ctx, False, roctx=ROCTX)
    for _ in range(warmup):
        scorer.score(db, G, out)
    torch.cuda.synchronize()
    rc = scorer.status()[0]
    if rc != 0:
        raise RuntimeError(f"device status {rc}: {cfabi.cf_last_error()}")
    if timing:
        cfabi.cf_timing_read(scorer.ctx)          # drop warm-up entries
        cfabi.cf_timing_enable(scorer.ctx, True, roctx=ROCTX)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        scorer.score(db, G, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = None
    if timing:
        stats = cfabi.cf_timing_read(scorer.ctx)
        cfabi.cf_timing_enable(scorer.ctx, False, roctx=ROCTX)
    rc = scorer.status()[0]
    if rc != 0:
        raise RuntimeError(f"device status {rc}: {cfabi.cf_last_error()}")
    return (t1 - t0) / steps, stats


def by_kernel(stats):
    """Merge per-layer conv entries ("conv<i>.<variant>") by kernel variant."""
    out = {}
    for k, v in stats.items():
        key = "conv." + k.split(".", 1)[1] if k.startswith("conv") else k
        e = out.setdefault(key, dict(launches=0, total_ms=0.0, flop=0.0, bytes=0.0))
        for f in e:
            e[f] += v[f]
    return out


def error_stats(got, want, n):
    import numpy as np
    want = np.asarray(want[:n], np.float64)
    err = np.abs(np.asarray(got[:n], dtype=np.float64) - want)
    rel = err / np.maximum(1.0, np.abs(want))
    return dict(n_poses=int(n), max_abs_pk=float(err.max()), mean_abs_pk=float(err.mean()),
                max_rel=float(rel.max()))


def cnn_latent_error(scorer, batch, gd, G, n):
    """CNN-branch latents through cf_voxelize + cf_cnn3d_fwd vs the oracle's."""
    import numpy as np
    from paper_2104_04547_amd import cfabi
    sub = batch.select(list(range(n)))
    db = cfabi.DeviceBatch.from_pose_batch(sub)
    lat = scorer.cnn3d(scorer.voxelize(db, G), G).cpu().numpy().astype(np.float64)
    want = np.array([p["cnn_lat"] for p in gd["poses"][:n]])
    return float(np.abs(lat - want).max() / np.abs(want).max())


def kernel_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed counter summary
    (profiles/traffic.json: FETCH_SIZE + WRITE_SIZE per dispatch, scaled by a plain
    copy's reading), or None when there is none for this kernel or its source file
    has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path)).get(kernel)
    if not t:
        return None
    src = os.path.join(ROOT, "paper_2104_04547_amd", "csrc", t["source"])
    if not os.path.exists(src) or t.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return round(t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"], 0)


def _cpu_worker(args):
    """One process of the CPU baseline: its share of the poses, one BLAS thread."""
    os.environ["OPENBLAS_NUM_THREADS"] = os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import oracle
    import synth
    from threadpoolctl import threadpool_limits
    cfg, poses, arch_name, calib, G = args
    arch = synth.ARCHS[arch_name]
    w = synth.apply_calibration(synth.make_weights(arch), calib["scale"], calib["shift"])
    out = []
    with threadpool_limits(1):
        for p in poses:
            b = synth.make_poses(cfg, 1, pose0=p, threads=1)
            t0 = time.perf_counter()
            oracle.score_pose(b.xyz, b.feat, b.is_lig, w, arch, G)
            out.append(time.perf_counter() - t0)
    return out


def cpu_baseline(cfg, arch_name, calib, G, n, workers):
    """The FP64 oracle as it stands, poses in parallel over this host's cores: the
    first n poses of the workload, one pose per process at a time, each process on
    one BLAS thread; plus the single-thread rate from the same per-pose times."""
    import multiprocessing as mp
    workers = max(1, min(workers, n))
    shares = [list(range(i, n, workers)) for i in range(workers)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_cpu_worker, [(cfg, [0], arch_name, calib, 24)] * workers)   # imports and page-in, untimed
        t0 = time.perf_counter()
        per_pose = sum(pool.map(_cpu_worker, [(cfg, sh, arch_name, calib, G) for sh in shares]), [])
        dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="poses/s", cores=int(workers), kind="oracle",
                sample=f"first {n} of the workload's poses, full path per pose (splat, conv stack, graphs, "
                       f"SG-CNN, fusion) in float64 numpy, {workers} processes of one thread each; {dt:.1f} s",
                value_1core=len(per_pose) / sum(per_pose),
                sample_1core=f"mean time per pose of the same {n} poses on one thread; "
                             f"{sum(per_pose) / len(per_pose):.2f} s each",
                seconds=dt)


def batching_leg(arch, w, n_poses, steps):
    """Batching form: ragged poses whose total atom counts are log-uniform in
    [200, 1500], packed CSR-style and scored 512 per launch in the precision form,
    with the conv variants autotuned per grid size (32^3, 48^3, 64^3)."""
    import numpy as np
    import torch
    import synth
    from paper_2104_04547_amd import Scorer, cfabi
    t0 = time.perf_counter()
    batch = synth.make_poses("c4", n_poses)
    log(f"batching: generated {n_poses} poses ({batch.n_atoms} atoms) in {time.perf_counter() - t0:.1f}s")
    db = cfabi.DeviceBatch.from_pose_batch(batch)
    out = torch.empty(n_poses, dtype=torch.float32, device="cuda")
    s = Scorer(arch, w, "bf16")
    res = {}
    try:
        for G in (32, 48, 64):
            t0 = time.perf_counter()
            v = s.autotune(G, 512)
            tune_s = time.perf_counter() - t0
            sec, _ = time_steps(s, db, G, steps, 1, out)
            r = dict(poses_per_s=round(n_poses / sec, 2), ms_per_step=round(sec * 1e3, 3), conv_variants=v,
                     autotune_s=round(tune_s, 2),
                     conv_tflops=round(arch.flops_per_pose(G) * n_poses / sec / 1e12, 1))
            want = load_scores("c4", G)
            if want is not None:
                r["error"] = error_stats(out.cpu().numpy().astype(np.float64), want, min(len(want), n_poses))
            res[f"G{G}"] = r
            log(f"batching G={G}: {r['poses_per_s']:.1f} poses/s, variants {v}, tuned in {tune_s:.1f}s")
    finally:
        s.close()
    return dict(poses=n_poses, atoms=int(batch.n_atoms), steps=steps, **res)


def paper_leg(db, n_poses, steps):
    """The paper-shaped model (Sec. 3.3.1, Tables II, III, V) on the same poses:
    both forms, conv variants autotuned, error against its stored oracle scores."""
    import numpy as np
    import torch
    import synth
    from paper_2104_04547_amd import Scorer
    arch = synth.ARCHS["paper"]
    w = synth.make_weights(arch)
    calib = json.load(open(os.path.join(ROOT, "tests", "golden", "calib.json")))["paper"]
    w = synth.apply_calibration(w, calib["scale"], calib["shift"])
    want = load_scores("c2", 48, "_paper")
    out = torch.empty(n_poses, dtype=torch.float32, device="cuda")
    res = {}
    for prec in ("bf16", "fp32"):
        s = Scorer(arch, w, prec)
        try:
            v = s.autotune(48, 512)
            sec, stats = time_steps(s, db, 48, steps, 1, out, timing=True)
            r = dict(poses_per_s=round(n_poses / sec, 2), ms_per_step=round(sec * 1e3, 3), conv_variants=v)
            st = by_kernel(stats)
            conv_ms = sum(x["total_ms"] for k, x in st.items() if k.startswith("conv"))
            r["conv_share"] = round(conv_ms / sum(x["total_ms"] for x in st.values()), 4)
            r["sgcnn_ms_per_step"] = round(st["sgcnn"]["total_ms"] / steps, 3)
            if want is not None:
                r["error"] = error_stats(out.cpu().numpy().astype(np.float64), want, min(len(want), n_poses))
            res[prec] = r
            log(f"paper model {prec}: {r['poses_per_s']:.1f} poses/s, variants {v}, error {r.get('error')}")
        finally:
            s.close()
    return res


def backward_leg(db, batch, arch, w, G, n_poses, steps):
    """Backward pass for fine-tuning (cf_backward, plain form): gradients of the squared
    error (s - y)^2 / 2 against synthetic labels y = 6 pK for every parameter, over the
    first n_poses poses of the workload."""
    import numpy as np
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    sub = cfabi.DeviceBatch.from_pose_batch(batch.select(list(range(n_poses))))
    s = Scorer(arch, w, "fp32")
    try:
        scores = s.score(sub, G)
        dscore = (scores - 6.0).contiguous()                    # d/ds of (s - y)^2 / 2 with y = 6
        g, _ = s.backward(sub, G, dscore)                        # warm-up (allocates scratch)
        s.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g, sc = s.backward(sub, G, dscore)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        s.check()
        gn = float(torch.linalg.vector_norm(g).item())
    finally:
        s.close()
    return dict(poses=n_poses, grid=G, steps=steps, ms_per_call=round(dt * 1e3, 3),
                poses_per_s=round(n_poses / dt, 2), grad_norm=gn,
                what="scores + gradients of every parameter (3D-CNN, SG-CNN, fusion head), float32")


def serve_leg(arch, w, res, seconds, stream_poses=0):
    """Open-loop Poisson serving: requests of U{1..256} poses (200-1500 atoms),
    grid 48^3 or 64^3 per request, continuous batching on 4 slots with hipGraph
    replay.  Each form's capacity on this request mix is measured first (a burst
    of requests, closed loop); then both forms run at equal load -- 0.7 x the
    plain form's capacity -- and the precision form also at 0.7 x its own
    (stream_poses > 0: that run streams about that many poses instead of
    `seconds` of arrivals)."""
    import numpy as np
    import synth
    from paper_2104_04547_amd.serve import Engine, make_requests, run_open_loop, warm_up
    mean_req = 128.5
    t0 = time.perf_counter()
    pool = synth.make_poses("c5", 2048)
    log(f"serving pool: {pool.n_poses} poses in {time.perf_counter() - t0:.1f}s")
    f48, f64 = arch.flops_per_pose(48), arch.flops_per_pose(64)
    mix = 2.0 / (1.0 + f64 / f48)            # rough capacity at the 48/64 mix relative to 48^3
    out = {}
    engines = {}
    cap = {}
    try:
        for prec in ("bf16", "fp32"):
            engines[prec] = Engine(arch, w, prec, n_slots=4, slot_poses=512, slot_atoms=512 * 1600,
                                   hbm_budget_bytes=64 << 30)
            t0 = time.perf_counter()
            warm_up(engines[prec], pool)
            log(f"serving {prec}: graphs captured in {time.perf_counter() - t0:.1f}s")
            # capacity: a burst sized for ~8 s of work at the rough estimate
            n_req = int(min(400, max(12, 8.0 * res[prec]["poses_per_s"] * mix / mean_req)))
            reqs = make_requests(pool, n_req, np.random.default_rng(5))
            t0 = time.perf_counter()
            tickets = [(engines[prec].submit(b, G), b.n_poses) for b, G in reqs]
            for t, n in tickets:
                engines[prec].result(t, n)
            dt = time.perf_counter() - t0
            cap[prec] = sum(n for _, n in tickets) / dt
            out[f"{prec}_capacity_poses_per_s"] = round(cap[prec], 2)
            log(f"serving {prec}: capacity {cap[prec]:.1f} poses/s on this mix ({n_req} requests in {dt:.1f}s)")
        runs = [("bf16", 0.7 * cap["fp32"], "equal_load"), ("fp32", 0.7 * cap["fp32"], "equal_load"),
                ("bf16", 0.7 * cap["bf16"], "own_capacity")]
        for prec, poses_rate, tag in runs:
            rps = poses_rate / mean_req
            n_req = max(20, int(rps * seconds))
            if stream_poses and tag == "own_capacity":
                n_req = max(20, int(stream_poses / mean_req))
            reqs = make_requests(pool, n_req, np.random.default_rng(7))
            r = run_open_loop(engines[prec], reqs, rps, seed=11)
            r["offered_poses_per_s"] = poses_rate
            r.update(engines[prec].info())
            out[f"{prec}_{tag}"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}
            log(f"serving {prec} {tag}: {r['poses_per_s']:.1f} poses/s, p50 {r['p50_ms']:.1f} ms, "
                f"p99 {r['p99_ms']:.1f} ms over {r['requests']} requests")
    finally:
        for e in engines.values():
            e.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--poses", type=int, default=4096)
    ap.add_argument("--G", type=int, default=48)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--cpu-poses", type=int, default=48)
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=25.0)
    ap.add_argument("--serve-poses", type=int, default=0,
                    help="stream about this many poses in the precision form's own-capacity run")
    ap.add_argument("--batch-poses", type=int, default=32768)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--backward-poses", type=int, default=64)
    ap.add_argument("--backward-steps", type=int, default=2)
    ap.add_argument("--paper-steps", type=int, default=3)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 10 device copies of MIB MiB (calibrates HBM byte counters) and exit")
    ap.add_argument("--json-out", default="")
    ap.add_argument("--roctx", action="store_true",
                    help="roctx ranges around each chunk's stages (for rocprofv3 --marker-trace)")
    ap.add_argument("--run-log", default="", metavar="PATH",
                    help="append the result line, with its provenance, to this JSONL file")
    a = ap.parse_args()
    global ROCTX
    ROCTX = a.roctx

    if a.gpus != 1:
        print(f"bench.py measures one GPU: the library scores poses on a single MI355X and has no "
              f"multi-GPU path (asked for --gpus {a.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2104_04547_amd import Scorer, cfabi

    if a.copy_probe:
        n = a.copy_probe << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 10 copies of {n} bytes")
        return

    cfg = "c2"
    G = a.G
    arch = synth.ARCHS["full"]
    w = synth.make_weights(arch)
    calib = json.load(open(os.path.join(ROOT, "tests", "golden", "calib.json")))["full"]
    w = synth.apply_calibration(w, calib["scale"], calib["shift"])

    t0 = time.perf_counter()
    batch = synth.make_poses(cfg, a.poses)
    log(f"generated {a.poses} poses ({batch.n_atoms} atoms) in {time.perf_counter() - t0:.1f}s")
    db = cfabi.DeviceBatch.from_pose_batch(batch)
    torch.cuda.synchronize()
    out = torch.empty(a.poses, dtype=torch.float32, device="cuda")

    res = {}
    variants = {}
    for prec, steps, warm in (("bf16", a.steps, a.warmup), ("fp32", a.fp32_steps, 1)):
        if prec == "fp32" and a.no_fp32:
            continue
        s = Scorer(arch, w, prec)
        if not a.no_autotune:
            t0 = time.perf_counter()
            v = s.autotune(G, 512)
            log(f"{prec}: autotuned conv variants {v} in {time.perf_counter() - t0:.1f}s")
        variants[prec] = s.variants(G)
        sec, stats = time_steps(s, db, G, steps, warm, out, timing=True)
        scores = out.cpu().numpy().astype(np.float64)
        res[prec] = dict(sec_per_step=sec, poses_per_s=a.poses / sec, stats=stats, scores=scores)
        log(f"{prec}: {sec * 1e3:.1f} ms/step, {a.poses / sec:.1f} poses/s")
        gd = load_golden(cfg, G)
        want = load_scores(cfg, G)
        if want is not None:
            n = min(len(want), a.poses)
            res[prec]["error"] = error_stats(scores, want, n)
        if gd is not None:
            res[prec]["cnn_latent_max_rel_error"] = cnn_latent_error(s, batch, gd, G, min(len(gd["poses"]), 16))
            log(f"{prec}: error vs oracle {res[prec].get('error')}, "
                f"cnn latent rel {res[prec].get('cnn_latent_max_rel_error')}")
        s.close()

    # dominant kernel of the precision form: the kernel (one template instance,
    # possibly several layers) with the most device time, as a profiler groups it;
    # its bound follows from its algorithmic FLOP per byte against the ridge point
    st = by_kernel(res["bf16"]["stats"])
    total_ms = sum(v["total_ms"] for v in st.values())
    dom = max(st, key=lambda k: st[k]["total_ms"])
    d = st[dom]
    avg_ms = d["total_ms"] / d["launches"]
    flop_per_launch = d["flop"] / d["launches"]
    bytes_per_launch = d["bytes"] / d["launches"]
    mfma_bound = flop_per_launch > 0 and (bytes_per_launch == 0 or flop_per_launch / bytes_per_launch >
                                          PEAK_BF16_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9))
    if mfma_bound:
        achieved, peak, unit = flop_per_launch / (avg_ms * 1e-3) / 1e12, PEAK_BF16_TFLOPS, "TFLOP/s"
    else:
        achieved, peak, unit = bytes_per_launch / (avg_ms * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"
    conv_ms = sum(v["total_ms"] for k, v in st.items() if k.startswith("conv"))
    conv_flop = sum(v["flop"] for k, v in st.items() if k.startswith("conv"))
    breakdown = {k: dict(launches=v["launches"], ms_per_step=v["total_ms"] / a.steps,
                         share=v["total_ms"] / total_ms,
                         **({"tflops": v["flop"] / (v["total_ms"] * 1e-3) / 1e12} if v["flop"] else {}),
                         **({"gbs": v["bytes"] / (v["total_ms"] * 1e-3) / 1e9} if v["bytes"] and not v["flop"] else {}))
                 for k, v in sorted(st.items())}

    paper = None
    if not a.no_paper:
        paper = paper_leg(db, a.poses, a.paper_steps)

    backward = None
    if not a.no_backward:
        backward = backward_leg(db, batch, arch, w, G, a.backward_poses, a.backward_steps)
        log(f"backward (fp32): {backward['poses_per_s']:.1f} poses/s, {backward['ms_per_call']:.1f} ms per "
            f"{backward['poses']}-pose call")

    batching = None
    if not a.no_batching:
        batching = batching_leg(arch, w, a.batch_poses, a.batch_steps)

    serving = None
    if not a.no_serve and "fp32" in res:
        serving = serve_leg(arch, w, res, a.serve_seconds, a.serve_poses)

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(cfg, "full", calib, G, a.cpu_poses, a.cpu_workers)
        log(f"cpu oracle: {cpu['value']:.4f} poses/s on {cpu['cores']} threads, "
            f"{cpu.get('value_1core', float('nan')):.4f} poses/s on one")

    bf = res["bf16"]
    line = {
        "metric": "poses scored/sec, BF16 batched vs FP32 plain at stated pK error; p50/p99 latency",
        "value": round(bf["poses_per_s"], 2),
        "unit": "poses/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(bf["sec_per_step"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded docked-pose stand-ins, random He-normal weights with pK calibration)",
        "config": {
            "workload": f"4096 poses c2-shaped (ligand 20-60, pocket 400-900 atoms), {G}^3 grid, full model, "
                        f"512 poses per launch",
            "poses": a.poses, "grid": G, "model": "coherent-fusion full (3D-CNN k7 64/128 + 2 res blocks, "
                                                 "SG-CNN H64 3+3 rounds, fusion 74-64-1)",
            "conv_variants_bf16": variants.get("bf16"), "conv_variants_fp32": variants.get("fp32"),
        },
        "roofline": {
            "bound": "mfma" if mfma_bound else "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4), "traffic": kernel_traffic(dom),
            "avg_launch_ms": round(avg_ms, 4), "flop_per_launch": flop_per_launch,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "conv_stack_tflops": round(conv_flop / (conv_ms * 1e-3) / 1e12, 2),
            "conv_share_of_step": round(conv_ms / total_ms, 4),
        },
        "cpu_baseline": None if cpu is None else {k: (round(v, 6) if isinstance(v, float) else v)
                                                  for k, v in cpu.items() if k != "seconds"},
        "score_error_vs_oracle": {p: res[p].get("error") for p in res},
        "cnn_latent_max_rel_error": {p: res[p].get("cnn_latent_max_rel_error") for p in res},
        "kernels_bf16": breakdown,
    }
    if "fp32" in res:
        f = res["fp32"]
        fst = by_kernel(f["stats"])
        fdom = max((k for k in fst if k.startswith("conv")), key=lambda k: fst[k]["total_ms"])
        fd = fst[fdom]
        f_ach = fd["flop"] / (fd["total_ms"] * 1e-3) / 1e12
        line["fp32_plain"] = {"value": round(f["poses_per_s"], 2), "unit": "poses/s",
                              "ms_per_step": round(f["sec_per_step"] * 1e3, 3), "steps": a.fp32_steps,
                              "dominant_kernel": fdom, "achieved_tflops": round(f_ach, 2),
                              "frac_of_fp32_peak": round(f_ach / PEAK_FP32_TFLOPS, 4)}
        line["speedup_bf16_vs_fp32"] = round(bf["poses_per_s"] / f["poses_per_s"], 3)
    if paper is not None:
        line["paper_model"] = paper
    if batching is not None:
        line["batching"] = batching
    if backward is not None:
        line["backward"] = backward
    if serving is not None:
        line["serving"] = serving
    line["provenance"] = provenance(batch, arch, w)
    if a.json_out:
        json.dump(line, open(a.json_out, "w"), indent=1)
    if a.run_log:
        with open(a.run_log, "a") as fh:
            fh.write(json.dumps(line) + "\n")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
