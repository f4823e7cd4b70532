"""Write the stored oracle values used by the tests and the benchmark.

Calls only `oracle/` (and the seeded generator `synth/`); nothing here comes from
the HIP path.  Outputs (JSON, floats written with repr so they round-trip):

  calib.json           per architecture: the affine output calibration that maps
                       the oracle scores of that config's first 64 poses to
                       mean 6.0 / std 1.5 pK (so a bound in pK units means
                       something for random weights)
  <cfg>_G<G>_oracle.json  per pose: oracle centre, CNN latent, SG latent and
                       calibrated score, for poses [0, n) of a workload config

  <cfg>_G<G>_scores.json calibrated oracle scores (and edge counts) of poses
                       [0, n) when only the first --latents of them are
                       stored with their latents

Usage:  python tests/golden/make_golden.py c1 24 64
        python tests/golden/make_golden.py c2 48 64 --calibrate
        python tests/golden/make_golden.py c4 32 8
        python tests/golden/make_golden.py c2 48 64 --arch paper --calibrate
            (the paper-shaped model on the config's poses)
        python tests/golden/make_golden.py c2 48 64 --head-arch full_mid
            (calibration only, for an architecture that shares the config's trunk
             -- same conv / SG-CNN weights, another fusion head -- computed from
             the stored oracle latents of that config)
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def _latents(args):
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    import numpy as np
    import oracle
    import synth
    cfg, G, p, arch_name = args
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    b = synth.make_poses(cfg, 1, pose0=p, threads=1)
    lig = b.is_lig.astype(bool)
    c = oracle.pose_center(b.xyz[lig])
    grid = oracle.splat_pose(b.xyz, b.feat, c, G)
    cnn, _ = oracle.cnn3d_forward(grid, w, arch)
    cov = oracle.radius_graph_pose(b.xyz, arch.r_cov_u)
    nc = oracle.radius_graph_pose(b.xyz, arch.r_nc_u)
    sg = oracle.sgcnn_pose(b.feat, b.is_lig, cov, nc, w, arch)
    return p, [int(v) for v in c], [float(v) for v in cnn], [float(v) for v in sg], int(cov[0][-1]), int(nc[0][-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cfg")
    ap.add_argument("G", type=int)
    ap.add_argument("n", type=int)
    ap.add_argument("--calibrate", action="store_true")
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--head-arch", default=None)
    ap.add_argument("--arch", default=None, help="another architecture on the config's poses")
    ap.add_argument("--latents", type=int, default=None,
                    help="store latents for the first this many poses; scores of all n go to _scores.json")
    ap.add_argument("--cache", default=None, help="append-only JSONL of computed rows (resumable runs)")
    a = ap.parse_args()
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    import numpy as np
    import oracle
    import synth

    if a.head_arch:
        calibrate_head(a.cfg, a.G, a.head_arch)
        return

    t0 = time.time()
    arch_name = a.arch or synth.CONFIGS[a.cfg]["arch"]
    tag = "" if arch_name == synth.CONFIGS[a.cfg]["arch"] else f"_{arch_name}"
    path = os.path.join(HERE, f"{a.cfg}_G{a.G}{tag}_oracle.json")
    have = {}
    if a.latents is not None and os.path.exists(path):   # rows stored earlier by this script
        for r in json.load(open(path))["poses"]:
            have[r["pose"]] = (r["pose"], r["center"], r["cnn_lat"], r["sg_lat"], r["n_cov_edges"], r["n_nc_edges"])
    if a.cache and os.path.exists(a.cache):
        for line in open(a.cache):
            r = json.loads(line)
            if r[0] < a.n:
                have[r[0]] = tuple(r)
    todo = [p for p in range(a.n) if p not in have]
    print(f"{len(have)} rows known, {len(todo)} to compute", flush=True)
    with get_context("spawn").Pool(a.workers) as pool:
        cache = open(a.cache, "a") if a.cache else None
        for i, r in enumerate(pool.imap_unordered(_latents, [(a.cfg, a.G, p, arch_name) for p in todo])):
            have[r[0]] = r
            if cache:
                cache.write(json.dumps(r) + "\n")
                cache.flush()
            if (i + 1) % 64 == 0:
                print(f"{i + 1}/{len(todo)} poses in {time.time() - t0:.0f}s", flush=True)
    rows = [have[p] for p in range(a.n)]
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    calib_path = os.path.join(HERE, "calib.json")
    calib = json.load(open(calib_path)) if os.path.exists(calib_path) else {}
    if a.calibrate or arch_name not in calib:
        assert a.n >= 64, "calibration uses the config's first 64 poses"
        raw = np.array([oracle.fusion_head(np.array(r[2]), np.array(r[3]), w, arch) for r in rows[:64]])
        scale = 1.5 / raw.std()
        shift = 6.0 - raw.mean() * scale
        calib[arch_name] = dict(scale=float(scale), shift=float(shift), raw_mean=float(raw.mean()),
                                raw_std=float(raw.std()), source=f"{a.cfg} poses 0..63, G={a.G}")
        json.dump(calib, open(calib_path, "w"), indent=1)
    cw = synth.apply_calibration(w, calib[arch_name]["scale"], calib[arch_name]["shift"])
    n_lat = a.n if a.latents is None else min(a.latents, a.n)
    out = dict(config=a.cfg, G=a.G, arch=arch_name, seed_poses=0, seed_weights=1,
               calibration=calib[arch_name], poses=[])
    scores = dict(config=a.cfg, G=a.G, arch=arch_name, seed_poses=0, seed_weights=1,
                  calibration=calib[arch_name], score=[], n_cov_edges=[], n_nc_edges=[])
    for (p, c, cnn, sg, ecov, enc) in rows:
        s = float(oracle.fusion_head(np.array(cnn), np.array(sg), cw, arch))
        if p < n_lat:
            out["poses"].append(dict(pose=p, center=c, cnn_lat=cnn, sg_lat=sg, score=s,
                                     n_cov_edges=ecov, n_nc_edges=enc))
        scores["score"].append(s)
        scores["n_cov_edges"].append(ecov)
        scores["n_nc_edges"].append(enc)
    json.dump(out, open(path, "w"))
    print(f"wrote {path} ({n_lat} poses) in {time.time() - t0:.1f}s")
    if a.latents is not None:
        spath = os.path.join(HERE, f"{a.cfg}_G{a.G}{tag}_scores.json")
        json.dump(scores, open(spath, "w"))
        print(f"wrote {spath} ({a.n} poses)")


def calibrate_head(cfg, G, head_arch):
    import numpy as np
    import oracle
    import synth
    base = synth.ARCHS[synth.CONFIGS[cfg]["arch"]]
    arch = synth.ARCHS[head_arch]
    wb, w = synth.make_weights(base), synth.make_weights(arch)
    trunk = [k for k in wb if not k.startswith("fusion.")]
    assert all(k in w and np.array_equal(wb[k], w[k]) for k in trunk), "architecture does not share the trunk"
    rows = json.load(open(os.path.join(HERE, f"{cfg}_G{G}_oracle.json")))["poses"][:64]
    assert len(rows) == 64
    raw = np.array([oracle.fusion_head(np.array(r["cnn_lat"]), np.array(r["sg_lat"]), w, arch) for r in rows])
    calib_path = os.path.join(HERE, "calib.json")
    calib = json.load(open(calib_path))
    scale = 1.5 / raw.std()
    calib[head_arch] = dict(scale=float(scale), shift=float(6.0 - raw.mean() * scale), raw_mean=float(raw.mean()),
                            raw_std=float(raw.std()), source=f"{cfg} poses 0..63, G={G}, stored oracle latents")
    json.dump(calib, open(calib_path, "w"), indent=1)
    print(f"calibrated {head_arch}: {calib[head_arch]}")


if __name__ == "__main__":
    main()
