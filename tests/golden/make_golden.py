"""Write the stored oracle values used by the tests and the benchmark.

Calls only `oracle/` (and the seeded generator `synth/`); nothing here comes from
the HIP path.  Outputs (JSON, floats written with repr so they round-trip):

  calib.json           per architecture: the affine output calibration that maps
                       the oracle scores of that config's first 64 poses to
                       mean 6.0 / std 1.5 pK (so a bound in pK units means
                       something for random weights)
  <cfg>_G<G>_oracle.json  per pose: oracle centre, CNN latent, SG latent and
                       calibrated score, for poses [0, n) of a workload config

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
    with get_context("spawn").Pool(a.workers) as pool:
        rows = sorted(pool.map(_latents, [(a.cfg, a.G, p, arch_name) for p in range(a.n)], chunksize=1))
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
    out = dict(config=a.cfg, G=a.G, arch=arch_name, seed_poses=0, seed_weights=1,
               calibration=calib[arch_name], poses=[])
    for (p, c, cnn, sg, ecov, enc) in rows:
        s = oracle.fusion_head(np.array(cnn), np.array(sg), cw, arch)
        out["poses"].append(dict(pose=p, center=c, cnn_lat=cnn, sg_lat=sg, score=float(s),
                                 n_cov_edges=ecov, n_nc_edges=enc))
    tag = "" if arch_name == synth.CONFIGS[a.cfg]["arch"] else f"_{arch_name}"
    path = os.path.join(HERE, f"{a.cfg}_G{a.G}{tag}_oracle.json")
    json.dump(out, open(path, "w"))
    print(f"wrote {path} ({a.n} poses) in {time.time() - t0:.1f}s")


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
