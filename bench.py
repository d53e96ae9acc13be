"""Benchmark of the path tracer on one MI355X.

A step is one pt_render of the 1920x1080 icosphere-field scene
(1,310,722 triangles, 64 icospheres of level 5 on a ground plane, metal and
coated-diffuse materials, 2048x1024 sky with a 0.5 degree sun) at 64 spp and
max depth 8: camera rays, BVH closest hits, OpenPBR shading, next-event
estimation with MIS, Russian roulette and the FP64 per-pixel sums.
Inputs are resident in HBM before the timed region.

Prints one JSON line: Mrays/s (extension + shadow rays per second) with
samples/s beside it, the roofline of the closest-hit kernel measured live
with HIP events on the library's stream, and the FP64 oracle timed on the
host's cores on a bounded sample of the same workload.
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s and samples/s at 1080p; time-to-equal-RMSE, radiance cache vs plain"
HBM_PEAK_GBS = 8000.0
NODE_BYTES, TRI_BYTES, RAY_BYTES, HIT_BYTES = 128, 48, 32, 16


def kernel_source_hash() -> str:
    """sha256 over the HIP kernel sources (file name + bytes, sorted)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2407_19977_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(os.path.basename(p).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per k_extend launch from the committed counter summary, or
    None when the kernel sources changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_extend_spheres_1080p.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    t = re.search(r"^traffic_bytes_per_launch: (\d+)", txt, re.M)
    h = re.search(r"^kernel_source_sha256: ([0-9a-f]+)", txt, re.M)
    if not t or not h or h.group(1) != kernel_source_hash():
        return None
    return int(t.group(1))


def cpu_baseline(sc, spp_cpu=12, crop=(0, 0, 1920, 1080)):
    """The oracle as it stands, on a centre crop of the same scene."""
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = max(1, min(cores, 16))
    os_ = O.OracleScene(sc)
    t0 = time.perf_counter()
    r = os_.render(spp_cpu, sc.max_depth, seed=sc.seed, crop=crop, n_threads=threads)
    dt = time.perf_counter() - t0
    st = r["stats"]
    rays = st["extension_rays"] + st["shadow_rays"]
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{crop[2]}x{crop[3]} pixels from ({crop[0]},{crop[1]}) of the 1920x1080 frame at {spp_cpu} spp, depth "
                      f"{sc.max_depth}, full 1.31M-triangle scene; {rays} rays in {dt:.2f} s "
                      f"({crop[2] * crop[3] * spp_cpu / dt:.3g} samples/s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--spp", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-count", action="store_true", help="skip the node-visit counting pass")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(samples are independent: a multi-GPU run would split the sample range and sum the FP64 "
              "accumulators once)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_19977_amd import pt, scenes

    sc = scenes.spheres(spp=args.spp)
    cam = sc.camera
    W, H = cam.width, cam.height
    torch.cuda.set_device(0)
    s = pt.scene_from(sc, device=0)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        s.render(cam, sc.spp, sc.max_depth, sc.seed, out)

    # algorithmic work of one step: node visits and triangle tests (same seed -> same paths)
    counts = None
    if not args.no_count:
        s.set_profiling(False, True)
        s.reset_stats()
        s.render(cam, sc.spp, sc.max_depth, sc.seed, out)
        counts = s.stats()
        s.set_profiling(False, False)

    s.set_profiling(True, False)
    s.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.render(cam, sc.spp, sc.max_depth, sc.seed, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = s.stats()
    rays = st["extension_rays"] + st["shadow_rays"]
    mrays = rays / dt / 1e6
    samples_s = W * H * sc.spp * args.steps / dt

    roofline = None
    if counts is not None and st["launches_extend"] > 0:
        ext_bytes = (counts["node_visits"] * NODE_BYTES + counts["tri_tests"] * TRI_BYTES +
                     counts["extension_rays"] * (RAY_BYTES + HIT_BYTES))
        launches_per_step = st["launches_extend"] / args.steps
        bytes_per_launch = ext_bytes / launches_per_step
        avg_ms = st["ms_extend"] / st["launches_extend"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                    "kernel": "k_extend (BVH4 closest hit)",
                    "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_ms, 4),
                    "node_visits_per_ray": round(counts["node_visits"] / max(1, counts["extension_rays"]), 2),
                    "tri_tests_per_ray": round(counts["tri_tests"] / max(1, counts["extension_rays"]), 2)}

    result = {
        "metric": METRIC, "value": round(mrays, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 sums)", "data": "synthetic",
        "config": {"workload": "icosphere field: 1,310,722 tris, 1920x1080, 64 spp, depth 8, sky + sun env",
                   "width": W, "height": H, "spp": sc.spp, "max_depth": sc.max_depth, "triangles": sc.n_triangles,
                   "parallelism": "single GPU"},
        "samples_per_s": round(samples_s, 1),
        "extension_rays_per_step": st["extension_rays"] // args.steps,
        "shadow_rays_per_step": st["shadow_rays"] // args.steps,
        "nonfinite_dropped": st["nonfinite_dropped"],
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
