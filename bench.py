"""Benchmark of the path tracer on one MI355X.

A step is one pt_render of the 1920x1080 icosphere-field scene
(1,310,722 triangles, 64 icospheres of level 5 on a ground plane, metal and
coated-diffuse materials, 2048x1024 sky with a 0.5 degree sun) at 64 spp and
max depth 8: camera rays, BVH closest hits, OpenPBR shading, next-event
estimation with MIS, Russian roulette and the FP64 per-pixel sums.
Inputs are resident in HBM before the timed region.

Prints one JSON line: Mrays/s (extension + shadow rays per second) with
samples/s beside it, the roofline of the closest-hit kernel measured live
with HIP events on the library's stream, the display kernel's roofline, the
instanced scene at 1080p (256 spp, depth 12) with its own traversal
roofline, the radiance cache against the plain tracer (time to equal RMSE,
averaged over independent seeds, with the cache's bias floor), and the FP64
oracle timed on the host's cores on a bounded sample of the same workload.
"""
import argparse
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s and samples/s at 1080p; time-to-equal-RMSE, radiance cache vs plain"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_WAVE_INSTR_S = 256 * 4 * 2.4e9 / 4  # 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per 4 cycles
NODE_BYTES, TRI_BYTES, RAY_BYTES, HIT_BYTES = 128, 48, 32, 16
INST_BYTES = 128        # instance record read when a walk enters an instance (two-level scenes)
SHADOW_RAY_BYTES = 48  # o + tmax, d + path slot, contribution + skip primitive (the L update is not counted)
DISPLAY_BYTES_PER_PIXEL = 3 * 8 + 4  # FP64 sums read, one RGBA8 word written


def kernel_source_hash() -> str:
    """sha256 over everything the kernels' behaviour depends on: the library
    sources (kernels, host code that sets grids, streams and defaults), the C
    header and the build flags (file name + bytes, sorted)."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2407_19977_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*")))
    files += [os.path.join(ROOT, "include", "pt.h"), os.path.join(pkg, "build.py")]
    for p in files:
        h.update(os.path.relpath(p, ROOT).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()


def profile_field(name: str, key: str, as_float=False):
    """A value recorded in profiles/<name>, or None when the summary is missing
    or the sources changed since its counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    v = re.search(rf"^{re.escape(key)}: ([-+0-9.eE]+)", txt, re.M)
    h = re.search(r"^kernel_source_sha256: ([0-9a-f]+)", txt, re.M)
    if not v or not h or h.group(1) != kernel_source_hash():
        return None
    return float(v.group(1)) if as_float else int(float(v.group(1)))


CPU_SHARE_PER_GPU = 16  # host CPUs a one-GPU job may keep busy on the GPU machines this runs on


def host_info():
    """CPUs this process may use: the affinity mask, capped by a cgroup CPU quota if one is set."""
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = max(1, int(int(q) / int(period)))
    except (OSError, ValueError):
        pass
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = min(affinity, quota) if quota else affinity
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cgroup_cpu_quota": quota, "cpu_model": model,
            "usable_cpus": usable, "thread_cap": CPU_SHARE_PER_GPU}


def cpu_baseline(sc, spp_cpu=12, crop=(0, 0, 1920, 1080)):
    """The oracle as it stands, one thread per usable hardware thread (at most the CPU share of one
    GPU), on the full frame at few spp."""
    from oracle import oracle as O
    info = host_info()
    threads = min(info["usable_cpus"], CPU_SHARE_PER_GPU)
    os_ = O.OracleScene(sc)
    t0 = time.perf_counter()
    r = os_.render(spp_cpu, sc.max_depth, seed=sc.seed, crop=crop, n_threads=threads)
    dt = time.perf_counter() - t0
    st = r["stats"]
    rays = st["extension_rays"] + st["shadow_rays"]
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{crop[2]}x{crop[3]} pixels from ({crop[0]},{crop[1]}) of the 1920x1080 frame at {spp_cpu} spp, depth "
                      f"{sc.max_depth}, full 1.31M-triangle scene; {rays} rays in {dt:.2f} s "
                      f"({crop[2] * crop[3] * spp_cpu / dt:.3g} samples/s)",
            "host": info}


CHECKPOINTS = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)
NRC_FLOP_PER_QUERY = 2 * (5 * 64 * 64 + 3 * 64)   # 41,344 multiply-adds x 2
MFMA_BF16_PEAK_TFLOPS = 2500.0


def _frames(s, cam, depth, seed, frames, ref, out, torch):
    """Samples of 1 spp each into the FP64 sums, one call per span between
    checkpoints (so the library overlaps consecutive passes or frames as a
    user's call would): rows (spp, cumulative ms, MSE, relMSE) against ref."""
    s.reset_accumulation()
    t = 0.0
    rows = []
    done = 0
    for cp in sorted({c for c in CHECKPOINTS if c < frames} | {frames}):
        t0 = time.perf_counter()
        s.accumulate(cam, done, cp - done, depth, seed)  # returns after the stream has drained
        t += time.perf_counter() - t0
        done = cp
        s.resolve(out)
        d = out.double() - ref
        mse = torch.mean(d * d).item()
        rel = torch.mean(d * d / (ref * ref + 0.01)).item()
        rows.append((cp, t * 1e3, mse, rel, torch.mean(d).item()))
    return rows


def _average(runs):
    """Mean time and mean MSE / relMSE over runs at each checkpoint; RMSE = sqrt(mean MSE)."""
    out = []
    for k in range(len(runs[0])):
        cp = runs[0][k][0]
        ms = sum(r[k][1] for r in runs) / len(runs)
        mse = sum(r[k][2] for r in runs) / len(runs)
        rel = sum(r[k][3] for r in runs) / len(runs)
        bias = sum(r[k][4] for r in runs) / len(runs)
        out.append((cp, ms, math.sqrt(mse), rel, bias))
    return out


def _time_to(rows, target, col=2):
    """Time at which an error-vs-time curve (column col) first reaches target
    (log-log interpolation from the previous checkpoint), or None."""
    prev = None
    for r in rows:
        ms, e = r[1], r[col]
        if e <= target:
            if prev is None or prev[1] <= e:
                return ms
            (m0, e0) = prev
            f = (math.log(target) - math.log(e0)) / (math.log(e) - math.log(e0))
            return math.exp(math.log(m0) + f * (math.log(ms) - math.log(m0)))
        prev = (ms, e)
    return None


def _error_at(rows, ms_target, col=2):
    """Error of a curve at a given time (log-log interpolation), or None outside it."""
    for a, b in zip(rows, rows[1:]):
        if a[1] <= ms_target <= b[1]:
            f = (math.log(ms_target) - math.log(a[1])) / (math.log(b[1]) - math.log(a[1]))
            return math.exp(math.log(a[col]) + f * (math.log(b[col]) - math.log(a[col])))
    return None


CACHE_VARIANTS = (
    ("refinements of the cited method: adaptive termination (spread 0.01) by vertex 2, training paths "
     "ending in the cache at vertex 3 (self-training), factorised by the reflectance",
     {"spread_c": 0.01, "train_end_bounce": 3, "factorize": 1}),
    ("adaptive termination only (spread 0.01)", {"spread_c": 0.01}),
)


def _cache_runs(pt, s, cam, depth, frames, seeds, ref, out, torch, cache_kw):
    """Frames of the cache for each seed (fresh network per seed); statistics summed over the runs."""
    runs = []
    st_all = {"cache_queries": 0, "cache_records": 0, "ms_cache_query": 0.0, "ms_cache_train": 0.0, "steps": 0}
    for seed in range(seeds):
        # untimed cache frames allocate the cache's buffers (the first frame runs alone, later ones
        # overlap on two path sets); configuring again resets weights and Adam state
        s.set_radiance_cache(pt.cache_config(init_seed=seed, **cache_kw))
        s.reset_accumulation()
        s.accumulate(cam, 0, 3, depth, seed)
        s.set_radiance_cache(pt.cache_config(init_seed=seed, **cache_kw))
        s.reset_stats()
        runs.append(_frames(s, cam, depth, seed, frames, ref, out, torch))
        st = s.stats()
        for k in ("cache_queries", "cache_records", "ms_cache_query", "ms_cache_train"):
            st_all[k] += st[k]
        st_all["steps"] += st["cache_adam_steps"]
        print(f"[cache] {cache_kw or 'defaults'} seed {seed}: {runs[-1][-1]}", file=sys.stderr, flush=True)
    return runs, st_all


def _compare(plain, cache, frames, seeds, ref_mean):
    """Time to the plain tracer's RMSE / relMSE at 4, 16 and 64 spp, RMSE at equal time, bias measures."""
    def floor(rows):
        n1 = max(1, frames // 4)
        r1 = [r for r in rows if r[0] == n1]
        if not r1 or n1 == frames:
            return None
        m1, m2 = r1[0][2] ** 2, rows[-1][2] ** 2
        b2 = (frames * m2 - n1 * m1) / (frames - n1)
        return math.sqrt(max(0.0, b2))

    bias_cache, bias_plain = floor(cache), floor(plain)
    trained = [r for r in cache if r[0] > 1]
    tte = []
    for col, name in ((2, "RMSE"), (3, "relMSE")):
        for target_spp in (4, 16, 64):
            row = [r for r in plain if r[0] == target_spp]
            if not row:
                continue
            target = row[0][col]
            t_plain = _time_to(plain, target, col)
            t_nrc = _time_to(trained, target, col)
            ent = {"target": f"plain {name} at {target_spp} spp (mean over {seeds} seeds)", "value": round(target, 6),
                   "plain_ms": None if t_plain is None else round(t_plain, 2),
                   "cache_ms": None if t_nrc is None else round(t_nrc, 2),
                   "speedup": None if (t_nrc is None or t_plain is None) else round(t_plain / t_nrc, 3)}
            if col == 2 and bias_cache is not None:
                ent["above_cache_bias_floor"] = target > bias_cache
            tte.append(ent)
    t_eq = min(plain[-1][1], trained[-1][1])

    def at(rows):
        return rows[-1][2] if rows[-1][1] <= t_eq else _error_at(rows, t_eq)
    return {
        "time_to_equal_rmse": tte,
        "rmse_at_equal_time": {"ms": round(t_eq, 2), "plain": None if at(plain) is None else round(at(plain), 6),
                               "cache": None if at(trained) is None else round(at(trained), 6)},
        "mean_bias": {"cache": round(cache[-1][4] / ref_mean, 6), "plain": round(plain[-1][4] / ref_mean, 6),
                      "what": f"(mean of the {frames}-spp image - mean of the reference) / mean of the reference, "
                              f"averaged over seeds"},
        "bias_floor_rmse": {"cache": None if bias_cache is None else round(bias_cache, 6),
                            "plain": None if bias_plain is None else round(bias_plain, 6),
                            "method": f"MSE(N) = V/N + B^2 fitted through the seed-averaged MSE at N = "
                                      f"{max(1, frames // 4)} and {frames}; the plain tracer's B is the "
                                      f"reference's own error"},
        "ms_per_frame_plain": round(plain[-1][1] / plain[-1][0], 3),
        "ms_per_frame_cache": round(cache[-1][1] / cache[-1][0], 3),
    }


def cache_experiment(pt, torch, sc, frames=256, ref_spp=4096, seeds=4, variants=CACHE_VARIANTS, **cache_kw):
    """Plain vs radiance-cache rendering, frames of 1 spp (consecutive frames
    of one call overlap in both modes), MSE against a ref_spp plain render with
    FP64 sums and an independent seed, averaged over `seeds` independent runs
    (sample seeds 0..seeds-1; the cache also starts from a different initial
    network per run).  The cache's first frame renders plain (nothing is
    trained yet), so its curve enters the time-to-target search from frame 2
    on.  Bias floor: with MSE(N) = V / N + B^2 per mode, B^2 from the averaged
    MSE at N1 = frames / 4 and N2 = frames.  The main comparison uses the
    library's cache settings (overridden by cache_kw); each variant changes
    some of them and is compared against the same plain runs."""
    cam = sc.camera
    W, H, depth = cam.width, cam.height, sc.max_depth
    s = pt.scene_from(sc, device=0)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")
    acc = torch.empty((H, W, 3), dtype=torch.float64, device="cuda:0")
    ref_seed = 1000
    s.set_radiance_cache(None)
    s.reset_accumulation()
    chunk = 256
    for k in range(0, ref_spp, chunk):
        s.accumulate(cam, k, min(chunk, ref_spp - k), depth, ref_seed)
    s.resolve(out, acc)
    ref = acc / ref_spp
    ref_mean = ref.mean().item()
    print(f"[cache] reference: {ref_spp} spp plain, seed {ref_seed}", file=sys.stderr, flush=True)
    s.set_profiling(True, False)
    plain_runs = []
    for seed in range(seeds):
        s.set_radiance_cache(None)
        plain_runs.append(_frames(s, cam, depth, seed, frames, ref, out, torch))
    plain = _average(plain_runs)
    cache_runs, st_all = _cache_runs(pt, s, cam, depth, frames, seeds, ref, out, torch, cache_kw)
    cache = _average(cache_runs)
    # the query kernel alone: frames of one call each (nothing beside them), 8 of them
    s.reset_stats()
    for k in range(8):
        s.accumulate(cam, frames + k, 1, depth, 0)
    st_iso = s.stats()
    fwd_2m = forward_rate(s, torch)
    var_out = []
    for name, kw in variants:
        vruns, _ = _cache_runs(pt, s, cam, depth, frames, seeds, ref, out, torch, {**kw, **cache_kw})
        v = _average(vruns)
        ent = {"name": name, "settings": kw, "rmse_final": round(v[-1][2], 6)}
        ent.update(_compare(plain, v, frames, seeds, ref_mean))
        var_out.append(ent)
    s.set_radiance_cache(None)
    table = [{"spp": a[0], "plain_ms": round(a[1], 2), "plain_rmse": round(a[2], 6), "plain_relmse": round(a[3], 6),
              "cache_ms": round(b[1], 2), "cache_rmse": round(b[2], 6), "cache_relmse": round(b[3], 6),
              "cache_frame_trained": a[0] > 1}
             for a, b in zip(plain, cache)]
    q_ms = st_iso["ms_cache_query"]
    achieved = st_iso["cache_queries"] * NRC_FLOP_PER_QUERY / (q_ms * 1e-3) / 1e12 if q_ms > 0 else None
    q_ms_frames = st_all["ms_cache_query"]
    achieved_frames = (st_all["cache_queries"] * NRC_FLOP_PER_QUERY / (q_ms_frames * 1e-3) / 1e12
                       if q_ms_frames > 0 else None)
    cfg = pt.cache_config(**cache_kw)
    train_samples = st_all["steps"] * cfg.batch_size
    result = {
        "workload": f"icosphere field {W}x{H}, depth {depth}, frames of 1 spp; cache: 64-feature encoding, "
                    "5x64 ReLU MLP (bf16 matrix cores), paths end in it by vertex 2, 65,536 training paths and "
                    "4 Adam steps of 16,384 records per frame",
        "reference": f"{ref_spp} spp plain tracer, FP64 sums, seed {ref_seed}",
        "seeds": seeds,
        "cache_config": {k: getattr(cfg, k) for k, _ in cfg._fields_},
        "rmse": table,
    }
    result.update(_compare(plain, cache, frames, seeds, ref_mean))
    result.update({
        "variants": var_out,
        "cache_queries_per_s": round(st_all["cache_queries"] / (sum(r[-1][1] for r in cache_runs) * 1e-3), 1),
        "training_records_per_frame": st_all["cache_records"] // (frames * seeds),
        "training_samples_per_s": round(train_samples / (st_all["ms_cache_train"] * 1e-3), 1)
        if st_all["ms_cache_train"] > 0 else None,
        "ms_train_steps_per_frame": round(st_all["ms_cache_train"] / (frames * seeds), 3),
        "roofline": None if achieved is None else {
            "bound": "mfma", "kernel": "k_nrc_infer<1> (cache queries: encoding + 6-layer bf16 MLP)",
            "achieved": round(achieved, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
            "flop_per_query": NRC_FLOP_PER_QUERY, "queries": st_iso["cache_queries"],
            "avg_launch_ms": round(q_ms / 8, 4),
            "measured_on": "8 frames of one call each (the query kernel with nothing beside it)",
            "pt_nrc_forward_2M_queries": fwd_2m,
            "in_overlapped_frames_tflops": None if achieved_frames is None else round(achieved_frames, 2)},
    })
    s.close()
    return result


def tail_info(counts, st, steps):
    """The persistent tail kernel (all vertices of the last few paths): time and closest-hit bytes."""
    info = {"kernel": "k_tail (remaining vertices once few paths are alive)",
            "ms_per_step": round(st["ms_tail"] / steps, 3), "launches_per_step": st["launches_tail"] / steps,
            "extension_rays_per_step": st["tail_extension_rays"] // steps}
    if st["ms_tail"] > 0 and counts is not None:
        b = (counts["tail_node_visits"] * NODE_BYTES + counts["tail_tri_tests"] * TRI_BYTES +
             counts["tail_instances_entered"] * INST_BYTES + counts["tail_extension_rays"] * (RAY_BYTES + HIT_BYTES))
        info["closest_hit_gbs"] = round(b / (st["ms_tail"] / steps * 1e-3) / 1e9, 1)
    return info


def traversal_roofline(counts, st, steps, kernel):
    """HBM roofline of the traversal kernel: algorithmic bytes of a step (counted on the same seeded
    paths by the counting variant) per launch, over the launches' HIP-event durations."""
    if counts is None or st["launches_extend"] <= 0:
        return None
    # the wavefront traversal kernel only: the tail kernel's rays and visits are counted apart
    ext_rays = counts["extension_rays"] - counts["tail_extension_rays"]
    sh_rays = counts["shadow_rays"] - counts["tail_shadow_rays"]
    ext_bytes = (counts["node_visits"] * NODE_BYTES + counts["tri_tests"] * TRI_BYTES +
                 ext_rays * (RAY_BYTES + HIT_BYTES))
    sh_bytes = (counts["shadow_node_visits"] * NODE_BYTES + counts["shadow_tri_tests"] * TRI_BYTES +
                sh_rays * SHADOW_RAY_BYTES)
    inst_bytes = counts["instances_entered"] * INST_BYTES
    launches_per_step = st["launches_extend"] / steps
    bytes_per_launch = (ext_bytes + sh_bytes + inst_bytes) / (counts["launches_extend"] or launches_per_step)
    avg_ms = st["ms_extend"] / st["launches_extend"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernel,
         "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_ms, 4),
         "launches_per_step": launches_per_step,
         "node_visits_per_ray": round(counts["node_visits"] / max(1, ext_rays), 2),
         "tri_tests_per_ray": round(counts["tri_tests"] / max(1, ext_rays), 2),
         "node_visits_per_shadow_ray": round(counts["shadow_node_visits"] / max(1, sh_rays), 2),
         "tri_tests_per_shadow_ray": round(counts["shadow_tri_tests"] / max(1, sh_rays), 2),
         "tail_kernel": tail_info(counts, st, steps)}
    if counts["instances_entered"]:
        r["instances_entered_per_walk"] = round(counts["instances_entered"] / max(1, ext_rays + sh_rays), 2)
    return r


def _counted(s, render, steps=1):
    """Statistics of `steps` renders with the counting variant of the kernels, timing on (launch counts)."""
    s.set_profiling(True, True)
    s.reset_stats()
    for _ in range(steps):
        render()
    c = s.stats()
    s.set_profiling(False, False)
    return c


def display_roofline(s, W, H, torch, reps=20):
    """The display kernel on the sums of the last render: HBM roofline from HIP events."""
    rgba = torch.empty((H, W, 4), dtype=torch.uint8, device="cuda:0")
    s.display(rgba)  # warm-up
    s.set_profiling(True, False)
    s.reset_stats()
    for _ in range(reps):
        s.display(rgba)
    st = s.stats()
    s.set_profiling(False, False)
    avg_ms = st["ms_display"] / st["launches_display"]
    b = DISPLAY_BYTES_PER_PIXEL * W * H
    gbs = b / (avg_ms * 1e-3) / 1e9
    return {"kernel": "k_display (PBR Neutral tone map, sRGB, 8-bit RGBA of the FP64 running mean)",
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": b, "avg_launch_ms": round(avg_ms, 4),
            "launches": st["launches_display"], "traffic": None}


def shade_valu():
    """VALU roofline of the shading kernels from the committed counter summary (None if stale)."""
    name = "k_shade_spheres_1080p.md"
    instr = profile_field(name, "valu_wave_instructions_per_step", True)
    ms = profile_field(name, "kernel_ms_per_step", True)
    util = profile_field(name, "valu_lane_utilisation", True)
    if instr is None or ms is None or ms <= 0:
        return None
    rate = instr / (ms * 1e-3)
    return {"kernel": "k_shade<class> (all classes)", "bound": "alu", "achieved": round(rate / 1e9, 1),
            "peak": round(VALU_PEAK_WAVE_INSTR_S / 1e9, 1), "unit": "G wave-instructions/s",
            "frac": round(rate / VALU_PEAK_WAVE_INSTR_S, 4), "valu_lane_utilisation": util,
            "source": f"profiles/{name} (SQ_INSTS_VALU over kernel-trace durations)"}


def instanced_1080p(pt, torch, spp, tail=None):
    """The instanced scene at 1920x1080, `spp` samples, depth 12: throughput and traversal roofline."""
    from paper_2407_19977_amd import scenes
    sc = scenes.instanced(spp=spp)
    cam = sc.camera
    s = pt.scene_from(sc, device=0)
    if tail is not None:
        s.set_tail(*tail)
    out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda:0")
    s.render(cam, 4, sc.max_depth, sc.seed, out)  # warm-up
    counts = _counted(s, lambda: s.render(cam, spp, sc.max_depth, sc.seed, out))
    s.set_profiling(True, False)
    s.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.render(cam, spp, sc.max_depth, sc.seed, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = s.stats()
    rays = st["extension_rays"] + st["shadow_rays"]
    res = {"workload": f"instanced scene: 400 instances of 5 meshes, {sc.n_triangles:,} instanced triangles, "
                       f"two-level BVH, {cam.width}x{cam.height}, {spp} spp, depth {sc.max_depth}",
           "Mrays_per_s": round(rays / dt / 1e6, 2), "samples_per_s": round(cam.width * cam.height * spp / dt, 1),
           "ms_per_render": round(dt * 1e3, 2), "extension_rays": st["extension_rays"],
           "shadow_rays": st["shadow_rays"],
           "roofline": traversal_roofline(counts, st, 1, "k_traverse<two-level> (top-level + per-mesh BVH4 walks)")}
    s.close()
    return res


def forward_rate(s, torch, n=1 << 21, calls=10):
    """pt_nrc_forward on n uniform inputs: average kernel time (HIP events on
    the library's stream) and the matrix-core roofline it reaches."""
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.rand((n, 12), generator=g, dtype=torch.float32).to("cuda:0")
    y = torch.empty((n, 3), dtype=torch.float32, device="cuda:0")
    s.nrc_forward(x, y)
    s.set_profiling(True, False)
    s.reset_stats()
    for _ in range(calls):
        s.nrc_forward(x, y)
    st = s.stats()
    ms = st["ms_cache_forward"] / calls
    tflops = n * NRC_FLOP_PER_QUERY / (ms * 1e-3) / 1e12
    return {"queries": n, "avg_launch_ms": round(ms, 4), "achieved_tflops": round(tflops, 2),
            "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4)}


def nrc_kernels(pt, torch, scenes, warm_frames=16, iso_frames=8, n_forward=1 << 21, forward_calls=20):
    """The radiance-cache kernels on their own (icosphere field 1080p, frames of
    1 spp): queries of frames run one call each (the query kernel with nothing
    beside it), the training steps of those frames, and pt_nrc_forward on
    n_forward uniform inputs (HIP events around each call).  Short
    enough to run under a counter profiler."""
    sc = scenes.spheres(spp=1)
    cam = sc.camera
    s = pt.scene_from(sc, device=0)
    s.set_radiance_cache(pt.cache_config())
    s.reset_accumulation()
    s.accumulate(cam, 0, warm_frames, sc.max_depth, 0)
    s.set_profiling(True, False)
    s.reset_stats()
    steps0 = s.stats()["cache_adam_steps"]  # the device's step counter is not reset
    for k in range(iso_frames):
        s.accumulate(cam, warm_frames + k, 1, sc.max_depth, 0)
    st = s.stats()
    s.set_profiling(False, False)
    cfg = pt.cache_config()
    q_ms = st["ms_cache_query"]
    res = {"workload": f"icosphere field {cam.width}x{cam.height}, depth {sc.max_depth}, cache after {warm_frames} "
                       f"frames; {iso_frames} frames of one call each",
           "queries_per_frame": st["cache_queries"] // iso_frames,
           "query_kernel_ms_per_frame": round(q_ms / iso_frames, 4),
           "query_tflops": round(st["cache_queries"] * NRC_FLOP_PER_QUERY / (q_ms * 1e-3) / 1e12, 2) if q_ms > 0
           else None,
           "train_ms_per_frame": round(st["ms_cache_train"] / iso_frames, 4),
           "train_samples_per_frame": (st["cache_adam_steps"] - steps0) * cfg.batch_size // iso_frames}
    res["pt_nrc_forward"] = forward_rate(s, torch, n_forward, forward_calls)
    s.set_radiance_cache(None)
    s.close()
    return res


def _cache_kw(args):
    """Cache settings given on the command line (the library's defaults otherwise)."""
    kw = {"ema_decay": args.cache_ema, "train_end_bounce": args.cache_train_end, "factorize": args.cache_factorize,
          "query_bounce": args.cache_query_bounce, "spread_c": args.cache_spread}
    return {k: v for k, v in kw.items() if v is not None}


def bvh_builds(pt, torch, sc_spheres, steps=2):
    """Host binned-SAH build vs the device builds (locally-ordered clustering, the default, and the linear
    BVH; soup in host memory -> BVH ready), and what each tree costs the traversal: the icosphere field
    rendered through each tree."""
    from paper_2407_19977_amd import scenes
    res = {"paper_context": "Table 1: CPU BVH set-up of 327.57 ms (Apple M1 Max) and 383.10 ms (Ryzen 5 5600X) "
                            "for 1,068,735 triangles; context only (other machines, other builder)"}
    cam = sc_spheres.camera
    out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda:0")
    for name, sc in (("icosphere field (1,310,722 triangles)", sc_spheres),
                     ("instanced scene (5 meshes, 135,000 unique triangles; top level on the host)", None)):
        if sc is None:
            sc = scenes.instanced()
        ent = {}
        for gpu in (False, "ploc", "lbvh"):
            s = pt.scene_from(sc, device=0, gpu_bvh=gpu)
            if gpu:  # a second build: the first one also loads the builder's kernels
                s.build_bvh(sc.meshes, sc.instances, on_device=True)
            info = s.bvh_info()
            e = {"build_ms": round(info["build_ms"], 2), "nodes": info["n_nodes"], "depth": info["depth"],
                 "max_leaf": info["max_leaf_tris"]}
            if info["sah_cost"]:
                e["sah_cost"] = round(info["sah_cost"], 3)
            if sc is sc_spheres:  # the traversal through this tree
                s.render(cam, sc.spp, sc.max_depth, sc.seed, out)
                s.set_profiling(True, False)
                s.reset_stats()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    s.render(cam, sc.spp, sc.max_depth, sc.seed, out)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                st = s.stats()
                e["render_Mrays_per_s"] = round((st["extension_rays"] + st["shadow_rays"]) / dt / 1e6, 1)
            ent[{"ploc": "device", "lbvh": "device_lbvh"}.get(gpu, "host")] = e
            s.close()
        ent["speedup"] = round(ent["host"]["build_ms"] / ent["device"]["build_ms"], 2)
        res[name] = ent
    return res


PAPER_TABLE2_RTX3080_MS = {1068735: 1058.73, 106873: 790.20, 10687: 790.83}  # 512x512, 100 spp, depth 5


def paper_shape(pt, torch, reps=10):
    """The shape of the paper's Table 2 (512x512, 100 spp, depth 5, a model at
    three levels of detail ~10x apart; Table 1 times the CPU BVH set-up of the
    same models): the icosphere field at subdivision levels 5, 3 and 2.  Render
    time is the mean (and standard deviation) of `reps` pt_render calls after
    one warm-up, as the paper averages 30 runs; BVH set-up on the host and on
    the device.  The paper's RTX 3080 times are context only (other models,
    machine and renderer)."""
    import numpy as np
    from paper_2407_19977_amd import scenes
    out = {"workload": "icosphere field at subdivision levels 5 / 3 / 2, 512x512, 100 spp, depth 5",
           "paper_context": "Table 2, RTX 3080 (WebGPU, no NEE): 1058.73 ms at 1,068,735 triangles, 790.20 ms at "
                            "106,873, 790.83 ms at 10,687; Table 1 CPU BVH set-up 383.10 / 41.77 / 8.43 ms "
                            "(Ryzen 5 5600X)",
           "levels": []}
    for level in (5, 3, 2):
        sc = scenes.spheres(width=512, height=512, spp=100, max_depth=5, level=level)
        cam = sc.camera
        ent = {"level": level, "triangles": sc.n_triangles}
        for gpu in (False, True):
            s = pt.scene_from(sc, device=0, gpu_bvh=gpu)
            if gpu:
                s.build_bvh(sc.meshes, sc.instances, on_device=True)  # the first build also loads the kernels
            ent["bvh_build_ms_" + ("device" if gpu else "host")] = round(s.bvh_info()["build_ms"], 2)
            if gpu:
                s.close()
                continue
            img = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda:0")
            s.render(cam, 100, 5, 0, img)
            s.set_profiling(False, False)
            s.reset_stats()
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.render(cam, 100, 5, 0, img)
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
            st = s.stats()
            ms = float(np.mean(times))
            ent.update({"render_ms": round(ms, 3), "render_ms_std": round(float(np.std(times)), 3),
                        "samples_per_s": round(cam.width * cam.height * 100 / (ms * 1e-3), 1),
                        "Mrays_per_s": round((st["extension_rays"] + st["shadow_rays"]) / reps / (ms * 1e-3) / 1e6,
                                             1)})
            s.close()
        out["levels"].append(ent)
    return out


def _tail_args(args):
    """(min_bounce, max_fraction) from the command line, None for the library's defaults."""
    if args.tail_min_bounce is None and args.tail_fraction is None:
        return None
    return (2 if args.tail_min_bounce is None else args.tail_min_bounce,
            0.15 if args.tail_fraction is None else args.tail_fraction)


def instanced_4k(pt, torch, spp, ref_spp, tail=None):
    """The instanced scene at 3840x2160: plain tracer and radiance cache side by
    side, each accumulated to `spp` samples (FP64 sums; the cache in frames of
    1 spp, as configured and with the first of CACHE_VARIANTS), against a
    `ref_spp` plain render with an independent seed.  Prints progress to
    stderr; returns the JSON object of the comparison."""
    from paper_2407_19977_amd import scenes
    sc = scenes.instanced(width=3840, height=2160, spp=spp)
    cam = sc.camera
    W, H, depth, seed = cam.width, cam.height, sc.max_depth, sc.seed
    s = pt.scene_from(sc, device=0)
    if tail is not None:
        s.set_tail(*tail)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")
    acc = torch.empty((H, W, 3), dtype=torch.float64, device="cuda:0")
    chunk = 32

    def run(n, sd, cache, kw=None):
        s.set_radiance_cache(pt.cache_config(**(kw or {})) if cache else None)
        s.reset_accumulation()
        s.reset_stats()
        s.set_profiling(True, False)
        t0 = time.perf_counter()
        for k in range(0, n, chunk):
            s.accumulate(cam, k, min(chunk, n - k), depth, sd)
            print(f"[4k] {'cache' if cache else 'plain'} seed {sd}: {min(n, k + chunk)}/{n} spp, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        st = s.stats()
        s.set_profiling(False, False)
        s.resolve(out, acc)
        return dt, st, (acc / n).clone()

    t_ref, _, ref = run(ref_spp, seed + 1, False)
    res = {"workload": f"instanced scene (400 instances of 5 meshes, 10.8M instanced triangles), {W}x{H}, depth {depth}",
           "reference": f"{ref_spp} spp plain tracer, FP64 sums, seed {seed + 1} ({t_ref:.1f} s)", "modes": {}}
    modes = (("plain", False, None), ("cache", True, None), ("cache_refined", True, CACHE_VARIANTS[0][1]))
    for name, cache, kw in modes:
        dt, st, img = run(spp, seed, cache, kw)
        d = img - ref
        rays = st["extension_rays"] + st["shadow_rays"]
        res["modes"][name] = {
            "spp": spp, "seconds": round(dt, 3), "Mrays_per_s": round(rays / dt / 1e6, 1),
            "samples_per_s": round(W * H * spp / dt, 1),
            "rmse": round(torch.sqrt(torch.mean(d * d)).item(), 6),
            "relmse": round(torch.mean(d * d / (ref * ref + 0.01)).item(), 6),
            "cache_queries": st["cache_queries"], "adam_steps": st["cache_adam_steps"],
            "mean_bias": round(((img.mean() - ref.mean()) / ref.mean()).item(), 6)}
        if kw:
            res["modes"][name]["settings"] = kw
    s.set_radiance_cache(None)
    s.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--spp", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-count", action="store_true", help="skip the node-visit counting pass")
    ap.add_argument("--no-cache", action="store_true", help="skip the radiance-cache vs plain experiment")
    ap.add_argument("--no-instanced", action="store_true", help="skip the instanced scene at 1080p")
    ap.add_argument("--no-display", action="store_true", help="skip the display kernel's roofline")
    ap.add_argument("--no-bvh", action="store_true", help="skip the host vs device BVH build comparison")
    ap.add_argument("--no-paper-shape", action="store_true",
                    help="skip the icosphere field at three levels of detail in the shape of the paper's Table 2")
    ap.add_argument("--cache-frames", type=int, default=256)
    ap.add_argument("--cache-seeds", type=int, default=4)
    ap.add_argument("--ref-spp", type=int, default=4096)
    ap.add_argument("--instanced-spp", type=int, default=256)
    ap.add_argument("--cache-ema", type=float, default=None, help="ema_decay of the cache (library default if omitted)")
    ap.add_argument("--cache-train-end", type=int, default=None,
                    help="train_end_bounce of the cache: vertex at which training paths end in it (self-training)")
    ap.add_argument("--cache-factorize", type=int, default=None, help="factorize of the cache (0 or 1)")
    ap.add_argument("--cache-query-bounce", type=int, default=None, help="query_bounce of the cache")
    ap.add_argument("--cache-spread", type=float, default=None, help="spread_c of the cache (adaptive termination)")
    ap.add_argument("--workload", choices=["spheres-1080p", "instanced-4k", "cache", "instanced-1080p", "nrc-kernels"],
                    default="spheres-1080p",
                    help="instanced-4k: plain vs cache on the instanced scene at 3840x2160 (minutes); cache: only "
                         "the radiance-cache experiment; instanced-1080p: only the instanced scene; nrc-kernels: "
                         "the cache kernels alone, short enough for counter profiling (none is the bench line)")
    ap.add_argument("--spp-4k", type=int, default=1024)
    ap.add_argument("--ref-spp-4k", type=int, default=2048)
    ap.add_argument("--tail-min-bounce", type=int, default=None,
                    help="first bounce at which the tail kernel may take over (library default if omitted)")
    ap.add_argument("--tail-fraction", type=float, default=None,
                    help="largest fraction of alive paths handed to the tail kernel (library default if omitted)")
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

    torch.cuda.set_device(0)
    if args.workload == "instanced-4k":
        print(json.dumps({"metric": "plain vs radiance cache, 4K instanced scene",
                          "result": instanced_4k(pt, torch, args.spp_4k, args.ref_spp_4k, _tail_args(args))}),
              flush=True)
        return
    if args.workload == "cache":
        sc = scenes.spheres(spp=args.spp)
        print(json.dumps({"metric": "radiance cache vs plain, icosphere field 1080p",
                          "result": cache_experiment(pt, torch, sc, args.cache_frames, args.ref_spp,
                                                     args.cache_seeds, **_cache_kw(args))}), flush=True)
        return
    if args.workload == "nrc-kernels":
        print(json.dumps({"metric": "radiance-cache kernels", "result": nrc_kernels(pt, torch, scenes)}), flush=True)
        return
    if args.workload == "instanced-1080p":
        print(json.dumps({"metric": "instanced scene 1080p",
                          "result": instanced_1080p(pt, torch, args.instanced_spp, _tail_args(args))}), flush=True)
        return

    sc = scenes.spheres(spp=args.spp)
    cam = sc.camera
    W, H = cam.width, cam.height
    s = pt.scene_from(sc, device=0)
    if _tail_args(args) is not None:
        s.set_tail(*_tail_args(args))
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def render():
        s.render(cam, sc.spp, sc.max_depth, sc.seed, out)

    for _ in range(args.warmup):
        render()

    # algorithmic work of one step: node visits and triangle tests (same seed -> same paths)
    counts = None if args.no_count else _counted(s, render)

    s.set_profiling(True, False)
    s.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        render()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = s.stats()
    s.set_profiling(False, False)
    rays = st["extension_rays"] + st["shadow_rays"]
    mrays = rays / dt / 1e6
    samples_s = W * H * sc.spp * args.steps / dt

    roofline = traversal_roofline(counts, st, args.steps,
                                  "k_traverse (BVH4 walks: closest hits of a bounce and the previous bounce's "
                                  "shadow rays)")
    if roofline is not None:
        roofline["traffic"] = profile_field("k_traverse_spheres_1080p.md", "traffic_bytes_per_launch")

    result = {
        "metric": METRIC, "value": round(mrays, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 sums)", "data": "synthetic",
        "config": {"workload": "icosphere field: 1,310,722 tris, 1920x1080, 64 spp, depth 8, sky + sun env",
                   "width": W, "height": H, "spp": sc.spp, "max_depth": sc.max_depth, "triangles": sc.n_triangles,
                   "parallelism": "single GPU",
                   "tail_hand_off": dict(zip(("min_bounce", "max_fraction"), _tail_args(args) or (2, 0.15)))},
        "samples_per_s": round(samples_s, 1),
        "extension_rays_per_step": st["extension_rays"] // args.steps,
        "shadow_rays_per_step": st["shadow_rays"] // args.steps,
        "nonfinite_dropped": st["nonfinite_dropped"],
        "roofline": roofline,
        "shade_valu": shade_valu(),
        "display": None if args.no_display else display_roofline(s, W, H, torch),
        "cpu_baseline": None,
        "bvh_build": None,
        "paper_table2_shape": None,
        "instanced_1080p": None,
        "radiance_cache": None,
    }
    s.close()
    if not args.no_bvh:
        print("[bench] BVH builds", file=sys.stderr, flush=True)
        result["bvh_build"] = bvh_builds(pt, torch, sc)
    if not args.no_paper_shape:
        print("[bench] the shape of the paper's Table 2", file=sys.stderr, flush=True)
        result["paper_table2_shape"] = paper_shape(pt, torch)
    if not args.no_instanced:
        print("[bench] instanced scene 1080p", file=sys.stderr, flush=True)
        result["instanced_1080p"] = instanced_1080p(pt, torch, args.instanced_spp, _tail_args(args))
    if not args.no_cache:
        print("[bench] radiance cache vs plain", file=sys.stderr, flush=True)
        result["radiance_cache"] = cache_experiment(pt, torch, sc, args.cache_frames, args.ref_spp, args.cache_seeds,
                                                    **_cache_kw(args))
    if not args.no_cpu_baseline:
        print("[bench] oracle on the host", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
