"""Benchmark of the K-pass recursive camera-painting render on one MI355X.

One step = one frame: the whole hot path (per-pixel displaced ray
generation, BVH traversal with watertight intersection, shading, the
convergence test, over all K passes on one stream) for the 1920x1080, K=6
render of the 1,000,418-triangle synthetic terrain scene.  The default
chain engine runs the frame as one persistent launch (k_chain); --engine
passes runs one launch per pass with compaction in HBM (k_pass).
The scene and BVH are built once (build time reported separately) and stay
resident; outputs are preallocated; inputs are in HBM before timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU peak of MI355X without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.32 T lane-operations per second (the 157.3 TFLOP/s FP32 figure
# counts an FMA as 2 and packed dual-FP32 issue as 2; the build disables
# packed FP32 and counts an FMA as one operation).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-operations the method needs per unit of work, counted from the
# arithmetic of each step as written (not from the compiled code):
#   inner-node visit: 4 children x (6 slab-plane FMAs, 3 max and 2 min for
#     the entry and exit, 2 compares) + 1 multiply of the best-hit bound = 53
#   triangle test (watertight): 9 subtractions to the origin, 6 x (multiply,
#     subtract) of the shear, 3 x (2 multiplies, subtract) edge functions,
#     3 zero tests, 6 sign tests, 2 adds and 1 test of det, 3 multiplies of
#     the z terms, 5 for T, 1 division, 1 test of t, 2 compares against the
#     best hit = 54
#   traced ray: its displaced camera ray (68), the traversal's ray constants
#     (72), the shade lookup and convergence test (10) = 150
OPS_PER_NODE = 53
OPS_PER_TRI = 54
OPS_PER_RAY = 150
KERNEL_OF_ENGINE = {"chain": "k_chain", "passes": "k_pass"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2312_12392_amd", "csrc", f)
                  for f in ("chain.hip", "trace.hip", "traverse.hpp", "rcp_internal.hpp", "bvh_build.hip")]


def traffic_file(kernel: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")


def counters_file(kernel: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")


def load_profile(path: str, workload: str):
    """A profile summary (JSON) if it was taken on the current kernel sources."""
    try:
        with open(path) as f:
            pr = json.load(f)
    except (OSError, ValueError):
        return None
    if pr.get("kernel_source_sha256") != kernel_source_hash() or pr.get("workload") != workload:
        return None
    return pr


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and blank space removed, so
    that a measurement stays attached to the code it was taken on."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def algorithmic_bytes(counts, engine="chain"):
    """Logical global-memory bytes of one frame from the traversal counters.

    Per pass k (counts[k] = rays traced, inner nodes visited, triangles
    tested, rays continued to pass k + 1), both engines:
      112 B per 4-wide node visited (four child boxes + four links)
      48 B per triangle tested (three vertices + index)
      16 B per traced ray: the shaded colour looked up (hit or miss constant)
      12 B + 4 B per traced ray: image k and its hit ID written
      16 B per remaining image for every pixel that converged at pass k
    and with one launch per pass ("passes"), the pass state in HBM:
      16 B per traced ray at k > 0: its {pixel, previous RGB} entry read
      16 B per continued ray: its entry written for pass k + 1
    The chain engine keeps that state in registers.
    """
    K = len(counts)
    total = 0.0
    for k in range(K):
        rays, nodes, tris, app = (float(x) for x in counts[k][:4])
        total += 112 * nodes + 48 * tris + (16 + 12 + 4) * rays
        if engine == "passes":
            total += 16 * app + (16 * rays if k > 0 else 0.0)
        converged = rays - app if k + 1 < K else 0.0
        total += 16 * converged * (K - 1 - k)
    return total


def algorithmic_ops(counts):
    """VALU lane-operations of one frame the method needs (OPS_PER_*)."""
    tot = counts[:, :3].astype("float64").sum(0)
    return OPS_PER_RAY * tot[0] + OPS_PER_NODE * tot[1] + OPS_PER_TRI * tot[2]


def logical_bytes_by_tier(counts):
    """Bytes the traversal reads and writes, by the memory that serves them:
    node visits staged in LDS; node visits, triangle tests and the shade
    lookup through the L1/L2 caches; the images and IDs written."""
    tot = counts.astype("float64").sum(0)
    rays, nodes, tris, _, lds_nodes = tot[:5]
    return {"lds": round(112 * lds_nodes), "l1_l2": round(112 * (nodes - lds_nodes) + 48 * tris + 16 * rays)}


def cpu_baseline(w, min_seconds=10.0, min_reps=3, max_reps=60):
    """The oracle on the host cores: whole frames until at least min_seconds
    of work (and min_reps frames) have run; the median frame is reported."""
    import numpy as np
    import oracle
    o = oracle.OracleScene(w.scene, use_bvh=True)
    times = []
    while len(times) < min_reps or (sum(times) < min_seconds and len(times) < max_reps):
        t0 = time.perf_counter()
        o.render(w.camera, w.width, w.height, w.passes, w.lambda_eye, w.lambda_dir)
        times.append(time.perf_counter() - t0)
    reps = len(times)
    t = float(np.median(times))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": w.nominal_rays / t / 1e6, "unit": "Mrays/s", "cores": oracle.default_threads(),
            "kind": "oracle", "cpu": model,
            "sample": f"full {w.width}x{w.height} K={w.passes} frames of the same scene, median of {reps} "
                      f"({t:.2f} s each, {sum(times):.1f} s in all; oracle BVH build not timed)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="terrain1m",
                    help="terrain1m (default: the K-pass frame), batch64, served, terrain16m, gather4k")
    ap.add_argument("--duration", type=float, default=6.0, help="served: seconds of arrivals per rate")
    ap.add_argument("--rates", default="20,50,100,200", help="served: arrival rates, requests per second")
    ap.add_argument("--frames", type=int, default=120, help="terrain16m: walk-through frames")
    ap.add_argument("--literal-eye", action="store_true", help="displace the eye as well (lambda_eye = lambda)")
    ap.add_argument("--engine", choices=["chain", "passes"], default="chain",
                    help="chain: one persistent launch per frame; passes: one launch per pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-leaf", type=int, default=3, help="BVH leaf size bound (build option)")
    ap.add_argument("--c-trav", type=float, default=1.0, help="SAH cost of a node visit (build option)")
    ap.add_argument("--c-isect", type=float, default=1.0, help="SAH cost of a triangle test (build option)")
    ap.add_argument("--collapse", choices=["sah", "greedy"], default="sah",
                    help="how the 4-wide tree is formed from the binary tree (build option)")
    ap.add_argument("--builder", choices=["ploc", "lbvh"], default="ploc", help="binary tree builder (build option)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--no-served", action="store_true", help="skip the served leg of the default line")
    ap.add_argument("--no-literal-eye", action="store_true",
                    help="skip the literal-eye leg (profiling runs: only the default frame's launches)")
    ap.add_argument("--served-seconds", type=float, default=3.0, help="served leg: seconds of arrivals at 200/s")
    ap.add_argument("--saturating-rate", type=float, default=600.0,
                    help="served leg: an arrival rate above what the GPU serves")
    ap.add_argument("--saturating-seconds", type=float, default=1.5,
                    help="served leg: seconds of arrivals at the saturating rate")
    ap.add_argument("--max-inflight", type=int, default=2, help="server: concurrent batched launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the render would shard "
              "by pixels with no exchange, but no multi-GPU path is implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.workload in EXTRA:
        print(json.dumps(EXTRA[args.workload](args)), flush=True)
        return
    bench_frame(args)


def copy_bandwidth_gbs(stream, reps: int = 3) -> float:
    """Best of `reps` 1 GiB device-to-device copies on `stream`, in GB/s of
    bytes read plus written."""
    import torch

    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    moved = 2 * a.numel() * a.element_size()
    del a, b
    return moved / (best * 1e-3) / 1e9


def build_options(args):
    """The BVH build options named on the command line."""
    from paper_2312_12392_amd import rcp
    return rcp.build_options(max_leaf=args.max_leaf, c_trav=args.c_trav, c_isect=args.c_isect,
                             builder=rcp.RCP_BUILDER_PLOC if args.builder == "ploc" else rcp.RCP_BUILDER_LBVH,
                             collapse=rcp.RCP_COLLAPSE_SAH if args.collapse == "sah" else rcp.RCP_COLLAPSE_GREEDY)


def bench_frame(args):
    import numpy as np
    import torch

    import scenegen
    from paper_2312_12392_amd import rcp

    stream = torch.cuda.current_stream()
    w = scenegen.workload(args.workload, literal_eye=args.literal_eye)
    log(f"workload {w.name}: {w.width}x{w.height} K={w.passes} tris={w.scene.n_tris}")
    scene = rcp.Scene(w.scene, build_options(args))
    scene.set_engine(rcp.RCP_ENGINE_CHAIN if args.engine == "chain" else rcp.RCP_ENGINE_PASSES)
    kernel = KERNEL_OF_ENGINE[args.engine]
    info = scene.info()
    log(f"scene built: {info}; engine {args.engine}")
    K, W, H = w.passes, w.width, w.height
    imgs = torch.empty((K, H, W, 3), dtype=torch.float32, device="cuda")
    ids = torch.empty((K, H, W), dtype=torch.int32, device="cuda")
    disp = rcp.make_displacement(w.lambda_eye, w.lambda_dir)

    def step():
        rcp.rcp_render(scene.handle, w.camera, W, H, K, disp, imgs, ids, stream)

    step()
    torch.cuda.synchronize()

    # traversal counters from the instrumented kernel (untimed)
    imgs_s = torch.empty_like(imgs)
    counts = rcp.rcp_render_stats(scene.handle, w.camera, W, H, K, disp, imgs_s, None, stream)
    same = bool(torch.equal(imgs_s, imgs))
    del imgs_s
    traced = int(counts[:, 0].sum())
    bytes_frame = algorithmic_bytes(counts, args.engine)
    launches = 1 if args.engine == "chain" else K
    log(f"counts per pass [rays, nodes, tris, continued]: {counts.tolist()} (stats image identical: {same})")

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the warm-up frames come last before the timed ones: after the host-side
    # work above the GPU has been idle, and its first frames then run at lower
    # clocks (measured: 1.34-1.41 ms against 1.27 ms for the following ones)
    for _ in range(args.warmup):
        step()
    # one event between consecutive frames: the total and the per-frame times
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms_total = ev[0].elapsed_time(ev[-1])
    ms = ms_total / args.steps
    per_frame = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    nominal = W * H * K
    value = nominal * args.steps / (ms_total * 1e-3) / 1e6
    # the frame is one k_chain launch (or K k_pass launches) plus one setup
    # launch of a few microseconds; the average launch lasts ms / launches
    # and carries 1 / launches of the frame's work, so the rates are the
    # frame's
    ops_frame = algorithmic_ops(counts)
    achieved_tops = ops_frame / (ms * 1e-3) / 1e12

    copy_gbs = copy_bandwidth_gbs(stream)

    # HBM traffic and SQ counters of this kernel from the committed profiles,
    # when they were taken on the current sources (null otherwise)
    tr = load_profile(traffic_file(kernel, w.name), w.name)
    traffic = tr["hbm_bytes_per_launch"] if tr else None
    write_bytes = round(tr["write_kib_per_dispatch"] * 1024 * tr["write_scale"]) if tr else None
    sq = load_profile(counters_file(kernel, w.name), w.name)
    compulsory_writes = 16 * W * H * K          # every image (12 B) and ID (4 B) of every pass
    literal = None if args.literal_eye or args.no_literal_eye else literal_eye_leg(args, scene, w, imgs, ids, stream)

    result = {
        "metric": "Mrays/s (nominal W*H*K rays) of the K=6 frame at 1080p/1M tris; frame ms in ms_per_step",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_median": round(float(np.median(per_frame)), 4),
        "ms_min": round(float(per_frame.min()), 4),
        "ms_p90": round(float(np.percentile(per_frame, 90)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {W}x{H}, K={K}, {w.scene.n_tris} triangles "
                               f"(fBm terrain + boxes, seeded), lambda_eye={w.lambda_eye}, lambda_dir={w.lambda_dir}",
                   "width": W, "height": H, "passes": K, "triangles": w.scene.n_tris},
        "traced_mrays_per_s": round(traced * args.steps / (ms_total * 1e-3) / 1e6, 2),
        "traced_rays_per_frame": traced,
        "active_per_pass": [int(c) for c in counts[:, 0]],
        "bvh_build_ms": round(info["build_ms"], 3),
        "bvh": {"nodes": info["n_nodes"], "sah_cost": round(info["sah_cost"], 3), "max_depth": info["max_depth"],
                "builder": args.builder, "collapse": args.collapse, "max_leaf": args.max_leaf,
                "c_trav": args.c_trav, "c_isect": args.c_isect},
        # The traversal is bound on chip by VALU issue (no dense contraction,
        # no MFMA; HBM runs far below its peak), so the roofline is the VALU
        # one: the method's lane-operations per frame (OPS_PER_*) over the
        # frame time, against the VALU peak.  Beside it, from the committed
        # counter profiles of the same sources: how busy the VALU issue is and
        # what fraction of its lanes is active, and the HBM side.
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved_tops, 3),
            "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "T lane-op/s",
            "frac": round(achieved_tops / VALU_PEAK_TOPS, 4),
            "traffic": traffic,
            "kernel": kernel,
            "launches_per_step": launches,
            "algorithmic_ops_per_launch": round(ops_frame / launches),
            "ops_per_unit": {"inner_node_visit": OPS_PER_NODE, "triangle_test": OPS_PER_TRI,
                             "traced_ray": OPS_PER_RAY},
            "valu_issue": None if sq is None else {
                "busy": sq["valu_busy"], "lane_utilisation": sq["lane_utilisation"],
                "useful_lane_frac": round(sq["valu_busy"] * sq["lane_utilisation"], 4),
                "ta_busy": sq["ta_busy"], "source": os.path.basename(counters_file(kernel, w.name))},
            "hbm": {
                "achieved": None if traffic is None else round(traffic / (ms * 1e-3) / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None if traffic is None else round(traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": traffic, "write_bytes": write_bytes,
                "compulsory_write_bytes": compulsory_writes,
                "write_amplification": None if write_bytes is None else round(write_bytes / compulsory_writes, 3),
                "source": os.path.basename(traffic_file(kernel, w.name)),
                # what a plain 1 GiB device copy reaches on the same GPU
                "copy_gbs": round(copy_gbs, 1),
            },
            "logical_bytes_per_launch": dict(logical_bytes_by_tier(counts),
                                             hbm_measured=traffic,
                                             total=round(bytes_frame / launches)),
        },
    }
    if literal is not None:
        result["literal_eye"] = literal
    scene.close()
    if not args.no_served and args.engine == "chain" and w.name == "terrain1m":
        result["served"] = served_leg(args)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores ...")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


def literal_eye_leg(args, scene, w, imgs, ids, stream, reps=10):
    """The same frame with the eye displaced too, lambda_eye = lambda_dir
    (the configuration's literal wording): mean of `reps` frames."""
    import torch

    from paper_2312_12392_amd import rcp
    d = rcp.make_displacement(w.lambda_dir, w.lambda_dir)
    for _ in range(2):
        rcp.rcp_render(scene.handle, w.camera, w.width, w.height, w.passes, d, imgs, ids, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        rcp.rcp_render(scene.handle, w.camera, w.width, w.height, w.passes, d, imgs, ids, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"lambda_eye": w.lambda_dir, "lambda_dir": w.lambda_dir, "ms_per_frame": round(ms, 4),
            "mrays_per_s": round(w.width * w.height * w.passes / (ms * 1e-3) / 1e6, 2), "frames": reps}


def served_leg(args):
    """Compact served measurement for the default line: the continuous-
    batching server against the plain per-request loop on the 4M-triangle
    scene, at 200 requests/s and at a rate above what the GPU can serve."""
    import torch

    import scenegen
    from paper_2312_12392_amd import rcp
    w = scenegen.workload("terrain4m")
    log(f"served leg: terrain4m, {w.scene.n_tris} triangles")
    scene = rcp.Scene(w.scene, build_options(args))
    rates = [(200.0, args.served_seconds), (args.saturating_rate, args.saturating_seconds)]
    out = {"scene": f"terrain4m: {w.scene.n_tris} triangles", "max_inflight": args.max_inflight,
           "requests": "Poisson arrivals; 512^2/720p/1080p/4K; K 3..8; spline cameras; lambda_dir 0.01"}
    for i, (rate, seconds) in enumerate(rates):
        r = served_rate(rcp, scene, w, rate, seconds, 5 + i, args.max_inflight, torch.cuda.current_stream())
        out[f"{int(rate)}_per_s"] = r
        log(f"served rate {rate}: {r}")
    scene.close()
    return out

def _percentiles(x):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    return {"p50": round(float(np.percentile(x, 50)), 3), "p99": round(float(np.percentile(x, 99)), 3),
            "mean": round(float(x.mean()), 3), "max": round(float(x.max()), 3)}


def bench_batch(args):
    """64 views of the 1M scene (orbit; 256^2, 512^2, 720p, 1024^2; K 1..8)
    in one batched launch, with the default launch parameters and with the
    ones the autotuner picks for this batch, against 64 sequential
    rcp_render calls."""
    import torch

    import scenegen
    from paper_2312_12392_amd import rcp

    stream = torch.cuda.current_stream()
    w = scenegen.workload("terrain1m")
    views = scenegen.orbit_views(3, 64)
    scene = rcp.Scene(w.scene, build_options(args))
    d = rcp.make_displacement(0.0, w.lambda_dir)
    outs = [torch.empty((K, H, W, 3), device="cuda") for (_, W, H, K) in views]
    batch = [(cam, W, H, K, d, o, None) for (cam, W, H, K), o in zip(views, outs)]
    rays = sum(W * H * K for (_, W, H, K) in views)

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def run_batch():
        rcp.rcp_render_batch(scene.handle, batch, stream)

    defaults = rcp.rcp_get_tuning(scene.handle)
    ms_default = timed(run_batch, args.steps)

    def seq():
        for (cam, W, H, K), o in zip(views, outs):
            rcp.rcp_render(scene.handle, cam, W, H, K, d, o, None, stream)
    ms_seq = timed(seq, max(1, args.steps // 4))
    t0 = time.perf_counter()
    tuned, _ = rcp.rcp_autotune_batch(scene.handle, batch, repeats=3, stream=stream)
    tune_s = time.perf_counter() - t0
    ms_tuned = timed(run_batch, args.steps)
    ms_batch = min(ms_tuned, ms_default)
    scene.close()
    return {
        "metric": "Mrays/s of a 64-view batch (1M-triangle scene, mixed resolution and K) in one launch",
        "value": round(rays / (ms_batch * 1e-3) / 1e6, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "ms_per_step": round(ms_batch, 4), "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch64: 64 orbit views of terrain1m, resolutions 256^2/512^2/720p/1024^2, K 1..8, "
                               "lambda_dir 0.01", "views": 64, "nominal_rays": rays},
        "default_tuning": defaults, "default_ms": round(ms_default, 4),
        "autotuned": tuned, "autotuned_ms": round(ms_tuned, 4), "autotune_seconds": round(tune_s, 1),
        "sequential_rcp_render_ms": round(ms_seq, 4),
        "speedup_vs_sequential": round(ms_seq / ms_batch, 3),
    }


def _retire(rcp, srv, pending, late, lat):
    still = []
    for t in pending:
        st, (ts, tb, td) = rcp.rcp_poll(srv, t)
        if st == rcp.RCP_REQ_FAILED:
            raise RuntimeError(f"served request {t} failed")
        if st == rcp.RCP_REQ_DONE:
            lat.append((td - ts + late[t]) * 1e3)
            rcp.rcp_release(srv, t)
        else:
            still.append(t)
    return still


def served_rate(rcp, scene, w, rate, duration, seed, max_inflight, stream):
    """One arrival rate: the server, then the plain loop, on the same trace.
    Latency = completion - arrival time (host clock); throughput = nominal
    rays / wall time from the first arrival to the last completion."""
    import time

    import torch

    import scenegen
    d = rcp.make_displacement(0.0, w.lambda_dir)
    trace = scenegen.served_trace(seed, rate, duration)
    rays = sum(W * H * K for (_, _, W, H, K) in trace)
    # warm-up of both paths (kernels loaded, workspaces sized)
    big = torch.empty((8, 2160, 3840, 3), device="cuda")
    rcp.rcp_render(scene.handle, trace[0][1], 3840, 2160, 8, d, big, None, stream)
    torch.cuda.synchronize()
    # --- server ---
    srv = rcp.rcp_server_create(scene.handle, 48 << 30, max_inflight=max_inflight)
    t0 = time.perf_counter()
    pending = []
    lat = []
    late = {}
    for (arr, cam, W, H, K) in trace:
        while time.perf_counter() - t0 < arr:
            time.sleep(0.0002)
        t = rcp.rcp_submit(srv, cam, W, H, K, d)
        late[t] = time.perf_counter() - t0 - arr        # submitted this long after its arrival time
        pending.append(t)
        if len(pending) > 16:                           # retire finished requests as we go
            pending = _retire(rcp, srv, pending, late, lat)
    while pending:
        pending = _retire(rcp, srv, pending, late, lat)
        time.sleep(0.0005)
    t_srv = time.perf_counter() - t0
    launches = rcp.rcp_server_stats(srv)["launches"]
    rcp.rcp_server_destroy(srv)
    log(f"  rate {rate}: server done ({len(trace)} requests, {t_srv:.1f} s); running the plain loop")
    # --- plain loop: one synchronous rcp_render at a time, in arrival order ---
    lat_loop = []
    t0 = time.perf_counter()
    for (arr, cam, W, H, K) in trace:
        now = time.perf_counter() - t0
        if now < arr:
            time.sleep(arr - now)
        out = big.view(-1)[:K * H * W * 3].view(K, H, W, 3)
        rcp.rcp_render(scene.handle, cam, W, H, K, d, out, None, stream)
        stream.synchronize()
        lat_loop.append((time.perf_counter() - t0 - arr) * 1e3)
        if len(lat_loop) % 2000 == 0:
            log(f"  loop: {len(lat_loop)} of {len(trace)} requests")
    t_loop = time.perf_counter() - t0
    del big
    return {"requests": len(trace), "seconds_of_arrivals": duration, "nominal_rays": rays, "launches": launches,
            "server_latency_ms": _percentiles(lat), "loop_latency_ms": _percentiles(lat_loop),
            "server_mrays_per_s": round(rays / t_srv / 1e6, 1), "loop_mrays_per_s": round(rays / t_loop / 1e6, 1)}


def bench_served(args):
    """Poisson arrivals on the 4M-triangle scene: the continuous-batching
    server vs a plain first-in-first-out loop of synchronous rcp_render."""
    import torch

    import scenegen
    from paper_2312_12392_amd import rcp

    stream = torch.cuda.current_stream()
    w = scenegen.workload("terrain4m")
    scene = rcp.Scene(w.scene, build_options(args))
    rates = [float(r) for r in args.rates.split(",")]
    per_rate = {}
    for ri, rate in enumerate(rates):
        per_rate[str(int(rate))] = served_rate(rcp, scene, w, rate, args.duration, 5 + ri, args.max_inflight, stream)
        log(f"rate {rate}: {per_rate[str(int(rate))]}")
    scene.close()
    top = per_rate[str(int(rates[-1]))]
    return {
        "metric": "served p50/p99 latency (ms) and Mrays/s vs a plain per-request loop, 4M-triangle scene",
        "value": top["server_latency_ms"]["p99"], "unit": "ms (p99 latency at the highest rate)",
        "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served: terrain4m ({w.scene.n_tris} triangles), Poisson arrivals at {args.rates} "
                               f"req/s for {args.duration} s each, 512^2/720p/1080p/4K, K 3..8, spline cameras",
                   "rates": rates, "duration_s": args.duration, "max_inflight": args.max_inflight},
        "per_rate": per_rate,
    }


def bench_walk(args):
    """The 16M-triangle scene: a walk-through of 4K, K=8 frames, each frame
    restarting from the grey seed with a new camera; timed with the default
    launch parameters and with the ones the autotuner picks on the first
    frame (the line's value is the faster of the two walks)."""
    import numpy as np
    import torch

    import scenegen
    from paper_2312_12392_amd import rcp

    stream = torch.cuda.current_stream()
    w = scenegen.workload("terrain16m")
    log(f"terrain16m: {w.scene.n_tris} triangles")
    scene = rcp.Scene(w.scene, build_options(args))
    info = scene.info()
    W, H, K = w.width, w.height, w.passes
    imgs = torch.empty((K, H, W, 3), device="cuda")
    d = rcp.make_displacement(0.0, w.lambda_dir)
    pts = scenegen.spline_path(7)
    cams = [scenegen.walk_camera(pts, i / args.frames) for i in range(args.frames)]
    rcp.rcp_render(scene.handle, cams[0], W, H, K, d, imgs, None, stream)
    torch.cuda.synchronize()

    def walk():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.frames + 1)]
        ev[0].record(stream)
        for i, cam in enumerate(cams):
            rcp.rcp_render(scene.handle, cam, W, H, K, d, imgs, None, stream)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        return np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.frames)])

    defaults = rcp.rcp_get_tuning(scene.handle)
    ms_default = walk()
    # launch parameters tuned on the first frame (scene and resolution), then
    # the whole walk-through again with them
    t0 = time.perf_counter()
    tuned, _ = rcp.rcp_autotune(scene.handle, cams[0], W, H, K, d, imgs, None, repeats=2, stream=stream)
    tune_s = time.perf_counter() - t0
    ms_tuned = walk()
    ms = ms_tuned if ms_tuned.sum() < ms_default.sum() else ms_default
    rays = W * H * K * args.frames
    scene.close()
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle (its own BVH, all host cores) on the walk-through's first
        # two frames
        import oracle
        log("timing the oracle on the first two frames ...")
        t0 = time.perf_counter()
        o = oracle.OracleScene(w.scene, use_bvh=True)
        t_bvh = time.perf_counter() - t0
        times = []
        for cam in cams[:2]:
            t0 = time.perf_counter()
            o.render(cam, W, H, K, 0.0, w.lambda_dir)
            times.append(time.perf_counter() - t0)
        o.close()
        cpu = {"value": round(2 * W * H * K / sum(times) / 1e6, 3), "unit": "Mrays/s",
               "cores": oracle.default_threads(), "kind": "oracle",
               "sample": f"the first 2 frames of the walk-through, {times[0]:.1f} s and {times[1]:.1f} s "
                         f"(oracle BVH build {t_bvh:.1f} s, not timed)"}
    return {
        "metric": "Mrays/s of a 4K K=8 walk-through of the 16M-triangle scene; frame ms p50/p99",
        "value": round(rays / (ms.sum() * 1e-3) / 1e6, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.frames,
        "ms_per_step": round(float(ms.mean()), 4), "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"terrain16m: {W}x{H}, K={K}, {w.scene.n_tris} triangles, {args.frames}-frame spline "
                               "walk-through, lambda_dir 0.01", "frames": args.frames},
        "frame_ms": _percentiles(ms), "bvh_build_ms": round(info["build_ms"], 2), "cpu_baseline": cpu,
        "default_tuning": defaults, "default_frame_ms": _percentiles(ms_default),
        "autotuned": tuned, "autotuned_frame_ms": _percentiles(ms_tuned), "autotune_seconds": round(tune_s, 1),
        "bvh": {"nodes": info["n_nodes"], "sah_cost": round(info["sah_cost"], 3), "max_depth": info["max_depth"],
                "builder": args.builder, "collapse": args.collapse, "max_leaf": args.max_leaf,
                "c_trav": args.c_trav, "c_isect": args.c_isect},
    }


def bench_gather(args):
    """Screen-space variant: K-1 = 5 gather passes over a rendered 4K image."""
    import torch

    import scenegen
    from paper_2312_12392_amd import rcp

    stream = torch.cuda.current_stream()
    w = scenegen.workload("terrain1m")
    scene = rcp.Scene(w.scene, build_options(args))
    W, H, n = 3840, 2160, 5
    base = torch.empty((1, H, W, 3), device="cuda")
    rcp.rcp_render(scene.handle, w.camera, W, H, 1, rcp.make_displacement(0.0, 0.0), base, None, stream)
    out = torch.empty((n, H, W, 3), device="cuda")
    for _ in range(3):
        rcp.rcp_gather_passes(base, W, H, n, 6.0, rcp.RCP_EDGE_MIRROR, True, out, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        rcp.rcp_gather_passes(base, W, H, n, 6.0, rcp.RCP_EDGE_MIRROR, True, out, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    bytes_pass = 32.0 * W * H          # own R, G (8 B) + source RGB (12 B) + written RGB (12 B)
    gbs = bytes_pass * n / (ms * 1e-3) / 1e9
    scene.close()
    return {
        "metric": "screen-space variant: pixels/s of 5 gather passes over a 4K image (mirror edges)",
        "value": round(W * H * n / (ms * 1e-3) / 1e9, 3), "unit": "Gpixel-passes/s", "n_gpus": 1,
        "steps": args.steps, "ms_per_step": round(ms, 4), "higher_is_better": True, "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gather4k: 3840x2160 render of terrain1m, 5 passes, max_smudge 6 px, mirror edges"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_gather",
                     "algorithmic_bytes_per_launch": round(bytes_pass)},
    }


EXTRA = {"batch64": bench_batch, "served": bench_served, "terrain16m": bench_walk, "gather4k": bench_gather}


if __name__ == "__main__":
    main()
