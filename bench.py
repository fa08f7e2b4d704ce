"""Benchmark: per-pixel RGBD plane fits on one MI355X.

One step = the whole per-frame path (integrands, integral-image sweep, box
sums, per-pixel solve, stores) over the 640x480 workload at every window size
it lists (k = 3, 5, 9, 15), in the default implicit mode with FP64 moments.
Inputs are seeded synthetic depth frames already resident in HBM; the timed
loop rotates through enough distinct input/output buffer sets to keep the
256 MB last-level cache from holding them.

Printed: one JSON line with the throughput (Mpixel/s over all fitted pixels),
the dominant kernel's roofline position (algorithmic HBM bytes per launch over
its average HIP-event duration), the FP64 CPU oracle timed on a bounded sample
on the host, and side measurements (explicit mode, FP32, the 1920x1080 frame).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E peak, GB/s
BYTES_PER_PIXEL = 4 + 12 + 4 + 4 + 1   # depth in; normals, offset, residual, status out
METRIC = ("Mpixel/s of per-pixel plane fits (normal+offset+residual) at 640×480 and "
          "1080p; % HBM peak")


def measured_traffic():
    """HBM bytes per headline launch from the committed FETCH_SIZE/WRITE_SIZE runs,
    or None when the kernel source has changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        src = open(os.path.join(ROOT, "paper_2103_06644_amd", "csrc", "planefit.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("kernel_source_sha256_prefix"):
        return None
    return (rec["fetch_kib_per_launch"] * rec["fetch_scale"] +
            rec["write_kib_per_launch"] * rec["write_scale"]) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sets", type=int, default=64, help="distinct buffer sets rotated")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device-to-device copy first (calibrates HBM counters)")
    return ap.parse_args()


class Rig:
    """Device buffers for `sets` copies of one frame and `per_set` output sets each."""

    def __init__(self, torch, depth_np, sets, per_set=1):
        self.torch = torch
        H, W = depth_np.shape
        base = torch.from_numpy(depth_np).cuda()
        self.depth = [base.clone() for _ in range(sets)]
        self.outs = [[(torch.empty((3, H, W), device="cuda"), torch.empty((H, W), device="cuda"),
                       torch.empty((H, W), device="cuda"),
                       torch.empty((H, W), dtype=torch.uint8, device="cuda"))
                      for _ in range(per_set)] for _ in range(sets)]
        self.sets = sets
        self.pixels = H * W


def time_launches(torch, pf, rig, intr, ks, mode, precision, steps, warmup, tuned=None):
    """One step = one launch fitting the frame at every k in ks (a batched launch
    when there are several).  The timed steps are replayed from captured HIP
    graphs, `chunk` consecutive steps (each on its own buffer set) per graph, so
    the kernels run back to back with no host gaps; HIP events on the replay
    stream bracket every replay.  tuned = (band height, launch shape) of a
    derived plan for a single-k step.  Returns (ms per step, ms per launch)."""
    H, W = rig.depth[0].shape
    for k in ks:
        pf.get_plan(intr, H, W, k, mode, precision)
    bh, sh = tuned if tuned else (None, None)

    def run(s):
        if len(ks) == 1:
            pf.fit_planes(rig.depth[s], intr, ks[0], mode=mode, precision=precision,
                          out=rig.outs[s][0], band_height=bh, shape=sh)
        else:
            pf.fit_planes_batch([rig.depth[s]] * len(ks), intr, list(ks), mode=mode,
                                precision=precision, outs=rig.outs[s])

    chunk = max(c for c in range(1, min(32, rig.sets, steps) + 1) if steps % c == 0)
    for i in range(warmup):
        run(i % rig.sets)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graphs = []
    n_graphs = min(steps // chunk, -(-rig.sets // chunk))
    with torch.cuda.stream(side):
        for gi in range(n_graphs):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                for j in range(chunk):
                    run((gi * chunk + j) % rig.sets)
            graphs.append(g)
    torch.cuda.current_stream().wait_stream(side)
    for g in graphs:
        g.replay()
    torch.cuda.synchronize()
    n_rep = steps // chunk
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n_rep)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for i in range(n_rep):
        a, b = evs[i]
        a.record()
        graphs[i % len(graphs)].replay()
        b.record()
    t_end.record()
    torch.cuda.synchronize()
    per_launch = float(sum(a.elapsed_time(b) for a, b in evs)) / (n_rep * chunk)
    time_launches.sets_used = min(rig.sets, n_rep * chunk, len(graphs) * chunk)
    return t_start.elapsed_time(t_end) / steps, per_launch


def batch_measure(torch, pf, np, frames_for, queued=False):
    """The 64-frame mixed workload (320x240, 640x480, 1280x720; per-frame k):
    one batched call, eager and replayed from a captured HIP graph; two
    input/output sets alternate.  queued=False: two launches of up to 32 frames
    each; queued=True: one persistent fit launch fed by a work queue (after its
    small job-table setup launches)."""
    frames = frames_for("batch_mixed_64")
    sets = []
    for _ in range(2):
        d = [torch.from_numpy(f.depth).cuda() for f in frames]
        o = [(torch.empty((3,) + f.depth.shape, device="cuda"),
              torch.empty(f.depth.shape, device="cuda"), torch.empty(f.depth.shape, device="cuda"),
              torch.empty(f.depth.shape, dtype=torch.uint8, device="cuda")) for f in frames]
        sets.append((d, o))
    intr = [f.intrinsics for f in frames]
    ks = [f.window for f in frames]
    px = sum(f.depth.size for f in frames)
    wss = [torch.empty(pf.batch_workspace_bytes(len(frames)), dtype=torch.uint8, device="cuda")
           for _ in range(2)]

    def call(s):
        pf.fit_planes_batch(sets[s][0], intr, ks, mode="implicit", outs=sets[s][1],
                            queued=queued, workspace=wss[s])

    for i in range(5):
        call(i % 2)
    torch.cuda.synchronize()
    n = 40
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(n):
        call(i % 2)
    b.record()
    torch.cuda.synchronize()
    eager = a.elapsed_time(b) / n
    graphs = []
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for s in range(2):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                call(s)
            graphs.append(g)
    torch.cuda.current_stream().wait_stream(side)
    for i in range(4):
        graphs[i % 2].replay()
    torch.cuda.synchronize()
    a.record()
    for i in range(n):
        graphs[i % 2].replay()
    b.record()
    torch.cuda.synchronize()
    graph = a.elapsed_time(b) / n
    return {"frames": len(frames), "pixels": px, "mode": "implicit", "precision": "fp64",
            "launch": "queued (one persistent fit launch)" if queued else "chunked (32 frames per launch)",
            "eager_ms": round(eager, 4), "graph_ms": round(graph, 4),
            "eager_Mpx_s": round(px / (eager * 1e-3) / 1e6, 1),
            "graph_Mpx_s": round(px / (graph * 1e-3) / 1e6, 1)}


def diff_measure(torch, pf, np, frames_for, diff_loss_inputs):
    """The differentiation workload: 8 frames of 640x480, k = 9, implicit FP64.
    One step = the forward fits of the 8 frames (one batched launch) and the
    batched backward pass of the 8 frames for L = sum W (1 - n . t) + 0.1 r (two
    launches), replayed from a captured HIP graph; the backward alone is timed
    the same way."""
    frames = frames_for("diff_8x640x480")
    k = frames[0].window
    intr = frames[0].intrinsics
    H, W = frames[0].depth.shape
    depth = [torch.from_numpy(f.depth).cuda() for f in frames]
    outs = [(torch.empty((3, H, W), device="cuda"), torch.empty((H, W), device="cuda"),
             torch.empty((H, W), device="cuda"), torch.empty((H, W), dtype=torch.uint8, device="cuda"))
            for _ in frames]
    ups = []
    for i in range(len(frames)):
        w, t = diff_loss_inputs(H, W, 6000 + i)
        wt = torch.from_numpy(w.astype(np.float32)).cuda()
        tt = torch.from_numpy(t.astype(np.float32)).cuda()
        ups.append(((-wt[None] * tt).contiguous(), (0.1 * wt).contiguous()))
    grads = [torch.empty((H, W), device="cuda") for _ in frames]
    pf.get_plan(intr, H, W, k, "implicit", "fp64")

    pf.get_plan(intr, H, W, k, "implicit", "fp32")

    def fwd(prec="fp64"):
        pf.fit_planes_batch(depth, intr, k, mode="implicit", precision=prec, outs=outs)

    def bwd():
        pf.fit_planes_backward_batch(depth, intr, k, [u[0] for u in ups], None,
                                     [u[1] for u in ups], outs=grads)

    def both():
        fwd()
        bwd()

    def both32():
        fwd("fp32")
        bwd()

    res = {"frames": len(frames), "pixels": len(frames) * H * W, "k": k, "mode": "implicit",
           "precision": "forward fp64 (fwd_bwd) or fp32 (fwd32_bwd); backward fp64"}
    for name, fn in (("fwd_bwd", both), ("fwd32_bwd", both32), ("bwd", bwd)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        n = 30
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / n
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_Mpx_s"] = round(res["pixels"] / (ms * 1e-3) / 1e6, 1)
    return res


def xyz_measure(torch, pf, frames_for):
    """The paper's comparison (Sec. II-E): the same fits in the standard XYZ
    formulation (nine depth-dependent window sums) against the RGBD one (four),
    FP64, one frame per launch, each timed over graph replays of 32 launches
    on rotating buffer sets."""
    res = {}
    for name, k in (("vga_640x480", 9), ("hd_1920x1080", 15)):
        f = frames_for(name)[0]
        sets = 8 if name.startswith("hd") else 32
        rig = Rig(torch, f.depth, sets)
        for mode in ("implicit", "explicit"):
            row = {}
            for kind, call in (("rgbd", pf.fit_planes), ("xyz", pf.fit_planes_xyz)):
                def run(s, call=call):
                    call(rig.depth[s], f.intrinsics, k, mode=mode, out=rig.outs[s][0])
                for i in range(5):
                    run(i % sets)
                torch.cuda.synchronize()
                side = torch.cuda.Stream()
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=side):
                        for j in range(32):
                            run(j % sets)
                torch.cuda.current_stream().wait_stream(side)
                g.replay()
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(5):
                    g.replay()
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / (5 * 32)
                row[f"{kind}_ms"] = round(ms, 5)
                row[f"{kind}_Mpx_s"] = round(f.depth.size / (ms * 1e-3) / 1e6, 1)
            row["xyz_over_rgbd_time"] = round(row["xyz_ms"] / row["rgbd_ms"], 3)
            res[f"{name}_k{k}_{mode}"] = row
        del rig
        torch.cuda.empty_cache()
    return res


def rects_measure(torch, pf, np, frames_for):
    """Fits to many rectangles of one 1080p frame (the paper's use of integral
    images, Sec. II-C): the FP64 integral images of the frame (three launches;
    44 algorithmic bytes per pixel: the depth in, five FP64 planes out), then
    100,000 seeded rectangles of 8..128 pixels a side, implicit and explicit;
    each timed over graph replays."""
    f = frames_for("hd_1920x1080")[0]
    H, W = f.depth.shape
    d = torch.from_numpy(f.depth).cuda()
    rng = np.random.Generator(np.random.PCG64(31))
    n = 100_000
    w = rng.integers(8, 129, n)
    h = rng.integers(8, 129, n)
    rects = np.stack([rng.integers(0, W - w + 1), rng.integers(0, H - h + 1), w, h], 1)
    r = torch.from_numpy(rects.astype(np.int32)).cuda()
    res = {"frame": "hd_1920x1080", "rects": n, "sides": "8..128"}
    for mode in ("implicit", "explicit"):
        ws = pf.integral_images(d, f.intrinsics, mode=mode)
        out = pf.fit_rects(ws, d.shape, f.intrinsics, r, mode=mode)
        for name, fn in (("integral", lambda: pf.integral_images(d, f.intrinsics, mode=mode,
                                                                 workspace=ws)),
                         ("rects", lambda: pf.fit_rects(ws, d.shape, f.intrinsics, r, mode=mode,
                                                        out=out))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=side):
                    for _ in range(10):
                        fn()
            torch.cuda.current_stream().wait_stream(side)
            g.replay()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(5):
                g.replay()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / 50
            res[f"{mode}_{name}_ms"] = round(ms, 5)
        res[f"{mode}_Mrects_s"] = round(n / (res[f"{mode}_rects_ms"] * 1e-3) / 1e6, 1)
        res[f"{mode}_integral_hbm_frac"] = round(
            44.0 * H * W / (res[f"{mode}_integral_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return res


def _time_calls(torch, run, sets, n_graph=16, reps=5):
    """ms per call of run(s) (s = buffer set), replayed from a captured HIP graph
    of n_graph consecutive calls on rotating sets."""
    for i in range(3):
        run(i % sets)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for j in range(n_graph):
                run(j % sets)
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (reps * n_graph)


def latency_measure(torch, pf, frames_for):
    """Single-frame latency of the 160x120 workload (k = 5, implicit FP64): the
    time from enqueue to completion of one fit, eager (host call + launch +
    synchronisation) and as one replay of a captured HIP graph; medians of 50."""
    f = frames_for("plain_160x120")[0]
    d = torch.from_numpy(f.depth).cuda()
    H, W = f.depth.shape
    out = (torch.empty((3, H, W), device="cuda"), torch.empty((H, W), device="cuda"),
           torch.empty((H, W), device="cuda"), torch.empty((H, W), dtype=torch.uint8, device="cuda"))
    run = lambda: pf.fit_planes(d, f.intrinsics, 5, out=out)
    for _ in range(5):
        run()
    torch.cuda.synchronize()
    eager = []
    for _ in range(50):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        eager.append((time.perf_counter() - t0) * 1e6)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            run()
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    graph, kern = [], []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(50):
        t0 = time.perf_counter()
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        graph.append((time.perf_counter() - t0) * 1e6)
        kern.append(a.elapsed_time(b) * 1e3)
    med = lambda v: round(sorted(v)[len(v) // 2], 1)
    return {"frame": "plain_160x120", "k": 5, "eager_us": med(eager), "graph_us": med(graph),
            "device_us": med(kern)}


def autotune_measure(torch, pf, frames_for):
    """Single-frame 640x480 launches at k = 9 with the plan's built-in launch
    shape, then with the band height and shape pf_plan_autotune picks (a derived
    plan; the shared one is not changed)."""
    f = frames_for("vga_640x480")[0]
    rig = Rig(torch, f.depth, 32)
    res = {}
    for mode in ("implicit", "explicit"):
        plan = pf.get_plan(f.intrinsics, 480, 640, 9, mode, "fp64")
        before = plan.tile_h
        run = lambda s, mode=mode: pf.fit_planes(rig.depth[s], f.intrinsics, 9, mode=mode,
                                                 out=rig.outs[s][0])
        t0 = _time_calls(torch, run, rig.sets)
        chosen, shape = plan.autotune(rig.depth[0])
        run = lambda s, mode=mode, bh=chosen, sh=shape: pf.fit_planes(
            rig.depth[s], f.intrinsics, 9, mode=mode, out=rig.outs[s][0], band_height=bh, shape=sh)
        t1 = _time_calls(torch, run, rig.sets)
        res[mode] = {"default_band_rows": before, "default_shape": plan.shape,
                     "default_Mpx_s": round(rig.pixels / (t0 * 1e-3) / 1e6, 1),
                     "tuned_band_rows": chosen, "tuned_shape": shape,
                     "tuned_Mpx_s": round(rig.pixels / (t1 * 1e-3) / 1e6, 1)}
    return res


def cpu_model():
    """The host CPU's model string (lscpu / /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frame, ks, mode, budget_s, threads=None):
    """The FP64 oracle on the host: random sample of window centres, growing until
    about budget_s seconds of work; returns Mpixel/s and what was sampled."""
    import numpy as np
    import oracle
    z = frame.depth.astype(np.float64)
    H, W = z.shape
    if threads is None:
        threads = os.cpu_count() or 1
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    rng = np.random.Generator(np.random.PCG64(7))
    n = 2000
    total_px, total_t = 0, 0.0
    while True:
        t0 = time.perf_counter()
        for k in ks:
            ys = rng.integers(0, H, n)
            xs = rng.integers(0, W, n)
            oracle.fit_points(z, frame.intrinsics, k, xs, ys, mode, threads=threads)
        dt = time.perf_counter() - t0
        total_px += n * len(ks)
        total_t += dt
        if total_t >= budget_s:
            break
        n = int(n * min(8.0, max(1.5, (budget_s - total_t) / max(dt, 1e-3))))
        n = min(n, 5_000_000)
    return dict(value=total_px / total_t / 1e6, unit="Mpixel/s", cores=threads, kind="oracle",
                cpu=cpu_model(),
                sample=f"{total_px} random window centres of the 640x480 frame, "
                       f"k in {list(ks)}, {mode} mode, FP64, {total_t:.1f} s")


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: frames are "
                          "independent, so N GPUs process N disjoint frame streams; "
                          "run it with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2103_06644_amd as pf
    from depthsynth import diff_loss_inputs, frames_for

    pf.load_library()
    copy_probe = None
    if args.copy_probe or not args.no_extras:
        # achievable HBM bandwidth: a 256 MiB device-to-device copy (read + write)
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 10
        nbytes = 2 * src.numel() * 4
        copy_probe = {"bytes_moved": nbytes, "ms": round(ms, 4),
                      "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                      "frac_of_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del src, dst
        torch.cuda.empty_cache()
    f = frames_for("vga_640x480")[0]
    ks = (3, 5, 9, 15)
    rig = Rig(torch, f.depth, args.sets, per_set=len(ks))
    ms_step, avg_launch_ms = time_launches(torch, pf, rig, f.intrinsics, ks, "implicit", "fp64",
                                           args.steps, args.warmup)
    px_step = rig.pixels * len(ks)
    value = px_step / (ms_step * 1e-3) / 1e6
    bytes_launch = px_step * BYTES_PER_PIXEL     # one launch fits the frame at all four k
    achieved = bytes_launch / (avg_launch_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "vga_640x480: one 640x480 depth frame (8 planar patches + 3 "
                               "spheres, 0.5-6 m, Kinect noise, 10% holes), windows k=3,5,9,15, "
                               "implicit fit, FP64 moments", "frame": [480, 640],
                   "windows": list(ks), "mode": "implicit", "precision": "fp64",
                   "buffer_sets": time_launches.sets_used},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(),
                     "kernel": "fit_planes_fused<double, implicit, no mask>",
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "bytes_per_pixel": BYTES_PER_PIXEL, "pixels_per_launch": px_step,
                     "avg_launch_ms": round(avg_launch_ms, 5)},
    }
    if not args.no_extras:
        progress("headline done; extras")
        extras = {"copy_probe_256MiB": copy_probe}
        # per-window throughput of single-frame launches at 640x480: the
        # integral-image fit's cost per pixel should not grow with the window
        per_k, per_k_tuned = {}, {}
        for mode in ("implicit", "explicit"):
            for k in ks:
                ms, avg = time_launches(torch, pf, rig, f.intrinsics, (k,), mode, "fp64", 64, 5)
                per_k[f"{mode}_k{k}"] = round(rig.pixels / (ms * 1e-3) / 1e6, 1)
                plan = pf.get_plan(f.intrinsics, 480, 640, k, mode, "fp64")
                tuned = plan.autotune(rig.depth[0])
                ms, avg = time_launches(torch, pf, rig, f.intrinsics, (k,), mode, "fp64", 64, 5,
                                        tuned=tuned)
                per_k_tuned[f"{mode}_k{k}"] = {"Mpx_s": round(rig.pixels / (ms * 1e-3) / 1e6, 1),
                                               "band_rows": tuned[0], "shape": tuned[1]}
        extras["vga_single_frame_per_k_Mpx_s"] = per_k
        extras["vga_single_frame_per_k_autotuned"] = per_k_tuned
        progress("per-k done")
        for mode, prec in (("explicit", "fp64"), ("implicit", "fp32"), ("explicit", "fp32"),
                           ("implicit", "compensated"), ("explicit", "compensated")):
            ms, _ = time_launches(torch, pf, rig, f.intrinsics, ks, mode, prec, 64, 5)
            extras[f"vga_{mode}_{prec}_Mpx_s"] = round(px_step / (ms * 1e-3) / 1e6, 1)
        # paper variants on the headline frame, k = 3, 5, 9, 15: partial windows (at
        # least half of each window valid), the literal |(a,b,c,d)| = 1 constraint,
        # and disparity input (D = f b / Z with f b = 39.375)
        variants = {}
        half = [max(3, k * k // 2) for k in ks]   # min_valid per window size
        for name, kw, mode in (("partial_half_implicit", "partial", "implicit"),
                               ("partial_half_explicit", "partial", "explicit"),
                               ("literal_implicit", None, "implicit_literal")):
            mv = half if kw == "partial" else None
            t = _time_calls(torch, lambda s, mode=mode, mv=mv: pf.fit_planes_batch(
                [rig.depth[s]] * len(ks), f.intrinsics, list(ks), mode=mode, min_valid=mv,
                outs=rig.outs[s]), rig.sets)
            variants[name] = {"ms_per_step": round(t, 5),
                              "Mpx_s": round(rig.pixels * len(ks) / (t * 1e-3) / 1e6, 1)}
        dsc = 1.0 / 39.375
        drig = [(39.375 / torch.clamp(d, min=1e-6)) * (d > 0) for d in rig.depth]
        t = _time_calls(torch, lambda s: pf.fit_planes_batch(
            [drig[s]] * len(ks), f.intrinsics, list(ks), outs=rig.outs[s],
            disparity_scale=dsc), rig.sets)
        variants["disparity_implicit"] = {"ms_per_step": round(t, 5),
                                          "Mpx_s": round(rig.pixels * len(ks) / (t * 1e-3) / 1e6, 1)}
        extras["variants_vga_k3-15"] = variants
        progress("variants done")
        del rig
        torch.cuda.empty_cache()
        hd = frames_for("hd_1920x1080")[0]
        rig_hd = Rig(torch, hd.depth, 8, per_set=1)
        for mode in ("implicit", "explicit"):
            for k in (15, 31):
                ms, avg = time_launches(torch, pf, rig_hd, hd.intrinsics, (k,), mode, "fp64",
                                        40, 5)
                rec = {"Mpx_s": round(rig_hd.pixels / (ms * 1e-3) / 1e6, 1),
                       "avg_launch_ms": round(avg, 5),
                       "hbm_frac": round(rig_hd.pixels * BYTES_PER_PIXEL / (avg * 1e-3) / 1e9 /
                                         HBM_PEAK_GBS, 4)}
                # the band height and launch shape pf_plan_autotune picks on this frame
                plan = pf.get_plan(hd.intrinsics, 1080, 1920, k, mode, "fp64")
                tuned = plan.autotune(rig_hd.depth[0])
                ms, avg = time_launches(torch, pf, rig_hd, hd.intrinsics, (k,), mode, "fp64",
                                        40, 5, tuned=tuned)
                rec["autotuned"] = {
                    "band_rows": tuned[0], "shape": tuned[1],
                    "Mpx_s": round(rig_hd.pixels / (ms * 1e-3) / 1e6, 1),
                    "avg_launch_ms": round(avg, 5),
                    "hbm_frac": round(rig_hd.pixels * BYTES_PER_PIXEL / (avg * 1e-3) / 1e9 /
                                      HBM_PEAK_GBS, 4)}
                extras[f"hd_{mode}_k{k}"] = rec
        for mode in ("implicit", "explicit"):
            t15 = extras[f"hd_{mode}_k15"]["autotuned"]["Mpx_s"]
            t31 = extras[f"hd_{mode}_k31"]["autotuned"]["Mpx_s"]
            # the integral-image fit's cost per pixel should not grow with the window
            extras[f"hd_{mode}_k31_over_k15_autotuned"] = round(t31 / t15, 3)
        del rig_hd
        torch.cuda.empty_cache()
        progress("1080p done")
        extras["batch_mixed_64"] = batch_measure(torch, pf, np, frames_for)
        extras["batch_mixed_64_queued"] = batch_measure(torch, pf, np, frames_for, queued=True)
        extras["latency_160x120"] = latency_measure(torch, pf, frames_for)
        progress("batches and latency done")
        extras["diff_8x640x480"] = diff_measure(torch, pf, np, frames_for, diff_loss_inputs)
        extras["xyz_vs_rgbd"] = xyz_measure(torch, pf, frames_for)
        extras["rects_1080p"] = rects_measure(torch, pf, np, frames_for)
        extras["autotune_vga_k9"] = autotune_measure(torch, pf, frames_for)
        out["extras"] = extras
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(f, ks, "implicit", args.cpu_seconds)
        one = cpu_baseline(f, ks, "implicit", max(2.0, args.cpu_seconds / 4), threads=1)
        out["cpu_baseline"]["one_thread"] = {"value": one["value"], "sample": one["sample"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
