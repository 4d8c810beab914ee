#!/usr/bin/env python
"""Light-field frame benchmark on one MI355X.

A step renders one light field of the clustered-Gaussian workload: 500,000 Gaussians,
512 x 512 views, N_chunk = 64 quantile planes, 45 horizontally sheared views over +-20 deg
(D_focal = 2, base fov 50 deg), nearest sampling.  The step is the whole forward hot path:
lf_build_mpi (cull, key, depth sort, chunking, tile binning, splat into planes) followed
by lf_composite (swizzle blending of all 45 views).  Inputs are seeded synthetic scenes
(scenegen) resident in HBM before timing starts.

The JSON line reports views/s of the FP32-plane form (FP32 views) as ``value`` and beside
it the FP16-, BF16- and UNORM8-plane forms (FP16 views), the FP32 form with bilinear
sampling, the roofline of the dominant kernel and of the composite against the 8 TB/s HBM
peak and against a measured device-copy rate, per-phase kernel times measured with HIP
events on the launch stream, and the FP64 CPU oracle's rate on the whole frame computed
by a pool of worker processes over the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s

# HBM traffic per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE; KiB
# per dispatch) of `bench.py --steps 2 --warmup 1 --forms f32 --extra "" --copy-calibration`,
# scaled by what the same counters read for a plain 256 MiB device copy (FETCH_SIZE
# 131084 KiB, WRITE_SIZE 262144 KiB): fetch x 2.0, write x 1.0.  Each entry records a digest
# of the kernel's source text; when the kernel has changed since, the traffic is reported as
# null.
COPY_FETCH_SCALE = 262144.0 / 131084.0
COPY_WRITE_SCALE = 262144.0 / 262144.0
_DEV = "paper_2508_18540_amd/csrc/build_device.h::"
MEASURED_TRAFFIC = {
    "splat_gs": dict(src="paper_2508_18540_amd/csrc/build_gs.hip", fetch_kib=50944, write_kib=286992,
                     helpers=("block_max_q", "reached_quadrants", "splat_stage", "splat_item", "bucket_segments",
                              "emit_items", _DEV + "seg_count", _DEV + "item_order", _DEV + "item_bucket",
                              _DEV + "xcd_item", "paper_2508_18540_amd/csrc/build_api.cpp::splat_item_shift"),
                     digest="b08401825c5240c4"),
    "composite_wave": dict(src="paper_2508_18540_amd/csrc/composite.hip", fetch_kib=88267, write_kib=184320,
                           helpers=("composite_wave_tile",), digest="2dadd58c87f87f47"),
}


def kernel_digest(path, name, helpers=()):
    """sha1 of a kernel's definition (from its signature to the closing brace in column 0),
    preceded by the definitions of the device functions and kernels it is built from or whose
    output decides its traffic (a helper "file::name" is looked up in that file)."""
    import hashlib
    import re

    parts = []
    for h in tuple(helpers) + (name,):
        src, fn = h.split("::") if "::" in h else (path, h)
        text = open(os.path.join(ROOT, src)).read()
        # (a helper from another file may be a host function: any definition in column 0)
        kind = "__global__" if h == name else ("[A-Za-z_]" if "::" in h else "__(?:device|global)__")
        m = re.search(r"^(template <[^\n]*>\n)?" + kind + r"[^\n]*\b" + re.escape(fn) + r"\(", text, re.M)
        if not m:
            return None
        end = text.find("\n}\n", m.start())
        if end < 0:
            return None
        parts.append(text[m.start():end])
    return hashlib.sha1("".join(parts).encode()).hexdigest()[:16]


def measured_traffic(name):
    """Counter-measured HBM bytes per launch of `name`, or None if the kernel changed since."""
    t = MEASURED_TRAFFIC.get(name)
    if t is None or kernel_digest(t["src"], name, t.get("helpers", ())) != t["digest"]:
        return None
    return int(round((t["fetch_kib"] * COPY_FETCH_SCALE + t["write_kib"] * COPY_WRITE_SCALE) * 1024))
# VALU wave-instructions per wave-sample from rocprofv3 --pmc SQ_INSTS_VALU (per dispatch, divided
# by samples / 64) of `bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-bilinear --forms f32
# --extra ""`, digest-gated like the traffic
MEASURED_VALU = {
    "composite_wave": dict(src="paper_2508_18540_amd/csrc/composite.hip", valu_per_wave_sample=7.99,
                           helpers=("composite_wave_tile",), digest="2dadd58c87f87f47"),
}


def measured_valu(name):
    t = MEASURED_VALU.get(name)
    if t is None or kernel_digest(t["src"], name, t.get("helpers", ())) != t["digest"]:
        return None
    return t["valu_per_wave_sample"]


SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: float32 lane-ops/s (no packed math)
FP32_PEAK_TFLOPS = 2 * VALU_LANE_OPS / 1e12   # one FMA = 2 flops per lane-op -> 78.6


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--interp", default="nearest", choices=["nearest", "bilinear"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-processes", type=int, default=0, help="oracle worker processes (0: the host's cores, "
                   "at most 16)")
    p.add_argument("--forms", default="f32,f16,bf16,u8",
                   help="plane storage forms to time (first one is `value`; f32 writes FP32 views, the others FP16)")
    p.add_argument("--no-bilinear", action="store_true", help="skip the bilinear-sampling row")
    p.add_argument("--extra", default="voxel256,grad200k,quilt2d,sh500k,batch8",
                   help="further workloads timed into the same line (voxel256, grad200k, quilt2d, sh500k, "
                        "batch8; empty for none)")
    p.add_argument("--extra-steps", type=int, default=5)
    p.add_argument("--only-extra", action="store_true",
                   help="time only the --extra workloads (for profiling them on their own)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain device copy of known size (for HBM counter scaling)")
    return p.parse_args()


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(config, n_views, interp, processes):
    """The FP64 oracle on the whole frame (every plane, every view), its per-plane and
    per-view work spread over worker processes.  The pool forks, so it runs as a child
    program (this process has used the GPU)."""
    import subprocess
    import tempfile

    with tempfile.TemporaryDirectory(prefix="lf_cpu_") as d:
        cmd = [sys.executable, "-m", "oracle.pool", "frame", "--config", config, "--out", d, "--no-save",
               "--interp", interp]
        if processes:
            cmd += ["--processes", str(processes)]
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            return dict(error=r.stderr[-2000:])
        t = json.load(open(os.path.join(d, "timing.json")))
    frame_s = t["partition_s"] + t["planes_s"] + t["views_s"]
    return dict(value=round(n_views / frame_s, 3), unit="views/s", cores=t["processes"], kind="oracle",
                cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                sample=(f"the whole {config} frame: partition of every Gaussian ({t['partition_s']:.2f} s, one "
                        f"process), every plane rasterised ({t['planes_s']:.2f} s) and every view composited "
                        f"({t['views_s']:.2f} s) on {t['processes']} worker processes; {frame_s:.1f} s wall"),
                measured_s=round(frame_s, 2))


def copy_rate(dev, nbytes=1 << 30, reps=5):
    """Best device-to-device copy rate (bytes read + written per second, GB/s) of a plain
    torch copy of nbytes, timed with HIP events: the achievable HBM bandwidth."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * nbytes / (best * 1e-3) / 1e9


def _passes(fn, steps, ctx, L):
    """The timed region, then the instrumented one: `steps` calls of fn with the library's
    per-phase HIP events off (the step time reported), then `steps` more with them on (the
    per-phase times, from events recorded on the launch stream; the events add about 0.03
    ms to a cluster500k frame, so they stay out of the step time).  Returns (ms per step,
    ms per step instrumented, {phase: (total ms, launches)})."""
    import torch
    L.lf_profile_enable(ctx.handle, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.lf_profile_read(ctx.handle, reset=True)
    L.lf_profile_enable(ctx.handle, True)
    t2 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    L.lf_profile_enable(ctx.handle, False)
    prof = L.lf_profile_read(ctx.handle, reset=True)
    return (t1 - t0) * 1e3 / steps, (t3 - t2) * 1e3 / steps, prof


def _timed(fn, warmup, steps, ctx, L):
    """Run fn warmup times, then _passes; returns (ms per step, {phase: ms per step})."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ms, _, prof = _passes(fn, steps, ctx, L)
    return ms, {k: round(v[0] / steps, 4) for k, v in prof.items() if v[1]}


def extra_voxel256(ctx, steps, warmup):
    """Sparse-voxel light field: 335,544 voxels (256^3 grid, 2 %), 512^2, 64 planes, 96 views,
    FP16 planes, build (with the plane low-pass) + composite."""
    import numpy as np
    import torch

    import scenegen
    from paper_2508_18540_amd import _lib as L
    from paper_2508_18540_amd import torch_api as T

    vox, cam, cfg = scenegen.config("voxel256")
    K, V = cfg["n_chunk"], cfg["vx"]
    vlist = L.lf_quilt_views(L.make_camera(cam), V, 1)
    ds = T.to_device(vox)
    ws = T.workspace_for(ds, cam, K)
    out = T.build_mpi(ctx, ds, cam, K, dtype=torch.float16, workspace=ws)
    img = torch.empty((V, cam.ny, cam.nx, 4), dtype=torch.float16, device="cuda")

    def step():
        T.build_mpi(ctx, ds, cam, K, dtype=torch.float16, workspace=ws, out=out)
        T.composite(ctx, out["rgba"], out["depth"], cam, vlist, "nearest", out=img)
    ms, ph = _timed(step, warmup, steps, ctx, L)
    T.build_stats(ctx, ws, check=True)
    return dict(workload="voxel256: 335,544 voxels, 512x512, 64 quantile planes, 96 views, FP16 planes and views",
                views_per_s=round(V / (ms * 1e-3), 1), ms_per_step=round(ms, 4), phases_ms=ph)


def extra_grad200k(ctx, steps, warmup):
    """Differentiation step: 200k Gaussians, 512^2, 128 planes, 45 views, FP32; forward
    (build + composite), L2 loss against a target light field, backward through the
    composite and the build to the five parameter tensors."""
    import torch

    import scenegen
    from paper_2508_18540_amd import _lib as L
    from paper_2508_18540_amd import torch_api as T

    scene, cam, cfg = scenegen.config("grad200k")
    K, V = cfg["n_chunk"], cfg["vx"]
    vlist = L.lf_quilt_views(L.make_camera(cam), V, 1)
    target = scenegen.perturbed_target(scene, cfg["target_seed"])
    with torch.no_grad():
        tout = T.build_mpi(ctx, T.to_device(target), cam, K)
        timg = T.composite(ctx, tout["rgba"], tout["depth"], cam, vlist, "nearest")
    del tout
    params = {k: v.clone().requires_grad_(True) for k, v in T.to_device(scene).items()}
    ws = T.workspace_for(params, cam, K)

    def step():
        img = T.render_light_field(ctx, params, cam, vlist, K, "nearest", workspace=ws)
        loss = ((img[..., :3] - timg[..., :3]) ** 2).sum()
        loss.backward()
    ms, ph = _timed(step, warmup, steps, ctx, L)
    return dict(workload="grad200k: 200k Gaussians, 512x512, 128 quantile planes, 45 views, FP32; forward + "
                         "L2 loss + backward to means, log-scales, quaternions, opacities, colours",
                ms_per_step=round(ms, 4), views_per_s=round(V / (ms * 1e-3), 1), phases_ms=ph)


def extra_quilt2d(ctx, steps, warmup):
    """2D parallax: the cluster500k scene, 512^2, 64 quantile planes, FP32, composited into a
    9 x 5 quilt (five vertical offsets); build + composite per step.  Beside it, the composite
    alone with the row kernel (views grouped by dy) and with the per-pixel kernel."""
    import os

    import torch

    import scenegen
    from paper_2508_18540_amd import _lib as L
    from paper_2508_18540_amd import torch_api as T

    scene, cam, cfg = scenegen.config("quilt2d")
    K, V = cfg["n_chunk"], cfg["vx"] * cfg["vy"]
    vlist = L.lf_quilt_views(L.make_camera(cam), cfg["vx"], cfg["vy"])
    ds = T.to_device(scene)
    ws = T.workspace_for(ds, cam, K)
    out = T.build_mpi(ctx, ds, cam, K, workspace=ws)
    info, st = T.build_stats(ctx, ws, check=False)
    if st == L.LF_ERR_CAPACITY:
        ws = T.workspace_for(ds, cam, K, entry_capacity=int(info.entries_needed * 1.25))
        out = T.build_mpi(ctx, ds, cam, K, workspace=ws)
    img = torch.empty((V, cam.ny, cam.nx, 4), dtype=torch.float32, device="cuda")

    def step():
        T.build_mpi(ctx, ds, cam, K, workspace=ws, out=out)
        T.composite(ctx, out["rgba"], out["depth"], cam, vlist, "nearest", out=img)
    ms, ph = _timed(step, warmup, steps, ctx, L)
    T.build_stats(ctx, ws, check=True)
    comp = {}
    for kern in ("rows", "general"):
        os.environ["LF_COMPOSITE_KERNEL"] = kern
        try:
            _, cph = _timed(lambda: T.composite(ctx, out["rgba"], out["depth"], cam, vlist, "nearest", out=img),
                            warmup, steps, ctx, L)
        finally:
            del os.environ["LF_COMPOSITE_KERNEL"]
        comp[kern] = cph.get("composite")
    return dict(workload="quilt2d: 500k clustered Gaussians, 512x512, 64 quantile planes, 9x5 views "
                         "(+-20 x +-10 deg), FP32",
                views_per_s=round(V / (ms * 1e-3), 1), ms_per_step=round(ms, 4), phases_ms=ph,
                composite_ms_row_kernel=comp["rows"], composite_ms_per_pixel_kernel=comp["general"])


def extra_sh500k(ctx, steps, warmup):
    """SH colour (the ablation of Fig. 6): the cluster500k scene with degree-3 spherical-
    harmonic colour (seeded coefficients), 512^2, 64 quantile planes of 52 float32s per
    texel, 45 views; build + composite per step, beside the RGB path's plane bytes."""
    import torch

    import scenegen
    from paper_2508_18540_amd import _lib as L
    from paper_2508_18540_amd import torch_api as T

    scene, cam, cfg = scenegen.config("cluster500k")
    K, V = cfg["n_chunk"], cfg["vx"]
    vlist = L.lf_quilt_views(L.make_camera(cam), V, 1)
    ds = T.to_device(scene)
    coef = torch.from_numpy(scenegen.sh_coefficients(scene["means"].shape[0], 3, 7)).cuda()
    ws = T.workspace_for(ds, cam, K)
    out = T.build_mpi_sh(ctx, ds, coef, cam, K, workspace=ws)
    info, st = T.build_stats(ctx, ws, check=False)
    if st == L.LF_ERR_CAPACITY:
        ws = T.workspace_for(ds, cam, K, entry_capacity=int(info.entries_needed * 1.25))
        out = T.build_mpi_sh(ctx, ds, coef, cam, K, workspace=ws)
    img = torch.empty((V, cam.ny, cam.nx, 4), dtype=torch.float32, device="cuda")

    def step():
        T.build_mpi_sh(ctx, ds, coef, cam, K, workspace=ws, out=out)
        T.composite_sh(ctx, out["planes"], out["depth"], 3, cam, vlist, "nearest", out=img)
    ms, ph = _timed(step, warmup, steps, ctx, L)
    T.build_stats(ctx, ws, check=True)
    return dict(workload="sh500k: cluster500k with degree-3 SH colour, 512x512, 64 quantile planes (52 float32 "
                         "per texel), 45 views",
                views_per_s=round(V / (ms * 1e-3), 1), ms_per_step=round(ms, 4), phases_ms=ph,
                plane_bytes=int(out["planes"].numel() * 4), rgb_plane_bytes=int(out["planes"][..., :4].numel() * 4))


def extra_batch8(ctx, steps, warmup):
    """Eight clustered-Gaussian scenes of uneven size in one batch (seeds 30+i): (N, res,
    N_chunk, views) from 50k / 256^2 / 64 / 9 up to 2M / 768^2 / 128 / 45, FP16 planes and
    views, autotuned view groups and row tiles, one HIP graph replay per step, in the
    work-list form (one splat, merge and composite launch over every scene's work items;
    `ms_per_step`) and the per-scene stream form; beside them the same scenes rendered one
    after another with the single-scene entry points."""
    import math

    import numpy as np
    import torch

    import scenegen
    from paper_2508_18540_amd import _lib as L
    from paper_2508_18540_amd import torch_api as T

    scenes = []
    for i, (n, res, K, V) in enumerate(scenegen.BATCH_SCENES):
        cam = scenegen.camera(res, res, 50.0, 2.0, math.radians(40.0))
        vl = L.lf_quilt_views(L.make_camera(cam), V, 1)
        scenes.append(dict(scene=T.to_device(scenegen.cluster_scene(n, seed=30 + i)), cam=cam, n_chunk=K, views=vl,
                           plane_dtype=torch.float16, out_dtype=torch.float16))
    b = T.Batch(ctx, scenes, graph=True, autotune=True, worklist=True)
    groups, tiles = b.groups(), b.tiles()
    ms, _ = _timed(b.run, warmup, steps, ctx, L)
    b.stats(check=True)
    total_views = sum(len(sc["views"]) for sc in scenes)
    # the stream form over the same scenes and buffers (the tuned choices come from the cache)
    bs = T.Batch(ctx, scenes, graph=True, autotune=True, worklist=False)
    ms_streams, _ = _timed(bs.run, warmup, steps, ctx, L)
    bs.stats(check=True)
    bs.close()

    def sequential():
        for sc, o in zip(scenes, b.outs):
            T.build_mpi(ctx, sc["scene"], sc["cam"], sc["n_chunk"], dtype=torch.float16, workspace=o["workspace"],
                        out=o)
            T.composite(ctx, o["rgba"], o["depth"], sc["cam"], sc["views"], "nearest", out=o["views"])
    ms_seq, _ = _timed(sequential, warmup, steps, ctx, L)
    b.close()
    return dict(workload="batch8: 8 scenes, 50k-2M Gaussians, 256^2-768^2, N_chunk 64/128/512, 9-100 views, "
                         "FP16 planes and views",
                # the step is the stream form, the library's default (the faster form)
                views_per_s=round(total_views / (ms_streams * 1e-3), 1), ms_per_step=round(ms_streams, 4),
                total_views=total_views,
                worklist_ms=round(ms, 4), streams_ms=round(ms_streams, 4), sequential_ms=round(ms_seq, 4),
                autotuned_view_groups=groups,
                autotuned_row_tiles=tiles)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a design note, "
                                   "not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen
    from paper_2508_18540_amd import _lib as L
    from paper_2508_18540_amd import torch_api as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    ctx = T.Context(0)
    if args.only_extra:
        line = {"only_extra": True}
        for name in [x.strip() for x in args.extra.split(",") if x.strip()]:
            fn = {"voxel256": extra_voxel256, "grad200k": extra_grad200k, "quilt2d": extra_quilt2d,
                  "sh500k": extra_sh500k, "batch8": extra_batch8}[name]
            line[name] = fn(ctx, args.extra_steps, 2)
        print(json.dumps(line), flush=True)
        return
    scene, cam, cfg = scenegen.config("cluster500k")
    K, V = cfg["n_chunk"], cfg["vx"] * cfg["vy"]
    camc = L.make_camera(cam)
    vlist = L.lf_quilt_views(camc, cfg["vx"], cfg["vy"])
    dx = np.array([v.dx for v in vlist], dtype=np.float32)
    dy = np.array([v.dy for v in vlist], dtype=np.float32)
    geo = L.lf_geometry(camc)
    ds = T.to_device(scene, dev)
    torch.cuda.synchronize()

    # size the workspace from one probe build (re-allocated once if the default is short)
    ws = T.workspace_for(ds, cam, K, device=dev)
    T.build_mpi(ctx, ds, cam, K, dtype=torch.float32, workspace=ws)
    info, st = T.build_stats(ctx, ws, check=False)
    if st == L.LF_ERR_CAPACITY:
        ws = T.workspace_for(ds, cam, K, entry_capacity=int(info.entries_needed * 1.25), device=dev)

    def one_form(form, interp):
        pdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16, "u8": torch.uint8}[form]
        vdt = torch.float32 if form == "f32" else torch.float16
        out = T.build_mpi(ctx, ds, cam, K, dtype=pdt, workspace=ws)
        img = torch.empty((V, cam.ny, cam.nx, 4), dtype=vdt, device=dev)

        def step():
            T.build_mpi(ctx, ds, cam, K, dtype=pdt, workspace=ws, out=out)
            T.composite(ctx, out["rgba"], out["depth"], cam, vlist, interp, out=img, out_dtype=vdt)

        for _ in range(args.warmup):
            step()
        info, st = T.build_stats(ctx, ws, check=True)
        ms, ms_instr, prof = _passes(step, args.steps, ctx, L)
        info, st = T.build_stats(ctx, ws, check=True)
        phases = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]}
        pb = {"f32": 16, "f16": 8, "bf16": 8, "u8": 4}[form]
        comp_bytes = K * geo.plane_height * geo.plane_width * pb + V * cam.ny * cam.nx * (16 if form == "f32" else 8)
        comp_ms = phases["composite"]
        gbs = comp_bytes / (comp_ms * 1e-3) / 1e9
        comp_roof = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS,
                         unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4), copy_peak=round(copy_gbs, 1),
                         frac_of_copy=round(gbs / copy_gbs, 4),
                         traffic=measured_traffic("composite_wave") if form == "f32" and interp == "nearest" else None,
                         kernel="composite_wave", bytes_per_launch=comp_bytes,
                         avg_ms=round(comp_ms, 4))
        # splat: algorithmic work = the support pairs, (Gaussian, texel) pairs with o G >= 1/255,
        # counted on the device over the frame's tile lists (outside the timed region), at 16
        # flop-equivalent slots each (Taylor-form quadratic 5 FMA, exp2, min, select, blend 4
        # FMA + T update); beside them the (entry, texel) evaluations the kernel performs and
        # the texels of the whole listed tiles, per support pair
        splat_ms = phases["splat"]
        work = T.splat_work(ctx, ds, cam, K, ws)
        pairs = work["support_pairs"]
        splat_roof = dict(bound="alu", achieved=round(pairs * 16 / (splat_ms * 1e-3) / 1e12, 3),
                          peak=round(FP32_PEAK_TFLOPS, 1), unit="TFLOP/s",
                          frac=round(pairs * 16 / (splat_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                          traffic=measured_traffic("splat_gs") if form == "f32" else None, kernel="splat_gs",
                          support_pairs=pairs, flops_per_launch=pairs * 16,
                          evaluations_per_pair=round(work["evaluations"] / max(pairs, 1), 3),
                          list_texels_per_pair=round(work["list_texels"] / max(pairs, 1), 3),
                          avg_ms=round(splat_ms, 4))
        # the composite's instruction-issue view: VALU wave-instructions per wave-sample (64
        # samples) from the rocprofv3 SQ_INSTS_VALU counter of the nearest FP32 composite kernel
        # (null once that kernel has changed), and the share of the SIMDs' VALU issue slots they
        # take (a wave64 VALU instruction occupies a SIMD for 4 cycles)
        samples = V * cam.ny * cam.nx * K
        vpw = measured_valu("composite_wave") if form == "f32" and interp == "nearest" else None
        comp_valu = dict(bound="alu", kernel="composite_wave", samples_per_launch=samples,
                         valu_per_wave_sample=vpw,
                         issue_frac=(round(samples / 64 * vpw * 4 / (comp_ms * 1e-3 * SIMDS * CLOCK_HZ), 4)
                                     if vpw else None))
        return dict(form=form, views="f32" if form == "f32" else "f16", interp=interp, ms_per_step=ms,
                    ms_per_step_instrumented=ms_instr, views_per_s=V / (ms * 1e-3), phases_ms=phases,
                    composite_roofline=comp_roof, splat_roofline=splat_roof, composite_valu=comp_valu,
                    entries=int(info.entries_needed), n_visible=int(info.n_visible))

    copy_gbs = copy_rate(dev)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    res = {f: one_form(f, args.interp) for f in forms}
    bil = one_form(forms[0], "bilinear") if args.interp == "nearest" and not args.no_bilinear else None
    main_r = res[forms[0]]
    ph = main_r["phases_ms"]
    dominant = max(("splat", "composite"), key=lambda k: ph.get(k, 0.0))
    roof = main_r["splat_roofline"] if dominant == "splat" else main_r["composite_roofline"]

    if args.copy_calibration:
        a = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    line = {
        "metric": "light-field views/sec at 512^2, N_chunk=64 (FP32 vs FP16 planes); % HBM peak",
        "value": round(main_r["views_per_s"], 1),
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 4),
        # the same steps again with the per-phase HIP events on: phases_ms and the rooflines'
        # kernel times come from that pass
        "ms_per_step_instrumented": round(main_r["ms_per_step_instrumented"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 64-cluster Gaussian mixture)",
        "config": {"workload": "cluster500k: 500k Gaussians, 512x512 views, N_chunk=64 quantile planes, "
                               "45x1 views over +-20 deg, D_focal=2, fov 50 deg, nearest sampling",
                   "planes": forms[0], "interp": args.interp, "n_gaussians": 500_000, "n_chunk": K,
                   "views": V, "resolution": [cam.nx, cam.ny]},
        "roofline": roof,
        "copy_gbs": round(copy_gbs, 1),
        "composite_roofline": main_r["composite_roofline"],
        "splat_roofline": main_r["splat_roofline"],
        "composite_valu": main_r["composite_valu"] if args.interp == "nearest" else None,
        "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "entries": main_r["entries"],
        "n_visible": main_r["n_visible"],
    }
    for f in forms[1:]:
        r = res[f]
        line[f"{f}_planes"] = {"value": round(r["views_per_s"], 1), "views": r["views"],
                               "ms_per_step": round(r["ms_per_step"], 4),
                               "speedup_vs_" + forms[0]: round(main_r["ms_per_step"] / r["ms_per_step"], 3),
                               "composite_speedup_vs_" + forms[0]:
                                   round(ph["composite"] / r["phases_ms"]["composite"], 3),
                               "composite_roofline": r["composite_roofline"],
                               "phases_ms": {k: round(v, 4) for k, v in r["phases_ms"].items()}}
    if bil is not None:
        line["bilinear"] = {"value": round(bil["views_per_s"], 1), "planes": forms[0], "views": bil["views"],
                            "ms_per_step": round(bil["ms_per_step"], 4),
                            "slowdown_vs_nearest": round(bil["ms_per_step"] / main_r["ms_per_step"], 3),
                            "composite_roofline": bil["composite_roofline"],
                            "phases_ms": {k: round(v, 4) for k, v in bil["phases_ms"].items()}}
    for name in [x.strip() for x in args.extra.split(",") if x.strip()]:
        fn = {"voxel256": extra_voxel256, "grad200k": extra_grad200k, "quilt2d": extra_quilt2d,
                  "sh500k": extra_sh500k, "batch8": extra_batch8}[name]
        line[name] = fn(ctx, args.extra_steps, 2)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline("cluster500k", V, args.interp, args.cpu_processes)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
