"""Benchmark: Mpath-segments/s of the generalized-ray tracer on the mid terrain workload.

Workload: 65,536-triangle value-noise terrain with 16x16 material tiles (smooth, Gaussian
rough, sinusoidal grating), one partially coherent area emitter, 512 x 512 sensor, 16 samples
per pixel, 8 wavelengths, path depth <= 4 (seeded, synthetic).  One step = one full trace of
that workload (33.6M paths) including the per-pixel reduction, inputs resident on the GPU.

Prints one JSON line.  Only one GPU is supported (--gpus > 1 exits with a message).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
NODE_BYTES = 112     # bytes of a 4-wide node the traversal reads (boxes + child links)
TRI_BYTES = 48       # bytes of a triangle record
HIT_BYTES = 48 + 48 + 32   # closest hit: triangle, shading normals, material
RECORD_BYTES = 4     # one float per path

# HBM traffic of one trace-kernel launch on this workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by a plain copy of known size; valid only for the kernel sources it was
# measured on (sha256 prefix of the files below).
TRAFFIC_BYTES = 1_256_000 * 1024
TRAFFIC_KERNEL_HASH = "576957f4c11260db"
KERNEL_SOURCES = ["paper_2303_15762_amd/csrc/trace.hip", "paper_2303_15762_amd/csrc/device_math.hpp",
                  "paper_2303_15762_amd/csrc/kernels.hpp"]


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for s in KERNEL_SOURCES:
        with open(os.path.join(root, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(st):
    """Scene and output bytes one trace-kernel launch requests, from the in-kernel counters:
    node and triangle fetches of both traversals, the shading reads of each closest hit
    (approximated by segments - paths: every path ends on at most one miss) and one float
    written per path.  Path state stays in registers and moves no memory."""
    hits = max(0, st["segments"] - st["paths"])
    return (st["node_visits"] * NODE_BYTES + st["tri_tests"] * TRI_BYTES + hits * HIT_BYTES
            + st["paths"] * RECORD_BYTES)


def cpu_baseline(wl, target_s=15.0):
    import oracle
    from workloads import scenes as W  # noqa: F401
    osc = oracle.OracleScene(wl.scene)
    rng = np.random.default_rng(123)
    threads = os.cpu_count() or 1

    def run(npx):
        pix = np.stack([rng.integers(0, wl.sensor.width, npx), rng.integers(0, wl.sensor.height, npx)], 1)
        t0 = time.perf_counter()
        _, st = oracle.render(wl, osc, pixels=pix, n_threads=threads)
        return time.perf_counter() - t0, st["segments"]

    dt, seg = run(64)
    npx = int(max(64, min(wl.sensor.width * wl.sensor.height, 64 * target_s / max(dt, 1e-3))))
    dt, seg = run(npx)
    return {"value": seg / dt / 1e6, "unit": "Mpath-segments/s", "cores": threads, "kind": "oracle",
            "sample": f"{npx} random pixels x {wl.spp} samples x {len(wl.lambdas_um)} wavelengths of the "
                      f"same workload ({seg} segments, {dt:.1f} s, FP64 C++ oracle, {threads} threads)"}


def surrogate_leg(R, wl, o_plain, img, st_plain, args):
    """Train the learned p_w (outside the timed region), then time the same workload with the
    surrogate path.  Its image is compared with the plain-path image of this GPU."""
    import torch
    from paper_2303_15762_amd.surrogate import Surrogate
    S = Surrogate(R)
    t0 = time.perf_counter()
    p, hist = S.train()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    S.install(p)
    o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p, bsdf_mode=1)
    plain = img.clone()
    img_s = torch.zeros_like(img)
    _, st = R.trace(wl.lambdas_um, o, image=img_s, stats=True)
    err = float((img_s - plain).norm() / plain.norm())
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(R.stream)
    for _ in range(args.steps):
        R.trace(wl.lambdas_um, o, image=img_s, stats=False)
    e1.record(R.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    return {"value": round(st["segments"] / (ms * 1e-3) / 1e6, 2), "unit": "Mpath-segments/s",
            "ms_per_step": round(ms, 3), "rel_l2_vs_plain_gpu_image": err,
            "surrogate_evals_per_step": st["surrogate_evals"], "fallbacks_per_step": st["fallbacks"],
            "train_s": round(t_train, 2), "train_steps": hist["step"][-1],
            "val_mse_log_pw": hist["val_loss"][-1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip the learned-p_w leg (training takes a few seconds)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (scales the "
                         "HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the tracer is data-parallel over samples and the "
              "multi-GPU split is not built (see the sharding notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_15762_amd import Renderer
    from workloads import mid_terrain

    wl = mid_terrain()
    R = Renderer(0)
    info = R.load_workload(wl)
    o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p)
    img = torch.zeros((len(wl.lambdas_um), wl.sensor.height, wl.sensor.width), device=R.dev)
    # warmup (also gives the deterministic counters of one step)
    st = None
    for _ in range(max(1, args.warmup)):
        img.zero_()
        _, st = R.trace(wl.lambdas_um, o, image=img, stats=True)
    segments = st["segments"]
    stream = R.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        R.trace(wl.lambdas_um, o, image=img, stats=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    value = segments / (ms_step * 1e-3) / 1e6

    # dominant kernel: the path-tracing kernel, timed alone with HIP events on its stream
    kms = []
    for _ in range(3):
        img.zero_()
        _, s2 = R.trace(wl.lambdas_um, o, image=img, stats=True)
        kms.append(s2["ms"])
    k_ms = float(np.mean(kms))
    abytes = algorithmic_bytes(st)
    achieved = abytes / (k_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": TRAFFIC_BYTES if kernel_hash() == TRAFFIC_KERNEL_HASH else None,
                "kernel": "trace_kernel", "kernel_ms": round(k_ms, 3),
                "algorithmic_bytes": int(abytes)}

    out = {
        "metric": "Mpath-segments/s, plain vs NN-surrogate BSDF, at <=1% rel. L2 image error",
        "value": round(value, 2),
        "unit": "Mpath-segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mid terrain: 65,536 triangles, 512x512 sensor, 16 spp, 8 wavelengths, "
                               "depth<=4, plain closed-form scattering",
                   "paths_per_step": st["paths"], "segments_per_step": segments,
                   "shadow_rays_per_step": st["shadow_rays"], "bvh_nodes": info["n_nodes"],
                   "bvh_depth": info["depth"]},
        "roofline": roofline,
    }
    if args.surrogate:
        out["surrogate"] = surrogate_leg(R, wl, o, img, st, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
