"""Benchmark: Mpath-segments/s of the generalized-ray tracer, plain against learned p_w.

Headline workload: the large instanced scene (4,194,300 triangles: 60 displaced terrain tiles
and 21,845 random boxes with the smooth / Gaussian rough / grating material mix, three
partially coherent emitters), 1920 x 1080 sensor, 64 samples per pixel, 16 wavelengths, path
depth <= 6 with Russian roulette (2.12G paths per frame; seeded, synthetic).  One step = one
full trace of that frame including the per-pixel reduction, inputs resident on the GPU.  The
learned-p_w legs (BF16 and FP8 matrix-core operands) render the same frame.  Each leg's image
is compared with the FP64 oracle on every 8th row and column of the sensor (1/64 of the
pixels, the same per-path random streams); a leg qualifies at rel. L2 <= 1e-3 (closed form)
or <= 1e-2 (learned p_w).  The mid terrain (65,536 triangles, 512 x 512, 16 spp, 8
wavelengths, depth <= 4) is reported as an extra leg.

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
# Dense matrix-core peaks of the MI355X and the network's multiply-add work per query:
# 2 x (10 x 64 + 3 x 64 x 64 + 64) flops.
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0}
MLP_FLOPS = 2 * (10 * 64 + 3 * 64 * 64 + 64)
# Vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (one wave64
# instruction occupies a 16-lane SIMD for 4 cycles; FMA counted as one op, no packed math).
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# Algorithmic vector operations per unit of work (counted from the algorithm's steps, not from
# the compiled code): a 4-wide node visit = 4 boxes x (6 plane distances + 6 min/max + 4
# interval bounds + 1 test) + 10 for ordering + 3 for pushes; a watertight triangle test = 9
# translations + 6 shears + 9 for the edge functions + 3 sign tests + 2 for the determinant + 5
# for the distance + 1 reciprocal + 4 scalings and compares; a path segment = ray set-up,
# hit refinement, free-space update, frame and footprint, two counter-based draws (2 x 60) and
# continuation = 300; a shadow ray = emitter sampling, one draw and the p_w closed form = 150.
NODE_OPS = 81
TRI_OPS = 40
SEGMENT_OPS = 300
SHADOW_OPS = 150
NODE_BYTES = 112     # bytes of a 4-wide node the traversal reads (boxes + child links)
TRI_BYTES = 48       # bytes of a triangle record
HIT_BYTES = 48 + 48 + 32   # closest hit: triangle, shading normals, material
RECORD_BYTES = 4     # one float per path
SHADOW_QUEUE_BYTES = 2 * 48 + 2 * 4   # a queued shadow ray written and read, its value stored and read

# HBM traffic of one frame's path-tracing launches on this workload (trace, shadow-ray and
# merge kernels), from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known
# size; valid only for the kernel sources it was measured on (sha256 prefix of the files
# below).
TRAFFIC_BYTES = {"mid": 2_897_092 * 1024, "large": 113_166_855 * 1024}
TRAFFIC_KERNEL_HASH = "f380417f462446ac"
KERNEL_SOURCES = ["paper_2303_15762_amd/csrc/trace.hip", "paper_2303_15762_amd/csrc/trace_core.hpp",
                  "paper_2303_15762_amd/csrc/device_math.hpp",
                  "paper_2303_15762_amd/csrc/kernels.hpp", "paper_2303_15762_amd/csrc/composite.hpp",
                  "paper_2303_15762_amd/csrc/bvh_build.cpp"]


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for s in KERNEL_SOURCES:
        with open(os.path.join(root, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(st):
    """Scene and output bytes one frame's path-tracing launches request, from the in-kernel
    counters: node and triangle fetches of both traversals, the shading reads of each closest
    hit (approximated by segments - paths: every path ends on at most one miss), each shadow
    ray through its queue with its measurement value, and one float written per path.  Path
    state stays in registers and moves no memory."""
    hits = max(0, st["segments"] - st["paths"])
    return (st["node_visits"] * NODE_BYTES + st["tri_tests"] * TRI_BYTES + hits * HIT_BYTES
            + st["shadow_rays"] * SHADOW_QUEUE_BYTES + st["paths"] * RECORD_BYTES)


def algorithmic_ops(st):
    """Vector operations one frame's path-tracing launches need by the counts above."""
    return (st["node_visits"] * NODE_OPS + st["tri_tests"] * TRI_OPS + st["segments"] * SEGMENT_OPS
            + st["shadow_rays"] * SHADOW_OPS)


def subset_pixels(wl, step=8):
    """Every step-th row and column of the sensor as (x, y) pairs (1/64 of the pixels at 8)."""
    ys = np.arange(0, wl.sensor.height, step)
    xs = np.arange(0, wl.sensor.width, step)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], 1)


def rel_l2_on(img_gpu, pix, ref):
    """Relative L2 error of a GPU image [n_lambda, H, W] on the pixels pix (x, y) against the
    oracle's [n_lambda, n_pixels]."""
    g = img_gpu.detach().double().cpu().numpy()[:, pix[:, 1], pix[:, 0]]
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


def worst_pixel(img_gpu, pix, ref):
    """The pixel carrying the largest share of the squared error, and the rel. L2 without it
    (a single bright, ill-conditioned path can dominate a frame's norm)."""
    g = img_gpu.detach().double().cpu().numpy()[:, pix[:, 1], pix[:, 0]]
    e2 = ((g - ref) ** 2).sum(0)
    i = int(np.argmax(e2))
    keep = np.ones(len(pix), bool)
    keep[i] = False
    rest = float(np.linalg.norm(g[:, keep] - ref[:, keep]) / np.linalg.norm(ref[:, keep]))
    return {"pixel": [int(pix[i, 0]), int(pix[i, 1])], "share_of_squared_error": round(float(e2[i] / e2.sum()), 4),
            "its_rel_error": float(np.linalg.norm(g[:, i] - ref[:, i]) / max(np.linalg.norm(ref[:, i]), 1e-300)),
            "its_share_of_norm2": round(float((ref[:, i] ** 2).sum() / (ref ** 2).sum()), 4),
            "rel_l2_without_it": rest}


def save_subset(args, name, img_gpu, pix, ref):
    if not args.save_images:
        return
    os.makedirs(args.save_images, exist_ok=True)
    g = img_gpu.detach().cpu().numpy()[:, pix[:, 1], pix[:, 0]]
    np.save(os.path.join(args.save_images, f"{name}_gpu.npy"), g)
    np.save(os.path.join(args.save_images, f"{name}_pixels.npy"), pix)
    if ref is not None:
        np.save(os.path.join(args.save_images, f"{name}_oracle.npy"), ref)


def oracle_subset(wl, pix, threads):
    """The FP64 oracle on the pixel subset (every per-path stream as in the full frame); returns
    (image [n_lambda, n_pixels], seconds, segments)."""
    import oracle
    osc = oracle.OracleScene(wl.scene)
    t0 = time.perf_counter()
    img, st = oracle.render(wl, osc, pixels=pix, n_threads=threads)
    return img, time.perf_counter() - t0, st["segments"], osc


def cpu_baseline_from(wl, pix, dt, seg, osc, threads, what):
    """The oracle's Mpath-segments/s on the subset it rendered for the image comparison, and on
    one thread over every 16th pixel of that subset."""
    import oracle
    pix1 = pix[::16]
    t0 = time.perf_counter()
    _, st1 = oracle.render(wl, osc, pixels=pix1, n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": seg / dt / 1e6, "unit": "Mpath-segments/s", "cores": threads, "kind": "oracle",
            "single_thread_value": st1["segments"] / dt1 / 1e6,
            "sample": f"{what}: {len(pix)} pixels (every 8th row and column) x {wl.spp} samples x "
                      f"{len(wl.lambdas_um)} wavelengths ({seg} segments, {dt:.1f} s, FP64 C++ oracle, "
                      f"{threads} threads); single thread: {len(pix1)} of those pixels "
                      f"({st1['segments']} segments, {dt1:.1f} s)"}


def time_frames(R, wl, o, img, steps):
    """Mean ms per frame over `steps` traces timed with HIP events on the renderer's stream."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(R.stream)
    for _ in range(steps):
        R.trace(wl.lambdas_um, o, image=img, stats=False)
    e1.record(R.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def surrogate_leg(R, wl, img_plain, ms_plain, pix, ref, steps, args):
    """Train the learned p_w (outside the timed region), then render the same frame with the
    network (bfloat16 and E4M3 matrix-core operands): frame time, each image against the FP64
    oracle on the pixel subset, and what the network can gain at most on this frame."""
    import torch
    from paper_2303_15762_amd.surrogate import Surrogate
    S = Surrogate(R)
    t0 = time.perf_counter()
    if args.surrogate_params:
        # parameters saved by an earlier run (profiler runs that leave out the training)
        p = torch.tensor(np.load(args.surrogate_params), device=R.dev)
        hist = {"step": [0], "val_loss": [None]}
    else:
        p, hist = S.train()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if args.save_surrogate:
        np.save(args.save_surrogate, p.cpu().numpy())
    S.install(p)
    legs = {}
    for name, mode in (("bf16", 1), ("fp8", 2)):
        o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
                   rr_enable=wl.rr_enable, rr_p=wl.rr_p, bsdf_mode=mode)
        img_s = torch.zeros_like(img_plain)
        _, st = R.trace(wl.lambdas_um, o, image=img_s, stats=True)
        err_o = rel_l2_on(img_s, pix, ref) if ref is not None else None
        err_p = float(torch.linalg.vector_norm((img_s - img_plain).double()) /
                      torch.linalg.vector_norm(img_plain.double()))
        ms = time_frames(R, wl, o, img_s, steps)
        legs[name] = {"value": round(st["segments"] / (ms * 1e-3) / 1e6, 2), "unit": "Mpath-segments/s",
                      "ms_per_step": round(ms, 3), "steps": steps,
                      "rel_l2_vs_oracle": err_o,
                      "qualifies": (err_o is not None and err_o <= 1e-2),
                      "rel_l2_vs_plain_gpu_image": err_p,
                      "surrogate_evals_per_step": st["surrogate_evals"],
                      "fallbacks_per_step": st["fallbacks"],
                      "frame_time_vs_plain": round(ms / ms_plain, 4)}
        meas = {k: st["measured_" + k] for k in ("smooth", "rough", "grating")}
    # measurements per material class: the network covers rough surfaces inside its trained
    # domain; smooth and grating surfaces and the other rough ones keep the closed form
    n_meas = max(1, sum(meas.values()))
    by_class = {"measurements_per_step": meas,
                "share_of_measurements": {k: round(v / n_meas, 4) for k, v in meas.items()},
                "rough_in_domain_share": round(legs["bf16"]["surrogate_evals_per_step"] / max(1, meas["rough"]), 4),
                "network_share_of_measurements": round(legs["bf16"]["surrogate_evals_per_step"] / n_meas, 4)}
    # the network alone on the matrix cores: 4M encoded queries, both operand types; and the
    # in-domain queries through gr_bsdf_eval, closed form against network
    x, _, q = S.samples(1 << 22, seed=77, with_queries=True)
    mfma = {}
    for name, dtype, peak in (("bf16", 1, MFMA_PEAK_TFLOPS["bf16"]), ("fp8", 2, MFMA_PEAK_TFLOPS["fp8"])):
        S.forward(p, x, dtype=dtype)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(R.stream)
        for _ in range(5):
            S.forward(p, x, dtype=dtype)
        e1.record(R.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        tf = x.shape[0] * MLP_FLOPS / (ms * 1e-3) / 1e12
        mfma[name] = {"bound": "mfma", "achieved": round(tf, 1), "peak": peak, "unit": "TFLOP/s",
                      "frac": round(tf / peak, 4), "rows": int(x.shape[0]), "ms": round(ms, 4)}
    per_query = {}
    for name, mode in (("closed_form", 0), ("bf16", 1), ("fp8", 2)):
        R.bsdf_eval(q, mode=mode)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(R.stream)
        for _ in range(5):
            R.bsdf_eval(q, mode=mode)
        e1.record(R.stream)
        torch.cuda.synchronize()
        per_query[name] = e0.elapsed_time(e1) / 5 / q.shape[0] * 1e6   # ns per query
    legs["bf16"]["roofline"] = mfma["bf16"]
    legs["fp8"]["roofline"] = mfma["fp8"]
    n_in = legs["bf16"]["surrogate_evals_per_step"]
    cf_ms = n_in * per_query["closed_form"] * 1e-6
    out = {"bf16": legs["bf16"], "fp8": legs["fp8"], "by_material": by_class,
           "train_s": round(t_train, 2), "train_steps": hist["step"][-1],
           "val_mse_log_pw": hist["val_loss"][-1],
           # the in-domain queries in full waves through gr_bsdf_eval: the closed form's cost the
           # network replaces, and the most the frame can gain from it (Amdahl)
           "in_domain_ns_per_query": {k: round(v, 4) for k, v in per_query.items()},
           "in_domain_speedup_per_query": {"bf16": round(per_query["closed_form"] / per_query["bf16"], 2),
                                           "fp8": round(per_query["closed_form"] / per_query["fp8"], 2)},
           "closed_form_pw_ms_replaced_per_frame_est": round(cf_ms, 3),
           "closed_form_pw_share_of_frame_est": round(cf_ms / ms_plain, 5),
           "amdahl_max_frame_speedup": round(ms_plain / max(ms_plain - cf_ms, 1e-9), 5)}
    return out


def hero_leg(R, wl, ms_plain, steps):
    """Hero-wavelength paths (one path per pixel, sample and rotation group of four wavelengths)
    on the same workload: the same image estimated from a quarter of the paths.  Reported: the
    frame time, path segments per second, and wavelength-segments per second (each hero segment
    carries four).  Both estimators are unbiased for the same image (checked by the tests); a
    single frame's totals are dominated by rare bright paths, so they are not compared here."""
    import torch
    o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p, hero=True)
    img = torch.zeros((len(wl.lambdas_um), wl.sensor.height, wl.sensor.width), device=R.dev)
    _, st = R.trace(wl.lambdas_um, o, image=img, stats=True)
    ms = time_frames(R, wl, o, img, steps)
    return {"value": round(st["segments"] / (ms * 1e-3) / 1e6, 2), "unit": "Mpath-segments/s",
            "ms_per_step": round(ms, 3), "steps": steps, "paths_per_step": st["paths"],
            "segments_per_step": st["segments"],
            "wavelength_segments_per_s_M": round(4 * st["segments"] / (ms * 1e-3) / 1e6, 2),
            "frame_speedup_vs_one_wavelength_paths": round(ms_plain / ms, 3)}


def aniso_leg(R, wl, ms_plain, img_plain, steps):
    """Anisotropic generalized rays (matrix beta, rho) on the same workload and random streams:
    frame time, path segments per second, and the image difference from the scalar rays."""
    import torch
    o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p, aniso=True)
    img = torch.zeros((len(wl.lambdas_um), wl.sensor.height, wl.sensor.width), device=R.dev)
    _, st = R.trace(wl.lambdas_um, o, image=img, stats=True)
    diff = float(torch.linalg.vector_norm((img - img_plain).double()) /
                 torch.linalg.vector_norm(img_plain.double()))
    ms = time_frames(R, wl, o, img, steps)
    return {"value": round(st["segments"] / (ms * 1e-3) / 1e6, 2), "unit": "Mpath-segments/s",
            "ms_per_step": round(ms, 3), "steps": steps, "segments_per_step": st["segments"],
            "frame_time_vs_scalar_rays": round(ms / ms_plain, 3), "rel_l2_vs_scalar_ray_image": diff}


def composite_leg(R, wl, ms_plain, img_plain, steps, threads, no_cpu, reach_m=2e-3, step=32):
    """Composite interactions at material boundaries (GR_TRACE_COMPOSITE) on the same frame:
    the boundary search on the host, the frame time and rate, the share of interactions that
    met a boundary, the image change against single-material interactions, and the image error
    against the FP64 oracle on every 32nd row and column (its composite p_w is ~40x slower per
    interaction than its closed form, so a sparser subset than the plain leg's)."""
    import torch
    t0 = time.perf_counter()
    n_edges = R.boundaries(reach_m)
    build_s = time.perf_counter() - t0
    o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p, composite=True)
    img = torch.zeros((len(wl.lambdas_um), wl.sensor.height, wl.sensor.width), device=R.dev)
    _, st = R.trace(wl.lambdas_um, o, image=img, stats=True)
    diff = float(torch.linalg.vector_norm((img - img_plain).double()) /
                 torch.linalg.vector_norm(img_plain.double()))
    out = {"reach_m": reach_m, "boundary_edges": n_edges, "boundary_build_s": round(build_s, 2),
           "composite_per_segment": round(st["composite"] / st["segments"], 4),
           "rel_l2_vs_single_material_image": diff}
    ms = time_frames(R, wl, o, img, steps)
    out.update({"value": round(st["segments"] / (ms * 1e-3) / 1e6, 2), "unit": "Mpath-segments/s",
                "ms_per_step": round(ms, 3), "steps": steps, "segments_per_step": st["segments"],
                "frame_time_vs_plain": round(ms / ms_plain, 3)})
    if not no_cpu:
        import oracle
        pix = subset_pixels(wl, step)
        osc = oracle.OracleScene(wl.scene)
        t0 = time.perf_counter()
        ref, ost = oracle.render(wl, osc, pixels=pix, n_threads=threads, composite=True, reach_m=reach_m)
        dt = time.perf_counter() - t0
        img.zero_()
        R.trace(wl.lambdas_um, o, image=img, stats=False)
        err = rel_l2_on(img, pix, ref)
        out.update({"rel_l2_vs_oracle": err, "qualifies": err <= 1e-3,
                    "rel_l2_pixels": f"{len(pix)} pixels: every {step}th row and column",
                    "worst_pixel": worst_pixel(img, pix, ref),
                    "oracle_mpath_segments_per_s": round(ost["segments"] / dt / 1e6, 3)})
    return out


# Coherent measurement: vector operations of one (sample, slit node) evaluation in the FP64
# mode, the way the kernel writes them: distance (1 FMA + a square root of ~6), phase (1),
# amplitude (a reciprocal of the distance, ~8, 3 multiplies, a square root of ~6), sincos with
# its range reduction (~40), the large-argument correction (1 multiply), complex product and
# accumulation (8).  FP64 vector operations issue at the FP32 rate on this chip (78.6 TFLOP/s
# counts an FMA as two).
COHERENT_NODE_OPS = 74


def coherent_leg(R, steps):
    """The precision-stress measurement (double slit, z = 1 m, 0.55 um, 1024 x 64 sensor, 64
    samples, 16 Gauss-Legendre nodes per slit) in its three phase modes."""
    from workloads import coherent_case
    case = coherent_case("slits", z_m=1.0, lambda_um=0.55)
    nodes = 16
    out = {"workload": "double slit b = 10 um, d = 50 um, z = 1 m, 0.55 um, 1024x64 sensor, 64 spp, "
                       "2 x 16 Gauss-Legendre nodes"}
    evals = case.width * case.height * case.spp * 2 * nodes
    for name, mode in (("fp32", 0), ("fp64", 1), ("two_float", 2)):
        R.coherent(case, phase_mode=mode, nodes_per_slit=nodes)
        ms = []
        for _ in range(max(1, steps)):
            _, t = R.coherent(case, phase_mode=mode, nodes_per_slit=nodes, timing=True)
            ms.append(t)
        m = float(np.median(ms))
        out[name] = {"ms": round(m, 3), "node_evals_per_s_G": round(evals / (m * 1e-3) / 1e9, 2)}
    ach = evals * COHERENT_NODE_OPS / (out["fp64"]["ms"] * 1e-3) / 1e9
    out["fp64"]["roofline"] = {"bound": "alu", "achieved": round(ach, 1), "peak": round(VALU_PEAK_GOPS, 1),
                               "unit": "Gop/s", "frac": round(ach / VALU_PEAK_GOPS, 4),
                               "ops_per_node_eval": COHERENT_NODE_OPS}
    return out


def plain_frame(R, wl, warmup, steps):
    """Warm up, time `steps` plain frames, then take the deterministic counters and the image of
    one frame and the path-tracing kernels' device time (HIP events around the trace, shadow-ray
    and merge launches on the renderer's stream) over three more frames."""
    import torch
    o = R.opts(spp_count=wl.spp, spp_norm=wl.spp, max_depth=wl.max_depth, seed=wl.seed,
               rr_enable=wl.rr_enable, rr_p=wl.rr_p)
    img = torch.zeros((len(wl.lambdas_um), wl.sensor.height, wl.sensor.width), device=R.dev)
    for _ in range(max(1, warmup)):
        R.trace(wl.lambdas_um, o, image=img, stats=False)
    ms_step = time_frames(R, wl, o, img, steps)
    kms = []
    for _ in range(3):
        img.zero_()
        _, st = R.trace(wl.lambdas_um, o, image=img, stats=True)
        kms.append(st["ms"])
    return o, img, st, ms_step, float(np.mean(kms))


def roofline_of(st, k_ms, workload):
    # The kernel issues vector-ALU work near the issue limit (see the committed counters) while
    # its scene fetches are served from the caches, so the bound is the vector ALU; the
    # requested-bytes view against HBM is reported beside it.
    aops = algorithmic_ops(st)
    achieved = aops / (k_ms * 1e-3) / 1e9
    abytes = algorithmic_bytes(st)
    traffic = (TRAFFIC_BYTES.get(workload) if kernel_hash() == TRAFFIC_KERNEL_HASH else None)
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": round(VALU_PEAK_GOPS, 1),
            "unit": "Gop/s", "frac": round(achieved / VALU_PEAK_GOPS, 4), "traffic": traffic,
            "kernel": "trace_kernel + shadow_kernel + shadow_merge_kernel", "kernel_ms": round(k_ms, 3),
            "algorithmic_ops": int(aops), "requested_bytes": int(abytes),
            "requested_gbs": round(abytes / (k_ms * 1e-3) / 1e9, 1), "hbm_peak_gbs": HBM_PEAK_GBS,
            "traffic_gbs": (round(traffic / (k_ms * 1e-3) / 1e9, 1) if traffic else None),
            "traffic_bytes_per_segment": (round(traffic / st["segments"], 1) if traffic else None)}


WORKLOAD_NAMES = {
    "large": ("large instanced scene: 4,194,300 triangles (60 displaced terrain tiles + 21,845 boxes, "
              "smooth / rough / grating mix), 1920x1080 sensor, 64 spp, 16 wavelengths, depth<=6 with "
              "Russian roulette, 3 partially coherent emitters; plain closed-form scattering, learned-p_w "
              "legs on the same frame"),
    "mid": ("mid terrain: 65,536 triangles, 512x512 sensor, 16 spp, 8 wavelengths, depth<=4, "
            "plain closed-form scattering"),
}


def load(workload):
    from workloads import mid_terrain
    from workloads import scenes as W
    # the oracle gets the float32-rounded values the library receives, so both render the same
    # scene (a grazing narrow-lobe path moves with the rounding of its inputs)
    if workload == "mid":
        return W.as_float32_inputs(mid_terrain())
    return W.as_float32_inputs(W.large_workload())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--leg-steps", type=int, default=3,
                    help="timed frames of each extra leg (learned p_w, hero, anisotropic, mid), "
                         "at most --steps")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the FP64 oracle (no rel. L2 against it, no CPU baseline)")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="skip the learned-p_w legs (training takes a few seconds)")
    ap.add_argument("--no-hero", dest="hero", action="store_false", help="skip the hero-wavelength leg")
    ap.add_argument("--no-aniso", dest="aniso", action="store_false", help="skip the anisotropic-ray leg")
    ap.add_argument("--no-composite", dest="composite", action="store_false",
                    help="skip the composite-interaction leg")
    ap.add_argument("--no-coherent", dest="coherent", action="store_false",
                    help="skip the coherent-measurement leg")
    ap.add_argument("--no-mid", dest="mid", action="store_false",
                    help="skip the mid-terrain leg of the large workload")
    ap.add_argument("--workload", choices=["large", "mid"], default="large",
                    help="large: the 4,194,300-triangle instanced scene at 1920x1080, 64 spp, 16 "
                         "wavelengths (the reported line); mid: the 65,536-triangle terrain alone")
    ap.add_argument("--surrogate-params", default=None,
                    help="load the learned p_w's parameters (.npy, float32 [13249]) instead of training")
    ap.add_argument("--save-surrogate", default=None, help="save the trained parameters (.npy)")
    ap.add_argument("--save-images", default=None,
                    help="directory: save each leg's image on the oracle's pixel subset and the "
                         "oracle's (.npy)")
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

    leg_steps = max(1, min(args.leg_steps, args.steps))
    threads = os.cpu_count() or 1
    wl = load(args.workload)
    pix = subset_pixels(wl)
    # the FP64 oracle on the pixel subset first (CPU only), so its image is at hand for every leg
    ref = None
    if not args.no_cpu:
        ref, dt_or, seg_or, osc = oracle_subset(wl, pix, threads)
    R = Renderer(0)
    info = R.load_workload(wl)
    o, img, st, ms_step, k_ms = plain_frame(R, wl, args.warmup, args.steps)
    segments = st["segments"]
    value = segments / (ms_step * 1e-3) / 1e6
    err_plain = rel_l2_on(img, pix, ref) if ref is not None else None
    save_subset(args, args.workload, img, pix, ref)

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
        "config": {"workload": WORKLOAD_NAMES[args.workload],
                   "paths_per_step": st["paths"], "segments_per_step": segments,
                   "shadow_rays_per_step": st["shadow_rays"], "bvh_nodes": info["n_nodes"],
                   "bvh_depth": info["depth"], "n_tris": info["n_tris"]},
        "rel_l2_vs_oracle": err_plain,
        "qualifies": (err_plain is not None and err_plain <= 1e-3),
        "rel_l2_pixels": f"{len(pix)} pixels: every 8th row and column, all samples and wavelengths",
        "worst_pixel": worst_pixel(img, pix, ref) if ref is not None else None,
        "roofline": roofline_of(st, k_ms, args.workload),
    }
    if args.surrogate:
        out["surrogate"] = surrogate_leg(R, wl, img, ms_step, pix, ref, leg_steps, args)
    if args.hero and len(wl.lambdas_um) % 4 == 0:
        out["hero"] = hero_leg(R, wl, ms_step, leg_steps)
    if args.aniso:
        out["aniso"] = aniso_leg(R, wl, ms_step, img, leg_steps)
    if args.composite:
        out["composite"] = composite_leg(R, wl, ms_step, img, leg_steps, threads, args.no_cpu)
    if args.coherent:
        out["coherent"] = coherent_leg(R, leg_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_from(wl, pix, dt_or, seg_or, osc, threads, args.workload)
    if args.workload == "large" and args.mid:
        wm = load("mid")
        pm = subset_pixels(wm)
        ref_m = None if args.no_cpu else oracle_subset(wm, pm, threads)[0]
        info_m = R.load_workload(wm)
        _, img_m, st_m, ms_m, k_ms_m = plain_frame(R, wm, 1, args.steps)
        err_m = rel_l2_on(img_m, pm, ref_m) if ref_m is not None else None
        save_subset(args, "mid", img_m, pm, ref_m)
        comp_m = None
        if args.composite:
            comp_m = composite_leg(R, wm, ms_m, img_m, args.steps, threads, args.no_cpu, step=8)
        out["mid"] = {"workload": WORKLOAD_NAMES["mid"], "value": round(st_m["segments"] / (ms_m * 1e-3) / 1e6, 2),
                      "unit": "Mpath-segments/s", "ms_per_step": round(ms_m, 3), "steps": args.steps,
                      "segments_per_step": st_m["segments"], "bvh_nodes": info_m["n_nodes"],
                      "rel_l2_vs_oracle": err_m, "qualifies": (err_m is not None and err_m <= 1e-3),
                      "rel_l2_pixels": f"{len(pm)} pixels: every 8th row and column",
                      "worst_pixel": worst_pixel(img_m, pm, ref_m) if ref_m is not None else None,
                      "roofline": roofline_of(st_m, k_ms_m, "mid"), "composite": comp_m}
    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
