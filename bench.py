"""Benchmark of the X-GS Perceiver hot path on one MI355X.

One step = one pass of every hot-path row over one batch of synthetic input:
  a1-a4  project -> tile sort -> render forward -> render backward of a
         1,000,000-Gaussian synthetic room at 1200x680 with 3 + 1 + 32
         channels, at the next pose of a random-walk trajectory;
  a5     bilinear grid sampling of a 512 x 30 x 40 feature map to 640 x 480;
  a6-a7  BF16-MFMA VQ assignment (top-4 + FP32 rescore) of 816,000 x 768
         features against 4,096 codewords, then one EMA update.
The headline value is fwd+bwd ms/frame (a1-a4, HIP events on the launch
stream, mean over the timed steps).  The backward's zeroing of its
accumulated gradients (a call of its own) runs on a side stream beside the
forward pass, inside the frame's events.  Everything is resident in HBM
before the timed region; nothing is skipped inside it.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/frame at 1M Gaussians 1200x680 32-ch"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
# FP32 lane operations per second with packed FP32 off (the build disables it):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; an FMA counts as one operation
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2603_09632_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, src: list[str], launches_bytes_alg: float):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    or None if it is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel)
    if not e or e.get("source_sha") != source_sha(*src):
        return None
    return float(e["bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-semantic", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2603_09632_amd as xgs
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    # ---------------------------------------------------------------- inputs
    log("generating the 1M-Gaussian room")
    scene = synth.room_scene(1_000_000, seed=2, c_sem=32)
    g = xgs.Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity), t(scene.colors),
                      t(scene.features))
    poses = synth.room_trajectory(100, seed=10)
    nframes = args.warmup + args.steps
    cams = [xgs.camera_from(synth.room_camera(1200, 680, 600.0, poses[(5 + k) % len(poses)]))
            for k in range(nframes)]
    hs, ws, ty, tx = xgs.grid_dims(cams[0])
    C = 4 + scene.c_sem
    p = xgs.Projected.alloc(g.n, dev)
    # capacity: the largest instance count over the poses, plus headroom
    mmax = 0
    for c in cams:
        xgs.xgs_project(g, c, out=p)
        mmax = max(mmax, int(p.tiles_touched.to(torch.int64).sum().item()))
    b = xgs.alloc_binning(g.n, int(mmax * 1.25) + 1024, cams[0], dev)
    out = torch.empty((C, hs, ws), device=dev)
    fT = torch.empty((hs, ws), device=dev)
    nl = torch.empty((hs, ws), dtype=torch.int32, device=dev)
    d_out = t(synth.upstream_grad(C, hs, ws, seed=1))
    grads = xgs.Gaussians.empty_like(g)
    bwd_ws = torch.empty(int(xgs.lib.xgs_render_bwd_workspace(g.n)), dtype=torch.uint8, device=dev)

    log("generating the feature map and the VQ features")
    P = t(synth.feature_map(512, 30, 40, seed=5))
    G = torch.empty((512, 480, 640), device=dev)
    V = torch.empty((480, 640), dtype=torch.uint8, device=dev)
    Xh = synth.vq_mixture(816_000, 768, 256, seed=30)
    Eh = synth.vq_codebook(4096, 768, 256, seed=31, centre_seed=30)
    X = t(Xh)
    E0 = t(Eh)
    E = E0.clone()
    Eb, en = xgs.xgs_vq_prepare(E)
    idx = torch.empty(X.shape[0], dtype=torch.int32, device=dev)
    dist = torch.empty(X.shape[0], device=dev)
    Nema = torch.ones(4096, device=dev)
    Mema = E0.clone()
    counts = torch.empty(4096, device=dev)
    ema_ws = torch.empty(int(xgs.lib.xgs_vq_ema_workspace(X.shape[0], 768, 4096)), dtype=torch.uint8, device=dev)
    vq_ws = xgs.vq_assign_workspace(X.shape[0], 768, 4096, xgs.VQ_BF16_RESCORE4, dev)
    if args.calib_copy:
        src = torch.empty(256 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
    torch.cuda.synchronize()

    names = ["project", "tile_sort", "render_fwd", "render_bwd", "grid_sample", "vq_stage", "vq_gemm", "vq_rescore",
             "vq_ema"]
    stream = torch.cuda.current_stream()
    # The backward's zeroing of the accumulated gradients runs on a side
    # stream beside this frame's forward pass (issued once the sort is done,
    # so inside the frame's events); the backward waits for it.
    side = torch.cuda.Stream(device=dev)

    def step(k, evs):
        c = cams[k]
        zeroed = torch.cuda.Event()
        evs[0].record(stream)
        xgs.xgs_project(g, c, out=p)
        evs[1].record(stream)
        xgs.xgs_tile_sort(p, c, g.n, b)
        evs[2].record(stream)
        side.wait_event(evs[2])
        xgs.xgs_render_bwd_zero(g, grads, bwd_ws, stream=side)
        zeroed.record(side)
        xgs.xgs_render_fwd(g, p, b, c, out=out, final_T=fT, n_last=nl)
        evs[3].record(stream)
        stream.wait_event(zeroed)
        xgs.xgs_render_bwd(g, p, b, c, d_out, fT, nl, flags=xgs.BWD_PREZEROED, grads=grads, workspace=bwd_ws)
        evs[4].record(stream)
        xgs.xgs_grid_sample(P, 480, 640, G=G, V=V)
        evs[5].record(stream)
        # xgs_vq_assign (BF16 + rescore) as its three stages, so that the
        # MFMA sweep is timed on its own
        xgs.xgs_vq_stage(X, Eb, en, vq_ws)
        evs[6].record(stream)
        xgs.xgs_vq_candidates(X.shape[0], 768, 4096, vq_ws)
        evs[7].record(stream)
        xgs.xgs_vq_rescore(X, E, vq_ws, idx=idx, dist=dist)
        evs[8].record(stream)
        xgs.xgs_vq_ema_update(X, idx, Nema, Mema, E, Eb, en, 0.99, 1e-5, xgs.EMA_LAPLACE, counts=counts,
                              workspace=ema_ws)
        evs[9].record(stream)

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
    log(f"warmup {args.warmup} steps")
    for k in range(args.warmup):
        step(k, mk())
    torch.cuda.synchronize()
    if int(b.status.item()) != 0:
        raise RuntimeError("binning capacity exceeded during warmup")
    log(f"timing {args.steps} steps")
    evs_all = [mk() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, evs_all[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int(b.status.item()) != 0:
        raise RuntimeError("binning capacity exceeded in the timed region")
    per = {n: [] for n in names}
    for evs in evs_all:
        for i, n in enumerate(names):
            per[n].append(evs[i].elapsed_time(evs[i + 1]))
    if args.calib_copy:
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # the FP32 plain form of the same assignment, once (for the precision
    # statement: the BF16 form must be faster at equal agreement)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    idx32 = torch.empty_like(idx)
    dist32 = torch.empty_like(dist)
    xgs.xgs_vq_assign(X, E, Eb, en, xgs.VQ_BF16_RESCORE4, idx=idx, dist=dist, workspace=vq_ws)
    e0.record(stream)
    xgs.xgs_vq_assign(X, E, Eb, en, xgs.VQ_FP32, idx=idx32, dist=dist32)
    e1.record(stream)
    torch.cuda.synchronize()
    vq_fp32_ms = e0.elapsed_time(e1)
    # a seeded row sample of both assignments and the codebook they used, for
    # the agreement with the FP64 oracle (computed in the CPU-baseline leg)
    vq_rows = np.sort(np.random.default_rng(33).choice(X.shape[0], 8192, replace=False))
    vq_sample = (Xh[vq_rows], E.cpu().numpy(), idx.cpu().numpy()[vq_rows], idx32.cpu().numpy()[vq_rows])
    vq_same = float((idx32 == idx).float().mean().item())

    ms = {n: float(np.mean(v)) for n, v in per.items()}
    ms["vq_assign"] = ms["vq_stage"] + ms["vq_gemm"] + ms["vq_rescore"]
    frame = [sum(per[n][k] for n in names[:4]) for k in range(args.steps)]
    value = float(np.mean(frame))
    m_inst = int(b.num_instances.item())

    # ------------------------------------------------------------ rooflines
    N, D, K = X.shape[0], 768, 4096
    vq_flop = 2.0 * N * K * D
    vq_tflops = vq_flop / (ms["vq_gemm"] * 1e-3) / 1e12
    vq_assign_tflops = vq_flop / (ms["vq_assign"] * 1e-3) / 1e12
    grid_bytes = 512 * 480 * 640 * 4 + 480 * 640 + 512 * 30 * 40 * 4
    grid_gbs = grid_bytes / (ms["grid_sample"] * 1e-3) / 1e9
    comp = compositing_work(xgs, g, p, b, cams[args.warmup + args.steps - 1], out, fT, nl, scene.c_sem, m_inst,
                            ms["render_fwd"], ms["render_bwd"])
    roofs = [
        {"kernel": "vq_gemm_ereg_kernel", "bound": "mfma", "achieved": round(vq_tflops, 2), "peak": BF16_PEAK_TFLOPS,
         "unit": "TFLOP/s", "frac": round(vq_tflops / BF16_PEAK_TFLOPS, 4),
         "traffic": traffic_for("vq_gemm_ereg_kernel", ["vq.hip"], vq_flop),
         "algorithmic": f"2*N*K*D = {vq_flop:.3e} flop per launch (N=816000, K=4096, D=768)", "ms": ms["vq_gemm"]},
        comp.pop("roofline_fwd"), comp.pop("roofline_bwd"),
    ]
    roof = dict(max(roofs, key=lambda r: r["ms"]))
    roof.pop("ms")

    result = {
        "metric": METRIC, "value": round(value, 4), "unit": "ms/frame", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded room scene, trajectory, VFM-like maps, mixture VQ features)",
        "config": {"workload": "1M-Gaussian synthetic room, 1200x680, 3+1+32 channels, fwd+bwd per frame; "
                               "grid_sample 512x30x40 -> 640x480; VQ 816000x768 vs K=4096 (bf16+rescore) + EMA",
                   "gaussians": g.n, "width": 1200, "height": 680, "c_sem": scene.c_sem,
                   "instances_last_frame": m_inst},
        "ms": {k: round(v, 4) for k, v in ms.items()},
        "frame_ms_median": round(float(np.median(frame)), 4),
        "frame_ms_p10": round(float(np.percentile(frame, 10)), 4),
        "frame_ms_p90": round(float(np.percentile(frame, 90)), 4),
        # FP32 bytes of X consumed per second by the whole assignment (stage + sweep + rescore)
        "vq_assign_GBps": round(N * D * 4 / (ms["vq_assign"] * 1e-3) / 1e9, 1),
        "vq_gemm_TFLOPs": round(vq_tflops, 1), "vq_assign_TFLOPs": round(vq_assign_tflops, 1),
        "vq_fp32_plain_ms": round(vq_fp32_ms, 3), "vq_bf16_vs_fp32_same_index": round(vq_same, 6),
        "grid_sample_GBps": round(grid_gbs, 1),
        "roofline": roof,
        "rooflines": roofs,
        "compositing": comp,
    }

    if not args.no_semantic:
        result["mapping_scale"] = mapping_scale(xgs, synth, dev)
        result["semantic_phase"] = semantic_phase(xgs, synth, dev, G)
        result["tracking_and_targets"] = tracking_and_targets(xgs, g, p, b, cams[args.warmup + args.steps - 1], out,
                                                              fT, nl, d_out, grads, bwd_ws, dev)

    if not args.no_serve:
        del X, Xh, G
        torch.cuda.empty_cache()
        result["serving"] = serving(xgs, synth, dev, args.serve_requests)

    # ------------------------------------------------------------ CPU baseline
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scene, synth)
        agree, vq_cpu = vq_agreement(*vq_sample)
        result["vq_index_agreement_fp64"] = agree
        result["cpu_baseline"].update(vq_cpu)
    print(json.dumps(result), flush=True)


SRC = {"render_fwd_mfma_kernel": ["render_fwd.hip", "render_common.h", "common.h"],
       "render_bwd_mfma_kernel": ["render_bwd.hip", "render_common.h", "common.h", "wave.h"]}


def compositing_work(xgs, g, p, b, cam, out, fT, nl, c_sem, m_inst, fwd_ms, bwd_ms):
    """Algorithmic work of the compositing calls on the last timed frame,
    counted outside the timed region from the forward's own outputs.

    M = (Gaussian, tile) instances.  E = pixel-Gaussian evaluations a walk
    needs: each pixel's list positions up to and including its last blended
    Gaussian (sum of n_last); E_list = the positions of every pixel's whole
    tile list (the work of a walk without early termination).
    Bytes (a3): per instance its list entry (4), splat record (32), colour
    (12) and features (4 c_sem); per pixel C + 2 outputs.  Bytes (a4): the
    instance reads again, per instance one gradient row (2 + 3 + 1 + 3 + 1 +
    c_sem floats), per pixel d_out, final_T and n_last, and per Gaussian the
    projection backward (11 parameter and 3 + 3 + 4 + 1 + 3 + c_sem gradient
    floats).  ALU: E (20 + C) FP32 lane operations forward and E (35 + 2 C)
    backward (recompute alpha, recover T, g.c, d alpha, the chain to conic,
    mean and opacity, w g), against VALU_PEAK_TOPS."""
    import torch
    xgs.xgs_render_fwd(g, p, b, cam, out=out, final_T=fT, n_last=nl)
    _, _, ty, tx = xgs.grid_dims(cam)
    torch.cuda.synchronize()
    C = 4 + c_sem
    hs, ws = nl.shape
    E = int(nl.to(torch.int64).sum().item())
    r = b.ranges.to(torch.int64)
    lens = (r[:, 1] - r[:, 0]).reshape(ty, tx)
    px = torch.ones((hs, ws), dtype=torch.int64, device=nl.device)
    per_tile = torch.nn.functional.pad(px, (0, tx * 16 - ws, 0, ty * 16 - hs)).reshape(ty, 16, tx, 16).sum((1, 3))
    E_list = int((lens * per_tile).sum().item())
    n = g.n
    inst_b = 4 + 32 + 12 + 4 * c_sem
    fwd_bytes = m_inst * inst_b + hs * ws * 4 * (C + 2)
    bwd_bytes = (m_inst * (inst_b + 4 * (10 + c_sem)) + hs * ws * 4 * (C + 2)
                 + n * 4 * (11 + 14 + c_sem))
    fwd_ops, bwd_ops = E * (20 + C), E * (35 + 2 * C)

    def roof(kernel, nbytes, ops, t_ms, what):
        gbs = nbytes / (t_ms * 1e-3) / 1e9
        tops = ops / (t_ms * 1e-3) / 1e12
        hbm, alu = gbs / HBM_PEAK_GBS, tops / VALU_PEAK_TOPS
        return {"kernel": kernel, "bound": "hbm" if hbm >= alu else "alu",
                "achieved": round(gbs, 1) if hbm >= alu else round(tops, 2),
                "peak": HBM_PEAK_GBS if hbm >= alu else round(VALU_PEAK_TOPS, 2),
                "unit": "GB/s" if hbm >= alu else "Tops/s", "frac": round(max(hbm, alu), 4),
                "hbm_GBps": round(gbs, 1), "hbm_frac": round(hbm, 4), "alu_Tops": round(tops, 2),
                "alu_frac": round(alu, 4), "traffic": traffic_for(kernel + "<32", SRC[kernel], nbytes),
                "algorithmic": what, "ms": t_ms}

    return {
        "instances_M": m_inst, "evaluations_E": E, "evaluations_E_list": E_list,
        "mean_walk_per_pixel": round(E / (hs * ws), 1),
        "fwd_bytes": fwd_bytes, "bwd_bytes": bwd_bytes, "fwd_ops": fwd_ops, "bwd_ops": bwd_ops,
        "valu_peak_Tops": round(VALU_PEAK_TOPS, 2),
        "roofline_fwd": roof("render_fwd_mfma_kernel", fwd_bytes, fwd_ops, fwd_ms,
                             f"M*{inst_b} + px*4*(C+2) = {fwd_bytes:.3e} B; E*(20+C) = {fwd_ops:.3e} ops"),
        "roofline_bwd": roof("render_bwd_mfma_kernel", bwd_bytes, bwd_ops, bwd_ms,
                             f"M*({inst_b}+4*(10+c_sem)) + px*4*(C+2) + N*4*(25+c_sem) = {bwd_bytes:.3e} B; "
                             f"E*(35+2C) = {bwd_ops:.3e} ops; time of the whole xgs_render_bwd call "
                             "(gradient fill, pixel kernel, projection backward)"),
    }


def mapping_scale(xgs, synth, dev, frames: int = 20, warm: int = 3):
    """Mapping-scale configuration: 300k-Gaussian room, 640x480, f = 525, 16
    semantic channels; project -> tile sort -> forward -> backward per frame
    over 20 poses of the trajectory (after 3 warm-up frames)."""
    import torch
    log("mapping scale: 300k room, 640x480, 16 semantic channels")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    scene = synth.room_scene(300_000, seed=2, c_sem=16)
    g = xgs.Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity), t(scene.colors),
                      t(scene.features))
    poses = synth.room_trajectory(100, seed=10)
    cams = [xgs.camera_from(synth.room_camera(640, 480, 525.0, poses[k])) for k in range(warm + frames)]
    p = xgs.Projected.alloc(g.n, dev)
    mmax = 0
    for c in cams:
        xgs.xgs_project(g, c, out=p)
        mmax = max(mmax, int(p.tiles_touched.to(torch.int64).sum().item()))
    b = xgs.alloc_binning(g.n, int(mmax * 1.25) + 1024, cams[0], dev)
    C = 20
    out = torch.empty((C, 480, 640), device=dev)
    fT = torch.empty((480, 640), device=dev)
    nl = torch.empty((480, 640), dtype=torch.int32, device=dev)
    d_out = t(synth.upstream_grad(C, 480, 640, seed=1))
    grads = xgs.Gaussians.empty_like(g)
    bws = torch.empty(int(xgs.lib.xgs_render_bwd_workspace(g.n)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cams]
    for c, (e0, e1) in zip(cams, evs):
        e0.record(stream)
        xgs.xgs_project(g, c, out=p)
        xgs.xgs_tile_sort(p, c, g.n, b)
        xgs.xgs_render_fwd(g, p, b, c, out=out, final_T=fT, n_last=nl)
        xgs.xgs_render_bwd(g, p, b, c, d_out, fT, nl, grads=grads, workspace=bws)
        e1.record(stream)
    torch.cuda.synchronize()
    if int(b.status.item()) != 0:
        raise RuntimeError("binning capacity exceeded in the mapping-scale leg")
    f = [e0.elapsed_time(e1) for e0, e1 in evs[warm:]]
    return {"workload": "300k-Gaussian synthetic room, 640x480, 3+1+16 channels, fwd+bwd per frame over 20 "
                        "trajectory poses", "frames": frames, "ms_per_frame_mean": round(float(np.mean(f)), 4),
            "ms_per_frame_median": round(float(np.median(f)), 4),
            "ms_per_frame_p10": round(float(np.percentile(f, 10)), 4),
            "ms_per_frame_p90": round(float(np.percentile(f, 90)), 4)}


def semantic_phase(xgs, synth, dev, G, reps: int = 10):
    """Semantic phase (geometry frozen): 300k-Gaussian room at 640x480, L = 16
    mixture weights over a 16 x 512 codebook, targets = the 512 x 480 x 640
    bilinear grid sample, blocky validity mask.  Per stage: softmax, render
    forward, fused decode + masked loss, feature-only backward, softmax
    backward (HIP events, mean of `reps` runs after 3 warm-up runs)."""
    import torch
    log("semantic phase: 300k room, 640x480, L=16, D=512")
    t = lambda a, dt=np.float32: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    scene = synth.room_scene(300_000, seed=2, c_sem=16)
    rng = np.random.default_rng(11)
    L, D = 16, 512
    z = t(rng.standard_normal((scene.n, L)) * 2)
    E = t(rng.standard_normal((L, D)))
    yy, xx = np.mgrid[0:480, 0:640]
    V = t((((yy // 60) + (xx // 80)) % 3 != 0), np.uint8)
    g = xgs.Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity), t(scene.colors),
                      t(scene.features))
    cam = xgs.camera_from(synth.room_camera(640, 480, 525.0, synth.room_trajectory(100, seed=10)[7]))
    p = xgs.xgs_project(g, cam)
    m = int(p.tiles_touched.to(torch.int64).sum().item())
    b = xgs.alloc_binning(g.n, m + 1024, cam, dev)
    xgs.xgs_tile_sort(p, cam, g.n, b)
    w = torch.empty_like(z)
    dz = torch.empty_like(z)
    gw = xgs.Gaussians(g.means, g.log_scales, g.quats, g.opacity, g.colors, w)
    out = torch.empty((4 + L, 480, 640), device=dev)
    fT = torch.empty((480, 640), device=dev)
    nl = torch.empty((480, 640), dtype=torch.int32, device=dev)
    d_out = torch.empty_like(out)
    loss = torch.empty(1, device=dev)
    lws = torch.empty(int(xgs.lib.xgs_semantic_loss_workspace(480, 640)), dtype=torch.uint8, device=dev)
    grads = xgs.Gaussians.empty_like(gw)
    bws = torch.empty(int(xgs.lib.xgs_render_bwd_workspace(g.n)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    names = ["softmax", "render_fwd", "decode_loss", "render_bwd_features", "softmax_bwd"]

    def run(evs):
        evs[0].record(stream)
        xgs.xgs_semantic_softmax(z, w)
        evs[1].record(stream)
        xgs.xgs_render_fwd(gw, p, b, cam, out=out, final_T=fT, n_last=nl)
        evs[2].record(stream)
        xgs.xgs_semantic_loss(out, E, G, V, 1.0, d_out=d_out, loss=loss, workspace=lws)
        evs[3].record(stream)
        xgs.xgs_render_bwd(gw, p, b, cam, d_out, fT, nl, flags=xgs.BWD_FEATURES_ONLY, grads=grads, workspace=bws)
        evs[4].record(stream)
        xgs.xgs_semantic_softmax_bwd(w, grads.features, dz)
        evs[5].record(stream)

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
    for _ in range(3):
        run(mk())
    torch.cuda.synchronize()
    evs_all = [mk() for _ in range(reps)]
    for evs in evs_all:
        run(evs)
    torch.cuda.synchronize()
    ms = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs_all])) for i, n in enumerate(names)}
    P_ = 480 * 640
    loss_bytes = 2 * D * P_ * 4 + L * P_ * 4 + P_ + (4 + L) * P_ * 4
    return {"workload": "300k-Gaussian room, 640x480, L=16 mixture weights, D=512 targets, geometry frozen",
            "ms": {k: round(v, 4) for k, v in ms.items()}, "total_ms": round(sum(ms.values()), 4),
            "instances": m, "loss": float(loss.item()),
            "decode_loss_GBps": round(loss_bytes / (ms["decode_loss"] * 1e-3) / 1e9, 1),
            "decode_loss_bytes": loss_bytes}


def tracking_and_targets(xgs, g, p, b, cam, out, fT, nl, d_out, grads, bwd_ws, dev, reps: int = 10):
    """Tracking pieces on the 1M-Gaussian 1200x680 frame (loss -> backward ->
    pose gradient), occluder pruning of the 1M Gaussians against a depth map,
    and region-indexed targets at 640x480 (D = 512, 100 regions)."""
    import torch
    log("tracking, occluder pruning, region targets")
    stream = torch.cuda.current_stream()
    torch.manual_seed(3)
    image = (out[:3] + 0.02 * torch.randn_like(out[:3])).contiguous()
    depth = (out[3] * 1.01).contiguous()
    loss = torch.empty(1, device=dev)
    tws = torch.empty(int(xgs.lib.xgs_tracking_loss_workspace(out.shape[1], out.shape[2])), dtype=torch.uint8,
                      device=dev)
    d_pose = torch.empty(6, device=dev)
    prune = torch.empty(g.n, dtype=torch.uint8, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    S = torch.randint(-1, 100, (480, 640), dtype=torch.int32, device=dev)
    Phi = torch.randn(100, 512, device=dev)
    Gr = torch.empty((512, 480, 640), device=dev)
    Vr = torch.empty((480, 640), dtype=torch.uint8, device=dev)
    # the four stride-2 target grids of the 512x30x40 map at 640x480, one launch
    import synth
    Pm = torch.from_numpy(synth.feature_map(512, 30, 40, seed=5)).to(dev)
    Go = torch.empty((4, 512, 240, 320), device=dev)
    Vo = torch.empty((4, 240, 320), dtype=torch.uint8, device=dev)
    names = ["tracking_loss", "render_bwd", "pose_grad", "occluder_mask", "region_targets", "targets_all_offsets"]

    def run(evs):
        evs[0].record(stream)
        xgs.xgs_tracking_loss(out, image, depth, 0.05, d_out=d_out, loss=loss, workspace=tws)
        evs[1].record(stream)
        xgs.xgs_render_bwd(g, p, b, cam, d_out, fT, nl, grads=grads, workspace=bwd_ws)
        evs[2].record(stream)
        xgs.xgs_pose_grad(g, p, cam, bwd_ws, d_pose=d_pose)
        evs[3].record(stream)
        xgs.xgs_occluder_mask(p, g.n, depth, 0.1, prune=prune, count=cnt)
        evs[4].record(stream)
        xgs.xgs_region_targets(S, Phi, G=Gr, V=Vr)
        evs[5].record(stream)
        xgs.xgs_grid_sample_offsets(Pm, 480, 640, 2, G=Go, V=Vo)
        evs[6].record(stream)

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
    for _ in range(3):
        run(mk())
    torch.cuda.synchronize()
    evs_all = [mk() for _ in range(reps)]
    for evs in evs_all:
        run(evs)
    torch.cuda.synchronize()
    ms = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs_all])) for i, n in enumerate(names)}
    reg_bytes = 512 * 480 * 640 * 4 + 480 * 640 * (4 + 1)
    return {"ms": {k: round(v, 4) for k, v in ms.items()},
            "tracking_step_ms": round(ms["tracking_loss"] + ms["render_bwd"] + ms["pose_grad"], 4),
            "pruned": int(cnt.item()), "region_targets_GBps": round(reg_bytes / (ms["region_targets"] * 1e-3) / 1e9, 1),
            "targets_all_offsets_GBps": round((Go.numel() * 4 + Vo.numel()) / (ms["targets_all_offsets"] * 1e-3) / 1e9,
                                              1),
            "workload": "1M room 1200x680 (tracking: L1 photo + 0.05 L1 depth, pose gradient; occluders vs a depth "
                        "map 1% behind the render), region targets 640x480 D=512 R=100, the four stride-2 target "
                        "grids of the 512x30x40 map at 640x480 in one launch"}


def serving(xgs, synth, dev, n_requests):
    """Serving form: 8 resident rooms of 100k..1M Gaussians (16 semantic
    channels), requests for a random scene, trajectory pose and resolution in
    {320x240, 640x480, 1200x680}, rendered in batches (continuous batching
    over four arenas).  Saturation throughput is measured with all requests
    queued at once (full batches) and as the highest Poisson rate the server
    sustains; Poisson arrivals at 50% and 80% of the sustained rate give
    p50/p99."""
    import torch

    from paper_2603_09632_amd.serve import Resolution, Server, poisson_load
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    sizes = (100_000, 150_000, 250_000, 350_000, 500_000, 650_000, 800_000, 1_000_000)
    log("generating the 8 served scenes")
    scenes = {}
    for k, n in enumerate(sizes):
        s = synth.room_scene(n, seed=40 + k, c_sem=16)
        scenes[f"room{k}"] = xgs.Gaussians(t(s.means), t(s.log_scales), t(s.quats), t(s.opacity), t(s.colors),
                                           t(s.features))
    res = [Resolution(320, 240, 262.5, 262.5, 160, 120), Resolution(640, 480, 525, 525, 320, 240),
           Resolution(1200, 680, 600, 600, 600, 340)]
    poses = synth.room_trajectory(100, seed=10)
    rng = np.random.default_rng(48)
    mk = lambda m: [(f"room{rng.integers(0, 8)}", poses[rng.integers(0, 100)], res[rng.integers(0, 3)])
                    for _ in range(m)]
    srv = Server(scenes, hbm_budget_bytes=4 << 30, max_inflight=8, streams=4)
    for f in [srv.submit(*r, discard=True) for r in mk(200)]:  # warm-up
        f.result()
    srv.completed.clear()
    burst = mk(n_requests)
    b0 = (srv.batches, srv.batched_requests)
    t0 = time.perf_counter()
    for f in [srv.submit(*r, discard=True) for r in burst]:
        f.result()
    sat = n_requests / (time.perf_counter() - t0)
    sat_batch = (srv.batched_requests - b0[1]) / max(srv.batches - b0[0], 1)
    srv.completed.clear()

    def poisson_run(qps, n, seed):
        """Completion rate and the rate the sample's own arrivals offered."""
        reqs = mk(n)
        t0 = time.perf_counter()
        futs = poisson_load(srv, reqs, qps, seed=seed, discard=True)
        t_arrived = time.perf_counter()
        for f in futs:
            f.result()
        return n / (time.perf_counter() - t0), n / (t_arrived - t0)

    # Sustained saturation: the highest Poisson arrival rate the server keeps
    # up with, by bisection between 30% and 100% of the burst rate (1,000
    # requests per probe).  A probe keeps up when its requests complete at
    # >= 97% of the rate at which that probe's arrivals came in: a 1,000-
    # arrival Poisson sample itself runs ~3% (one sigma) off its nominal rate,
    # so a bar against the nominal rate would fail or pass some seeds whatever
    # the server does.  Burst batches are full, Poisson batches smaller, so the
    # sustained rate is the lower one.
    lo, hi = 0.3 * sat, sat
    for it in range(5):
        mid = 0.5 * (lo + hi)
        got, offered = poisson_run(mid, 1000, 60 + it)
        srv.completed.clear()
        if got >= 0.97 * offered:
            lo = mid
        else:
            hi = mid
    sustained = lo
    log(f"serving: burst {sat:.0f} frames/s, sustained Poisson {sustained:.0f} req/s")
    points = []
    for frac, seed in ((0.5, 49), (0.8, 50)):
        qps = frac * sustained
        log(f"serving: Poisson run at {frac:.0%} of the sustained rate = {qps:.0f} req/s")
        c0 = (srv.batches, srv.batched_requests, srv.graphs_captured, srv.overflows)
        reqs = mk(n_requests)
        t0 = time.perf_counter()
        futs = poisson_load(srv, reqs, qps, seed=seed, discard=True)
        for f in futs:
            f.result()
        wall = time.perf_counter() - t0
        del futs
        st = srv.stats()
        srv.completed.clear()
        c1 = (srv.batches, srv.batched_requests, srv.graphs_captured, srv.overflows)
        d = [b - a for a, b in zip(c0, c1)]
        points.append({"load": frac, "offered_qps": round(qps, 1),
                       "achieved_frames_per_s": round(n_requests / wall, 1), "p50_ms": round(st["p50_ms"], 3),
                       "p99_ms": round(st["p99_ms"], 3), "p99_over_p50": round(st["p99_ms"] / st["p50_ms"], 2),
                       "p50_queued_ms": round(st["p50_queued_ms"], 3), "p99_queued_ms": round(st["p99_queued_ms"], 3),
                       "batches": d[0], "mean_batch": round(d[1] / max(d[0], 1), 2), "graphs_captured": d[2],
                       "overflows": d[3]})
    peak = srv.peak_ledger_bytes / 2 ** 20
    overflows = srv.overflows
    growths = srv.arena_growths
    srv.close()
    return {"scenes": "8 rooms, 100k-1M Gaussians, 16 semantic channels",
            "resolutions": "320x240 / 640x480 / 1200x680 uniform", "requests": n_requests, "warmup_requests": 200,
            "saturation_frames_per_s": round(sat, 1), "saturation_mean_batch": round(sat_batch, 2),
            "sustained_poisson_req_per_s": round(sustained, 1),
            "sustained_criterion": "highest nominal Poisson rate (bisection, 5 probes of 1,000 requests) whose "
                                   "requests complete at >= 97% of the probe's own arrival rate",
            "load_reference": "load points are fractions of the sustained Poisson rate",
            "load_points": points, "p99_ms_at_80pct": points[-1]["p99_ms"], "peak_hbm_MB": round(peak, 1),
            "hbm_budget_MB": 4096, "capacity_overflows": overflows, "arena_growths": growths, "max_slots": 8,
            "arenas": 4, "hip_graphs": True,
            "batching": "one project + tile sort + compositing launch sequence per batch, keyed by (slot, tile, "
                        "depth); one HIP graph per arena and capacity bucket"}


def vq_agreement(Xs, Es, idx_bf16, idx_fp32):
    """Index agreement of the BF16 + rescore and the FP32 plain assignments
    with the FP64 oracle (brute force) on a seeded row sample; tie-adjusted
    counts rows whose two best FP64 distances are within 1e-6 relative as
    agreeing.  The oracle's assignment of the sample is also the CPU
    baseline's VQ term: timed with every thread, and on one thread over the
    first 512 rows, as FP32 bytes of X consumed per second."""
    import oracle

    threads = oracle.set_threads(0)
    t0 = time.perf_counter()
    ri, d1, d2 = oracle.vq_assign(Xs, Es)
    t_all = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.vq_assign(Xs[:512], Es)
    t_one = time.perf_counter() - t0
    oracle.set_threads(threads)
    tie = (d2 - d1) <= 1e-6 * np.maximum(d1, 1e-30)
    agree = lambda a: (round(float((a == ri).mean()), 6), round(float(((a == ri) | tie).mean()), 6))
    b_raw, b_adj = agree(idx_bf16)
    f_raw, f_adj = agree(idx_fp32)
    row_b = Xs.shape[1] * 4
    return ({"rows": int(len(ri)), "bf16_rescore": b_raw, "bf16_rescore_tie_adjusted": b_adj, "fp32_plain": f_raw,
             "fp32_plain_tie_adjusted": f_adj},
            {"vq_assign_GBps": round(len(ri) * row_b / t_all / 1e9, 5),
             "vq_assign_GBps_one_thread": round(512 * row_b / t_one / 1e9, 6),
             "vq_sample": f"FP64 brute force of {len(ri)} rows x K = {Es.shape[0]}, D = {Xs.shape[1]} "
                          f"({t_all:.1f} s on {threads} threads; 512 rows on one thread {t_one:.1f} s)"})


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, synth):
    """The FP64 oracle on one frame of the same workload (1M-Gaussian room,
    1200x680, 36 channels, the bench's first pose).  All threads: projection,
    binning, forward and backward compositing of the whole frame and the
    projection backward.  One thread: the per-Gaussian parts (projection,
    binning, channels, projection backward) timed whole, the compositing
    walks on every 3rd row of tiles and scaled by the tile fraction."""
    import oracle

    cam = synth.room_camera(1200, 680, 600.0, synth.room_trajectory(100, seed=10)[5])
    hs, ws, ty, tx = oracle.grid_info(cam)
    g = synth.upstream_grad(4 + scene.c_sem, hs, ws, seed=1).astype(np.float64)

    def frame(tile_mask):
        ts = {}
        t0 = time.perf_counter()
        pr = oracle.project(scene, cam)
        keys, order, ranges = oracle.bin_instances(pr.rect, oracle.depth_bits(pr.depth), tx, ty)
        chan = oracle.channels(scene, pr.depth)
        t1 = time.perf_counter()
        out, fT, nl, amb = oracle.composite_fwd(pr, scene.opacity, chan, order, ranges, cam, tile_mask)
        r = oracle.Render(pr, keys, order, ranges, out, fT, nl, amb, chan)
        d_m2, d_co, d_op, d_ch = oracle.composite_bwd(scene, cam, g, r, tile_mask)
        t2 = time.perf_counter()
        oracle.project_bwd(scene, cam, d_m2, d_co, np.ascontiguousarray(d_ch[:, 3]))
        t3 = time.perf_counter()
        ts["per_gaussian"] = (t1 - t0) + (t3 - t2)
        ts["walks"] = t2 - t1
        return ts

    threads = oracle.set_threads(0)
    log(f"cpu baseline: oracle frame on {threads} threads")
    a = frame(None)
    all_ms = (a["per_gaussian"] + a["walks"]) * 1e3
    oracle.set_threads(1)
    log("cpu baseline: oracle frame sample on one thread")
    mask = np.zeros((ty, tx), np.uint8)
    mask[::3] = 1
    frac = float(mask.mean())
    o = frame(mask.ravel())
    oracle.set_threads(threads)
    one_ms = (o["per_gaussian"] + o["walks"] / frac) * 1e3
    return {"value": round(all_ms, 1), "unit": "ms/frame", "cores": threads, "kind": "oracle",
            "sample": f"one whole 1200x680 frame of the 1M-Gaussian room (fwd+bwd, FP64 C with OpenMP over grid "
                      f"rows on {threads} threads: per-Gaussian parts {a['per_gaussian']:.2f} s, compositing "
                      f"walks {a['walks']:.2f} s)",
            "cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
            "one_thread_ms_per_frame": round(one_ms, 1),
            "one_thread_sample": f"per-Gaussian parts of the whole frame ({o['per_gaussian']:.2f} s, unscaled) + "
                                 f"the walks of every 3rd tile row ({frac:.3f} of the tiles, {o['walks']:.2f} s) "
                                 f"scaled to the frame"}


if __name__ == "__main__":
    main()
