#!/usr/bin/env python3
"""Benchmark of the SLIC superpixel path on one MI355X.

One step = one frame through slic_segment: CIELAB conversion, seeding with
3x3 gradient perturbation, association, `iters` rounds of (centre update,
association), and connectivity enforcement, on a synthetic image already
resident in HBM.  Prints ONE JSON line (rank 0, one GPU):

  value       frames/s of the headline workload (c2: 640x480, S=16, m=10,
              10 iterations, perturbed seeds, connectivity)
  roofline    the dominant kernel (the fused association + accumulation),
              bound by its vector arithmetic: algorithmic FP32 operations per
              launch / its average duration inside frames ((frame with 10
              rounds - frame with 0 rounds) / 10, HIP events on the launch
              stream) against the non-packed FP32 peak; with its HBM fraction
              and its VALU instruction rate (committed counters)
  cpu_baseline the CPU oracle on a bounded sample of frames, on every OpenMP
              thread (and on one)
  extra       Mpix/s per iteration at 640x480 and 1920x1080, per-kernel
              times (events around each launch, so each includes about 2-3 us
              of event overhead), the 1080p frame rate, the 64-image batch

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# FP32 vector peak without packed instructions (the library is built without
# them): 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane
# instructions per second, x 2 for a fused multiply-add = 78.6 T ops/s
VALU_ISSUE_PEAK_T = 39.32
ALU_PEAK_TFLOPS = 78.64
# algorithmic FP32 operations per pixel of one association launch: Eq. 1 for
# each of 9 candidates (3 colour and 2 position differences, 5 squares, 3
# additions, 2 square roots, the product with m/S and the final sum: 17),
# 8 comparisons for the argmin, and 5 additions into the centre sums
ASSIGN_OPS_PER_PIXEL = 9 * 17 + 8 + 5
VALU_FILE = os.path.join(ROOT, "profiles", "assign_valu_counters.json")
METRIC = "frames/s & Mpix/s/iter at 640x480 and 1080p; learned vs plain at equal energy"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assign_c2_traffic.json")
ASSIGN_SRC = os.path.join(ROOT, "paper_1509_04232_amd", "csrc", "assign.hip")


def assign_bytes(n_pixels: int, n_clusters: int) -> int:
    """Algorithmic bytes of one association launch that another association
    follows (every launch these timings measure): read Lab (12 B/pixel),
    read each centre (20 B) and add its five sums and count (48 B).  The
    labels (4 B/pixel more) are written by the last launch of a frame only."""
    return 12 * n_pixels + 68 * n_clusters


class Frame:
    """Preallocated buffers for repeated slic_segment calls on one image."""

    def __init__(self, slic, wl, device, squared_distance: bool = False, tune: bool = False):
        import numpy as np  # noqa: F401
        import torch

        import synth
        self.slic = slic
        self.wl = wl
        img = synth.image_for(wl)
        self.rgb = torch.from_numpy(img.reshape(-1)).to(device)
        self.p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m, perturb=wl.perturb,
                             min_segment=wl.min_segment, squared_distance=squared_distance)
        self.cp = self.p.c()
        self.ws = slic.workspace_for(self.p, device)
        self.labels = torch.empty((wl.height, wl.width), dtype=torch.int32, device=device)
        self.nseg = torch.empty(1, dtype=torch.int32, device=device)
        self.stream = torch.cuda.current_stream().cuda_stream
        self.K = self.p.n_clusters
        # the association launch variant: the library's default for this
        # size and step (it follows the autotuner's picks and, unlike a
        # timed choice, is the same under a profiler), or with `tune` the
        # autotuner's pick (recorded process-wide)
        if tune:
            self.variant, self.tuned_ms_per_iter = slic.slic_autotune(
                self.cp, self.rgb.data_ptr(), wl.iters, 5, self.stream, self.ws.data_ptr(),
                self.ws.numel())
        else:
            self.variant = slic.slic_get_assign_variant(wl.width, wl.height, wl.S)
            self.tuned_ms_per_iter = None

    def run(self, iters: int, enforce: bool) -> None:
        self.slic.slic_segment(self.cp, self.rgb.data_ptr(), iters, 1 if enforce else 0,
                               self.labels.data_ptr(), None, None,
                               self.nseg.data_ptr() if enforce else None, self.stream,
                               self.ws.data_ptr(), self.ws.numel())


def time_frames(torch, frame: Frame, steps: int, warmup: int, iters: int, enforce: bool) -> float:
    """Seconds per frame over `steps` timed frames."""
    for _ in range(warmup):
        frame.run(iters, enforce)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        frame.run(iters, enforce)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_frames_ms(torch, frame: Frame, steps: int, iters: int, enforce: bool) -> float:
    """Milliseconds per frame between two HIP events recorded on the launch
    stream around `steps` back-to-back frames."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    frame.run(iters, enforce)
    start.record()
    for _ in range(steps):
        frame.run(iters, enforce)
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / steps


def assign_from_frames_ms(torch, frame: Frame, steps: int, reps: int = 5) -> float:
    """Average duration (ms) of one association launch inside frames: each
    round of a frame is one association launch, so (frame with 10 rounds -
    frame with 0 rounds) / 10, both timed with HIP events on the launch
    stream (no connectivity); median of `reps` repetitions."""
    runs = []
    for _ in range(reps):
        t10 = event_frames_ms(torch, frame, steps, 10, False)
        t0 = event_frames_ms(torch, frame, steps, 0, False)
        runs.append((t10 - t0) / 10)
    runs.sort()
    return runs[len(runs) // 2]


def time_frames_with_upload(torch, frame: Frame, steps: int, warmup: int) -> float:
    """Seconds per frame when every frame is first copied from pinned host
    memory to the device on the launch stream (the listing of Section 4
    uploads each frame inside its timed segmentation)."""
    host = frame.rgb.cpu().pin_memory()
    wl = frame.wl
    for _ in range(warmup):
        frame.rgb.copy_(host, non_blocking=True)
        frame.run(wl.iters, wl.connectivity)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        frame.rgb.copy_(host, non_blocking=True)
        frame.run(wl.iters, wl.connectivity)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


KERNELS = ("lab_seed", "assign", "ccl_", "energy")


def kernel_times(slic, torch, frame: Frame, steps: int, iters: int, enforce: bool):
    """Per-kernel average launch durations (ms) with HIP events recorded on
    the launch stream, over `steps` frames."""
    slic.slic_timing_enable(True)
    try:
        for _ in range(steps):
            frame.run(iters, enforce)
        torch.cuda.synchronize()
    finally:
        slic.slic_timing_enable(False)
    out = {}
    for name in KERNELS:
        total, n = slic.slic_timing_read(name)
        if n:
            out[name] = {"avg_ms": total / n, "launches_per_frame": n / steps}
    return out


def bench_c4(slic, torch, dev, reps: int):
    """Workload c4: 64 uneven images through one batch plan (autotuned, one
    HIP graph per run) against 64 sequential slic_segment calls."""
    import synth
    wls = synth.batch_workload()
    imgs = [torch.from_numpy(synth.image_for(w).reshape(-1)).to(dev) for w in wls]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb) for w in wls]
    iters = wls[0].iters
    b = slic.Batch(params, imgs, iters, use_graph=True)
    variant, _ = b.autotune(reps=2)
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    # per-launch association time, from a run without the graph
    nb = slic.Batch(params, imgs, iters, variant=variant, use_graph=False)
    nb.run()
    torch.cuda.synchronize()
    slic.slic_timing_enable(True)
    for _ in range(reps):
        nb.run()
    torch.cuda.synchronize()
    slic.slic_timing_enable(False)
    a_ms, a_n = slic.slic_timing_read("assign")
    nb.close()
    # sequential per-image calls, each with its own autotuned variant
    frames = []
    for w, img in zip(wls, imgs):
        f = Frame.__new__(Frame)
        f.slic, f.wl, f.rgb = slic, w, img
        f.p = params[len(frames)]
        f.cp = f.p.c()
        f.ws = slic.workspace_for(f.p, dev)
        f.labels = torch.empty((w.height, w.width), dtype=torch.int32, device=dev)
        f.nseg = torch.empty(1, dtype=torch.int32, device=dev)
        f.stream = torch.cuda.current_stream().cuda_stream
        f.variant, _ = slic.slic_autotune(f.cp, img.data_ptr(), 3, 2, f.stream, f.ws.data_ptr(),
                                          f.ws.numel())
        frames.append(f)
    for f in frames:
        f.run(iters, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for f in frames:
            f.run(iters, False)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    b.close()
    npx = sum(w.n_pixels for w in wls)
    nbytes = sum(assign_bytes(w.n_pixels, p.n_clusters) for w, p in zip(wls, params))
    avg = a_ms / max(a_n, 1)
    return {"images": len(wls), "mpix": round(npx / 1e6, 2), "iters": iters,
            "variant": variant, "batch_graph_ms": round(t_batch * 1e3, 3),
            "sequential_ms": round(t_seq * 1e3, 3),
            "images_per_s": round(len(wls) / t_batch, 1),
            "speedup_vs_sequential": round(t_seq / t_batch, 2),
            "assign_avg_us": round(avg * 1e3, 2),
            "mpix_per_s_per_iter": round(npx / (avg * 1e-3) / 1e6, 1),
            "assign_gbps": round(nbytes / (avg * 1e-3) / 1e9, 1),
            "assign_hbm_frac": round(nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def bench_c2_batched(slic, torch, dev, n_frames: int, reps: int):
    """c2-sized frames (each its own seeded image) segmented together through
    one batch plan with connectivity: every launch covers all frames, so the
    small-launch latency of a single 640x480 frame is shared.  Frames/s of
    the batch, beside the sequential rate of the headline."""
    import dataclasses

    import synth
    base = synth.WORKLOADS["c2"]
    wls = [dataclasses.replace(base, seed=base.seed + 1000 + j) for j in range(n_frames)]
    imgs = [torch.from_numpy(synth.image_for(w).reshape(-1)).to(dev) for w in wls]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb,
                          min_segment=w.min_segment) for w in wls]
    b = slic.Batch(params, imgs, base.iters, enforce=True, use_graph=True)
    variant, _ = b.autotune(reps=2)
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    b.close()
    return {"frames": n_frames, "variant": variant, "ms_per_batch": round(t * 1e3, 3),
            "frames_per_s": round(n_frames / t, 1)}


def bench_c5(slic, torch, dev, train_steps: int, n_train: int, n_eval: int, reps: int):
    """Workload c5: the learned warm start.  Trains the net on the GPU (crops
    of c5 training images, targets from plain 10-iteration SLIC), then on
    ``n_eval`` evaluation images, at 640x480 and at 1920x1080, compares plain
    SLIC (convert + seed + 10 iterations) with the warm start (convert + net
    + 2 iterations + energy): frames/s of each, the per-image energy ratio,
    the gate's pass rate (E_warm <= 1.01 E_plain), frames/s with failing
    images charged warm + plain time, and label agreement with plain SLIC."""
    import synth
    from synth.configs import warm_train_workload
    S, plain_iters = 16, 10
    t0 = time.perf_counter()
    data = None
    # images generated on host threads (the generator releases the
    # interpreter) in chunks, each chunk's targets computed on the GPU
    from concurrent.futures import ThreadPoolExecutor
    chunk = 512
    with ThreadPoolExecutor(max_workers=8) as pool:
        for c0 in range(0, n_train, chunk):
            wls = [warm_train_workload(j) for j in range(c0, min(n_train, c0 + chunk))]
            imgs = list(pool.map(synth.image_for, wls))
            part = [(torch.from_numpy(img.reshape(-1)).to(dev),
                     slic.Params(w.width, w.height, S=S, m=w.m, perturb=w.perturb))
                    for w, img in zip(wls, imgs)]
            more = slic.warm.TrainingSet(part, plain_iters)
            if data is None:
                data = more
            else:
                data.items.extend(more.items)
            del part
            print(f"c5: {len(data)} of {n_train} training images ready", file=sys.stderr,
                  flush=True)
    net = slic.warm.Net(S, 32, 128, 128, seed=1)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    log = slic.warm.train(net, data, train_steps, seed=2, log_every=max(1, train_steps // 4))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    taus, validation = c5_pick_confidence(slic, torch, dev, net, n_train, 8, (2, 3, 4))
    tau = taus[2]
    result = {"images": n_eval, "S": S,
              "train": {"images": n_train, "steps": train_steps, "crops": "32 x 128x128",
                        "training_set": "the first %d of the workload's 20,000 training images%s"
                                        % (n_train, "" if n_train >= 20000 else
                                           " (a reduced set)"),
                        "data_s": round(t_data, 2), "train_s": round(t_train, 2),
                        "ms_per_step": round(t_train / max(train_steps, 1) * 1e3, 3),
                        "loss": [[s, round(v, 4)] for s, v in log]},
              "min_confidence": tau,
              "min_confidence_by_rounds": {str(r): t for r, t in taus.items()},
              "validation": {"images": "8 held-out training images (640x480)",
                             "energy_ratio_mean_by_rounds_and_min_confidence": validation}}
    result.update(c5_evaluate(slic, torch, dev, net, n_eval, reps, hd=False, taus=taus))
    result["1920x1080"] = c5_evaluate(slic, torch, dev, net, n_eval, reps, hd=True, taus=taus)
    # the learned start against plain 10-round SLIC at the fewest warm rounds
    # whose gate passes on at least 90% of the images
    summary = {}
    for key, ev in (("640x480", result), ("1920x1080", result["1920x1080"])):
        ok = [int(r) for r, v in ev["rounds"].items() if v["gate_pass_rate"] >= 0.9]
        if not ok:
            summary[key] = {"rounds": None, "note": "the gate passes on fewer than 90% of "
                                                     "the images at 2 to 4 rounds"}
            continue
        r = str(min(ok))
        v = ev["rounds"][r]
        summary[key] = {"rounds": int(r), "gate_pass_rate": v["gate_pass_rate"],
                        "warm_frames_per_s_fallback_charged": v["warm_frames_per_s_fallback_charged"],
                        "plain10_frames_per_s": ev["plain_frames_per_s"],
                        "speedup": round(v["warm_frames_per_s_fallback_charged"] /
                                         ev["plain_frames_per_s"], 3)}
    result["learned_vs_plain10"] = summary
    return result


C5_CONFIDENCES = (0.0, 0.5, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85)


def c5_pick_confidence(slic, torch, dev, net, first: int, n_val: int, rounds=(2,)):
    """Per warm round count, the decode's minimum confidence with the lowest
    mean energy ratio (against plain 10 rounds) on training-distribution
    images the net never saw (training images first .. first + n_val - 1).
    Returns ({rounds: tau}, {rounds: {tau: ratio}})."""
    import synth
    from synth.configs import warm_train_workload
    S = net.S
    vals = [warm_train_workload(first + j) for j in range(n_val)]
    imgs = [torch.from_numpy(synth.image_for(w).reshape(-1)).to(dev) for w in vals]
    params = [slic.Params(w.width, w.height, S=S, m=w.m, perturb=w.perturb) for w in vals]
    plain = [float(slic.segment(r, p, 10, want_energy=True)["energy"].cpu()[0])
             for r, p in zip(imgs, params)]
    table = {str(n): {} for n in rounds}
    for tau in C5_CONFIDENCES:
        prepared = slic.warm.prepare(net.params, S, tau)
        for n in rounds:
            ratios = [float(slic.warm.warm_segment(r, p, prepared, n)["energy"].cpu()[0]) / e
                      for r, p, e in zip(imgs, params, plain)]
            table[str(n)][str(tau)] = round(sum(ratios) / len(ratios), 4)
    best = {n: min(C5_CONFIDENCES, key=lambda t: table[str(n)][str(t)]) for n in rounds}
    return best, table


def c5_evaluate(slic, torch, dev, net, n_eval: int, reps: int, hd: bool, taus: dict):
    """The trained net against plain SLIC on ``n_eval`` evaluation images of
    640x480 (or 1920x1080 with ``hd``), one image at a time, with the
    decode's minimum confidence ``taus[rounds]``; then the warm start at 2..4
    rounds beside plain SLIC after as many associations (one round fewer)
    and after as many rounds, and the plain argmax decode (every pixel
    votes) at 2 rounds.  Both paths are timed without the energy (the
    gate's input, taken in untimed runs)."""
    import numpy as np

    import synth
    from synth.configs import warm_eval_workload
    S, warm_iters, plain_iters = net.S, 2, 10
    evals = [warm_eval_workload(j, hd) for j in range(n_eval)]
    imgs = [torch.from_numpy(synth.image_for(w).reshape(-1)).to(dev) for w in evals]
    params = [slic.Params(w.width, w.height, S=S, m=w.m, perturb=w.perturb) for w in evals]
    cps = [p.c() for p in params]
    stream = torch.cuda.current_stream().cuda_stream
    ws_plain = torch.empty(slic.slic_workspace_bytes(cps[0]), dtype=torch.uint8, device=dev)
    ws_warm = torch.empty(slic.slic_warm_workspace_bytes(cps[0]), dtype=torch.uint8, device=dev)
    lab_plain = [torch.empty((w.height, w.width), dtype=torch.int32, device=dev) for w in evals]
    lab_warm = [torch.empty((w.height, w.width), dtype=torch.int32, device=dev) for w in evals]
    e_plain = torch.empty(n_eval, dtype=torch.float64, device=dev)
    e_warm = torch.empty(n_eval, dtype=torch.float64, device=dev)
    slic.slic_autotune(cps[0], imgs[0].data_ptr(), plain_iters, 3, stream, ws_plain.data_ptr(),
                       ws_plain.numel())

    def run_plain(with_energy):
        for i in range(n_eval):
            slic.slic_segment(cps[i], imgs[i].data_ptr(), plain_iters, 0, lab_plain[i].data_ptr(),
                              None, e_plain[i:].data_ptr() if with_energy else None, None, stream,
                              ws_plain.data_ptr(), ws_plain.numel())

    tau = taus[warm_iters]
    prepared = slic.warm.prepare(net.params, S, tau)

    def run_warm(rounds=warm_iters, net_buf=prepared, out=e_warm):
        # out=None: no energy (the timed runs, like plain SLIC's; the energy
        # only feeds the gate, an evaluation device, and is taken untimed)
        for i in range(n_eval):
            slic.slic_warm_segment(cps[i], imgs[i].data_ptr(), net_buf.data_ptr(), rounds,
                                   0, lab_warm[i].data_ptr(), None,
                                   out[i:].data_ptr() if out is not None else None, None,
                                   stream, ws_warm.data_ptr(), ws_warm.numel())

    def run_plain_n(rounds, out):
        for i in range(n_eval):
            slic.slic_segment(cps[i], imgs[i].data_ptr(), rounds, 0, lab_plain[i].data_ptr(), None,
                              out[i:].data_ptr(), None, stream, ws_plain.data_ptr(),
                              ws_plain.numel())

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        runs = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t)
        runs.sort()
        return runs[len(runs) // 2]

    t_plain = timed(lambda: run_plain(False))
    t_warm = timed(lambda: run_warm(out=None))
    run_plain(True)
    run_warm()
    torch.cuda.synchronize()
    ep, ew = e_plain.cpu().numpy(), e_warm.cpu().numpy()
    ratio = ew / ep
    passed = ratio <= 1.01
    agree = [float((a == b).float().mean()) for a, b in zip(lab_warm, lab_plain)]
    # plain energies at the warm start's iteration count, for the gain
    e2 = torch.empty(n_eval, dtype=torch.float64, device=dev)
    run_plain_n(warm_iters, e2)
    e2 = e2.cpu().numpy()
    t_charged = t_warm + t_plain * float((~passed).sum()) / n_eval
    # more warm rounds, against plain SLIC after as many associations
    sweep = {}
    e_tmp = torch.empty(n_eval, dtype=torch.float64, device=dev)
    for rounds in (2, 3, 4):
        net_r = slic.warm.prepare(net.params, S, taus[rounds])
        t_r = timed(lambda: run_warm(rounds, net_r, None))
        run_warm(rounds, net_r, e_tmp)
        r_w = e_tmp.cpu().numpy() / ep
        run_plain_n(rounds - 1, e_tmp)
        r_p = e_tmp.cpu().numpy() / ep
        run_plain_n(rounds, e_tmp)
        r_same = e_tmp.cpu().numpy() / ep
        sweep[str(rounds)] = {
            "min_confidence": taus[rounds],
            "plain_same_rounds_energy_ratio_mean": round(float(r_same.mean()), 4),
            "plain_same_rounds_gate_pass_rate": round(float((r_same <= 1.01).mean()), 4),
            "warm_frames_per_s": round(n_eval / t_r, 1),
            "warm_frames_per_s_fallback_charged": round(
                n_eval / (t_r + t_plain * float((r_w > 1.01).sum()) / n_eval), 1),
            "energy_ratio_mean": round(float(r_w.mean()), 4),
            "energy_ratio_max": round(float(r_w.max()), 4),
            "gate_pass_rate": round(float((r_w <= 1.01).mean()), 4),
            "plain_equal_associations_energy_ratio_mean": round(float(r_p.mean()), 4),
            "warm_below_plain_equal_associations": int((r_w < r_p).sum())}
    argmax_net = slic.warm.prepare(net.params, S, 0.0)
    run_warm(warm_iters, argmax_net, e_tmp)
    r_argmax = e_tmp.cpu().numpy() / ep
    w0 = evals[0]
    return {"size": f"{w0.width}x{w0.height}", "min_confidence": tau,
            "plain_iters": plain_iters, "warm_iters": warm_iters,
            "plain_frames_per_s": round(n_eval / t_plain, 1),
            "warm_frames_per_s": round(n_eval / t_warm, 1),
            "warm_frames_per_s_fallback_charged": round(n_eval / t_charged, 1),
            "gate_pass_rate": round(float(passed.mean()), 4),
            "energy_ratio_mean": round(float(ratio.mean()), 4),
            "energy_ratio_max": round(float(ratio.max()), 4),
            "plain_2iter_energy_ratio_mean": round(float((e2 / ep).mean()), 4),
            "warm_below_plain_2iter": int((ew < e2).sum()),
            "label_agreement_mean": round(float(np.mean(agree)), 4),
            "argmax_decode_energy_ratio_mean": round(float(r_argmax.mean()), 4),
            "rounds": sweep}


def bench_video(slic, torch, dev, n_frames: int, rounds: int, reps: int):
    """Row f3, the video warm start: a shaking hand-held camera (c2-sized
    frames, S=16, m=10).  Plain: every frame from seeds, 10 rounds.  Warm:
    the first frame plain, every later frame from the previous frame's
    centres with `rounds` rounds.  Frames/s of both chains, and each warm
    frame's energy against plain 10-round energy of the same frame."""
    import numpy as np

    import synth
    from synth.configs import video_workload
    canvas, origins = video_workload(n_frames)
    img = synth.image_for(canvas)
    frames = [torch.from_numpy(np.ascontiguousarray(img[oy:oy + 480, ox:ox + 640]).reshape(-1)).to(dev)
              for ox, oy in origins]
    p = slic.Params(640, 480, S=16, m=10.0)
    cp = p.c()
    K = p.n_clusters
    stream = torch.cuda.current_stream().cuda_stream
    ws = slic.workspace_for(p, dev)
    labels = torch.empty((480, 640), dtype=torch.int32, device=dev)
    cen = [torch.empty((K, 5), dtype=torch.float32, device=dev) for _ in range(2)]
    e_plain = torch.empty(n_frames, dtype=torch.float64, device=dev)
    e_warm = torch.empty(n_frames, dtype=torch.float64, device=dev)

    def plain(with_energy):
        for i, f in enumerate(frames):
            slic.slic_segment(cp, f.data_ptr(), 10, 0, labels.data_ptr(), None,
                              e_plain[i:].data_ptr() if with_energy else None, None, stream,
                              ws.data_ptr(), ws.numel())

    def warm(with_energy):
        for i, f in enumerate(frames):
            if i == 0:
                ctx = slic.slic_init(cp, f.data_ptr(), stream, ws.data_ptr(), ws.numel())
                slic.slic_iterate(ctx, 10)
            else:
                ctx = slic.slic_init_from_centres(cp, f.data_ptr(), cen[(i - 1) % 2].data_ptr(),
                                                  stream, ws.data_ptr(), ws.numel())
                slic.slic_iterate(ctx, rounds)
            if with_energy:
                slic.slic_energy(ctx, e_warm[i:].data_ptr())
            slic.slic_get_centres(ctx, cen[i % 2].data_ptr(), None)
            slic.slic_get_labels(ctx, labels.data_ptr())
            slic.slic_destroy(ctx)

    def timed(fn):
        fn(False)
        torch.cuda.synchronize()
        runs = []
        for _ in range(reps):
            t = time.perf_counter()
            fn(False)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t)
        runs.sort()
        return runs[len(runs) // 2]

    t_plain, t_warm = timed(plain), timed(warm)
    plain(True)
    warm(True)
    torch.cuda.synchronize()
    ratio = (e_warm.cpu().numpy() / e_plain.cpu().numpy())[1:]
    return {"frames": n_frames, "size": "640x480", "S": 16, "warm_rounds": rounds,
            "plain_frames_per_s": round(n_frames / t_plain, 1),
            "warm_frames_per_s": round(n_frames / t_warm, 1),
            "energy_ratio_mean": round(float(ratio.mean()), 4),
            "energy_ratio_max": round(float(ratio.max()), 4),
            "frames_within_1pct": int((ratio <= 1.01).sum())}


def bench_cleanup(slic, torch, dev, reps: int):
    """Row f2: the paper's stray-pixel filter (two passes) against the
    connectivity merge on c2 labels after 10 rounds: kernel time per frame
    (HIP events around each launch) and the 4-connected components each
    leaves, with those under the merge threshold S*S/4."""
    import numpy as np
    from scipy import ndimage

    import synth
    wl = synth.WORKLOADS["c2"]
    rgb = torch.from_numpy(synth.image_for(wl).reshape(-1)).to(dev)
    p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m)

    def run(kind, timed):
        ctx = slic.Context(p, rgb)
        ctx.iterate(wl.iters)
        if timed:
            slic.slic_timing_enable(True)
        if kind == "stray":
            ctx.filter_stray(2)
        else:
            ctx.enforce_connectivity()
        if timed:
            slic.slic_timing_enable(False)
        out = ctx.labels()
        ctx.close()
        return out

    def components(lb):
        n_all = n_small = 0
        for v in np.unique(lb):
            comp, n = ndimage.label(lb == v)
            sizes = np.bincount(comp.ravel())[1:]
            n_all += n
            n_small += int((4 * sizes < wl.S * wl.S).sum())
        return n_all, n_small

    res = {}
    for kind, prefix in (("stray", "stray"), ("merge", "ccl_")):
        run(kind, False)
        total, launches = 0.0, 0
        for _ in range(reps):
            run(kind, True)
            ms, n = slic.slic_timing_read(prefix)
            total += ms
            launches += n
        lb = run(kind, False).cpu().numpy()
        n_all, n_small = components(lb)
        res[kind] = {"us_per_frame": round(total / reps * 1e3, 2), "launches": launches // reps,
                     "components": n_all, "components_below_threshold": n_small}
    raw = slic.segment(rgb, p, wl.iters)["labels"].cpu().numpy()
    res["before"] = dict(zip(("components", "components_below_threshold"), components(raw)))
    return res


def traffic_from_profile():
    """HBM bytes per association launch from the committed PMC summary, or
    None if it is missing or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        src = hashlib.sha256(open(ASSIGN_SRC, "rb").read()).hexdigest()
        if t.get("assign_src_sha256") != src:
            return None
        return t.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, seconds: float):
    """The oracle (built -O3, its independent loops split over OpenMP
    threads; results identical for any thread count) on whole frames of the
    workload: one thread, then every thread OpenMP is given, each for about
    `seconds`."""
    import oracle
    import synth
    img = synth.image_for(wl)
    all_threads = oracle.threads()

    def rate(threads):
        oracle.threads(threads)
        oracle.segment(img, wl.S, wl.m, wl.iters, wl.perturb, wl.connectivity, wl.min_segment)
        n = 0
        t0 = time.perf_counter()
        while True:
            oracle.segment(img, wl.S, wl.m, wl.iters, wl.perturb, wl.connectivity,
                           wl.min_segment)
            n += 1
            dt = time.perf_counter() - t0
            if dt >= seconds:
                return n, dt

    n1, t1 = rate(1)
    nn, tn = rate(all_threads)
    oracle.threads(all_threads)
    return {"value": nn / tn, "unit": "frames/s", "cores": all_threads, "kind": "oracle",
            "single_thread_value": n1 / t1,
            "sample": f"{nn} frames of {wl.name} ({wl.width}x{wl.height}, {wl.iters} "
                      f"iterations, connectivity) on {all_threads} OpenMP threads, and {n1} "
                      f"frames on one thread; oracle built -O3 -fopenmp; host CPU: "
                      f"{cpu_model()}, {os.cpu_count()} logical CPUs visible"}


def valu_from_profile():
    """VALU instructions per pixel of the c2 association from the committed
    counter summary, or None if it is missing or the kernel source changed
    since the counters were taken."""
    try:
        with open(VALU_FILE) as f:
            v = json.load(f)
        src = hashlib.sha256(open(ASSIGN_SRC, "rb").read()).hexdigest()
        if v.get("assign_src_sha256") != src:
            return None
        return v
    except (OSError, ValueError):
        return None


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--train-steps", type=int, default=8000,
                    help="Adam steps of the warm-start net in the c5 leg")
    ap.add_argument("--train-images", type=int, default=20000,
                    help="c5 training images for the warm-start net (the workload's 20,000)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run a plain device copy of this many bytes (PMC calibration)")
    ap.add_argument("--workload-only", default=None, metavar="NAME",
                    help="profiling mode: run warmup+steps frames of workload NAME (c1, c2, c3, "
                         "c4: the 64-image batch, or c5warm: the warm-start path) and the "
                         "optional copy, print one line per phase, no JSON")
    ap.add_argument("--c5-only", action="store_true",
                    help="run only the learned warm-start leg (c5) and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the SLIC path has no multi-GPU mode "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        return 2

    import torch

    import paper_1509_04232_amd as slic
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.workload_only == "c5warm":
        # the warm-start path (untrained parameters: the timing does not
        # depend on their values) on the first 640x480 evaluation image
        from synth.configs import warm_eval_workload
        w = warm_eval_workload(0)
        rgb = torch.from_numpy(synth.image_for(w).reshape(-1)).to(dev)
        p = slic.Params(w.width, w.height, S=w.S, m=w.m)
        net = slic.warm.Net(w.S, 1, 16, 16, seed=1)
        ws = torch.empty(slic.slic_warm_workspace_bytes(p.c()), dtype=torch.uint8, device=dev)
        prepared = slic.warm.prepare(net.params, w.S)
        for _ in range(args.warmup + args.steps):
            slic.warm.warm_segment(rgb, p, prepared, 2, workspace=ws)
        torch.cuda.synchronize()
        print(f"ran {args.warmup + args.steps} warm-start frames of {w.name}", flush=True)
        return 0
    if args.c5_only:
        res = bench_c5(slic, torch, dev, args.train_steps, args.train_images, 32,
                       reps=max(3, args.steps // 100))
        print(json.dumps({"c5": res}), flush=True)
        return 0
    if args.workload_only == "c4":
        # the 64-image batch through one HIP graph, the variant the batch
        # autotuner picks (as in the c4 leg), without connectivity
        wls = synth.batch_workload()
        imgs = [torch.from_numpy(synth.image_for(w).reshape(-1)).to(dev) for w in wls]
        params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb) for w in wls]
        b = slic.Batch(params, imgs, wls[0].iters, use_graph=True)
        variant, _ = b.autotune(reps=2)
        for _ in range(args.warmup + args.steps):
            b.run()
        torch.cuda.synchronize()
        print(f"ran {args.warmup + args.steps} batches of c4 (variant {variant})", flush=True)
        return 0
    if args.workload_only:
        w = synth.WORKLOADS[args.workload_only]
        f = Frame(slic, w, dev)
        for _ in range(args.warmup + args.steps):
            f.run(w.iters, w.connectivity)
        torch.cuda.synchronize()
        print(f"ran {args.warmup + args.steps} frames of {w.name}", flush=True)
        if args.copy_bytes > 0:
            src = torch.ones(args.copy_bytes, dtype=torch.uint8, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            print(f"copied {args.copy_bytes} bytes 3 times", flush=True)
        return 0

    wl = synth.WORKLOADS["c2"]
    frame = Frame(slic, wl, dev)
    sec = time_frames(torch, frame, args.steps, args.warmup, wl.iters, wl.connectivity)
    value = 1.0 / sec

    ktimes = kernel_times(slic, torch, frame, min(args.steps, 200), wl.iters, wl.connectivity)
    a_ms = assign_from_frames_ms(torch, frame, max(args.steps, 20))
    nbytes = assign_bytes(wl.n_pixels, frame.K)
    gbps = nbytes / (a_ms * 1e-3) / 1e9
    ops = ASSIGN_OPS_PER_PIXEL * wl.n_pixels
    tflops = ops / (a_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(tflops, 3), "peak": ALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tflops / ALU_PEAK_TFLOPS, 4),
                "traffic": traffic_from_profile(),
                "kernel": f"assign_kernel (variant {frame.variant}: "
                          f"{'x'.join(map(str, slic.slic_assign_variant_info(frame.variant)[:2]))} "
                          f"pixels per thread)",
                "avg_launch_us": round(a_ms * 1e3, 3),
                "ops_per_pixel": ASSIGN_OPS_PER_PIXEL, "ops_per_launch": ops,
                "hbm": {"bytes_per_launch": nbytes, "achieved_gbps": round(gbps, 1),
                        "peak_gbps": HBM_PEAK_GBPS, "frac": round(gbps / HBM_PEAK_GBPS, 4)}}
    valu = valu_from_profile()
    if valu:
        per_px = valu["c2"]["valu_per_pixel"]
        lane_t = per_px * wl.n_pixels / (a_ms * 1e-3) / 1e12
        roofline["valu"] = {"instructions_per_pixel": per_px,
                            "transcendental_per_pixel": valu["c2"]["trans_per_pixel"],
                            "achieved_t_lane_instr_per_s": round(lane_t, 2),
                            "peak_t_lane_instr_per_s": VALU_ISSUE_PEAK_T,
                            "frac": round(lane_t / VALU_ISSUE_PEAK_T, 4),
                            "counters": os.path.relpath(VALU_FILE, ROOT)}

    extra = {"kernels_c2_event_bracketed": {k: {"avg_us": round(v["avg_ms"] * 1e3, 3),
                                "per_frame": v["launches_per_frame"]} for k, v in ktimes.items()}}
    up = time_frames_with_upload(torch, frame, args.steps, args.warmup)
    extra["c2_with_upload"] = {"frames_per_s": round(1.0 / up, 2), "ms_per_frame": round(up * 1e3, 4),
                               "upload": "921,600-byte frame from pinned host memory, on the "
                                         "launch stream, inside every timed frame"}
    if not args.no_extra:
        for name in ("c1", "c2", "c3"):
            w = synth.WORKLOADS[name]
            f = frame if name == "c2" else Frame(slic, w, dev)
            steps = max(20, args.steps // (5 if name == "c3" else 1))
            t10 = time_frames(torch, f, steps, 5, 10, False)
            t0 = time_frames(torch, f, steps, 5, 0, False)
            t_iter = (t10 - t0) / 10
            entry = {"mpix_per_s_per_iter": round(w.n_pixels / t_iter / 1e6, 1),
                     "us_per_iter": round(t_iter * 1e6, 3)}
            if name != "c2":
                tf = time_frames(torch, f, steps, 5, w.iters, w.connectivity)
                entry["frames_per_s"] = round(1.0 / tf, 1)
                a = assign_from_frames_ms(torch, f, steps)
                b = assign_bytes(w.n_pixels, f.K)
                entry["assign_avg_us"] = round(a * 1e3, 3)
                entry["assign_variant"] = f.variant
                entry["assign_gbps"] = round(b / (a * 1e-3) / 1e9, 1)
                entry["assign_hbm_frac"] = round(b / (a * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
            if name == "c3":
                # row f4: the squared-sum distance (no square roots) at 1080p
                fq = Frame(slic, w, dev, squared_distance=True)
                tq = (time_frames(torch, fq, steps, 5, 10, False) -
                      time_frames(torch, fq, steps, 5, 0, False)) / 10
                aq = assign_from_frames_ms(torch, fq, steps)
                entry["squared_distance"] = {
                    "mpix_per_s_per_iter": round(w.n_pixels / tq / 1e6, 1),
                    "us_per_iter": round(tq * 1e6, 3), "assign_avg_us": round(aq * 1e3, 3),
                    "assign_variant": fq.variant}
            extra[name] = entry
        extra["c4"] = bench_c4(slic, torch, dev, reps=max(5, args.steps // 50))
        extra["c2_batched"] = bench_c2_batched(slic, torch, dev, 16, reps=max(5, args.steps // 50))
        extra["c5"] = bench_c5(slic, torch, dev, args.train_steps, args.train_images, 32,
                               reps=max(3, args.steps // 100))
        extra["video"] = bench_video(slic, torch, dev, 32, 2, reps=max(3, args.steps // 100))
        extra["cleanup_c2"] = bench_cleanup(slic, torch, dev, reps=20)
    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2: one 640x480 seeded Voronoi image (256 regions, sigma 8), "
                               "S=16 (K=1200), m=10, 10 iterations, perturbed seeds, "
                               "connectivity (S*S/4 merge)",
                   "global_batch": 1, "parallelism": "none (one GPU)"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    line["extra"] = extra
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
