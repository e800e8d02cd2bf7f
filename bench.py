#!/usr/bin/env python3
"""Throughput of the uplink receiver (fft -> csi -> ZF detect -> max-log demod)
on one MI355X, in subcarrier-detections per second.

One step = the whole receiver over one batch of 100 frames of the
64-antenna, 16-user workload (N_FFT 2048, 1200 used subcarriers, 14 symbols,
16-QAM, i.i.d. Rayleigh, per-user SNR uniform in [10, 30] dB), with the
complex64 samples already resident in HBM.  One subcarrier-detection is one
(frame, data symbol, used subcarrier) turned into K*Q LLRs.

Prints one JSON line.  Per-stage kernel times come from HIP events recorded
on the stream the kernels run on; the dominant stage is priced against the
HBM roofline.  The FP64 oracle is timed on a bounded sample on the host.
"""
import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "subcarrier-detections/s (64×16, FFT→ZF→LLR), mixed/batched vs plain FP32"
HBM_PEAK_GBS = 8000.0


def _gen(args):
    cfg, f = args
    fr = synth.make_frame(cfg, f)
    return fr.x, fr.pilots


def gen_frames(cfg, n, workers):
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_gen, [(cfg, f) for f in range(n)], chunksize=max(1, n // (4 * workers))))
    return np.stack([r[0] for r in res]), np.stack([r[1] for r in res])


def stage_bytes(s):
    """Compulsory HBM bytes of each stage's interface tensors for one frame."""
    M, K, N, n_sc, S, cp, Q = s.M, s.K, s.n_fft, s.n_sc, s.n_sym, s.cp_len, s.qam_bits
    D = S - 1
    return {
        "fft": M * S * (cp + N) * 8 + M * S * n_sc * 8,
        "csi": M * n_sc * 8 + n_sc * 8 + M * K * n_sc * 8,
        "detect": M * K * n_sc * 8 + M * D * n_sc * 8 + K * D * n_sc * 8 + K * n_sc * 4 + n_sc,
        "demod": K * D * n_sc * 8 + K * n_sc * 4 + K * D * n_sc * Q * 4,
    }


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(cfg, det, budget_s):
    import oracle as O
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:  # pragma: no cover
        lim = None
    t_total, n, dets = 0.0, 0, 0
    while t_total < budget_s:
        fo = synth.make_frame(cfg, n)
        t0 = time.perf_counter()
        O.forward(fo.x, fo.pilots, fo.shape, 1.0, det)
        t_total += time.perf_counter() - t0
        dets += fo.shape.detections
        n += 1
    if lim is not None:
        lim.unregister() if hasattr(lim, "unregister") else None
    return {"value": dets / t_total, "unit": "subcarrier-detections/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d frame(s) of the same workload through the FP64 oracle "
                      "(fft, csi, %s, brute-force max-log), %.1f s of one core" %
                      (n, "ZF" if det == 0 else "MMSE", t_total)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the plain device copy timed as the bandwidth reference (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: frames are independent, so more GPUs would each "
              "run this same single-GPU path on their own share of frames (see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    cfg, det = 2, 0
    shape = synth.config_shape(cfg)
    F = args.frames
    t0 = time.time()
    x_h, p_h = gen_frames(cfg, F, args.workers)
    gen_s = time.time() - t0

    import torch
    import paper_2603_20481_amd as rx
    rx.load()
    torch.cuda.init()
    fr = rx.Frame.of(shape, det, 1.0)
    x = torch.from_numpy(x_h).cuda()
    p = torch.from_numpy(p_h).cuda()
    del x_h
    D = shape.n_data
    yf = torch.empty((F, shape.M, shape.n_sym, shape.n_sc), dtype=torch.complex64, device="cuda")
    h = torch.empty((F, shape.M, shape.K, shape.n_sc), dtype=torch.complex64, device="cuda")
    xt = torch.empty((F, shape.K, D, shape.n_sc), dtype=torch.complex64, device="cuda")
    nu = torch.empty((F, shape.K, shape.n_sc), dtype=torch.float32, device="cuda")
    fl = torch.empty((F, shape.n_sc), dtype=torch.uint8, device="cuda")
    llr = torch.empty((F, shape.K, D, shape.n_sc, shape.qam_bits), dtype=torch.float32, device="cuda")

    names = ["fft", "csi", "detect", "demod"]

    def step(ev=None):
        if ev: ev[0].record()
        rx.fft(fr, x, yf)
        if ev: ev[1].record()
        rx.csi(fr, yf, p, h)
        if ev: ev[2].record()
        rx.detect(fr, h, yf, "fp32", 1e3, xt, nu, fl)
        if ev: ev[3].record()
        rx.demod(fr, xt, nu, llr)
        if ev: ev[4].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_stage = {n: 0.0 for n in names}
    for ev in evs:
        for j, n in enumerate(names):
            per_stage[n] += ev[j].elapsed_time(ev[j + 1]) / args.steps   # ms
    ms_per_step = wall * 1e3 / args.steps
    dets = F * shape.detections
    value = dets / (ms_per_step * 1e-3)

    sb = stage_bytes(shape)
    dom = max(names, key=lambda n: per_stage[n])
    achieved = sb[dom] * F / (per_stage[dom] * 1e-3) / 1e9
    stages = {n: {"us": round(per_stage[n] * 1e3, 2),
                  "GBps": round(sb[n] * F / (per_stage[n] * 1e-3) / 1e9, 1),
                  "bytes_per_launch": sb[n] * F} for n in names}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "subcarrier-detections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator: Rayleigh block channel, comb pilots, AWGN)",
        "config": {"workload": "64x16 MIMO, N_FFT 2048, 1200 used subcarriers, 14 symbols, 16-QAM, "
                               "Rayleigh, SNR U[10,30] dB, 100 frames, ZF, FP32",
                   "frames": F, "M": shape.M, "K": shape.K, "n_fft": shape.n_fft,
                   "n_sc": shape.n_sc, "n_sym": shape.n_sym, "qam_bits": shape.qam_bits,
                   "detector": "zf", "precision": "fp32"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom), "traffic_unit": "bytes/launch",
                     "algorithmic_bytes": sb[dom] * F},
        "stages": stages,
        "staged_roofline_frac": round(sum(sb.values()) * F / (sum(per_stage.values()) * 1e-3) / 1e9
                                      / HBM_PEAK_GBS, 4),
        "gen_seconds": round(gen_s, 1),
    }
    if args.copy_mib > 0:
        # plain device-to-device copy of a known size: the achievable-bandwidth
        # reference, and the calibration kernel for the HBM byte counters
        n = args.copy_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(2):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        out["copy_reference"] = {"bytes_per_launch": 2 * n, "us": round(ms * 1e3, 1),
                                 "GBps": round(2 * n / (ms * 1e-3) / 1e9, 1)}
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, det, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
