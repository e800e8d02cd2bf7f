#!/usr/bin/env python3
"""Throughput of the uplink receiver (fft -> csi -> ZF detect -> max-log demod)
on one MI355X, in subcarrier-detections per second.

Headline step = the whole receiver over one batch of 100 frames of the
64-antenna, 16-user workload (N_FFT 2048, 1200 used subcarriers, 14 symbols,
16-QAM, i.i.d. Rayleigh, per-user SNR uniform in [10, 30] dB), plain FP32 ZF,
with the complex64 samples already resident in HBM: the FFT call and the
fused CSI + detector + demod call (the channel estimate is formed in the
detector and never stored, and each equalised symbol is demapped as it is
formed, so neither H nor x_tilde goes through memory).  One
subcarrier-detection is one (frame, data symbol, used subcarrier) turned into
K*Q LLRs.

Beside the headline the same line reports the other forms, each timed the same
way: the four separate stage calls on the same frames; csi + detect fused with
demod as its own call; MMSE; the BF16 / FP16 detector with FP64 refinement on
the 64x16 N_FFT 4096 64-QAM correlated workload (and plain FP32 there); 256
uneven frames in one persistent launch replayed from a hipGraph, with
autotuned and default item sizes and against a loop of per-frame calls; and
forward + adjoint on the 64x8 cascaded-channel workload; and the downlink
(QAM mapping, ZF precoder from the uplink estimate, inverse transform with
prefix) over the headline frames; and the real-time form: one task of C
frames released per frame period into a ping-pong stream, with the p99
latency against the period, for host-memory and device-resident samples;
the headline step with 16-bit I/Q samples (the fronthaul format); and the
paper's own sensing pipeline on (2000, 1024) TF plots: a batch of
plots per call, single-plot latency against the 20.48 ms window, detection
quality and the oracle on one core.

Before the W warm-up steps the headline runs untimed for --settle-s seconds
(0.5 s by default; the count is reported as settle_steps): the first few
hundred milliseconds of GPU work after the host-side set-up run about 9 %
slower while the clocks ramp, which a handful of warm-up steps does not cover.

Prints one JSON line.  Kernel times come from HIP events recorded on the
stream the kernels run on; the dominant stage is priced against the HBM
roofline.  The FP64 oracle is timed on a bounded sample on the host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "subcarrier-detections/s (64×16, FFT→ZF→LLR), mixed/batched vs plain FP32"
HBM_PEAK_GBS = 8000.0
# the calls of each way of running the chain
MODES = {"staged": ["fft", "csi", "detect", "demod"],          # the four stage calls
         "csi_detect": ["fft", "csi_detect", "demod"],        # csi and detect fused
         "full": ["fft", "csi_detect_demod"]}                 # csi, detect and demod fused


def gen_frames(cfg, n, workers, shape=None):
    res = synth.draw_inputs(cfg, range(n), [shape] * n if shape is not None else None, workers)
    return np.stack([r[0] for r in res]), np.stack([r[1] for r in res])


def stage_bytes(s):
    """Compulsory HBM bytes of each stage's interface tensors for one frame
    (csi_detect: the fused csi + detect call, which never stores H;
    csi_detect_demod: csi, detect and demod fused, which stores neither H nor
    x_tilde)."""
    M, K, N, n_sc, S, cp, Q = s.M, s.K, s.n_fft, s.n_sc, s.n_sym, s.cp_len, s.qam_bits
    D = S - 1
    return {
        "fft": M * S * (cp + N) * 8 + M * S * n_sc * 8,
        "csi": M * n_sc * 8 + n_sc * 8 + M * K * n_sc * 8,
        "detect": M * K * n_sc * 8 + M * D * n_sc * 8 + K * D * n_sc * 8 + K * n_sc * 4 + n_sc,
        "csi_detect": M * n_sc * 8 + n_sc * 8 + M * D * n_sc * 8 + K * D * n_sc * 8 + K * n_sc * 4 + n_sc,
        "csi_detect_demod": M * n_sc * 8 + n_sc * 8 + M * D * n_sc * 8 + K * n_sc * 4 + n_sc
                            + K * D * n_sc * Q * 4,
        "demod": K * D * n_sc * 8 + K * n_sc * 4 + K * D * n_sc * Q * 4,
    }


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when a source of the kernel has changed since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None
    return rec["traffic_bytes_per_launch"]


# GPU outputs of sampled frames of each form, kept (on the host, outside the
# timed regions) for the oracle leg: {form: dict(kind, ...)}
SAMPLES = {}


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_frame(job):
    """One frame through the FP64 oracle on one thread; returns the seconds."""
    import oracle as O
    from threadpoolctl import threadpool_limits
    cfg, f, det = job
    fo = synth.make_frame(cfg, f)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.forward(fo.x, fo.pilots, fo.shape, 1.0, det)
        return time.perf_counter() - t0


def _errors(ref, llr, xt=None, nu=None, flags=None, band_u=None):
    """Error of one frame's GPU outputs against the oracle's: EVM over the
    subcarriers with kappa_2 <= 1e3 that neither side erased, the relative LLR
    error |d| / max(|ref|, 0.01 RMS), the largest absolute LLR error and the
    hard-bit mismatches outside the guard band (1e-5 RMS, or band_u * kappa
    RMS for the mixed forms)."""
    r = ref["llr"]
    rms = float(np.sqrt(np.mean(r ** 2)))
    d = np.abs(llr.astype(np.float64) - r)
    out = {"llr_rel": float(np.max(d / np.maximum(np.abs(r), 0.01 * rms))), "llr_max_abs": float(d.max())}
    good = ref["flags"] == 0
    if "kappa" in ref:
        good &= ref["kappa"] <= 1e3
    if flags is not None:
        good &= (flags & 6) == 0
    if xt is not None and np.any(good):
        a, b = xt[..., good].astype(np.complex128), ref["xt"][..., good]
        out["evm_rel"] = float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))
    if nu is not None and np.any(good):
        out["nu_rel"] = float(np.sqrt(np.sum((nu[:, good] - ref["nu"][:, good]) ** 2)
                                      / np.sum(ref["nu"][:, good] ** 2)))
    tau = 1e-5 * rms
    if band_u is not None and "kappa" in ref:
        tau = max(tau, band_u * float(ref["kappa"][ref["flags"] == 0].max()) * rms)
    outside = np.abs(r) > tau
    out["hard_bit_mismatches"] = int(np.sum(((llr < 0) != (r < 0)) & outside))
    out["bits_in_band"] = int(np.sum(~outside))
    return out


def cpu_baseline(cfg, det, budget_s, workers):
    """The FP64 oracle as it stands, timed on the host: the headline workload on
    one core and on `workers` cores (one process per core, frames spread over
    them); then each kept sample of the other forms, timed on one core, with
    the GPU's error on that sample."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import oracle as O
    from threadpoolctl import threadpool_limits
    head = SAMPLES.get("headline")
    errs = []
    t_total, n, dets = 0.0, 0, 0
    with threadpool_limits(1):
        while t_total < budget_s:
            fo = synth.make_frame(cfg, n)
            t0 = time.perf_counter()
            O.forward(fo.x, fo.pilots, fo.shape, 1.0, det)
            t_total += time.perf_counter() - t0
            dets += fo.shape.detections
            if head is not None and n in head["frames"]:          # untimed: with the exact kappa_2
                k = head["frames"].index(n)
                ref = O.forward(fo.x, fo.pilots, fo.shape, 1.0, det, want_kappa=True)
                errs.append(_errors(ref, head["llr"][k], head["xt"][k], head["nu"][k], head["flags"][k]))
            n += 1
    one = dets / t_total
    # all cores: a process per core, each frame on one thread
    per_frame = fo.shape.detections
    jobs = [(cfg, f, det) for f in range(max(workers * 8, 1))]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        list(ex.map(_oracle_frame, [(cfg, 0, det)] * workers))        # start the workers
        t0 = time.perf_counter()
        secs = list(ex.map(_oracle_frame, jobs))
        wall = time.perf_counter() - t0
    many = len(jobs) * per_frame / wall
    out = {"value": many, "unit": "subcarrier-detections/s", "cores": workers, "kind": "oracle",
           "sample": "%d frames of the headline workload through the FP64 oracle (fft, csi, %s, brute-force "
                     "max-log), one process per core, one thread each, %.1f s wall" %
                     (len(jobs), "ZF" if det == 0 else "MMSE", wall),
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "single_core": {"value": one, "cores": 1,
                           "sample": "%d frame(s), %.1f s of one core" % (n, t_total)},
           "mean_frame_s_per_core": float(np.mean(secs))}
    if errs:
        out["headline_error"] = {k: max(e[k] for e in errs) for k in errs[0]}
        out["headline_error"]["frames"] = head["frames"]
    forms = {}
    with threadpool_limits(1):
        for name, smp in SAMPLES.items():
            if name == "headline":
                continue
            t0 = time.perf_counter()
            if smp["kind"] == "forward":
                per = []
                dets = 0
                for k, fo in enumerate(smp["inputs"]):
                    ref = O.forward(fo.x, fo.pilots, fo.shape, 1.0, smp["det"][k], want_kappa=True)
                    dets += fo.shape.detections
                    for lab, o in smp["outputs"][k].items():
                        per.append((lab, _errors(ref, o["llr"], o.get("xt"), o.get("nu"), o.get("flags"),
                                                 o.get("band_u"))))
                secs = time.perf_counter() - t0
                res = {}
                for lab, e in per:
                    cur = res.setdefault(lab, {})
                    for key, v in e.items():
                        cur[key] = max(cur.get(key, v), v)
                forms[name] = {"oracle_1core": {"value": dets / secs, "unit": "subcarrier-detections/s",
                                                "seconds": round(secs, 2), "frames": len(smp["inputs"])},
                               "error": res}
            elif smp["kind"] == "ldpc":             # bit-exact against the FP32-mode oracle; FP64 timed
                from oracle import ldpc_oracle as LO
                same = True
                for k in range(len(smp["index"])):
                    rp, rb, ri = LO.decode(smp["base"], smp["z"], smp["llr"][k], smp["max_iter"], smp["alpha"],
                                           dtype=np.float32)
                    same = same and ri == smp["iters"][k] and np.array_equal(rb, smp["bits"][k]) and \
                        np.array_equal(rp.view(np.uint32), smp["post"][k].view(np.uint32))
                t1 = time.perf_counter()
                for k in range(len(smp["index"])):
                    LO.decode(smp["base"], smp["z"], smp["llr"][k], smp["max_iter"], smp["alpha"])
                secs = time.perf_counter() - t1
                kb = smp["base"].shape[1] - smp["base"].shape[0]
                forms[name] = {"oracle_1core": {"value": len(smp["index"]) * kb * smp["z"] / secs / 1e9,
                                                "unit": "Gbit/s (FP64 oracle)", "seconds": round(secs, 2),
                                                "codewords": len(smp["index"])},
                               "error": {"bit_exact_vs_fp32_oracle": bool(same), "codewords": smp["index"]}}
            else:                                   # backward: dL/dx against the oracle adjoint
                fo = smp["input"]
                gx, _ = O.backward(fo.x, fo.pilots, fo.shape, 1.0, smp["det"], smp["dllr"].astype(np.float64))
                secs = time.perf_counter() - t0
                got = smp["dx"].astype(np.complex128)
                rms = float(np.sqrt(np.mean(np.abs(gx) ** 2)))
                forms[name] = {"oracle_1core": {"value": fo.shape.detections / secs,
                                                "unit": "subcarrier-detections/s (forward + adjoint)",
                                                "seconds": round(secs, 2), "frames": 1},
                               "error": {"dx_rel_rms": float(np.sqrt(np.sum(np.abs(got - gx) ** 2)
                                                                     / np.sum(np.abs(gx) ** 2))),
                                         "dx_elem_rel": float(np.max(np.abs(got - gx)
                                                                     / np.maximum(np.abs(gx), 0.01 * rms)))}}
    out["forms"] = forms
    return out


class Chain:
    """Device buffers of F same-shape frames and the four stage calls."""

    def __init__(self, rx, torch, shape, x_h, p_h):
        self.rx, self.torch, self.shape = rx, torch, shape
        F = x_h.shape[0]
        self.F = F
        dev = "cuda"
        D = shape.n_data
        self.x = torch.from_numpy(x_h).to(dev)
        self.p = torch.from_numpy(p_h).to(dev)
        c64, f32 = torch.complex64, torch.float32
        self.yf = torch.empty((F, shape.M, shape.n_sym, shape.n_sc), dtype=c64, device=dev)
        self.h = torch.empty((F, shape.M, shape.K, shape.n_sc), dtype=c64, device=dev)
        self.xt = torch.empty((F, shape.K, D, shape.n_sc), dtype=c64, device=dev)
        self.nu = torch.empty((F, shape.K, shape.n_sc), dtype=f32, device=dev)
        self.fl = torch.empty((F, shape.n_sc), dtype=torch.uint8, device=dev)
        self.llr = torch.empty((F, shape.K, D, shape.n_sc, shape.qam_bits), dtype=f32, device=dev)
        self.ws = None
        self.thr = 1e3                     # condition-estimate threshold of the BF16 / FP16 forms

    def step(self, fr, prec="fp32", ev=None, mode="full"):
        rx = self.rx
        kind = {"staged": rx.WS_DETECT, "csi_detect": rx.WS_CSI_DETECT, "full": rx.WS_CSI_DETECT_DEMOD}[mode]
        need = rx.workspace_bytes(fr, self.F, kind, prec)
        if need and (self.ws is None or self.ws.numel() < need):
            self.ws = self.torch.empty((need,), dtype=self.torch.uint8, device="cuda")
        ws = self.ws if need else None
        if ev: ev[0].record()
        rx.fft(fr, self.x, self.yf)
        if ev: ev[1].record()
        if mode == "full":
            rx.csi_detect_demod(fr, self.yf, self.p, prec, self.thr, llr=self.llr, nu=self.nu, flags=self.fl,
                                ws=ws)
            if ev: ev[2].record()
            return
        if mode == "csi_detect":
            rx.csi_detect(fr, self.yf, self.p, prec, self.thr, self.xt, self.nu, self.fl, ws)
        else:
            rx.csi(fr, self.yf, self.p, self.h)
            if ev: ev[2].record()
            rx.detect(fr, self.h, self.yf, prec, self.thr, self.xt, self.nu, self.fl, ws)
        if ev: ev[len(MODES[mode]) - 1].record()
        rx.demod(fr, self.xt, self.nu, self.llr)
        if ev: ev[len(MODES[mode])].record()

    def settle(self, fr, prec, seconds, mode="full", max_steps=2000):
        """Untimed steps until `seconds` of wall time have passed: the first
        few hundred milliseconds of work after the host-side set-up run
        measurably slower (clocks ramping), which a handful of warm-up steps
        does not cover.  Returns the number of steps run."""
        torch = self.torch
        t0 = time.perf_counter()
        n = 0
        while n < max_steps and time.perf_counter() - t0 < seconds:
            for _ in range(10):
                self.step(fr, prec, mode=mode)
            torch.cuda.synchronize()
            n += 10
        return n

    def time(self, fr, prec, steps, warmup, mode="full"):
        torch = self.torch
        names = MODES[mode]
        for _ in range(warmup):
            self.step(fr, prec, mode=mode)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(fr, prec, evs[k], mode=mode)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = {n: 0.0 for n in names}
        for ev in evs:
            for j, n in enumerate(names):
                per[n] += ev[j].elapsed_time(ev[j + 1]) / steps   # ms
        return wall * 1e3 / steps, per


def stage_report(shape, F, per):
    sb = stage_bytes(shape)
    return {n: {"us": round(per[n] * 1e3, 2),
                "GBps": round(sb[n] * F / (per[n] * 1e-3) / 1e9, 1),
                "bytes_per_launch": sb[n] * F} for n in per}


def form_summary(shape, F, ms, per, extra=None):
    sb = stage_bytes(shape)
    dets = F * shape.detections
    out = {"value": dets / (ms * 1e-3), "unit": "subcarrier-detections/s", "ms_per_step": round(ms, 4),
           "frames": F, "stages": stage_report(shape, F, per),
           "hbm_frac": round(sum(sb[n] for n in per) * F / (sum(per.values()) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             4)}
    if extra:
        out.update(extra)
    return out


def downlink_bytes(s):
    """Compulsory HBM bytes of each downlink call for one frame (bits are one
    byte each; precode reads symbol 0 of yf and the pilots, never stores H)."""
    M, K, N, n_sc, cp, Q = s.M, s.K, s.n_fft, s.n_sc, s.cp_len, s.qam_bits
    D = s.n_sym - 1
    return {"modulate": K * D * n_sc * (Q + 8),
            "precode": M * n_sc * 8 + n_sc * 8 + K * D * n_sc * 8 + M * D * n_sc * 8 + n_sc,
            "ifft": M * D * n_sc * 8 + M * D * (cp + N) * 8}


def run_downlink(rx, torch, chain, args):
    """Modulate -> precode -> inverse transform over the headline frames, the
    precoder built from the uplink estimate of the same frames' yf."""
    shape, F = chain.shape, chain.F
    D = shape.n_data
    fr = rx.Frame.of(shape, rx.ZF, 1.0)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    bits = torch.randint(0, 2, (F, shape.K, D, shape.n_sc, shape.qam_bits), generator=g,
                         device="cuda", dtype=torch.uint8)
    rx.fft(fr, chain.x, chain.yf)
    sym = rx.modulate(fr, bits)
    xf, fl = rx.precode(fr, chain.yf, chain.p, sym)
    x = rx.ifft(fr, xf)
    ws = torch.empty((rx.workspace_bytes(fr, F, rx.WS_PRECODE, "fp32"),), dtype=torch.uint8, device="cuda")
    names = ("modulate", "precode", "ifft")

    def step(ev=None):
        if ev: ev[0].record()
        rx.modulate(fr, bits, sym)
        if ev: ev[1].record()
        rx.precode(fr, chain.yf, chain.p, sym, xf, fl, ws)
        if ev: ev[2].record()
        rx.ifft(fr, xf, x)
        if ev: ev[3].record()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.form_steps)]
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    per = {n: sum(ev[j].elapsed_time(ev[j + 1]) for ev in evs) / len(evs) for j, n in enumerate(names)}
    ms = sum(per.values())
    db = downlink_bytes(shape)
    flagged = int(fl.ne(0).sum().item())
    # TDD reciprocity: the precoder reuses the factor records the uplink's fused
    # call left in its workspace for the same frames (the factorisation skipped)
    wsu = torch.empty((rx.workspace_bytes(fr, F, rx.WS_CSI_DETECT_DEMOD, "fp32"),), dtype=torch.uint8,
                      device="cuda")
    rx.csi_detect_demod(fr, chain.yf, chain.p, ws=wsu)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.form_steps):
        rx.precode(fr, chain.yf, chain.p, sym, xf, fl, wsu, reuse_factors=True)
    e1.record()
    torch.cuda.synchronize()
    reuse_us = e0.elapsed_time(e1) / args.form_steps * 1e3
    # modulation fused into the precoder (the symbols never stored), factors reused
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rx.modulate_precode(fr, chain.yf, chain.p, bits, xf, fl, wsu, reuse_factors=True)
    e0.record()
    for _ in range(args.form_steps):
        rx.modulate_precode(fr, chain.yf, chain.p, bits, xf, fl, wsu, reuse_factors=True)
    e1.record()
    torch.cuda.synchronize()
    fused_us = e0.elapsed_time(e1) / args.form_steps * 1e3
    # the time samples as 16-bit I/Q for the radio (power-of-two step with
    # one bit of headroom over the peak sample)
    peak = float(torch.max(torch.abs(torch.view_as_real(x))).item())
    q_scale = 2.0 ** np.ceil(np.log2(peak * 2.0 / 32767.0))
    x16 = rx.ifft_sc16(fr, xf, q_scale)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.form_steps):
        rx.ifft_sc16(fr, xf, q_scale, x16)
    e1.record()
    torch.cuda.synchronize()
    ifft16_us = e0.elapsed_time(e1) / args.form_steps * 1e3
    ifft16_bytes = F * shape.M * D * (shape.n_sc * 8 + (shape.cp_len + shape.n_fft) * 4)
    out = {"value": F * shape.detections / (ms * 1e-3), "unit": "subcarrier-precodings/s",
           "ms_per_step": round(ms, 4), "frames": F,
           "stages": {n: {"us": round(per[n] * 1e3, 2),
                          "GBps": round(db[n] * F / (per[n] * 1e-3) / 1e9, 1),
                          "bytes_per_launch": db[n] * F} for n in names},
           "hbm_frac": round(sum(db.values()) * F / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "flagged_subcarriers": flagged,
           "after_uplink": {"precode_us": round(reuse_us, 2),
                            "ms_per_step": round(per["modulate"] + reuse_us * 1e-3 + per["ifft"], 4),
                            "note": "precode reusing the uplink fused call's factor records "
                                    "(same frames, ZF): the factorisation is skipped"},
           "modulate_precode": {"us": round(fused_us, 2),
                                "ms_per_step_after_uplink": round((fused_us + per["ifft"] * 1e3) * 1e-3, 4),
                                "ms_per_step_after_uplink_sc16_out": round((fused_us + ifft16_us) * 1e-3, 4),
                                "note": "modulation fused into the precoder (the symbols never stored), "
                                        "the uplink's factor records reused"},
           "sc16_out": {"ifft_us": round(ifft16_us, 2), "scale": q_scale,
                        "GBps": round(ifft16_bytes / (ifft16_us * 1e-6) / 1e9, 1), "bytes_per_launch": ifft16_bytes,
                        "ms_per_step_after_uplink": round(per["modulate"] + (reuse_us + ifft16_us) * 1e-3, 4),
                        "note": "time samples written as 16-bit I/Q (round to nearest, saturating)"},
           "workload": "headline frames (64x16, N_FFT 2048, 1200 subcarriers, 13 data symbols, "
                       "16-QAM): random bits -> QAM -> ZF precoder from the uplink LS estimate "
                       "-> unscaled inverse transform with prefix, FP32"}
    del bits, sym, xf, fl, x, ws, wsu, x16
    torch.cuda.empty_cache()
    return out


SCS_HZ = 15e3      # subcarrier spacing of the streaming form: f_s = N_FFT x 15 kHz


def run_streaming(rx, torch, chain, args):
    """Real-time form: one task (C frames of the headline shape) becomes
    available every frame period P = n_sym (cp + N) / f_s; a producer thread
    releases task k at t0 + k P into a ping-pong stream (2 slots) and the
    runtime stamps its completion.  A configuration is real-time when at
    least 99 % of tasks finish within P (nearest-rank p99 <= P)."""
    shape, F = chain.shape, chain.F
    fs = shape.n_fft * SCS_HZ
    period_us = shape.n_sym * (shape.cp_len + shape.n_fft) / fs * 1e6
    fr = rx.Frame.of(shape, rx.ZF, 1.0)
    runs = []
    for host_io, sc16, counts in ((True, False, (1, 2, 3, 4)), (True, True, (2, 3, 4, 5)),
                                  (False, False, (1, 25, 50, 100))):
        for C in counts:
            if C > F:
                continue
            xh = chain.x[:C].cpu().numpy() if host_io else None
            q, scale = synth.quantize_sc16(xh) if sc16 else (None, 0.0)
            st = rx.Stream(fr, C, depth=2, host_io=host_io, sc16_scale=scale)
            outs = None
            if host_io:
                ph = chain.p[:C].cpu().numpy()
                for slot in range(2):
                    h = st.host(slot)
                    h["x"][...] = q if sc16 else xh
                    h["pilots"][...] = ph
            else:
                outs = [(torch.empty((C, fr.K, fr.n_data, fr.n_sc, fr.qam_bits), device="cuda"),
                         torch.empty((C, fr.K, fr.n_sc), device="cuda"),
                         torch.empty((C, fr.n_sc), dtype=torch.uint8, device="cuda")) for _ in range(2)]
                xs, ps = chain.x[:C], chain.p[:C]
                torch.cuda.synchronize()

            def produce(n):
                t0 = rx.clock_ns() + 1_000_000
                step = int(round(period_us * 1e3))
                for k in range(n):
                    t = t0 + k * step
                    while rx.clock_ns() < t:
                        pass
                    slot = st.acquire()
                    if host_io:
                        st.submit(slot, t)
                    else:
                        st.submit(slot, t, xs, ps, *outs[slot])
                st.drain()
            produce(args.stream_warmup)
            st.reset_latencies()
            produce(args.stream_tasks)
            lat = st.latencies()
            st.close()
            summ = rx.latency_summary(lat, period_us)
            io = "device-resident" if not host_io else \
                ("host, 16-bit I/Q in" if sc16 else "host (PCIe in and out)")
            runs.append({"io": io,
                         "frames_per_task": C, "tasks": int(summ["count"]),
                         "p50_us": round(summ["p50_us"], 1), "p99_us": round(summ["p99_us"], 1),
                         "max_us": round(summ["max_us"], 1), "mean_us": round(summ["mean_us"], 1),
                         "on_time": int(summ["on_time"]), "real_time": bool(summ["meets_99"]),
                         "detections_per_s": C * shape.detections / (period_us * 1e-6)})
            print("[bench] streaming %s C=%d p99 %.1f us (period %.1f)" %
                  (io, C, summ["p99_us"], period_us), file=sys.stderr, flush=True)
            del st, outs
    best = {}
    for r in runs:
        if r["real_time"]:
            k = r["io"]
            if k not in best or r["frames_per_task"] > best[k]["frames_per_task"]:
                best[k] = {"frames_per_task": r["frames_per_task"], "detections_per_s": r["detections_per_s"],
                           "p99_us": r["p99_us"]}
    torch.cuda.empty_cache()
    return {"period_us": round(period_us, 2), "sample_rate_msps": fs / 1e6, "depth": 2, "runs": runs,
            "largest_real_time": best,
            "workload": "tasks of C headline frames (64x16, N_FFT 2048, 1200 subcarriers, 14 symbols, "
                        "16-QAM, ZF, FP32), one task released per frame period (14 symbols at 15 kHz "
                        "subcarrier spacing, f_s = 30.72 MS/s); task = fft + fused csi/detect/demod, with "
                        "the samples copied in from and the LLRs, noise variances and flags copied back "
                        "to pinned host memory (host) or read and written in HBM (device-resident); "
                        "latency = completion - release; real time = at least 99 % within the period; the "
                        "16-bit runs carry the samples as quantised I/Q pairs (power-of-two scale)"}


SENSE_DEADLINE_US = 20480.0   # (T, F) = (2000, 1024) at 100 MS/s: T * F / f_s


def sense_bytes(T, F):
    """Compulsory HBM bytes of one plot per kernel of rxphy_sense.  The
    morphology reads the mask and writes the morphed mask, plus per 64x64
    tile its component list (784 bytes) and its border labels (1 KiB); the
    labelling passes read the lists three times and touch pixels only in
    tiles whose list overflowed (not counted, nor the union-find's chains)."""
    px = T * F
    tiles = -(-T // 64) * (F // 64)
    return {"fft_mag": px * 12, "colstat": px * 4 + F * 12, "otsu": px * 5 + F * 4,
            "morph": px * 2 + tiles * (784 + 1024), "ccl": tiles * 784 * 3}


def run_sensing(rx, torch, args):
    """The paper's sensing pipeline on (T, F) = (2000, 1024) plots: a batch
    of plots in one call (throughput), single plots (latency against the
    20.48 ms window) and the oracle on one host core."""
    from synth import sensing as SS
    T, F, P = 2000, 1024, args.sense_plots
    cfg = rx.SenseConfig(n_fft=F, n_rows=T)
    distinct = min(P, 16)
    t0 = time.time()
    scenes = [SS.make_scene(900 + i, "mixed", T=T, F=F) for i in range(distinct)]
    gen_s = time.time() - t0
    xh = np.stack([scenes[i % distinct].x for i in range(P)])
    x = torch.from_numpy(xh).cuda()
    ws = torch.empty((rx.sense_workspace_bytes(cfg, P),), dtype=torch.uint8, device="cuda")
    nb = torch.empty((P,), dtype=torch.int32, device="cuda")
    bx = torch.empty((P, 1024, 4), dtype=torch.int32, device="cuda")

    def call(xx, n, b):
        rx.sense(cfg, xx, max_boxes=1024, ws=ws, boxes=b, n_boxes=n)
    for _ in range(args.warmup):
        call(x, nb, bx)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.form_steps):
        call(x, nb, bx)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.form_steps
    sb = sense_bytes(T, F)
    byts = sum(sb.values()) * P
    # quality of the batch's boxes against the scenes' ground truth
    n_h, b_h = nb.cpu().numpy(), bx.cpu().numpy()
    pd, pfa, miou = [], [], []
    for i in range(distinct):
        m = rx.box_metrics(scenes[i].boxes, b_h[i][:min(int(n_h[i]), 1024)], 0.4)
        pd.append(m["p_d"])
        pfa.append(m["p_fa"])
        miou.append(m["mean_iou"])
    # single plots, each call synchronised: latency of one plot
    x1, n1, b1 = x[:1], nb[:1], bx[:1]
    lat = []
    for k in range(args.sense_latency_calls + 5):
        t1 = time.perf_counter()
        call(x1, n1, b1)
        torch.cuda.synchronize()
        if k >= 5:
            lat.append((time.perf_counter() - t1) * 1e6)
    summ = rx.latency_summary(lat, SENSE_DEADLINE_US)
    out = {"value": P / (ms * 1e-3), "unit": "TF plots/s", "ms_per_step": round(ms, 4), "plots": P,
           "algorithmic_bytes": byts, "GBps": round(byts / (ms * 1e-3) / 1e9, 1),
           "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "bytes_per_plot": sb,
           "single_plot_latency_us": {"p50": round(summ["p50_us"], 1), "p99": round(summ["p99_us"], 1),
                                      "max": round(summ["max_us"], 1), "calls": int(summ["count"]),
                                      "deadline_us": SENSE_DEADLINE_US, "real_time": bool(summ["meets_99"])},
           "detection": {"p_d": round(float(np.mean(pd)), 4), "p_fa": round(float(np.mean(pfa)), 4),
                         "mean_iou": round(float(np.mean(miou)), 4), "theta_iou": 0.4,
                         "scenes": distinct},
           "gen_seconds": round(gen_s, 1),
           "workload": "(T, F) = (2000, 1024) TF plots of synthetic captures (noise + BLE / OFDM / DSSS "
                       "energy blocks, mixed scenario, 16 distinct scenes), Savitzky-Golay 21/1, theta_PSD "
                       "1.1 N0, 256 Otsu bins; %d plots per call, FP32" % P}
    if not args.no_cpu_baseline:
        from oracle import sensing_oracle as SO
        t1 = time.perf_counter()
        SO.sense(scenes[0].x, SO.SenseConfig(F=F, T=T))
        dt = time.perf_counter() - t1
        out["cpu_oracle"] = {"value": 1.0 / dt, "unit": "TF plots/s", "cores": 1,
                             "sample": "one (2000, 1024) plot through the sensing oracle, %.2f s" % dt}
    del x, ws, nb, bx
    torch.cuda.empty_cache()
    return out


def run_sc16(rx, torch, chain, args):
    """The headline step with the samples as 16-bit I/Q (the fronthaul format
    of Section IV-D): the headline frames quantised with a power-of-two
    scale, then fft_sc16 and the fused csi + detect + demod call."""
    shape, F = chain.shape, chain.F
    fr = rx.Frame.of(shape, rx.ZF, 1.0)
    xh = chain.x.cpu().numpy()
    q_h, scale = synth.quantize_sc16(xh)
    q = torch.from_numpy(q_h).cuda()
    del q_h
    ws = torch.empty((rx.workspace_bytes(fr, F, rx.WS_CSI_DETECT_DEMOD, "fp32"),), dtype=torch.uint8,
                     device="cuda")

    def step(ev=None):
        if ev: ev[0].record()
        rx.fft_sc16(fr, q, scale, chain.yf)
        if ev: ev[1].record()
        rx.csi_detect_demod(fr, chain.yf, chain.p, "fp32", 1e3, llr=chain.llr, nu=chain.nu, flags=chain.fl, ws=ws)
        if ev: ev[2].record()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.form_steps)]
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    per = {n: sum(ev[j].elapsed_time(ev[j + 1]) for ev in evs) / len(evs)
           for j, n in enumerate(("fft_sc16", "csi_detect_demod"))}
    ms = sum(per.values())
    sb = stage_bytes(shape)
    M, S, N, n_sc, cp = shape.M, shape.n_sym, shape.n_fft, shape.n_sc, shape.cp_len
    byts = {"fft_sc16": M * S * (cp + N) * 4 + M * S * n_sc * 8, "csi_detect_demod": sb["csi_detect_demod"]}
    out = {"value": F * shape.detections / (ms * 1e-3), "unit": "subcarrier-detections/s",
           "ms_per_step": round(ms, 4), "frames": F, "scale": scale,
           "stages": {n: {"us": round(per[n] * 1e3, 2), "GBps": round(byts[n] * F / (per[n] * 1e-3) / 1e9, 1),
                          "bytes_per_launch": byts[n] * F} for n in per},
           "workload": "as the headline, with the samples as 16-bit I/Q pairs (power-of-two scale, "
                       "converted to FP32 in the FFT's loads)"}
    del q, ws
    torch.cuda.empty_cache()
    return out


def run_batched(rx, torch, args):
    """256 uneven frames: one persistent launch, replayed from a hipGraph."""
    from paper_2603_20481_amd.autotune import Tuner
    shapes = synth.draw_batch_shapes(args.batch_frames)
    frames = [rx.Frame.of(s, rx.MMSE, 1.0) for s in shapes]
    t0 = time.time()
    inputs = synth.draw_inputs(4, range(len(shapes)), shapes, args.workers)
    gen_s = time.time() - t0
    tuner = Tuner(args.tile_cache, fuse=True)
    tinfo = tuner.tune(frames)
    tuner.save()
    res = {}
    dets = sum(s.detections for s in shapes)
    # algorithmic bytes of each dataflow: the four stages (H and x_tilde
    # stored and read back); the FFT, the detector forming the estimate
    # itself, the demod; the FFT and the detector forming the estimate and
    # demapping (neither H nor x_tilde stored); the four stages with the demod
    # fused into the detector
    byts_staged = sum(stage_bytes(s)[k] for s in shapes for k in MODES["staged"])
    byts_fused = sum(stage_bytes(s)[k] for s in shapes for k in MODES["csi_detect"])
    byts_full = sum(stage_bytes(s)[k] for s in shapes for k in MODES["full"])
    byts_dm = sum(stage_bytes(s)[k] for s in shapes for k in ("fft", "csi")) + \
        sum(stage_bytes(s)["csi_detect_demod"] - stage_bytes(s)["csi_detect"] + stage_bytes(s)["detect"]
            for s in shapes)

    def flow(plan):
        if plan.fuse_csi and plan.fuse_demod:
            return "csi and demod fused into the detector (neither H nor x_tilde stored)", byts_full
        if plan.fuse_csi:
            return "csi fused into the detector (H never stored)", byts_fused
        if plan.fuse_demod:
            return "demod fused into the detector (x_tilde never stored)", byts_dm
        return "four stages (H and x_tilde stored and read back)", byts_staged
    bufs = rx.Plan(frames).alloc()
    lay = rx.Plan(frames)
    for f, (x, p) in enumerate(inputs):
        lay.view(bufs, "x", f).copy_(torch.from_numpy(x))
        lay.view(bufs, "pilots", f).copy_(torch.from_numpy(p))
    del lay
    pick = tuner.tune_plan(frames, bufs)
    variants = (("tuned", dict(tiles=pick["tiles"], grid=pick["grid"], fuse_csi=pick["fuse_csi"],
                               fuse_demod=pick["fuse_demod"])),
                ("fused_default_tiles", dict(fuse_csi=True, fuse_demod=True)),
                ("default", dict()))
    for label, kw in variants:
        plan = rx.Plan(frames, **kw)
        dataflow, byts = flow(plan)
        plan.graph(bufs)
        for _ in range(args.warmup):
            plan.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.form_steps):
            plan.replay()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / args.form_steps
        ms = e0.elapsed_time(e1) / args.form_steps
        status = plan.device_status()
        res[label] = {"value": dets / (ms * 1e-3), "ms_per_step": round(ms, 4),
                      "wall_ms_per_step": round(wall, 4), "items": plan.counts, "grid": plan.grid,
                      "dataflow": dataflow, "algorithmic_bytes": byts,
                      "hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "device_status": status}
        del plan
    # frames 0 and 1 of the last replay (the staged default plan, which writes
    # every tensor) for the oracle leg
    plan = rx.Plan(frames)
    keep = {}
    for f in (0, 1):
        keep[f] = {k: plan.view(bufs, k, f).cpu().numpy() for k in ("llr", "xt", "nu", "flags")}
    del plan
    SAMPLES["batched_256_uneven"] = {
        "kind": "forward", "inputs": [synth.make_frame(4, f, shape=shapes[f]) for f in (0, 1)],
        "det": [rx.MMSE, rx.MMSE],
        "outputs": [{"fp32": {"llr": keep[f]["llr"], "xt": keep[f]["xt"], "nu": keep[f]["nu"],
                              "flags": keep[f]["flags"]}} for f in (0, 1)]}
    # each stage alone over the same buffers (a plan with one stage in its mask)
    tiles = tuner.tiles_for(frames)
    stage_ms = {}
    for name, bit, fc, fd in (("fft", rx.STAGE_FFT, False, False), ("csi", rx.STAGE_CSI, False, False),
                              ("detect", rx.STAGE_DETECT, False, False),
                              ("csi_detect", rx.STAGE_DETECT, True, False),
                              ("csi_detect_demod", rx.STAGE_DETECT, True, True),
                              ("demod", rx.STAGE_DEMOD, False, False)):
        ps = rx.Plan(frames, tiles=tiles, stages=bit, fuse_csi=fc, fuse_demod=fd)
        ps.forward(bufs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.form_steps):
            ps.forward(bufs)
        e1.record()
        torch.cuda.synchronize()
        sms = e0.elapsed_time(e1) / args.form_steps
        sb = sum(stage_bytes(sh)[name] for sh in shapes)
        stage_ms[name] = {"us": round(sms * 1e3, 1), "GBps": round(sb / (sms * 1e-3) / 1e9, 1),
                          "bytes": sb}
        del ps
    # the same frames as a loop of per-frame single-frame calls (4 launches each)
    plan = rx.Plan(frames)
    views = []
    for f, fr in enumerate(frames):
        views.append({k: plan.view(bufs, k, f)[None] for k in plan.TENSORS})

    def loop():
        for fr, v in zip(frames, views):
            rx.fft(fr, v["x"], v["yf"])
            rx.csi(fr, v["yf"], v["pilots"], v["h"])
            rx.detect(fr, v["h"], v["yf"], "fp32", 1e3, v["xt"], v["nu"], v["flags"])
            rx.demod(fr, v["xt"], v["nu"], v["llr"])
    loop()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.form_steps):
        loop()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.form_steps
    res["per_frame_calls"] = {"value": dets / (ms * 1e-3), "ms_per_step": round(ms, 4),
                              "launches_per_step": 4 * len(frames)}
    out = dict(res["tuned"])
    out.update({"frames": len(frames), "detections_per_step": dets,
                "default": res["default"], "fused_default_tiles": res["fused_default_tiles"],
                "plan_knobs": {k: v for k, v in pick.items() if k != "tiles"}, "per_frame_calls": res["per_frame_calls"],
                "stages_alone": stage_ms,
                "autotune": tinfo, "gen_seconds": round(gen_s, 1),
                "workload": "256 uneven frames: M in {8,16,32,64}, K in 1..min(16,M), "
                            "300..3276 subcarriers, N_FFT next power of two >= 1.2 n_sc, "
                            "QPSK/16/64-QAM, Rayleigh, SNR U[5,30] dB, MMSE, FP32"})
    del bufs, views, plan
    torch.cuda.empty_cache()
    return out


def backward_bytes(s):
    """Compulsory HBM bytes of each kernel of rxphy_backward for one frame,
    given the forward's yf, h, x_tilde and nu (its interface tensors; the
    detector adjoint keeps X_hat, V = A^-1 G, A^-1 and the weights e of every
    subcarrier for the C kernel, and V and C for the apply kernel)."""
    M, K, N, n_sc, S, cp, Q = s.M, s.K, s.n_fft, s.n_sc, s.n_sym, s.cp_len, s.qam_bits
    D = S - 1
    xt, nu = K * D * n_sc * 8, K * n_sc * 4
    h, yd = M * K * n_sc * 8, M * D * n_sc * 8
    kd, kk = n_sc * K * D * 8, n_sc * K * K * 8
    return {
        "demod_adjoint": xt + nu + K * D * n_sc * Q * 4 + xt + nu,
        "detect_adjoint": h + yd + xt + nu + 2 * kd + kk + n_sc * K * 4,
        "detect_adjoint_c": 2 * kd + kk + n_sc * K * 4 + kk,
        "detect_adjoint_apply": h + yd + kd + kk + yd + h,
        "csi_adjoint": h + n_sc * 8 + M * n_sc * 8,
        "ifft": M * S * n_sc * 8 + M * S * (cp + N) * 8,
    }


def run_fwd_bwd(rx, torch, args):
    cfg = 5
    shape = synth.config_shape(cfg)
    F = args.bwd_frames
    x_h, p_h = gen_frames(cfg, F, args.workers)
    fr = rx.Frame.of(shape, rx.MMSE, 1.0)
    x = torch.from_numpy(x_h).cuda()
    p = torch.from_numpy(p_h).cuda()
    del x_h, p_h
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    dllr = torch.randn((F, shape.K, shape.n_data, shape.n_sc, shape.qam_bits), generator=g,
                       device="cuda")

    def step(ev=None):
        if ev: ev[0].record()
        out = rx.forward(fr, x, p)
        if ev: ev[1].record()
        dx = rx.backward(fr, x, p, dllr, saved=dict(yf=out["yf"], h=out["h"], xt=out["xt"], nu=out["nu"]))
        if ev: ev[2].record()
        return dx
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.form_steps)]
    for k in range(args.form_steps):
        dx = step(evs[k])
    torch.cuda.synchronize()
    fwd = sum(e[0].elapsed_time(e[1]) for e in evs) / args.form_steps
    bwd = sum(e[1].elapsed_time(e[2]) for e in evs) / args.form_steps
    ms = fwd + bwd
    sb, bb = stage_bytes(shape), backward_bytes(shape)
    fbytes = sum(sb[k] for k in MODES["staged"]) * F
    bbytes = sum(bb.values()) * F
    SAMPLES["fwd_bwd_64x8_cascaded"] = {"kind": "backward", "input": synth.make_frame(cfg, 0),
                                         "det": rx.MMSE, "dllr": dllr[0].cpu().numpy(),
                                         "dx": dx[0].cpu().numpy()}
    out = {"value": F * shape.detections / (ms * 1e-3), "unit": "subcarrier-detections/s",
           "ms_per_step": round(ms, 4), "frames": F,
           "forward": {"ms": round(fwd, 4), "algorithmic_bytes": fbytes,
                       "GBps": round(fbytes / (fwd * 1e-3) / 1e9, 1),
                       "hbm_frac": round(fbytes / (fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "calls": "fft, csi, detect, demod (H, x_tilde and nu kept for the adjoint)"},
           "backward": {"ms": round(bwd, 4), "algorithmic_bytes": bbytes,
                        "bytes_per_kernel_per_frame": bb,
                        "GBps": round(bbytes / (bwd * 1e-3) / 1e9, 1),
                        "hbm_frac": round(bbytes / (bwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "calls": "rxphy_backward with the forward's yf, h, x_tilde and nu"},
           "workload": "64x8 MIMO, N_FFT 2048, 1200 subcarriers, 16-QAM, cascaded channel "
                       "(256-element phase vector), 5 dB, MMSE; forward + adjoint to dL/dx, FP32"}
    del x, p, dllr
    torch.cuda.empty_cache()
    return out


ALU_PEAK_TOPS = 256 * 64 * 2.4e-3  # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: vector lane operations, 1e12/s


def run_detect_shapes(rx, torch, args):
    """The staged general detector alone across (M, K): per-subcarrier
    channels (random, so no tile shares a factor), 1200 subcarriers, 13 data
    symbols, 16-QAM, MMSE, about 1 GB of interface bytes per call.  Shows the
    per-tile floor that sets the uneven batch's detector rate (small M K
    tiles move few bytes through the same serial chain)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    rows = []
    for M, K in ((8, 1), (8, 2), (8, 4), (8, 8), (16, 4), (16, 12), (32, 2), (32, 8), (64, 4), (64, 8), (64, 16)):
        s = synth.Shape(M, K, 2048, 1200, 14, 0, 4)
        per = stage_bytes(s)["detect"]
        F = max(1, int(1.0e9 // per))
        fr = rx.Frame.of(s, rx.MMSE, 1.0)
        h = torch.randn((F, M, K, s.n_sc), dtype=torch.complex64, device="cuda", generator=g)
        yf = torch.randn((F, M, s.n_sym, s.n_sc), dtype=torch.complex64, device="cuda", generator=g)
        xt, nu, fl = rx.detect(fr, h, yf)
        for _ in range(2):
            rx.detect(fr, h, yf, xt=xt, nu=nu, flags=fl)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.form_steps):
            rx.detect(fr, h, yf, xt=xt, nu=nu, flags=fl)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / args.form_steps * 1e3
        tiles = F * ((s.n_sc + 15) // 16)
        rows.append({"M": M, "K": K, "frames": F, "us": round(us, 1), "GBps": round(F * per / us / 1e3, 1),
                     "hbm_frac": round(F * per / us / 1e3 / 8000, 3), "ns_per_tile": round(us * 1e3 / tiles, 2)})
        del h, yf, xt, nu, fl
    torch.cuda.empty_cache()
    return {"shapes": rows, "unit": "interface bytes / call time",
            "workload": "rxphy_detect, per-subcarrier random channels, 1200 subcarriers, 13 data symbols, "
                        "MMSE, FP32, about 1 GB per call"}


def run_ldpc(rx, torch, args):
    """Layered min-sum decoding of n_cw codewords of a 46 x 68 quasi-cyclic
    code at lifting size 384 (the shape of the largest 3GPP base graph, random
    shifts), BPSK over AWGN."""
    from synth import ldpc as SL
    z, mb, kb = 384, 46, 22
    base = SL.random_base(mb, kb, z, 7, seed=61)
    n_cw = args.ldpc_codewords
    t0 = time.time()
    cw = SL.make_codewords(base, z, n_cw, seed=62)
    llr_h = SL.bpsk_awgn_llrs(cw, args.ldpc_snr, seed=63)
    gen_s = time.time() - t0
    code = rx.LdpcCode(base, z)
    llr = torch.from_numpy(llr_h).cuda()
    N = code.n
    post = torch.empty((n_cw, N), dtype=torch.float32, device="cuda")
    bits = torch.empty((n_cw, N), dtype=torch.uint8, device="cuda")
    its = torch.empty((n_cw,), dtype=torch.int32, device="cuda")
    ws = torch.empty((code.workspace_bytes(n_cw),), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        rx.ldpc_decode(code, llr, args.ldpc_iters, 0.75, post, bits, its, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.form_steps):
        rx.ldpc_decode(code, llr, args.ldpc_iters, 0.75, post, bits, its, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.form_steps
    it_h = its.cpu().numpy()
    bits_h = bits.cpu().numpy()
    n_edges = int(np.sum(base >= 0))
    # Algorithmic vector operations: per edge and layer update 7 (Q = L - R,
    # the magnitude against the minimum, the second-minimum select, the sign
    # parity, the new message's magnitude select and sign, L = Q + R); per
    # edge and syndrome test 2 (the hard decision, the parity); the syndrome
    # is tested before the first iteration and after each one
    sum_it = float(np.sum(it_h))
    mean_it = float(np.mean(it_h))
    alu_ops = n_edges * z * (7.0 * sum_it + 2.0 * (sum_it + n_cw))
    hbm = n_cw * N * 9                                                      # LLRs in, posteriors and bits out
    msg = n_cw * mb * z * 12 * 2 * float(np.mean(np.maximum(it_h - 1, 0)))   # compressed messages read + written
    keep = [0, n_cw - 1]
    SAMPLES["ldpc_46x68_z384"] = {"kind": "ldpc", "base": base, "z": z, "max_iter": args.ldpc_iters,
                                  "alpha": 0.75, "llr": llr_h[keep], "post": post[keep].cpu().numpy(),
                                  "bits": bits_h[keep], "iters": it_h[keep], "index": keep}
    out = {"value": n_cw * kb * z / (ms * 1e-3) / 1e9, "unit": "Gbit/s (information bits decoded)",
           "ms_per_step": round(ms, 4), "codewords": n_cw, "codewords_per_s": n_cw / (ms * 1e-3),
           "mean_iterations": round(mean_it, 3), "max_iterations": int(it_h.max()),
           "codewords_in_error": int(np.sum(np.any(bits_h != cw, axis=1))),
           "raw_bit_errors": int(np.sum((llr_h < 0) != cw)),
           "roofline": {"bound": "alu", "achieved": round(alu_ops / (ms * 1e-3) / 1e12, 3),
                        "peak": ALU_PEAK_TOPS, "unit": "Tops/s (vector lane operations)",
                        "frac": round(alu_ops / (ms * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4),
                        "ops_per_step": alu_ops},
           "hbm": {"algorithmic_bytes": hbm, "GBps": round(hbm / (ms * 1e-3) / 1e9, 1),
                   "message_bytes": msg, "message_GBps": round(msg / (ms * 1e-3) / 1e9, 1)},
           "gen_seconds": round(gen_s, 1),
           "workload": "%d codewords of a 46 x 68 quasi-cyclic LDPC code, lifting size 384 (N = 26112, "
                       "K = 8448, random shifts, staircase parity), BPSK over AWGN at %.1f dB, layered "
                       "normalised min-sum (alpha 0.75), at most %d iterations, early stop on a zero "
                       "syndrome, FP32" % (n_cw, args.ldpc_snr, args.ldpc_iters)}
    del llr, post, bits, its, ws, code
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-s", type=float, default=0.5,
                    help="untimed steps for this many seconds before the warm-up steps (clock ramp)")
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--form-steps", type=int, default=10)
    ap.add_argument("--mixed-frames", type=int, default=100)
    ap.add_argument("--batch-frames", type=int, default=256)
    ap.add_argument("--bwd-frames", type=int, default=100)
    ap.add_argument("--ldpc-codewords", type=int, default=1024)
    ap.add_argument("--ldpc-snr", type=float, default=2.5)
    ap.add_argument("--ldpc-iters", type=int, default=10)
    ap.add_argument("--forms", default="staged,mmse,sc16,streaming,downlink,mixed,batched,detect_shapes,fwd_bwd,ldpc,"
                    "sensing",
                    help="comma list of extra forms to time ('' for the headline only)")
    ap.add_argument("--sense-plots", type=int, default=64)
    ap.add_argument("--sense-latency-calls", type=int, default=200)
    ap.add_argument("--stream-tasks", type=int, default=400)
    ap.add_argument("--stream-warmup", type=int, default=20)
    ap.add_argument("--tile-cache", default=None)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=min(16, len(os.sched_getaffinity(0))),
                    help="processes of the all-cores oracle timing (one thread each)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the plain device copy timed as the bandwidth reference (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: frames are independent, so more GPUs would each "
              "run this same single-GPU path on their own share of frames",
              file=sys.stderr)
        sys.exit(2)
    forms = [f for f in args.forms.split(",") if f]

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
    chain = Chain(rx, torch, shape, x_h, p_h)
    del x_h, p_h
    fr = rx.Frame.of(shape, det, 1.0)
    settle_steps = chain.settle(fr, "fp32", args.settle_s, mode="full") if args.settle_s > 0 else 0
    ms_per_step, per_stage = chain.time(fr, "fp32", args.steps, args.warmup, mode="full")
    dets = F * shape.detections
    value = dets / (ms_per_step * 1e-3)

    sb = stage_bytes(shape)
    dom = max(per_stage, key=lambda n: per_stage[n])
    achieved = sb[dom] * F / (per_stage[dom] * 1e-3) / 1e9

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
                               "Rayleigh, SNR U[10,30] dB, 100 frames, ZF, FP32; fft, then csi + "
                               "detect + demod fused (neither H nor x_tilde stored)",
                   "frames": F, "M": shape.M, "K": shape.K, "n_fft": shape.n_fft,
                   "n_sc": shape.n_sc, "n_sym": shape.n_sym, "qam_bits": shape.qam_bits,
                   "detector": "zf", "precision": "fp32"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom), "traffic_unit": "bytes/launch",
                     "algorithmic_bytes": sb[dom] * F},
        "stages": stage_report(shape, F, per_stage),
        "staged_roofline_frac": round(sum(sb[n] for n in per_stage) * F / (sum(per_stage.values()) * 1e-3)
                                      / 1e9 / HBM_PEAK_GBS, 4),
        "gen_seconds": round(gen_s, 1),
        "settle_steps": settle_steps,
        "forms": {},
    }
    print("[bench] headline %.4g det/s (%.3f ms/step)" % (value, ms_per_step), file=sys.stderr, flush=True)
    # outputs of the first and last frame for the oracle leg (one more untimed
    # call that also writes x_tilde)
    rx.csi_detect_demod(fr, chain.yf, chain.p, "fp32", 1e3, llr=chain.llr, nu=chain.nu, flags=chain.fl,
                        xt=chain.xt, ws=chain.ws)
    torch.cuda.synchronize()
    keep = [0, 1]
    SAMPLES["headline"] = {"frames": keep, "llr": [chain.llr[k].cpu().numpy() for k in keep],
                           "xt": [chain.xt[k].cpu().numpy() for k in keep],
                           "nu": [chain.nu[k].cpu().numpy() for k in keep],
                           "flags": [chain.fl[k].cpu().numpy() for k in keep]}
    if "staged" in forms:
        ms, per = chain.time(fr, "fp32", args.form_steps, 1, mode="staged")
        out["forms"]["staged_fp32"] = form_summary(
            shape, F, ms, per, {"workload": "as the headline, the four stage calls (H stored by csi, "
                                            "read back by detect; x_tilde stored by detect, read back "
                                            "by demod)"})
        ms, per = chain.time(fr, "fp32", args.form_steps, 1, mode="csi_detect")
        out["forms"]["csi_detect_fp32"] = form_summary(
            shape, F, ms, per, {"workload": "as the headline, csi + detect fused, demod its own call "
                                            "(x_tilde stored and read back)"})
        print("[bench] staged done", file=sys.stderr, flush=True)
    if "mmse" in forms:
        frm = rx.Frame.of(shape, rx.MMSE, 1.0)
        ms, per = chain.time(frm, "fp32", args.form_steps, 1, mode="full")
        out["forms"]["mmse_fp32"] = form_summary(shape, F, ms, per, {"workload": "as the headline, MMSE"})
        print("[bench] mmse done", file=sys.stderr, flush=True)
    if "sc16" in forms:
        out["forms"]["sc16_ingest_fp32"] = run_sc16(rx, torch, chain, args)
        print("[bench] sc16 done", file=sys.stderr, flush=True)
    if "streaming" in forms:
        out["forms"]["streaming_fp32"] = run_streaming(rx, torch, chain, args)
        print("[bench] streaming done", file=sys.stderr, flush=True)
    if "downlink" in forms:
        out["forms"]["downlink_zf_fp32"] = run_downlink(rx, torch, chain, args)
        print("[bench] downlink done", file=sys.stderr, flush=True)
    del chain
    torch.cuda.empty_cache()
    if "mixed" in forms:
        s3 = synth.config_shape(3)
        x3, p3 = gen_frames(3, args.mixed_frames, args.workers)
        c3 = Chain(rx, torch, s3, x3, p3)
        del x3, p3
        fr3 = rx.Frame.of(s3, rx.ZF, 1.0)
        kept = {}
        for prec in ("fp32", "bf16", "fp16"):
            ms, per = c3.time(fr3, prec, args.form_steps, 1, mode="full")
            refined = int((c3.fl & rx.FLAG_REFINED).ne(0).sum().item())
            rx.csi_detect_demod(fr3, c3.yf, c3.p, prec, 1e3, llr=c3.llr, nu=c3.nu, flags=c3.fl, xt=c3.xt,
                                ws=c3.ws)
            torch.cuda.synchronize()
            kept[prec] = {"llr": c3.llr[0].cpu().numpy(), "xt": c3.xt[0].cpu().numpy(),
                          "nu": c3.nu[0].cpu().numpy(), "flags": c3.fl[0].cpu().numpy(),
                          "band_u": {"fp32": None, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}[prec]}
            out["forms"]["kronecker_64x16_n4096_64qam_" + prec] = form_summary(
                s3, args.mixed_frames, ms, per,
                {"refined_subcarriers": refined, "refined_fraction": refined / c3.fl.numel(),
                 "workload": "64x16 MIMO, N_FFT 4096, 3276 subcarriers, 64-QAM, Kronecker "
                             "(0.7, 0.3), 25 dB, ZF, %s products, FP64 refinement above "
                             "condition estimate 1e3" % prec})
        # the FP64 refinement's cost: lower thresholds refine a growing share
        # of the pilot groups (0 refines every subcarrier)
        sweep = []
        for thr in (300.0, 100.0, 0.0):
            c3.thr = thr
            ms, per = c3.time(fr3, "bf16", args.form_steps, 1, mode="full")
            refined = int((c3.fl & rx.FLAG_REFINED).ne(0).sum().item())
            sweep.append({"cond_threshold": thr, "ms_per_step": round(ms, 4),
                          "csi_detect_demod_us": round(per["csi_detect_demod"] * 1e3, 2),
                          "refined_fraction": round(refined / c3.fl.numel(), 6),
                          "value": s3.detections * args.mixed_frames / (ms * 1e-3)})
        c3.thr = 1e3
        out["forms"]["kronecker_64x16_n4096_64qam_bf16"]["refinement_sweep"] = sweep
        SAMPLES["kronecker_64x16_n4096_64qam"] = {"kind": "forward", "inputs": [synth.make_frame(3, 0)],
                                                  "det": [rx.ZF], "outputs": [kept]}
        del c3
        torch.cuda.empty_cache()
        print("[bench] mixed done", file=sys.stderr, flush=True)
    if "batched" in forms:
        out["forms"]["batched_fp32"] = run_batched(rx, torch, args)
        print("[bench] batched done", file=sys.stderr, flush=True)
    if "fwd_bwd" in forms:
        out["forms"]["fwd_bwd_fp32"] = run_fwd_bwd(rx, torch, args)
        print("[bench] fwd+bwd done", file=sys.stderr, flush=True)
    if "detect_shapes" in forms:
        out["forms"]["detect_shapes_fp32"] = run_detect_shapes(rx, torch, args)
        print("[bench] detect shapes done", file=sys.stderr, flush=True)
    if "ldpc" in forms:
        out["forms"]["ldpc_decode_fp32"] = run_ldpc(rx, torch, args)
        print("[bench] ldpc done", file=sys.stderr, flush=True)
    if "sensing" in forms:
        out["forms"]["sensing_fp32"] = run_sensing(rx, torch, args)
        print("[bench] sensing done", file=sys.stderr, flush=True)
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
        out["cpu_baseline"] = cpu_baseline(cfg, det, args.cpu_budget, args.cpu_workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
