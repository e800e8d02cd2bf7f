"""Work-item size autotuner for batched plans (rxphy_plan_*).

Each stage's best item size depends only on the part of the frame shape that
stage sees, so the search is split by stage and by shape class:

  fft     key (n_fft, M)                       knob fft_iters
  csi     key (M, K padded to 4/8/16)          knob csi_tiles
  detect  key (M, K padded, ZF or MMSE)        knob det_tiles
  demod   key (qam_bits, K padded)             knob dem_groups

A class is timed on a plan of identical frames of that class that runs only
the stage being tuned (the other stages' outputs are filled once beforehand),
every candidate with HIP events on the current stream, and the fastest median
wins.  The detector class is tuned in the dataflow the tuner is built for
(fuse=True: the detector items form the channel estimate themselves and
demap their tiles, and the CSI and demod stages have no items).

tune_plan then chooses the plan-wide knobs on the actual frames and buffers:
the dataflow (CSI, demod, both or neither fused into the detector items) and
the grid of the persistent launch (one, two or three workgroups per CU)
and the item sizes (the tuned ones or the defaults), timing each
combination.

Every candidate gives bit-identical results for every output but H and
x_tilde (not written by the fused dataflows; the K padding is never
changed), so tuning affects speed only.  Results live in a JSON cache keyed
by device name.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import (STAGE_CSI, STAGE_DEMOD, STAGE_DETECT, STAGE_FFT, Frame, Plan, Tiles)

STAGES = ("fft", "csi", "detect", "demod")
STAGE_BIT = {"fft": STAGE_FFT, "csi": STAGE_CSI, "detect": STAGE_DETECT, "demod": STAGE_DEMOD}
KNOB = {"fft": "fft_iters", "csi": "csi_tiles", "detect": "det_tiles", "demod": "dem_groups"}
CANDIDATES = {"fft": (1, 2, 4, 8, 16), "csi": (1, 2, 4, 8), "detect": (1, 2, 4),
              "demod": (1, 2, 4, 8, 16)}
CACHE_VERSION = 4


def kp_of(K: int) -> int:
    return 4 if K <= 4 else 8 if K <= 8 else 16


def class_key(stage: str, fr: Frame, fused: bool = False) -> str:
    if stage == "fft":
        return "fft:N=%d,M=%d" % (fr.n_fft, fr.M)
    if stage == "csi":
        return "csi:M=%d,KP=%d" % (fr.M, kp_of(fr.K))
    if stage == "detect":
        return "detect:M=%d,KP=%d,%s%s" % (fr.M, kp_of(fr.K), "mmse" if fr.detector else "zf",
                                           ",fused" if fused else "")
    return "demod:Q=%d,KP=%d" % (fr.qam_bits, kp_of(fr.K))


def default_cache_path() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "rxphy", "tiles.json")


class Tuner:
    def __init__(self, cache_path: str | None = None, fuse: bool = True):
        self.path = cache_path or default_cache_path()
        self.fuse = bool(fuse)
        self.device = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
        self.entries: dict = {}
        try:
            with open(self.path) as fh:
                d = json.load(fh)
            if d.get("version") == CACHE_VERSION and d.get("device") == self.device:
                self.entries = dict(d.get("entries", {}))
        except (OSError, ValueError):
            pass

    def save(self):
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump({"version": CACHE_VERSION, "device": self.device, "entries": self.entries},
                      fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def tiles_for(self, frames) -> list:
        """Tiles per frame from the cache (0 = library default where untuned)."""
        out = []
        for fr in frames:
            kw = {}
            for st in STAGES:
                e = self.entries.get(class_key(st, fr, self.fuse))
                if e is not None:
                    kw[KNOB[st]] = int(e["value"])
            out.append(Tiles(**kw))
        return out

    # ------------------------------------------------------------ measuring
    @staticmethod
    def _time(plan: Plan, bufs, reps: int) -> float:
        plan.forward(bufs)                                # warm-up
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            plan.forward(bufs)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e3)
        ts.sort()
        return ts[len(ts) // 2]

    def tune_class(self, stage: str, fr: Frame, copies: int = 16, reps: int = 5) -> dict:
        frames = [fr] * copies
        full = Plan(frames)                               # staged: fills every intermediate
        bufs = full.alloc()
        g = torch.Generator(device="cuda")
        g.manual_seed(1234)
        for k in ("x", "pilots"):
            n = full.totals[k] // 4
            bufs[k][: n * 4].view(torch.float32).copy_(
                torch.randn(n, generator=g, device="cuda", dtype=torch.float32))
        full.forward(bufs)                                # realistic intermediates
        torch.cuda.synchronize()
        res = {}
        fuse = self.fuse and stage == "detect"
        for v in CANDIDATES[stage]:
            p = Plan(frames, tiles=Tiles(**{KNOB[stage]: v}), stages=STAGE_BIT[stage], fuse_csi=fuse,
                     fuse_demod=fuse)
            res[v] = self._time(p, bufs, reps)
            del p
        best = min(res, key=lambda v: (res[v], v))
        entry = {"value": best, "us": round(res[best], 2),
                 "candidates_us": {str(k): round(t, 2) for k, t in res.items()}}
        self.entries[class_key(stage, fr, fuse)] = entry
        return entry

    def tune(self, frames, force: bool = False, copies: int = 16, reps: int = 5) -> dict:
        """Tunes every (stage, class) present in `frames` that the cache lacks."""
        t0 = time.time()
        done = 0
        for st in STAGES:
            if st in ("csi", "demod") and self.fuse:
                continue                                   # no CSI or demod items in the fused dataflow
            seen = {}
            for fr in frames:
                seen.setdefault(class_key(st, fr, self.fuse), fr)
            for key, fr in seen.items():
                if force or key not in self.entries:
                    self.tune_class(st, fr, copies, reps)
                    done += 1
        return {"classes_tuned": done, "seconds": round(time.time() - t0, 2)}

    def tune_plan(self, frames, bufs, reps: int = 5) -> dict:
        """Plan-wide knobs on the given frames and packed buffers (x and the
        pilots filled; allocated by a staged plan, so that H and x_tilde have
        room): the dataflow (CSI and / or demod fused into the detector items),
        the grid (1, 2 or 3 workgroups per CU) and the item sizes (the cached
        per-class ones or the defaults: a class tuned alone on a plan of its
        own can lose inside the mixed plan).  Returns the winner (tiles None
        for the defaults) and every candidate's median time (us)."""
        tiles = self.tiles_for(frames)
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        res = {}
        for ts, tl in (("tuned", tiles), ("default", None)):
            for fc, fd in ((True, True), (True, False), (False, True), (False, False)):
                for per_cu in (1, 2, 3):
                    p = Plan(frames, tiles=tl, grid=per_cu * cus, fuse_csi=fc, fuse_demod=fd)
                    res[(fc, fd, per_cu, ts)] = self._time(p, bufs, reps)
                    del p
        best = min(res, key=lambda k: res[k])
        name = {(True, True): "csi+demod fused", (True, False): "csi fused", (False, True): "demod fused",
                (False, False): "staged"}
        return {"fuse_csi": best[0], "fuse_demod": best[1], "grid": best[2] * cus, "item_sizes": best[3],
                "tiles": tiles if best[3] == "tuned" else None,
                "candidates_us": {"%s,%d/CU,%s" % (name[k[:2]], k[2], k[3]): round(v, 1) for k, v in res.items()}}
