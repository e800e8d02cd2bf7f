"""Host-side logic of the work-item autotuner: class keys and the JSON cache."""
import json

import paper_2603_20481_amd as rx
from paper_2603_20481_amd import autotune as at


def test_class_keys_split_by_what_each_stage_sees():
    a = rx.Frame(64, 16, 2048, 1200, 14, 0, 4, rx.ZF)
    b = rx.Frame(64, 13, 2048, 700, 14, 0, 6, rx.ZF)      # same N, M; K pads to 16 too
    c = rx.Frame(64, 16, 2048, 1200, 14, 0, 4, rx.MMSE)
    assert at.class_key("fft", a) == at.class_key("fft", b)
    assert at.class_key("csi", a) == at.class_key("csi", b)
    assert at.class_key("detect", a) == at.class_key("detect", b)
    assert at.class_key("detect", a) != at.class_key("detect", c)
    assert at.class_key("detect", a) != at.class_key("detect", a, fused=True)
    assert at.class_key("fft", a) == at.class_key("fft", a, fused=True)
    assert at.class_key("demod", a) != at.class_key("demod", b)
    assert [at.kp_of(k) for k in (1, 4, 5, 8, 9, 16)] == [4, 4, 8, 8, 16, 16]


def test_cache_round_trip_and_tiles(tmp_path):
    path = str(tmp_path / "t.json")
    t = at.Tuner(path, fuse=False)
    fr = rx.Frame(32, 5, 1024, 800, 14, 0, 2, rx.MMSE)
    t.entries[at.class_key("fft", fr)] = {"value": 8}
    t.entries[at.class_key("demod", fr)] = {"value": 32}
    t.save()
    t2 = at.Tuner(path, fuse=False)
    assert t2.entries == t.entries
    tiles = t2.tiles_for([fr, rx.Frame(8, 2, 512, 300)])
    assert tiles[0] == rx.Tiles(fft_iters=8, dem_groups=32)
    assert tiles[1] == rx.Tiles()
    # a cache written for another device is ignored
    d = json.load(open(path))
    d["device"] = "some other device"
    json.dump(d, open(path, "w"))
    assert at.Tuner(path).entries == {}
