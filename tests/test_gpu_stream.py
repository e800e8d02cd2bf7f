"""GPU checks of the real-time streaming runtime (rxphy_stream_*): every
streamed task returns exactly what the direct calls (rxphy_fft, then
rxphy_csi_detect_demod) return on the same frames, through pinned host
buffers or device tensors, with ping-pong and deeper slot rings and
back-pressure; every task gets a finite positive latency."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-stream]", *a, flush=True)


def frames(cfg, first, n):
    fs = [synth.make_frame(cfg, first + i) for i in range(n)]
    return np.stack([f.x for f in fs]), np.stack([f.pilots for f in fs]), fs[0].shape


def direct(rx, fr, x, p):
    """The task's reference: the two direct calls on torch's stream."""
    xd = torch.from_numpy(x).cuda()
    pd = torch.from_numpy(p).cuda()
    yf = rx.fft(fr, xd)
    llr, nu, fl, _ = rx.csi_detect_demod(fr, yf, pd)
    torch.cuda.synchronize()
    return llr.cpu().numpy(), nu.cpu().numpy(), fl.cpu().numpy()


@pytest.mark.parametrize("cfg,nf,depth", [(1, 3, 2), (2, 2, 2), (2, 1, 3), (1, 2, 1)])
def test_host_io_tasks_equal_direct_calls(rx, cfg, nf, depth):
    _, _, shape = frames(cfg, 0, 1)
    fr = rx.Frame.of(shape, rx.ZF, 1.0)
    st = rx.Stream(fr, nf, depth=depth, host_io=True)
    try:
        task = 0
        for rnd in range(2):
            refs = {}
            for _ in range(depth):
                x, p, _ = frames(cfg, 10 * task, nf)
                slot = st.acquire()
                assert slot == task % depth
                h = st.host(slot)
                h["x"][...] = x
                h["pilots"][...] = p
                h["llr"][...] = np.nan                     # must be overwritten by the task
                st.submit(slot)
                refs[slot] = direct(rx, fr, x, p)
                task += 1
            st.drain()
            for slot, (llr, nu, fl) in refs.items():
                h = st.host(slot)
                assert np.array_equal(h["llr"], llr), (slot, "llr")
                assert np.array_equal(h["nu"], nu), (slot, "nu")
                assert np.array_equal(h["flags"], fl), (slot, "flags")
        lat = st.latencies()
        say("host io cfg", cfg, "frames", nf, "depth", depth, "latencies us", np.round(lat, 1))
        assert lat.size == task and np.all(np.isfinite(lat)) and np.all(lat > 0)
    finally:
        st.close()


def test_device_resident_ring_and_back_pressure(rx):
    """Depth 3, ten tasks submitted back to back (acquire blocks on busy
    slots), each into its own output tensors."""
    cfg, nf, depth, n_tasks = 2, 2, 3, 10
    _, _, shape = frames(cfg, 0, 1)
    fr = rx.Frame.of(shape, rx.MMSE, 1.0)
    st = rx.Stream(fr, nf, depth=depth, host_io=False)
    try:
        ins, outs, refs = [], [], []
        for t in range(n_tasks):
            x, p, _ = frames(cfg, 3 * t + 1, nf)
            ins.append((torch.from_numpy(x).cuda(), torch.from_numpy(p).cuda()))
            outs.append((torch.full((nf, fr.K, fr.n_data, fr.n_sc, fr.qam_bits), float("nan"), device="cuda"),
                         torch.empty((nf, fr.K, fr.n_sc), device="cuda"),
                         torch.empty((nf, fr.n_sc), dtype=torch.uint8, device="cuda")))
            refs.append(direct(rx, fr, x, p))
        torch.cuda.synchronize()
        t0 = rx.clock_ns()
        for t in range(n_tasks):
            slot = st.acquire()
            assert slot == t % depth
            st.submit(slot, t0, ins[t][0], ins[t][1], *outs[t])
        st.drain()
        for t in range(n_tasks):
            llr, nu, fl = (o.cpu().numpy() for o in outs[t])
            assert np.array_equal(llr, refs[t][0]), t
            assert np.array_equal(nu, refs[t][1]), t
            assert np.array_equal(fl, refs[t][2]), t
        lat = st.latencies()
        say("device ring latencies us (common arrival)", np.round(lat, 1))
        assert lat.size == n_tasks and np.all(np.isfinite(lat)) and np.all(lat > 0)
        # a common arrival time: later tasks cannot have finished earlier
        assert lat[-1] >= lat[0]
        s = rx.latency_summary(lat, 1e9)
        assert s["count"] == n_tasks and s["meets_99"] == 1
        st.reset_latencies()
        assert st.latencies().size == 0
    finally:
        st.close()


def test_misuse_is_rejected(rx):
    _, _, shape = frames(1, 0, 1)
    fr = rx.Frame.of(shape, rx.ZF, 1.0)
    st = rx.Stream(fr, 1, depth=1, host_io=True)
    try:
        with pytest.raises(rx.RxphyError, match="not acquired"):
            st.submit(0)
        slot = st.acquire()
        with pytest.raises(rx.RxphyError, match="not yet submitted"):
            st.acquire()
        d = torch.zeros(1, dtype=torch.complex64, device="cuda")
        lib = rx.load()
        assert lib.rxphy_stream_submit(st._h, slot, 0, rx._ptr(d), None, None, None, None) == 1
        assert lib.rxphy_stream_submit(st._h, 5, 0, None, None, None, None, None) == 1
        assert lib.rxphy_stream_submit(st._h, slot, -1, None, None, None, None, None) == 1
        with pytest.raises(rx.RxphyError):
            st.host(1)
        st.host(slot)["x"][...] = 0
        st.host(slot)["pilots"][...] = 1
        st.submit(slot)                                  # still acquired after the rejected submits
        st.drain()
        assert (st.host(slot)["flags"] == rx.FLAG_BREAKDOWN).all()   # zero samples: H = 0, ZF breaks down
    finally:
        st.close()
    dev = rx.Stream(fr, 1, depth=2, host_io=False)
    try:
        with pytest.raises(rx.RxphyError):
            dev.host(0)
        slot = dev.acquire()
        assert rx.load().rxphy_stream_submit(dev._h, slot, 0, None, None, None, None, None) == 1
    finally:
        dev.close()


def test_close_with_tasks_outstanding_drains(rx):
    _, _, shape = frames(2, 0, 1)
    fr = rx.Frame.of(shape, rx.ZF, 1.0)
    st = rx.Stream(fr, 4, depth=2, host_io=True)
    for _ in range(5):
        slot = st.acquire()
        st.host(slot)["pilots"][...] = 1
        st.submit(slot)
    st.close()                                           # waits for the outstanding tasks
    torch.cuda.synchronize()
