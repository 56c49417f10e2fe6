"""Serving loop (continuous batching) on the GPU: results are the same alone and
in the mix, admission respects the HBM budget, and oversized frames are
refused."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1702_04458_amd import inputs  # noqa: E402

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1702_04458_amd import _native, api  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


SHAPES = [(64, 8, 4, 72), (128, 16, 8, 300), (256, 32, 8, 72), (128, 32, 4, 300), (256, 16, 16, 72),
          (512, 64, 8, 72), (64, 16, 4, 300), (256, 32, 4, 300), (512, 32, 16, 72), (128, 8, 16, 300)]


def make_frames(pinned=True):
    frames = []
    for i, (B, U, C, n_sc) in enumerate(SHAPES):
        fr = inputs.uplink_frame(inputs.frame_seed(5, i, 10), n_sc, B, U, 16, 10.0)
        H = torch.from_numpy(fr.H)
        y = torch.from_numpy(fr.y)
        if pinned:
            H, y = H.pin_memory(), y.pin_memory()
        else:
            H, y = H.cuda(), y.cuda()
        frames.append(dict(H=H, y=y, C=C, N0=fr.N0, U=U, n_sc=n_sc))
    return frames


def out_bufs(f, pinned):
    if pinned:
        s = torch.empty((f["n_sc"], 1, f["U"]), dtype=torch.complex64, pin_memory=True)
        h = torch.empty((f["n_sc"], 1, f["U"]), dtype=torch.uint8, pin_memory=True)
    else:
        s = torch.empty((f["n_sc"], 1, f["U"]), dtype=torch.complex64, device="cuda")
        h = torch.empty((f["n_sc"], 1, f["U"]), dtype=torch.uint8, device="cuda")
    return s, h


@pytest.mark.parametrize("pinned", [True, False])
def test_alone_equals_mix(pinned):
    say(f"[gpu] serving alone vs mix pinned={pinned}")
    frames = make_frames(pinned)
    # reference: direct library calls, one at a time
    refs = []
    for f in frames:
        s, h = api.detect(f["H"].cuda(), f["y"].cuda(), f["N0"], f["C"], 1.0, 5, qam=16)
        refs.append((s.cpu(), h.cpu()))
    torch.cuda.synchronize()
    srv = api.Server(hbm_budget_bytes=1 << 30, n_slots=4)
    # alone: one frame in flight at a time
    alone = []
    for f in frames:
        s, h = out_bufs(f, pinned)
        t = srv.submit(f["H"], f["y"], s, h, f["C"], 5, 1.0, f["N0"], qam=16)
        lat, _ = srv.wait(t)
        assert lat > 0
        alone.append((s.cpu().clone(), h.cpu().clone()))
    # mix: everything submitted at once, overlapping on the device
    outs = [out_bufs(f, pinned) for f in frames]
    tickets = [srv.submit(f["H"], f["y"], o[0], o[1], f["C"], 5, 1.0, f["N0"], qam=16) for f, o in zip(frames, outs)]
    lats = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["peak_inflight"] >= 2
    for (sa, ha), (s, h), (sr, hr) in zip(alone, outs, refs):
        assert torch.equal(sa, sr) and torch.equal(ha, hr)
        assert torch.equal(s.cpu(), sa) and torch.equal(h.cpu(), ha)
    assert all(x > 0 for x in lats)


def test_budget_admission_serialises():
    say("[gpu] serving tiny budget")
    frames = make_frames(True)
    sizes = []
    for f in frames:
        n_sc, B, U = f["H"].shape
        al = lambda n: (n + 255) // 256 * 256  # noqa: E731
        ws = _native.lib().dbp_detect_workspace_bytes(n_sc, U, f["C"])     # FP64 re-slice workspace
        sizes.append(al(ws) + al(n_sc * B * U * 8) + al(n_sc * B * 8) + al(n_sc * U * 8) + al(n_sc * U))
    budget = max(sizes)
    srv = api.Server(hbm_budget_bytes=budget, n_slots=4)
    outs = [out_bufs(f, True) for f in frames]
    tickets = [srv.submit(f["H"], f["y"], o[0], o[1], f["C"], 5, 1.0, f["N0"], qam=16) for f, o in zip(frames, outs)]
    q = [srv.wait(t)[1] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(frames)
    assert st["peak_bytes"] <= budget
    assert max(q) > 0


def test_oversized_frame_refused():
    f = make_frames(True)[5]
    srv = api.Server(hbm_budget_bytes=1 << 20, n_slots=2)
    s, h = out_bufs(f, True)
    with pytest.raises(_native.DbpError) as e:
        srv.submit(f["H"], f["y"], s, h, f["C"], 5, 1.0, f["N0"], qam=16)
    assert e.value.code == 3
    srv.close()


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("h16", [False, True])
def test_resident_channel_frames(pinned, h16):
    """A static channel loaded once (complex64, or the packed FP16 form); four
    received frames against it, mixed with ordinary frames, each bit-identical
    to the library's factored call."""
    say(f"[gpu] serving resident channel pinned={pinned} h16={h16}")
    B, U, C, n_sc = 256, 32, 8, 120
    fr = inputs.uplink_frame(inputs.frame_seed(5, 99, 25), n_sc, B, U, 64, 25.0, n_sym=4)
    Hd = torch.from_numpy(fr.H).cuda()
    fac = api.factor(Hd, C, 1.0)
    packed = api.pack_channel_h16(Hd, C)
    srv = api.Server(hbm_budget_bytes=1 << 30, n_slots=4)
    H = torch.from_numpy(fr.H).pin_memory() if pinned else Hd
    ch = srv.load_channel(H, C, 1.0, h16=h16)
    others = make_frames(pinned)[:3]
    tickets, outs, refs = [], [], []
    for n in range(4):
        yn = torch.from_numpy(np.ascontiguousarray(fr.y[:, n:n + 1]))
        yd = yn.cuda()
        if h16:
            r = api.detect_factored_h16(packed, fac, yd, fr.N0, B, U, C, 1.0, 5, qam=64)
        else:
            r = api.detect_factored(Hd, fac, yd, fr.N0, C, 1.0, 5, qam=64)
        refs.append((r[0].cpu(), r[1].cpu()))
        y = yn.pin_memory() if pinned else yd
        s, h = out_bufs(dict(n_sc=n_sc, U=U), pinned)
        tickets.append(srv.submit_factored(ch, y, s, h, 5, fr.N0, qam=64))
        outs.append((s, h, y))
        f = others[n % 3]
        so, ho = out_bufs(f, pinned)
        tickets.append(srv.submit(f["H"], f["y"], so, ho, f["C"], 5, 1.0, f["N0"], qam=16))
        outs.append((so, ho, None))
    for t in tickets:
        lat, _ = srv.wait(t)
        assert lat > 0
    for n in range(4):
        s, h, _ = outs[2 * n]
        assert torch.equal(s.cpu(), refs[n][0]) and torch.equal(h.cpu(), refs[n][1])
    with pytest.raises(_native.DbpError) as e:
        srv.free_channel(ch + 1000)
    assert e.value.code == 6
    srv.free_channel(ch)
    with pytest.raises(_native.DbpError) as e:
        srv.free_channel(ch)
    assert e.value.code == 6
    st = srv.stats()
    srv.close()
    assert st["completed"] == 8


def test_channel_too_large_refused():
    f = make_frames(True)[5]
    srv = api.Server(hbm_budget_bytes=1 << 20, n_slots=2)
    with pytest.raises(_native.DbpError) as e:
        srv.load_channel(f["H"], f["C"], 1.0)
    assert e.value.code == 3
    srv.close()


def test_refused_configuration_fails_at_submit():
    """A frame the library would refuse (mixed precision is built for U = 32
    and 64 only; a regulariser code out of range) is refused by submit itself
    with the library's error, so no caller waits on a frame that cannot run;
    the server keeps serving valid frames afterwards."""
    say("[gpu] serving refused configuration")
    f = make_frames(True)[1]                      # B = 128, U = 16, C = 8
    srv = api.Server(hbm_budget_bytes=1 << 30, n_slots=2)
    s, h = out_bufs(f, True)
    with pytest.raises(_native.DbpError) as e:
        srv.submit(f["H"], f["y"], s, h, f["C"], 5, 1.0, f["N0"], qam=16, prec="fp16")
    assert e.value.code == 2
    with pytest.raises(KeyError):
        srv.submit(f["H"], f["y"], s, h, f["C"], 5, 1.0, f["N0"], qam=16, reg="lasso")
    t = srv.submit(f["H"], f["y"], s, h, f["C"], 5, 1.0, f["N0"], qam=16)
    lat, _ = srv.wait(t)
    assert lat > 0
    srv.close()
