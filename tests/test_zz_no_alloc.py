"""dbp_detect_admm_noalloc (the detection entry point that allocates nothing:
its FP64 re-slice workspace is a static device array) against
dbp_detect_admm with a workspace, bit for bit, through the C ABI: two calls in
a row, the second with fewer subcarriers, at an SNR where the re-slice runs."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1702_04458_amd import inputs  # noqa: E402

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1702_04458_amd import _native, api  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def call_noalloc(H, y, N0, C, T, qam, with_status):
    n_sc, B, U = H.shape
    n_sym = y.shape[1]
    s = torch.empty((n_sc, n_sym, U), dtype=torch.complex64, device=DEV)
    h = torch.empty((n_sc, n_sym, U), dtype=torch.uint8, device=DEV)
    st = torch.empty(n_sc, dtype=torch.int32, device=DEV) if with_status else None
    L = _native.lib()
    code = L.dbp_detect_admm_noalloc(H.data_ptr(), y.data_ptr(), s.data_ptr(), h.data_ptr(),
                                     st.data_ptr() if st is not None else None, n_sc, n_sym, B, U, C, T,
                                     1.0, 1.0, float(N0), 1.0, 0, qam, 0,
                                     torch.cuda.current_stream().cuda_stream or None)
    _native.check(code)
    return s, h, st


def call_reference(H, y, N0, C, T, qam):
    n_sc, B, U = H.shape
    n_sym = y.shape[1]
    s = torch.empty((n_sc, n_sym, U), dtype=torch.complex64, device=DEV)
    h = torch.empty((n_sc, n_sym, U), dtype=torch.uint8, device=DEV)
    st = torch.empty(n_sc, dtype=torch.int32, device=DEV)
    ws = api.workspace(n_sc, U, C, DEV)
    L = _native.lib()
    code = L.dbp_detect_admm(H.data_ptr(), y.data_ptr(), s.data_ptr(), h.data_ptr(), st.data_ptr(), ws.data_ptr(),
                             ws.numel(), n_sc, n_sym, B, U, C, T, 1.0, 1.0, float(N0), 1.0, 0, qam, 0,
                             torch.cuda.current_stream().cuda_stream or None)
    _native.check(code)
    return s, h, st


@pytest.mark.parametrize("with_status", [False, True])
def test_noalloc_matches_detect_admm(with_status):
    for i, (n_sc, B, U, C, qam, snr) in enumerate([(1200, 128, 16, 8, 16, 0.0), (300, 128, 16, 8, 16, 0.0)]):
        say(f"[gpu] noalloc call {i}: n_sc={n_sc} B={B} U={U} C={C} status={with_status}")
        fr = inputs.uplink_frame(inputs.frame_seed(50, i, int(snr)), n_sc, B, U, qam, snr)
        H = torch.from_numpy(fr.H).to(DEV)
        y = torch.from_numpy(fr.y).to(DEV)
        s0, h0, st0 = call_reference(H, y, fr.N0, C, 5, qam)
        s1, h1, st1 = call_noalloc(H, y, fr.N0, C, 5, qam, with_status)
        torch.cuda.synchronize()
        n_res = int(((st0 & 2) != 0).sum().item())
        say(f"    re-sliced {n_res} of {n_sc}")
        assert torch.equal(s0, s1)
        assert torch.equal(h0, h1)
        if with_status:
            assert torch.equal(st0, st1)
        if i == 0:
            assert n_res > 0            # the static scratch was used by the FP64 pass


def test_noalloc_refuses_oversized():
    L = _native.lib()
    cap = L.dbp_noalloc_scratch_bytes()
    assert cap == 16 << 20
    # flags of 4.2 M subcarriers exceed the array without a status array (host check, nothing queued)
    n_sc = (cap // 4) + 1
    code = L.dbp_detect_admm_noalloc(1, 1, 1, 1, None, n_sc, 1, 64, 8, 4, 3, 1.0, 1.0, 0.1, 1.0, 0, 4, 0, None)
    assert code == 2
    assert b"static" in L.dbp_last_error()
