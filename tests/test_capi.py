"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/dbp.h, and rejects malformed arguments before touching the
device (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1702_04458_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbp.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_native.LIB_PATH), reason="libdbp.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dbp_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(_native.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 6
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding knows every declared entry point
    assert set(syms) <= set(_native.SIGNATURES)


def test_version_and_strerror():
    L = _native.lib()
    assert b"gfx950" in L.dbp_version()
    for code in range(7):
        assert L.dbp_strerror(code)


def _admm(**kw):
    args = dict(H=1, y=1, s=1, hard=None, status=None, ws=None, ws_bytes=0, n_sc=4, n_sym=1, B=64, U=8, C=4, T=3,
                rho=1.0, gamma=1.0, N0=0.1, Es=1.0, reg=0, qam=4, prec=0)
    args.update(kw)
    L = _native.lib()
    return L.dbp_detect_admm(args["H"], args["y"], args["s"], args["hard"], args["status"], args["ws"],
                             args["ws_bytes"], args["n_sc"], args["n_sym"],
                             args["B"], args["U"], args["C"], args["T"], args["rho"], args["gamma"],
                             args["N0"], args["Es"], args["reg"], args["qam"], args["prec"], None)


@pytest.mark.parametrize("kw,code", [
    (dict(B=63), 1), (dict(U=128, B=64), 1), (dict(T=0), 1), (dict(rho=0.0), 1), (dict(rho=-1.0), 1),
    (dict(N0=-1.0), 1), (dict(Es=0.0), 1), (dict(gamma=0.0), 1), (dict(qam=8), 1), (dict(reg=7), 1),
    (dict(prec=9), 1), (dict(H=None), 1), (dict(y=None), 1), (dict(s=None), 1), (dict(n_sc=-1), 1),
    (dict(n_sym=0), 1), (dict(U=12, B=96, C=4), 2), (dict(B=64, C=8, U=16), 2), (dict(C=32, B=512), 2),
    (dict(rho=float("nan")), 1), (dict(prec=1, U=16, B=128, C=8), 2), (dict(prec=0x40), 1),
    (dict(prec=0x20), 2), (dict(prec=0x13), 1), (dict(prec=0x21, U=64, B=512, C=8), 1),
    # the FP64 factor rule (mixed, U/S > 0.8; explicit FP64 at U = 64) needs a workspace
    (dict(prec=1, U=32, B=256, C=8), 1), (dict(prec=2, U=64, B=512, C=8), 1),
])
def test_detect_admm_rejects(kw, code):
    assert _admm(**kw) == code
    assert _native.lib().dbp_last_error()


def test_detect_admm_empty_is_noop():
    assert _admm(n_sc=0, H=None, y=None, s=None) == 0
    # n_sc = 0 still validates every other argument (the serving loop relies on it)
    assert _admm(n_sc=0, H=None, y=None, s=None, prec=1, U=16, B=128, C=8) == 2


def test_workspace_bytes():
    L = _native.lib()
    # a 256-byte aligned flag region of n_sc int32, min(n_sc, 256) blocks of C U^2 complex FP64, and
    # room for 256 aligned int32 (the subcarriers recomputed with one workgroup per cluster)
    assert L.dbp_detect_workspace_bytes(1200, 32, 8) == 4864 + 256 * 8 * 32 * 32 * 16 + 1536
    assert L.dbp_detect_workspace_bytes(16, 8, 4) == 256 + 16 * 4 * 8 * 8 * 16 + 1536
    assert L.dbp_detect_workspace_bytes(0, 8, 4) == 256 * 0 + 1 * 4 * 8 * 8 * 16 + 1536
    assert L.dbp_detect_workspace_bytes(-1, 8, 4) == 0


def test_hard_decisions_need_a_workspace():
    need = _native.lib().dbp_detect_workspace_bytes(4, 8, 4)
    assert _admm(hard=1) == 1                                    # no workspace
    assert "workspace" in _native.lib().dbp_last_error().decode()
    assert _admm(hard=1, ws=256, ws_bytes=need - 1) == 1         # too small
    assert _admm(hard=1, ws=257, ws_bytes=need) == 1             # misaligned


def test_detect_cg_rejects():
    L = _native.lib()
    # (H, y, x, hard, status, ws, ws_bytes, n_sc, n_sym, B, U, C, T, N0, Es, reg, qam, stream)
    base = [1, 1, 1, None, None, None, 0, 4, 1, 64, 8, 4, 3, 0.1, 1.0, 0, 4, None]
    bad = list(base)
    bad[15] = 2
    assert L.dbp_detect_cg(*bad) == 1                                          # BOX is not quadratic
    bad = list(base)
    bad[11] = 3
    assert L.dbp_detect_cg(*bad) == 1                                          # B % C
    bad = list(base)
    bad[2] = None
    assert L.dbp_detect_cg(*bad) == 1                                          # null x
    bad = list(base)
    bad[3] = 1
    assert L.dbp_detect_cg(*bad) == 1                                          # hard without workspace


def test_precode_rejects():
    L = _native.lib()
    # (H, h_layout, s, x, beta, P, power_mode, n_sc, n_sym, B, U, C, T, rho, gamma, eps, stream)
    ok = [1, 0, 1, 1, None, None, 0, 4, 1, 256, 32, 16, 5, 1.0, 1.0, 0.0, None]
    bad_S = list(ok)
    bad_S[11] = 4         # C = 4 -> S = 64 > U = 32 (U x U branch)
    assert L.dbp_precode_admm(*bad_S) == 2
    bad_rho = list(ok)
    bad_rho[13] = 0.0
    assert L.dbp_precode_admm(*bad_rho) == 1
    bad_ptr = list(ok)
    bad_ptr[3] = None
    assert L.dbp_precode_admm(*bad_ptr) == 1
    for e in (-0.1, float("nan"), float("inf")):
        bad_eps = list(ok)
        bad_eps[15] = e
        assert L.dbp_precode_admm(*bad_eps) == 1
    bad_mode = list(ok)
    bad_mode[6] = 2
    assert L.dbp_precode_admm(*bad_mode) == 1
    bad_layout = list(ok)
    bad_layout[1] = 2
    assert L.dbp_precode_admm(*bad_layout) == 1


def test_factor_entry_points_reject():
    L = _native.lib()
    assert L.dbp_factor_bytes(1200, 32, 8) == 1200 * 8 * (32 * 33 // 2) * 8
    # dbp_factor_admm(H, factors, n_sc, B, U, C, rho, prec, stream)
    assert L.dbp_factor_admm(1, 1, 4, 256, 32, 8, 0.0, 0, None) == 1          # rho <= 0
    assert L.dbp_factor_admm(1, None, 4, 256, 32, 8, 1.0, 0, None) == 1       # null factors
    assert L.dbp_factor_admm(1, 1, 4, 256, 32, 16, 1.0, 0, None) == 2         # S = 16 < U
    assert L.dbp_factor_admm(1, 1, 4, 256, 32, 8, 1.0, 0x20, None) == 2       # FP64 inverse needs a mixed Gram
    assert L.dbp_factor_admm(1, 1, 4, 512, 64, 8, 1.0, 0x21, None) == 2       # no stored FP64 inverse at U = 64
    assert L.dbp_factor_admm(None, None, 0, 256, 32, 8, 1.0, 0, None) == 0    # empty is a no-op
    # dbp_factor_admm_h16(H, factors, packed, n_sc, B, U, C, rho, prec, stream)
    assert L.dbp_factor_admm_h16(1, 1, None, 4, 256, 32, 8, 1.0, 0, None) == 1   # null packed
    assert L.dbp_factor_admm_h16(1, 1, 1, 4, 256, 32, 8, 0.0, 0, None) == 1      # rho <= 0
    assert L.dbp_factor_admm_h16(1, 1, 1, 4, 256, 32, 16, 1.0, 0, None) == 2     # S = 16 < U
    assert L.dbp_factor_admm_h16(None, None, None, 0, 256, 32, 8, 1.0, 0, None) == 0
    # dbp_detect_admm_factored(H, F, y, s, hard, status, ws, ws_bytes, n_sc, n_sym, B, U, C, T, rho, gamma, N0,
    #                          Es, reg, qam, stream)
    ok = [1, 1, 1, 1, None, None, None, 0, 4, 1, 256, 32, 8, 5, 1.0, 1.0, 0.1, 1.0, 0, 64, None]
    for i, v, code in ((1, None, 1), (13, 0, 1), (19, 8, 1), (11, 12, 2), (4, 1, 1)):
        bad = list(ok)
        bad[i] = v
        assert L.dbp_detect_admm_factored(*bad) == code, (i, v)


def test_h16_channel_entry_points_reject():
    L = _native.lib()
    assert L.dbp_channel_h16_bytes(1200, 256, 32, 8) == 1200 * 256 * 32 * 4 + 1200 * 8 * 4
    assert L.dbp_channel_h16_bytes(4, 250, 32, 8) == 0                          # B % C
    # dbp_pack_channel_h16(H, packed, n_sc, B, U, C, stream)
    assert L.dbp_pack_channel_h16(1, None, 4, 256, 32, 8, None) == 1            # null packed
    assert L.dbp_pack_channel_h16(1, 1, 4, 256, 24, 8, None) == 2               # U not built
    assert L.dbp_pack_channel_h16(None, None, 0, 256, 32, 8, None) == 0         # empty: no-op
    # dbp_detect_admm_factored_h16(packed, factors, y, s_hat, hard, status, n_sc, n_sym, B, U, C, T, rho, gamma,
    #                              N0, Es, reg, qam, stream)
    ok = [1, 1, 1, 1, None, None, 4, 1, 256, 32, 8, 5, 1.0, 1.0, 0.1, 1.0, 0, 64, None]
    for i, v, code in ((1, None, 1), (12, 0.0, 1), (17, 8, 1), (9, 64, 2)):
        bad = list(ok)
        bad[i] = v
        assert L.dbp_detect_admm_factored_h16(*bad) == code, (i, v)
    small = list(ok)
    small[10] = 16                                                               # S = 16 < U = 32
    assert L.dbp_detect_admm_factored_h16(*small) == 2


def test_flag_nonfinite_rejects():
    L = _native.lib()
    # dbp_flag_nonfinite(x, n_sc, per_sc, status, stream)
    assert L.dbp_flag_nonfinite(1, -1, 4, 1, None) == 1
    assert L.dbp_flag_nonfinite(1, 4, 0, 1, None) == 1
    assert L.dbp_flag_nonfinite(None, 4, 4, 1, None) == 1
    assert L.dbp_flag_nonfinite(1, 4, 4, None, None) == 1
    assert L.dbp_flag_nonfinite(None, 0, 4, None, None) == 0


def test_autotune_rejects_and_defaults():
    L = _native.lib()
    # dbp_autotune(kind, H, in, out, n_sc, B, U, C, T, reps, stream, best)
    assert L.dbp_autotune(7, 1, 1, 1, 4, 128, 16, 8, 5, 3, None, None) == 1       # kind
    assert L.dbp_autotune(0, None, 1, 1, 4, 128, 16, 8, 5, 3, None, None) == 1    # null H
    assert L.dbp_autotune(0, 1, 1, 1, 4, 128, 16, 8, 5, 0, None, None) == 1       # reps
    assert L.dbp_autotune(0, 1, 1, 1, 4, 128, 12, 8, 5, 3, None, None) == 2       # U not built
    # the build-time default plan: at least four waves per workgroup
    assert L.dbp_autotune_get(0, 16, 8) == 4
    assert L.dbp_autotune_get(1, 32, 8) == 4
    assert L.dbp_autotune_get(2, 32, 16) == 4
    assert L.dbp_autotune_get(0, 12, 8) == -1


def test_detect_batch_rejects():
    import ctypes
    L = _native.lib()
    assert L.dbp_detect_admm_batch(None, 0, 32, None) == 0                      # empty: no-op
    assert L.dbp_detect_admm_batch(None, 25, 32, None) == 1                     # above DBP_MAX_BATCH
    arr = (_native.Frame * 2)()
    for e in arr:
        e.H = e.y = e.s_hat = 1
        e.n_sc, e.n_sym, e.B, e.C, e.T, e.reg, e.qam = 4, 1, 256, 8, 5, 0, 64
        e.rho, e.gamma, e.N0, e.Es = 1.0, 1.0, 0.1, 1.0
    assert L.dbp_detect_admm_batch(arr, 2, 12, None) == 2                       # U not built
    arr[1].C = 16                                                               # S = 16 < U = 32
    assert L.dbp_detect_admm_batch(arr, 2, 32, None) == 2
    assert b"frame 1" in L.dbp_last_error()
    arr[1].C = 8
    arr[0].hard = 1                                                             # hard without workspace
    assert L.dbp_detect_admm_batch(arr, 2, 32, None) == 1
