"""Python binding over the C ABI (``include/dbp.h``).

Argument marshalling only: every step of detection and precoding runs in the
HIP library.  torch provides device memory and the stream; inputs must be
contiguous complex64 CUDA (HIP) tensors already resident on the device.
"""
from __future__ import annotations

import torch

from . import _native

REG = {"mmse": 0, "zf": 1, "box": 2}
PREC = {"fp32": 0, "fp16": 1, "bf16": 2, "mixed_fp16": 1, "mixed_bf16": 2}
FACTOR = {None: 0, "auto": 0, "fp32": 0x10, "fp64": 0x20, "f16x2": 0x30}


def _dev(t: torch.Tensor, name: str, dtype=torch.complex64) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes_ptr(s.cuda_stream)


def ctypes_ptr(v):
    return v if v else None


def _shapes(H, y):
    if H.dim() != 3:
        raise ValueError("H must be [n_sc, B, U]")
    n_sc, B, U = H.shape
    if y.dim() == 2:
        y = y.unsqueeze(1)
    if y.dim() != 3 or y.shape[0] != n_sc or y.shape[2] != B:
        raise ValueError("y must be [n_sc, n_sym, B] (or [n_sc, B])")
    return n_sc, y.shape[1], B, U, y


def _check_out(t, name, shape, dtype, device):
    """An output buffer the kernels write in full: exact shape, dtype, device
    and contiguity (a wrong buffer would be written out of bounds)."""
    _dev(t, name, dtype)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}")
    return t


def _outputs(out, n_sc, n_sym, U, device, hard, status):
    """(s_hat, hard, status) buffers: from ``out`` (a tuple of 2 or 3 tensors,
    None entries allowed for hard / status) or freshly allocated."""
    shape = (n_sc, n_sym, U)
    if out is None:
        s_hat = torch.empty(shape, dtype=torch.complex64, device=device)
        hd = torch.empty(shape, dtype=torch.uint8, device=device) if hard else None
        stt = torch.empty(n_sc, dtype=torch.int32, device=device) if status else None
        return s_hat, hd, stt
    s_hat, hd = out[0], out[1]
    stt = out[2] if len(out) > 2 else None
    _check_out(s_hat, "s_hat", shape, torch.complex64, device)
    if hd is not None:
        _check_out(hd, "hard", shape, torch.uint8, device)
    if stt is not None:
        _check_out(stt, "status", (n_sc,), torch.int32, device)
    return s_hat, hd, stt


def workspace(n_sc, U, C, device="cuda"):
    """Device workspace of the FP64 re-slice (``dbp_detect_workspace_bytes``),
    reusable across calls of the same or smaller size that do not overlap."""
    nbytes = _native.lib().dbp_detect_workspace_bytes(n_sc, U, C)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def _workspace(ws, need_ws, n_sc, U, C, device):
    """(pointer, bytes, tensor) of the workspace of the FP64 pass, needed with
    hard decisions and by the mixed modes' FP64 factor rule.  The caller keeps
    the tensor referenced until the call that uses it has been queued (a
    workspace allocated here must not return to the allocator before that)."""
    if not need_ws:
        return None, 0, None
    need = _native.lib().dbp_detect_workspace_bytes(n_sc, U, C)
    if ws is None:
        ws = workspace(n_sc, U, C, device)
    _dev(ws, "workspace", torch.uint8)
    if ws.device != device or ws.numel() < need:
        raise ValueError(f"workspace must be a device uint8 tensor of >= {need} bytes on {device}")
    return ws.data_ptr(), ws.numel(), ws


def _mark_stream(ws, given, stream):
    """A workspace allocated here on the current stream but used on another
    one must not be handed out again before that stream's work is done."""
    if ws is not None and given is None and stream is not None:
        ws.record_stream(stream)


def _ret(s_hat, hd, stt, status):
    return (s_hat, hd, stt) if status else (s_hat, hd)


def detect(H, y, N0, C, rho=1.0, T=5, *, algo="admm", reg="mmse", qam=16, Es=1.0, gamma=1.0,
           prec="fp32", factor=None, hard=True, status=False, out=None, workspace=None, stream=None):
    """Decentralized uplink detection.

    ``algo="admm"`` runs Algorithm 1 (``rho`` is the ADMM penalty),
    ``algo="cg"`` runs Algorithm 2 (regulariser N0/Es, ``rho`` unused).
    ``prec`` selects the Gram arithmetic ("fp32", "fp16", "bf16"); in the mixed
    modes ``factor`` ("auto", "fp32", "fp64", "f16x2") selects the inverse's precision.
    Hard decisions are exact (near-threshold subcarriers recomputed in FP64,
    which needs a ``workspace``; one is allocated when none is given).
    Returns ``(s_hat [n_sc, n_sym, U] complex64, hard [n_sc, n_sym, U] uint8 or None)``,
    plus ``status [n_sc] int32`` (DBP_STATUS_* bits) with ``status=True``.
    """
    _dev(H, "H")
    _dev(y, "y")
    n_sc, n_sym, B, U, y = _shapes(H, y)
    s_hat, hd, stt = _outputs(out, n_sc, n_sym, U, H.device, hard, status)
    # the mixed modes may send ill-conditioned subcarriers to the FP64 pass
    need_ws = hd is not None or (algo == "admm" and prec != "fp32")
    wp, wb, _ws_keep = _workspace(workspace, need_ws, n_sc, U, C, H.device)
    _mark_stream(_ws_keep, workspace, stream)
    L = _native.lib()
    st = _stream(stream)
    hp = hd.data_ptr() if hd is not None else None
    sp = stt.data_ptr() if stt is not None else None
    if algo == "admm":
        code = L.dbp_detect_admm(H.data_ptr(), y.data_ptr(), s_hat.data_ptr(), hp, sp, wp, wb, n_sc, n_sym, B, U,
                                 C, T, float(rho), float(gamma), float(N0), float(Es), REG[reg], qam,
                                 PREC[prec] | FACTOR[factor], st)
    elif algo == "cg":
        code = L.dbp_detect_cg(H.data_ptr(), y.data_ptr(), s_hat.data_ptr(), hp, sp, wp, wb, n_sc, n_sym, B, U, C,
                               T, float(N0), float(Es), REG[reg], qam, st)
    else:
        raise ValueError(algo)
    _native.check(code)
    return _ret(s_hat, hd, stt, status)


def factor(H, C, rho=1.0, *, prec="fp32", factor=None, out=None, stream=None):
    """Algorithm 1's preprocessing for a static channel: B_c^{-1} for every
    (subcarrier, cluster), kept resident for :func:`detect_factored`.  Returns a
    complex64 device tensor [n_sc, C, U (U + 1) / 2] in the library's internal
    layout: the upper triangle of each Hermitian block, column by column
    (entry (i, v), i <= v, at v (v + 1) / 2 + i)."""
    _dev(H, "H")
    n_sc, B, U = H.shape
    f = out if out is not None else torch.empty((n_sc, C, U * (U + 1) // 2), dtype=torch.complex64,
                                                 device=H.device)
    _dev(f, "factors")
    if f.device != H.device:
        raise ValueError(f"factors must be on {H.device}")
    if f.numel() * 8 != _native.lib().dbp_factor_bytes(n_sc, U, C):
        raise ValueError("factors must hold n_sc * C * U (U + 1) / 2 complex64")
    _native.check(_native.lib().dbp_factor_admm(H.data_ptr(), f.data_ptr(), n_sc, B, U, C, float(rho),
                                                PREC[prec] | FACTOR[factor], _stream(stream)))
    return f


def detect_batch(frames, *, stream=None):
    """Uneven batch of ADMM detection frames in one launch
    (``dbp_detect_admm_batch``).  ``frames`` is a list of dicts with keys H
    [n_sc, B, U], y [n_sc, n_sym, B], N0, C and optionally rho, T, qam, reg,
    Es, gamma, hard (default True), status (default False), workspace; every
    frame must have the same U.  Returns a list of (s_hat, hard[, status])
    per frame, as :func:`detect`."""
    import ctypes

    if not frames:
        return []
    if len(frames) > 24:
        raise ValueError("at most 24 frames per batch (DBP_MAX_BATCH)")
    arr = (_native.Frame * len(frames))()
    results, keep = [], []
    U = None
    for i, f in enumerate(frames):
        H, y = _dev(f["H"], "H"), _dev(f["y"], "y")
        n_sc, n_sym, B, Uf, y = _shapes(H, y)
        if U is None:
            U = Uf
        elif Uf != U:
            raise ValueError("every frame of a batch must have the same U")
        C = int(f["C"])
        s_hat, hd, stt = _outputs(None, n_sc, n_sym, U, H.device, f.get("hard", True), f.get("status", False))
        wp, wb, wt = _workspace(f.get("workspace"), hd is not None, n_sc, U, C, H.device)
        _mark_stream(wt, f.get("workspace"), stream)
        keep.append((H, y, wt))
        e = arr[i]
        e.H, e.y, e.s_hat = H.data_ptr(), y.data_ptr(), s_hat.data_ptr()
        e.hard = hd.data_ptr() if hd is not None else None
        e.status = stt.data_ptr() if stt is not None else None
        e.workspace, e.workspace_bytes = wp, wb
        e.n_sc, e.n_sym, e.B, e.C, e.T = n_sc, n_sym, B, C, int(f.get("T", 5))
        e.reg, e.qam = REG[f.get("reg", "mmse")], int(f.get("qam", 16))
        e.rho, e.gamma, e.N0, e.Es = (float(f.get("rho", 1.0)), float(f.get("gamma", 1.0)), float(f["N0"]),
                                      float(f.get("Es", 1.0)))
        results.append(_ret(s_hat, hd, stt, f.get("status", False)))
    code = _native.lib().dbp_detect_admm_batch(arr, len(frames), U, _stream(stream))
    _native.check(code)
    return results


def detect_factored(H, factors, y, N0, C, rho=1.0, T=5, *, reg="mmse", qam=16, Es=1.0, gamma=1.0, hard=True,
                    status=False, out=None, workspace=None, stream=None):
    """Algorithm 1's iterations against resident factors from :func:`factor`
    (same ``rho``); forms no Gram and no inverse.  Outputs as :func:`detect`."""
    _dev(H, "H")
    _dev(y, "y")
    _dev(factors, "factors")
    n_sc, n_sym, B, U, y = _shapes(H, y)
    if factors.numel() * 8 != _native.lib().dbp_factor_bytes(n_sc, U, C):
        raise ValueError("factors do not match (n_sc, U, C)")
    s_hat, hd, stt = _outputs(out, n_sc, n_sym, U, H.device, hard, status)
    wp, wb, _ws_keep = _workspace(workspace, hd is not None, n_sc, U, C, H.device)
    _mark_stream(_ws_keep, workspace, stream)
    code = _native.lib().dbp_detect_admm_factored(
        H.data_ptr(), factors.data_ptr(), y.data_ptr(), s_hat.data_ptr(), hd.data_ptr() if hd is not None else None,
        stt.data_ptr() if stt is not None else None, wp, wb,
        n_sc, n_sym, B, U, C, T, float(rho), float(gamma), float(N0), float(Es), REG[reg], qam, _stream(stream))
    _native.check(code)
    return _ret(s_hat, hd, stt, status)


def nonfinite_status(x, *, out=None, stream=None):
    """Per-subcarrier flags of a result x [n_sc, ...] (complex64, device):
    int32 tensor [n_sc], 1 where any part of subcarrier k is NaN or infinite
    (``dbp_flag_nonfinite``)."""
    _dev(x, "x")
    n_sc = x.shape[0]
    per_sc = x.numel() // n_sc if n_sc else 1
    st = out if out is not None else torch.empty(n_sc, dtype=torch.int32, device=x.device)
    _check_out(st, "status", (n_sc,), torch.int32, x.device)
    _native.check(_native.lib().dbp_flag_nonfinite(x.data_ptr(), n_sc, per_sc, st.data_ptr(), _stream(stream)))
    return st


def pack_channel_h16(H, C, *, out=None, stream=None):
    """Packs the channel H [n_sc, B, U] into the library's mixed-precision
    resident form (complex FP16 with one power-of-two scale per subcarrier and
    cluster; ``dbp_pack_channel_h16``).  Returns a uint8 device tensor of
    ``dbp_channel_h16_bytes`` bytes."""
    _dev(H, "H")
    n_sc, B, U = H.shape
    nbytes = _native.lib().dbp_channel_h16_bytes(n_sc, B, U, C)
    if nbytes == 0 and n_sc > 0:
        raise ValueError("malformed (n_sc, B, U, C)")
    p = out if out is not None else torch.empty(nbytes, dtype=torch.uint8, device=H.device)
    if p.numel() * p.element_size() != nbytes or not p.is_contiguous():
        raise ValueError("packed must be a contiguous buffer of dbp_channel_h16_bytes bytes")
    _native.check(_native.lib().dbp_pack_channel_h16(H.data_ptr(), p.data_ptr(), n_sc, B, U, C, _stream(stream)))
    return p


def factor_h16(H, C, rho=1.0, *, prec="fp32", factor=None, out=None, stream=None):
    """:func:`factor` and :func:`pack_channel_h16` of the same channel in one
    call (``dbp_factor_admm_h16``; one launch at U = 32 with the FP32
    preprocessing).  ``out`` is an optional (factors, packed) pair.  Returns
    (factors, packed), bit for bit those of the two separate calls."""
    _dev(H, "H")
    n_sc, B, U = H.shape
    f, p = out if out is not None else (None, None)
    if f is None:
        f = torch.empty((n_sc, C, U * (U + 1) // 2), dtype=torch.complex64, device=H.device)
    _dev(f, "factors")
    if f.numel() * 8 != _native.lib().dbp_factor_bytes(n_sc, U, C):
        raise ValueError("factors must hold n_sc * C * U (U + 1) / 2 complex64")
    nbytes = _native.lib().dbp_channel_h16_bytes(n_sc, B, U, C)
    if nbytes == 0 and n_sc > 0:
        raise ValueError("malformed (n_sc, B, U, C)")
    if p is None:
        p = torch.empty(nbytes, dtype=torch.uint8, device=H.device)
    if p.numel() * p.element_size() != nbytes or not p.is_contiguous() or p.device != H.device:
        raise ValueError("packed must be a contiguous buffer of dbp_channel_h16_bytes bytes on H's device")
    if f.device != H.device:
        raise ValueError(f"factors must be on {H.device}")
    _native.check(_native.lib().dbp_factor_admm_h16(H.data_ptr(), f.data_ptr(), p.data_ptr(), n_sc, B, U, C,
                                                    float(rho), PREC[prec] | FACTOR[factor], _stream(stream)))
    return f, p


def detect_factored_h16(packed, factors, y, N0, B, U, C, rho=1.0, T=5, *, reg="mmse", qam=16, Es=1.0, gamma=1.0,
                        hard=True, status=False, out=None, stream=None):
    """Algorithm 1's iterations against resident factors and the packed FP16
    channel from :func:`pack_channel_h16` (low-precision path, <= 1e-3)."""
    _dev(packed, "packed", torch.uint8)
    _dev(y, "y")
    _dev(factors, "factors")
    if y.dim() == 2:
        y = y.unsqueeze(1)
    n_sc, n_sym = y.shape[0], y.shape[1]
    if y.shape[2] != B or not y.is_contiguous():
        raise ValueError("y must be a contiguous [n_sc, n_sym, B] tensor")
    L = _native.lib()
    if packed.numel() * packed.element_size() != L.dbp_channel_h16_bytes(n_sc, B, U, C):
        raise ValueError("packed channel does not match (n_sc, B, U, C)")
    if factors.numel() * 8 != L.dbp_factor_bytes(n_sc, U, C):
        raise ValueError("factors do not match (n_sc, U, C)")
    s_hat, hd, stt = _outputs(out, n_sc, n_sym, U, y.device, hard, status)
    code = L.dbp_detect_admm_factored_h16(
        packed.data_ptr(), factors.data_ptr(), y.data_ptr(), s_hat.data_ptr(), hd.data_ptr() if hd is not None else None,
        stt.data_ptr() if stt is not None else None,
        n_sc, n_sym, B, U, C, T, float(rho), float(gamma), float(N0), float(Es), REG[reg], qam, _stream(stream))
    _native.check(code)
    return _ret(s_hat, hd, stt, status)


POWER = {"common_gain": 0, "per_cluster": 1}


def precode(H, s, C, rho=1.0, T=5, *, gamma=1.0, eps=0.0, P_cluster=None, power="common_gain", layout="uplink",
            out=None, stream=None):
    """Decentralized ADMM beamforming (Algorithm 3; ``eps`` > 0 uses the
    z-update of Lemma 2 for the constraint ||s - H^d x|| <= eps).

    ``H`` is the uplink-layout channel [n_sc, B, U] (``layout="uplink"``,
    used as H^d = H^T) or the downlink channel H^d [n_sc, U, B]
    (``layout="downlink"``); ``s`` the targets [n_sc, n_sym, U] (or [n_sc, U]).  ``P_cluster`` optional device float32
    tensor [C] of per-cluster budgets, met by a common gain after the
    algorithm (``power="common_gain"``) or by the budgeted step (P1) in every
    x-update (``power="per_cluster"``).  Returns ``(x [n_sc, n_sym, B], beta [n_sc, n_sym])``.
    """
    _dev(H, "H")
    _dev(s, "s")
    if H.dim() != 3:
        raise ValueError("H must be [n_sc, B, U] (uplink) or [n_sc, U, B] (downlink)")
    if layout == "uplink":
        n_sc, B, U = H.shape
    elif layout == "downlink":
        n_sc, U, B = H.shape
    else:
        raise ValueError(layout)
    if s.dim() == 2:
        s = s.unsqueeze(1)
    n_sym = s.shape[1]
    if s.shape[0] != n_sc or s.shape[2] != U:
        raise ValueError("s must be [n_sc, n_sym, U]")
    if P_cluster is not None:
        _dev(P_cluster, "P_cluster", torch.float32)
        if P_cluster.numel() != C or P_cluster.device != H.device:
            raise ValueError(f"P_cluster must hold C = {C} budgets on {H.device}")
    if out is None:
        x = torch.empty((n_sc, n_sym, B), dtype=torch.complex64, device=H.device)
        beta = torch.empty((n_sc, n_sym), dtype=torch.float32, device=H.device)
    else:
        x, beta = out
        _check_out(x, "x", (n_sc, n_sym, B), torch.complex64, H.device)
        _check_out(beta, "beta", (n_sc, n_sym), torch.float32, H.device)
    L = _native.lib()
    code = L.dbp_precode_admm(H.data_ptr(), 0 if layout == "uplink" else 1, s.data_ptr(), x.data_ptr(), beta.data_ptr(),
                              P_cluster.data_ptr() if P_cluster is not None else None, POWER[power],
                              n_sc, n_sym, B, U, C, T, float(rho), float(gamma), float(eps),
                              _stream(stream))
    _native.check(code)
    return x, beta


class Server:
    """Continuous-batching detection server (``dbp_server_*``).

    Frames are submitted either from pinned host tensors (``torch.empty(...,
    pin_memory=True)``; the server copies them into its HBM arena) or from
    device tensors already resident in HBM (no copies).  They must stay alive
    until :meth:`wait` returns for their ticket.
    """

    def __init__(self, hbm_budget_bytes: int, n_slots: int = 8, device: int = 0):
        import ctypes

        self._ct = ctypes
        h = ctypes.c_void_p()
        _native.check(_native.lib().dbp_server_create(device, int(hbm_budget_bytes), int(n_slots), ctypes.byref(h)))
        self._h = h

    def submit(self, H, y, s_out, hard_out, C, T=5, rho=1.0, N0=0.0, *, reg="mmse", qam=16, prec="fp32",
               factor=None) -> int:
        ct = self._ct
        dev = H.is_cuda
        for t, n in ((H, "H"), (y, "y"), (s_out, "s_out")) + (((hard_out, "hard_out"),) if hard_out is not None else ()):
            if not t.is_contiguous():
                raise ValueError(f"{n} must be contiguous")
            if dev and not t.is_cuda:
                raise ValueError(f"{n} must be a device tensor like H")
            if not dev and (t.is_cuda or not t.is_pinned()):
                raise ValueError(f"{n} must be a pinned host tensor like H")
        n_sc, B, U = H.shape
        n_sym = y.shape[1]
        tk = ct.c_uint64()
        code = _native.lib().dbp_server_submit(
            self._h, H.data_ptr(), y.data_ptr(), s_out.data_ptr(),
            hard_out.data_ptr() if hard_out is not None else None,
            n_sc, n_sym, B, U, C, T, float(rho), float(N0), REG[reg], qam, PREC[prec] | FACTOR[factor],
            1 if dev else 0, ct.byref(tk))
        _native.check(code)
        return tk.value

    def load_channel(self, H, C, rho=1.0, *, prec="fp32", factor=None, h16=False) -> int:
        """Copy a static channel H (pinned host or device tensor) into the arena
        and factor it once; returns a channel handle for :meth:`submit_factored`.
        ``h16=True`` keeps H resident in the packed FP16 form (low-precision path)."""
        ct = self._ct
        if not H.is_contiguous():
            raise ValueError("H must be contiguous")
        if not H.is_cuda and not H.is_pinned():
            raise ValueError("H must be a pinned host tensor or a device tensor")
        n_sc, B, U = H.shape
        ch = ct.c_uint64()
        _native.check(_native.lib().dbp_channel_load(self._h, H.data_ptr(), n_sc, B, U, C, float(rho),
                                                     PREC[prec] | FACTOR[factor],
                                                     (1 if H.is_cuda else 0) | (2 if h16 else 0), ct.byref(ch)))
        return ch.value

    def free_channel(self, channel: int):
        _native.check(_native.lib().dbp_channel_free(self._h, self._ct.c_uint64(channel)))

    def submit_factored(self, channel: int, y, s_out, hard_out, T=5, N0=0.0, *, reg="mmse", qam=16) -> int:
        """Queue a frame of received vectors y [n_sc, n_sym, B] against a loaded channel."""
        ct = self._ct
        dev = y.is_cuda
        for t, n in ((y, "y"), (s_out, "s_out")) + (((hard_out, "hard_out"),) if hard_out is not None else ()):
            if not t.is_contiguous():
                raise ValueError(f"{n} must be contiguous")
            if dev != t.is_cuda or (not dev and not t.is_pinned()):
                raise ValueError(f"{n} must be a pinned host tensor, or a device tensor like y")
        tk = ct.c_uint64()
        code = _native.lib().dbp_server_submit_factored(
            self._h, ct.c_uint64(channel), y.data_ptr(), s_out.data_ptr(),
            hard_out.data_ptr() if hard_out is not None else None, y.shape[1], T, float(N0), REG[reg], qam,
            1 if dev else 0, ct.byref(tk))
        _native.check(code)
        return tk.value

    def poll(self, ticket: int):
        ct = self._ct
        done, lat = ct.c_int(), ct.c_double()
        _native.check(_native.lib().dbp_server_poll(self._h, ct.c_uint64(ticket), ct.byref(done), ct.byref(lat)))
        return bool(done.value), lat.value

    def wait(self, ticket: int):
        """Blocks until done; returns (latency_us, queue_us)."""
        ct = self._ct
        lat, q = ct.c_double(), ct.c_double()
        _native.check(_native.lib().dbp_server_wait(self._h, ct.c_uint64(ticket), ct.byref(lat), ct.byref(q)))
        return lat.value, q.value

    def set_batching(self, max_frames: int):
        """Frames one launch may take at admission (1: no batching)."""
        _native.check(_native.lib().dbp_server_set_batching(self._h, int(max_frames)))

    def stats(self):
        ct = self._ct
        pb, pi, c = ct.c_size_t(), ct.c_int(), ct.c_uint64()
        _native.check(_native.lib().dbp_server_stats(self._h, ct.byref(pb), ct.byref(pi), ct.byref(c)))
        return {"peak_bytes": pb.value, "peak_inflight": pi.value, "completed": c.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _native.check(_native.lib().dbp_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


TUNE = {"admm": 0, "cg": 1, "precode": 2}


def autotune(kind, H, inp, out, C, T=5, reps=10, stream=None):
    """Times the launch-plan candidates of a kernel family on the given device
    data and keeps the fastest for later calls (``dbp_autotune``); returns
    the chosen minimum waves per workgroup.  ``inp`` is y [n_sc, 1, B] (ADMM,
    CG) or the targets s [n_sc, 1, U] (precode); ``out`` the matching output
    buffer, overwritten."""
    import ctypes

    for t, n in ((H, "H"), (inp, "input"), (out, "output")):
        _dev(t, n)
    n_sc, B, U = H.shape
    best = ctypes.c_int()
    _native.check(_native.lib().dbp_autotune(TUNE[kind], H.data_ptr(), inp.data_ptr(), out.data_ptr(), n_sc, B, U,
                                             C, T, reps, _stream(stream), ctypes.byref(best)))
    return best.value


def autotune_get(kind, U, C):
    return _native.lib().dbp_autotune_get(TUNE[kind], U, C)
