"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars (FP32 path):
* soft outputs: frame-level relative Frobenius error ||gpu - oracle|| / ||oracle||
  <= 1e-5, and every vector within 1e-4 relative;
* hard decisions: identical to the oracle's FP64 decisions on every symbol.
  The library makes them exact by recomputing in FP64 every subcarrier with a
  soft value within a guard of a decision threshold (DBP_STATUS_RESLICED); the
  oracle is evaluated with the kernel's own FP32 value of N0.  On subcarriers
  that were not recomputed the decision is also the FP32 slicer applied to the
  kernel's soft output, bit for bit, and that soft output lies well inside the
  guard (its largest error, in the slicer's units, is below a quarter of the
  guard).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import dbp_oracle as O
from paper_1702_04458_amd import inputs

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1702_04458_amd import api  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel_err(gpu, ref):
    return float(np.linalg.norm(gpu - ref) / np.linalg.norm(ref))


def per_vec_rel(gpu, ref):
    num = np.linalg.norm(gpu - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return float(np.max(num / np.maximum(den, 1e-30)))


def threshold_gap(x, M):
    """Distance of the oracle value to the nearest decision threshold, in the
    slicer's units t = (kappa x + L) / 2 (thresholds at t = 1 .. L-1)."""
    L = int(math.sqrt(M))
    kappa = math.sqrt(2 * (M - 1) / 3)

    def gap(v):
        t = (kappa * v + L) / 2
        return np.abs(t - np.clip(np.round(t), 1, L - 1))
    return np.minimum(gap(x.real), gap(x.imag))


STATUS_NONFINITE, STATUS_RESLICED = 1, 2


def guard_t(U):
    """Re-slice guard of the FP32 path (slicer units) at U users."""
    return 2.0 ** -14 if U <= 16 else (2.0 ** -13 if U == 32 else 2.0 ** -12)


def t_units(x, M):
    return (math.sqrt(2 * (M - 1) / 3) * x + int(math.sqrt(M))) / 2


def check_hard(shat, hard, ref, M, status=None, guard=None):
    """Exact hard decisions (see the module docstring).  Returns the number of
    re-sliced subcarriers."""
    ref_hard = O.slice_qam(ref, M)
    diff = hard != ref_hard
    assert not np.any(diff), f"{int(np.sum(diff))} hard decisions differ from the FP64 oracle"
    if status is None:
        return 0
    if guard is None:
        guard = guard_t(shat.shape[-1])
    plain = (status & STATUS_RESLICED) == 0
    assert np.array_equal(hard[plain], O.slice_qam_f32(shat[plain], M)), "kernel slicer differs from FP32 slicer"
    if np.any(plain):
        err = np.maximum(np.abs(t_units(shat[plain].real, M) - t_units(ref[plain].real, M)),
                         np.abs(t_units(shat[plain].imag, M) - t_units(ref[plain].imag, M)))
        say(f"    largest soft error {err.max():.2e} (slicer units, guard {guard:.1e})")
        assert err.max() < guard / 4, f"FP32 error {err.max():.2e} too close to the guard {guard:.2e}"
    # a subcarrier that was not re-sliced has no soft value inside the guard
    gap = threshold_gap(shat[plain].astype(np.complex128), M)
    assert np.all(gap >= guard * (1 - 1e-3))
    return int(np.sum(~plain))


def check_hard_low_precision(shat, hard, ref, M, guard=1e-3):
    """Hard-decision rule of the low-precision paths that are not re-sliced
    (the FP16 resident channel, factors made with a BF16 Gram): the decision
    is the FP32 slicer applied to the kernel's own soft output bit for bit,
    and equals the oracle's FP64 decision on every symbol whose oracle value
    lies farther than `guard` (slicer units) from a threshold; at most 1e-4 of
    the symbols may differ (identical decisions on >= 99.99 %)."""
    assert np.array_equal(hard, O.slice_qam_f32(shat, M)), "kernel slicer differs from FP32 slicer"
    diff = hard != O.slice_qam(ref, M)
    near = threshold_gap(ref, M) < guard
    assert not np.any(diff & ~near), f"{int(np.sum(diff & ~near))} hard decisions differ away from thresholds"
    assert np.sum(diff) <= max(1, 1e-4 * diff.size)


def n0_f32(N0):
    """The kernel receives N0 as an FP32 argument; the oracle takes that value."""
    return float(np.float32(N0))


def run_detect(fr, C, T, algo, reg="mmse", rho=1.0, sel=None):
    H, y = to_dev(fr.H), to_dev(fr.y)
    s, h, st = api.detect(H, y, fr.N0, C, rho, T, algo=algo, reg=reg, qam=fr.qam, status=True)
    torch.cuda.synchronize()
    s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    assert not np.any(st & STATUS_NONFINITE)
    return s, h, st


def oracle_detect(fr, C, T, algo, reg="mmse", rho=1.0, sel=None):
    Hs = fr.H if sel is None else fr.H[sel]
    ys = fr.y if sel is None else fr.y[sel]
    box_r = O.box_radius(fr.qam)
    if algo == "admm":
        return O.admm_ul_frame(Hs, ys, C, rho, T, n0_f32(fr.N0), reg=reg, box_r=box_r)
    return O.dcg_ul_frame(Hs, ys, C, T, n0_f32(fr.N0), reg=reg)


# -- configuration 1: B=64, C=4, U=8, 16 subcarriers, QPSK, 10 dB, rho=1, T=3, 4 seeds
@pytest.mark.parametrize("seed", range(4))
def test_cfg1_admm(seed):
    say(f"[gpu] cfg1 admm seed={seed}")
    fr = inputs.uplink_frame(inputs.frame_seed(1, seed, 10), 16, 64, 8, 4, 10.0)
    s, h, st = run_detect(fr, 4, 3, "admm")
    ref = oracle_detect(fr, 4, 3, "admm")
    assert rel_err(s, ref) <= 1e-5
    assert per_vec_rel(s, ref) <= 1e-4
    check_hard(s, h, ref, 4, st)


# -- configuration 2: B=128, C=8, U=16, 16-QAM, SNR 0..20, T=5; ADMM and DCG side by side.
# 75 subcarriers (a ragged tail of the 2-subcarrier workgroups) per SNR point.
@pytest.mark.parametrize("snr", [0, 5, 10, 15, 20])
@pytest.mark.parametrize("algo", ["admm", "cg"])
def test_cfg2(snr, algo):
    say(f"[gpu] cfg2 {algo} snr={snr}")
    fr = inputs.uplink_frame(inputs.frame_seed(2, 0, snr), 75, 128, 16, 16, float(snr))
    s, h, st = run_detect(fr, 8, 5, algo)
    ref = oracle_detect(fr, 8, 5, algo)
    assert rel_err(s, ref) <= 1e-5
    assert per_vec_rel(s, ref) <= 1e-4
    nres = check_hard(s, h, ref, 16, st)
    say(f"    re-sliced {nres} of {len(st)} subcarriers")


def test_cfg2_full_size_sampled():
    """1200 subcarriers in one launch; the oracle checks a sample of them."""
    say("[gpu] cfg2 full size sampled")
    fr = inputs.uplink_frame(inputs.frame_seed(2, 1, 10), 1200, 128, 16, 16, 10.0)
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(1200, 48, replace=False))
    for algo in ("admm", "cg"):
        s, h, st = run_detect(fr, 8, 5, algo)
        ref = oracle_detect(fr, 8, 5, algo, sel=sel)
        assert rel_err(s[sel], ref) <= 1e-5
        check_hard(s[sel], h[sel], ref, 16, st[sel])


# -- headline shape: B=256, U=32, 64-QAM, 25 dB, T=5, C=8 (S=32) and C=4 (S=64)
@pytest.mark.parametrize("C", [8, 4])
def test_headline_shape(C):
    say(f"[gpu] headline C={C}")
    fr = inputs.uplink_frame(inputs.frame_seed(6, C, 25), 41, 256, 32, 64, 25.0)
    s, h, st = run_detect(fr, C, 5, "admm")
    ref = oracle_detect(fr, C, 5, "admm")
    assert rel_err(s, ref) <= 1e-5
    assert per_vec_rel(s, ref) <= 1e-4
    check_hard(s, h, ref, 64, st)


# -- configuration 4 shape (B=512, C=8, U=64), FP32 path, i.i.d. and correlated
@pytest.mark.parametrize("corr", [0.0, 0.7])
def test_cfg4_shape_fp32(corr):
    say(f"[gpu] cfg4 fp32 corr={corr}")
    fr = inputs.uplink_frame(inputs.frame_seed(4, 0, 25), 9, 512, 64, 64, 25.0, corr=corr)
    s, h, st = run_detect(fr, 8, 5, "admm")
    ref = oracle_detect(fr, 8, 5, "admm")
    assert rel_err(s, ref) <= 1e-5
    check_hard(s, h, ref, 64, st)


@pytest.mark.parametrize("reg", ["zf", "box"])
def test_other_regularisers(reg):
    say(f"[gpu] reg={reg}")
    fr = inputs.uplink_frame(inputs.frame_seed(7, 0, 15), 21, 64, 8, 16, 15.0)
    s, h, st = run_detect(fr, 4, 4, "admm", reg=reg)
    ref = oracle_detect(fr, 4, 4, "admm", reg=reg)
    assert rel_err(s, ref) <= 1e-5
    check_hard(s, h, ref, 16, st)


def test_cg_zf():
    say("[gpu] cg zf")
    fr = inputs.uplink_frame(inputs.frame_seed(7, 1, 15), 13, 64, 8, 16, 15.0)
    s, h, st = run_detect(fr, 4, 4, "cg", reg="zf")
    ref = oracle_detect(fr, 4, 4, "cg", reg="zf")
    assert rel_err(s, ref) <= 1e-5
    check_hard(s, h, ref, 16, st)


# (54, 16, 3), (99, 32, 3), (195, 64, 3): S = 18, 33, 65 leave a partial last
# row group in the matrix-core Gram prologues, and C = 3 of 4 cluster slots
# leaves an inactive problem in the waves (both read as zero by the range
# check of the buffer loads).
@pytest.mark.parametrize("B,U,C", [(64, 16, 4), (128, 32, 4), (512, 64, 8), (128, 8, 16), (96, 8, 3),
                                   (54, 16, 3), (99, 32, 3), (195, 64, 3)])
@pytest.mark.parametrize("algo", ["admm", "cg"])
def test_shapes(B, U, C, algo):
    say(f"[gpu] shape B={B} U={U} C={C} {algo}")
    fr = inputs.uplink_frame(inputs.frame_seed(8, B + U + C, 10), 11, B, U, 16, 10.0)
    s, h, st = run_detect(fr, C, 3, algo)
    ref = oracle_detect(fr, C, 3, algo)
    assert rel_err(s, ref) <= 1e-5
    check_hard(s, h, ref, 16, st)


def test_multi_symbol_reuse():
    """N_sym = 3 receive vectors share one channel (and one factorisation)."""
    say("[gpu] n_sym=3")
    fr = inputs.uplink_frame(inputs.frame_seed(9, 0, 10), 10, 128, 16, 16, 10.0, n_sym=3)
    for algo in ("admm", "cg"):
        s, h, st = run_detect(fr, 8, 4, algo)
        ref = oracle_detect(fr, 8, 4, algo)
        assert rel_err(s, ref) <= 1e-5
        check_hard(s, h, ref, 16, st)


def test_T1_and_C1():
    say("[gpu] T=1, C=1")
    fr = inputs.uplink_frame(inputs.frame_seed(9, 1, 10), 7, 32, 8, 4, 10.0)
    for C, T in ((1, 1), (1, 4), (4, 1)):
        for algo in ("admm", "cg"):
            s, h, st = run_detect(fr, C, T, algo)
            ref = oracle_detect(fr, C, T, algo)
            assert rel_err(s, ref) <= 1e-5
            check_hard(s, h, ref, 4, st)


def test_empty_batch():
    H = torch.zeros((0, 64, 8), dtype=torch.complex64, device=DEV)
    y = torch.zeros((0, 1, 64), dtype=torch.complex64, device=DEV)
    s, h = api.detect(H, y, 0.1, 4, 1.0, 3)
    assert s.shape == (0, 1, 8)


# Largest shapes the kernels accept: every cluster group of a subcarrier
# shares one 512-lane workgroup (C <= 8 at U = 64, C <= 16 below), B = 1024.
@pytest.mark.parametrize("B,U,C", [(1024, 64, 8), (1024, 32, 16), (1024, 16, 16), (1024, 8, 16)])
@pytest.mark.parametrize("algo", ["admm", "cg"])
def test_max_shapes(B, U, C, algo):
    say(f"[gpu] max shape B={B} U={U} C={C} {algo}")
    fr = inputs.uplink_frame(inputs.frame_seed(12, B + U + C, 15), 5, B, U, 64, 15.0)
    s, h, st = run_detect(fr, C, 5, algo)
    ref = oracle_detect(fr, C, 5, algo)
    assert rel_err(s, ref) <= 1e-5
    check_hard(s, h, ref, 64, st)


@pytest.mark.parametrize("B,U,C", [(512, 64, 8), (512, 32, 16), (256, 32, 8)])
def test_precode_max_shapes(B, U, C):
    say(f"[gpu] precode max shape B={B} U={U} C={C}")
    fr = inputs.downlink_frame(inputs.frame_seed(13, B + U, C), 5, B, U, 64)
    x, _ = api.precode(to_dev(fr.H), to_dev(fr.s), C, 1.0, 5)
    torch.cuda.synchronize()
    ref = O.admm_dl_frame(fr.H, fr.s, C, 1.0, 5)
    err = rel_err(x.cpu().numpy(), ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-5
    assert per_vec_rel(x.cpu().numpy(), ref) <= 1e-4


def test_degenerate_inputs():
    """y = 0 gives s = 0 exactly (every step is linear in y); H = 0 leaves
    B_c = rho I and also gives s = 0; a user whose channel column is zero gets
    s_u = 0 while the others match the oracle."""
    say("[gpu] degenerate inputs")
    fr = inputs.uplink_frame(inputs.frame_seed(14, 0, 10), 9, 128, 16, 16, 10.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    for algo in ("admm", "cg"):
        s, h = api.detect(H, torch.zeros_like(y), fr.N0, 8, 1.0, 5, algo=algo, qam=16)
        s0, _ = api.detect(torch.zeros_like(H), y, fr.N0, 8, 1.0, 5, algo=algo, qam=16)
        torch.cuda.synchronize()
        assert torch.count_nonzero(s).item() == 0
        assert torch.count_nonzero(s0).item() == 0
        assert np.array_equal(h.cpu().numpy(), O.slice_qam_f32(np.zeros(h.shape, np.complex64), 16))
    Hz = fr.H.copy()
    Hz[:, :, 3] = 0
    s, _ = api.detect(to_dev(Hz), y, fr.N0, 8, 1.0, 5, qam=16)
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    ref = O.admm_ul_frame(Hz, fr.y, 8, 1.0, 5, fr.N0)
    assert np.all(s[:, :, 3] == 0) and np.all(ref[:, :, 3] == 0)
    assert rel_err(s, ref) <= 1e-5


def test_nonfinite_status():
    """Per-subcarrier flags are exact for planted NaN / infinite parts, zero
    for a finite result, and set exactly on the subcarriers whose FP32 Gram
    overflows (H scaled by 1e22 there)."""
    say("[gpu] non-finite status")
    x = torch.full((9, 2, 16), 1 + 1j, dtype=torch.complex64, device=DEV)
    x[2, 1, 5] = complex(float("nan"), 0.0)
    x[4, 0, 0] = complex(0.0, float("inf"))
    x[8, 1, 15] = complex(-float("inf"), 1.0)
    assert api.nonfinite_status(x).cpu().tolist() == [0, 0, 1, 0, 1, 0, 0, 0, 1]
    fr = inputs.uplink_frame(inputs.frame_seed(15, 0, 10), 6, 128, 16, 16, 10.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    s, _ = api.detect(H, y, fr.N0, 8, 1.0, 5, qam=16)
    assert api.nonfinite_status(s).cpu().tolist() == [0] * 6
    Hbig = H.clone()
    Hbig[1:3] *= 1e22
    s2, _ = api.detect(Hbig, y, fr.N0, 8, 1.0, 5, qam=16)
    assert api.nonfinite_status(s2).cpu().tolist() == [0, 1, 1, 0, 0, 0]
    assert torch.equal(s2[[0, 3, 4, 5]], s[[0, 3, 4, 5]])


def test_launch_shape_independence():
    """Same inputs as one batch or split in pieces give identical bits."""
    say("[gpu] tiling independence")
    fr = inputs.uplink_frame(inputs.frame_seed(10, 0, 10), 33, 128, 16, 16, 10.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    full, _ = api.detect(H, y, fr.N0, 8, 1.0, 5)
    parts = [api.detect(H[i:i + 7].contiguous(), y[i:i + 7].contiguous(), fr.N0, 8, 1.0, 5)[0] for i in range(0, 33, 7)]
    torch.cuda.synchronize()
    assert torch.equal(full, torch.cat(parts))


# -- configuration 3: downlink B=256, C=16 (S=16), U=32, 64-QAM targets, T=5, power budgets
@pytest.mark.parametrize("budget", [False, True])
def test_cfg3_precode(budget):
    say(f"[gpu] cfg3 precode budget={budget}")
    B, U, C = 256, 32, 16
    fr = inputs.downlink_frame(inputs.frame_seed(3, 0, 0), 37, B, U, 64)
    H, s = to_dev(fr.H), to_dev(fr.s)
    P = None
    # budgets below the typical per-cluster energy (about U / (B - U) / C) so
    # that the common gain is active on most subcarriers
    Pc = [0.007] * C
    if budget:
        P = torch.tensor(Pc, dtype=torch.float32, device=DEV)
    x, beta = api.precode(H, s, C, 1.0, 5, P_cluster=P)
    torch.cuda.synchronize()
    x, beta = x.cpu().numpy(), beta.cpu().numpy()
    ref = O.admm_dl_frame(fr.H, fr.s, C, 1.0, 5)
    if budget:
        refb = np.zeros_like(beta, dtype=np.float64)
        for k in range(ref.shape[0]):
            ref[k, 0], refb[k, 0] = O.power_scale(ref[k, 0], C, Pc)
        assert np.abs(beta - refb).max() <= 1e-5
        assert np.any(refb < 1.0)
    else:
        assert np.all(beta == 1.0)
    assert rel_err(x, ref) <= 1e-5
    assert per_vec_rel(x, ref) <= 1e-4


# -- Lemma 2 with eps > 0 at the configuration-3 shape.  ||s - w|| runs about
# 1.2 .. 2.1 on these frames, so eps = 1.5 leaves the constraint active on some
# subcarriers and iterations and inactive on others; eps = 100 makes it
# inactive everywhere (z_c = w_c).
@pytest.mark.parametrize("eps", [0.5, 1.5, 100.0])
def test_cfg3_precode_eps(eps):
    say(f"[gpu] cfg3 precode eps={eps}")
    B, U, C = 256, 32, 16
    fr = inputs.downlink_frame(inputs.frame_seed(3, 1, 0), 29, B, U, 64)
    H, s = to_dev(fr.H), to_dev(fr.s)
    x, _ = api.precode(H, s, C, 1.0, 5, eps=eps)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    ref = O.admm_dl_frame(fr.H, fr.s, C, 1.0, 5, eps=eps)
    err = rel_err(x, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-5
    assert per_vec_rel(x, ref) <= 1e-4


def test_precode_eps0_is_algorithm3():
    fr = inputs.downlink_frame(inputs.frame_seed(3, 2, 0), 7, 128, 16, 16)
    H, s = to_dev(fr.H), to_dev(fr.s)
    a, _ = api.precode(H, s, 8, 1.0, 5)
    b, _ = api.precode(H, s, 8, 1.0, 5, eps=0.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("B,U,C", [(64, 8, 8), (128, 16, 8), (256, 32, 8), (64, 16, 8), (256, 64, 8)])
def test_precode_shapes(B, U, C):
    say(f"[gpu] precode B={B} U={U} C={C}")
    fr = inputs.downlink_frame(inputs.frame_seed(11, B + U, C), 9, B, U, 16)
    for eps in (0.0, 0.3):
        x, _ = api.precode(to_dev(fr.H), to_dev(fr.s), C, 1.0, 4, eps=eps)
        torch.cuda.synchronize()
        ref = O.admm_dl_frame(fr.H, fr.s, C, 1.0, 4, eps=eps)
        assert rel_err(x.cpu().numpy(), ref) <= 1e-5


# -- mixed precision (split FP16 / BF16 Gram on the matrix cores), U = 32.
# Bar: frame-level relative error <= 1e-3 and hard decisions as above; the FP16
# split is expected to be close to the FP32 path, BF16 looser.  Inverses: FP32
# and split-FP16 matrix cores, FP64 vector units ("auto" is the FP32 inverse
# with the FP64 factor rule at C = 8, where U/S = 1 > 0.8: at rho = 1 no
# cluster is poorly conditioned enough for it; plain FP32 at C = 4).
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("C,factor", [(8, "auto"), (8, "fp32"), (8, "f16x2"), (4, "auto"), (4, "fp64"), (4, "f16x2")])
def test_mixed_headline_shape(prec, C, factor):
    say(f"[gpu] mixed prec={prec} C={C} factor={factor}")
    fr = inputs.uplink_frame(inputs.frame_seed(6, 10 + C, 25), 41, 256, 32, 64, 25.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    s, h, st = api.detect(H, y, fr.N0, C, 1.0, 5, qam=64, prec=prec, factor=factor, status=True)
    torch.cuda.synchronize()
    s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    ref = O.admm_ul_frame(fr.H, fr.y, C, 1.0, 5, n0_f32(fr.N0))
    err = rel_err(s, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= mixed_bar(prec, factor)
    check_hard(s, h, ref, 64, st, mixed_guard(prec, factor, s.shape[-1]))


# A partial last row group (S = 33, 65) and an inactive cluster slot (C = 3 of
# 4) in the split-precision Gram prologues (buffer loads read both as zero).
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("B,U", [(99, 32), (195, 64)])
def test_mixed_ragged_shapes(prec, B, U):
    say(f"[gpu] mixed ragged prec={prec} B={B} U={U} C=3")
    fr = inputs.uplink_frame(inputs.frame_seed(6, 50 + U, 25), 13, B, U, 64, 25.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    s, h, st = api.detect(H, y, fr.N0, 3, 1.0, 5, qam=64, prec=prec, factor="auto", status=True)
    torch.cuda.synchronize()
    s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    ref = O.admm_ul_frame(fr.H, fr.y, 3, 1.0, 5, n0_f32(fr.N0))
    err = rel_err(s, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= mixed_bar(prec, "auto")
    check_hard(s, h, ref, 64, st, mixed_guard(prec, "auto", U))


def mixed_guard(prec, factor, U):
    """Re-slice guard of a mixed mode (slicer units): wider than the FP32
    path's for the split-FP16 inverse and the BF16 Gram."""
    if factor == "f16x2":
        return 2.0 ** -4
    if prec == "bf16":
        return 2.0 ** -8
    return guard_t(U)


def mixed_bar(prec, factor):
    """Frame-level bar of the mixed modes: the FP16 split Gram with an FP32 or
    FP64 inverse stays at the FP32 path's level (1e-5); the split-FP16 inverse
    (FP16 matrix-core accumulation is not correctly rounded under
    cancellation; measured 4e-6 .. 2e-4) and the BF16 Gram are held to the
    low-precision bar of 1e-3."""
    if prec == "bf16" or factor == "f16x2":
        return 1e-3
    return 1e-5


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_correlated_channel(prec):
    say(f"[gpu] mixed correlated prec={prec}")
    fr = inputs.uplink_frame(inputs.frame_seed(4, 1, 25), 23, 256, 32, 64, 25.0, corr=0.7)
    s, h, st = api.detect(to_dev(fr.H), to_dev(fr.y), fr.N0, 8, 1.0, 5, qam=64, prec=prec, status=True)
    torch.cuda.synchronize()
    ref = O.admm_ul_frame(fr.H, fr.y, 8, 1.0, 5, n0_f32(fr.N0))
    assert rel_err(s.cpu().numpy(), ref) <= 1e-3
    check_hard(s.cpu().numpy(), h.cpu().numpy(), ref, 64, st.cpu().numpy(), mixed_guard(prec, "auto", 32))


@pytest.mark.parametrize("prec,factor", [("fp32", None), ("fp16", "auto"), ("bf16", "fp32"), ("fp16", "f16x2"),
                                         ("bf16", "f16x2")])
def test_power_of_two_scaling_bit_exact(prec, factor):
    """(H, y, N0, rho) -> (2^k H, 2^k y, 4^k N0, 4^k rho) leaves the output bits
    unchanged: every step scales exactly, including the mixed path's
    per-cluster power-of-two normalisation."""
    say(f"[gpu] scaling invariance prec={prec}")
    fr = inputs.uplink_frame(inputs.frame_seed(12, 0, 15), 17, 256, 32, 64, 15.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    s0, h0 = api.detect(H, y, fr.N0, 8, 1.0, 5, qam=64, prec=prec, factor=factor)
    s1, h1 = api.detect(H * 4.0, y * 4.0, fr.N0 * 16.0, 8, 16.0, 5, qam=64, prec=prec, factor=factor)
    torch.cuda.synchronize()
    assert torch.equal(s0, s1)
    assert torch.equal(h0, h1)


# -- configuration 4: B=512, C=8 (S=64), U=64, 64-QAM, 25 dB, mixed FP16 / BF16
# Gram with FP32 accumulation; the inverse on the FP32 (default) or split-FP16
# matrix cores (the FP64 inverse is built for U=32 only); i.i.d. and correlated
# 0.7 channels.
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("corr,factor", [(0.0, "auto"), (0.7, "auto"), (0.0, "f16x2"), (0.7, "f16x2")])
def test_cfg4_mixed(prec, corr, factor):
    say(f"[gpu] cfg4 mixed prec={prec} corr={corr} factor={factor}")
    fr = inputs.uplink_frame(inputs.frame_seed(4, 2, 25), 9, 512, 64, 64, 25.0, corr=corr)
    s, h, st = api.detect(to_dev(fr.H), to_dev(fr.y), fr.N0, 8, 1.0, 5, qam=64, prec=prec, factor=factor,
                          status=True)
    torch.cuda.synchronize()
    s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    ref = O.admm_ul_frame(fr.H, fr.y, 8, 1.0, 5, n0_f32(fr.N0))
    err = rel_err(s, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= mixed_bar(prec, factor)
    check_hard(s, h, ref, 64, st, mixed_guard(prec, factor, s.shape[-1]))


# -- the FP64 factor rule of the mixed modes (U/S > 0.8): clusters whose bound
# kappa_hat = tr(B_c) ||B_c^{-1}||_F exceeds 2^14 send their subcarrier to the
# FP64 pass.  A small ADMM penalty rho makes B_c = G_c + rho I poorly
# conditioned at S = U; those subcarriers must come out at FP64 accuracy
# (FP64 result rounded to FP32), the others at the mixed bar.
def _ill_conditioned_frame(B, U, C):
    return inputs.uplink_frame(inputs.frame_seed(19, U, C), 24, B, U, 16, 20.0)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("B,U,C", [(256, 32, 8), (512, 64, 8)])
@pytest.mark.parametrize("hard", [True, False])
def test_fp64_factor_rule(prec, B, U, C, hard):
    say(f"[gpu] FP64 factor rule prec={prec} B={B} U={U} C={C} hard={hard}")
    fr = _ill_conditioned_frame(B, U, C)
    rho = 0.01
    H, y = to_dev(fr.H), to_dev(fr.y)
    s, h, st = api.detect(H, y, fr.N0, C, rho, 5, qam=16, prec=prec, hard=hard, status=True)
    torch.cuda.synchronize()
    s, st = s.cpu().numpy(), st.cpu().numpy()
    ref = O.admm_ul_frame(fr.H, fr.y, C, rho, 5, n0_f32(fr.N0))
    ill = (st & 4) != 0
    say(f"    flagged {int(ill.sum())} of {ill.size}")
    assert ill.any(), "rho = 0.01 at S = U makes some clusters poorly conditioned"
    assert np.all((st[ill] & 2) != 0), "an ill-conditioned subcarrier is recomputed in FP64"
    assert per_vec_rel(s[ill], ref[ill]) <= 1e-6
    assert rel_err(s, ref) <= 1e-3
    if hard:
        # exact decisions everywhere: the guard of the unflagged subcarriers
        # grows with their clusters' kappa_hat, so the FP32 errors that
        # conditioning brings stay inside it
        assert np.array_equal(h.cpu().numpy(), O.slice_qam(ref, 16))
    else:
        assert h is None


@pytest.mark.parametrize("B,U,C", [(256, 32, 8), (512, 64, 8)])
def test_fp64_factor_rule_idle_at_rho_one(B, U, C):
    """At the configurations' rho = 1 the i.i.d. clusters stay far below the
    bound (kappa_hat about 2e3 at U = 32, 8e3 at U = 64): nothing is flagged."""
    say(f"[gpu] FP64 factor rule idle B={B} U={U}")
    fr = inputs.uplink_frame(inputs.frame_seed(19, 1, U), 24, B, U, 64, 25.0)
    s, h, st = api.detect(to_dev(fr.H), to_dev(fr.y), fr.N0, C, 1.0, 5, qam=64, prec="fp16", status=True)
    torch.cuda.synchronize()
    assert not np.any(st.cpu().numpy() & 4)


def test_fp64_factor_explicit_u64():
    """DBP_FACTOR_FP64 at U = 64: every subcarrier recomputed in FP64."""
    say("[gpu] explicit FP64 factor at U = 64")
    fr = inputs.uplink_frame(inputs.frame_seed(19, 2, 64), 6, 512, 64, 64, 25.0)
    s, h, st = api.detect(to_dev(fr.H), to_dev(fr.y), fr.N0, 8, 1.0, 5, qam=64, prec="fp16", factor="fp64",
                          status=True)
    torch.cuda.synchronize()
    s, st = s.cpu().numpy(), st.cpu().numpy()
    assert np.all((st & 6) == 6)
    ref = O.admm_ul_frame(fr.H, fr.y, 8, 1.0, 5, n0_f32(fr.N0))
    assert per_vec_rel(s, ref) <= 1e-6
    check_hard(s, h.cpu().numpy(), ref, 64, st)


def test_fp64_factor_rule_needs_workspace():
    """Through the C ABI: the rule without hard decisions and without a
    workspace is refused before any work is queued."""
    say("[gpu] FP64 factor rule without workspace")
    from paper_1702_04458_amd import _native
    fr = _ill_conditioned_frame(256, 32, 8)
    H, y = to_dev(fr.H), to_dev(fr.y)
    out = torch.empty((H.shape[0], 1, 32), dtype=torch.complex64, device=DEV)
    L = _native.lib()
    code = L.dbp_detect_admm(H.data_ptr(), y.data_ptr(), out.data_ptr(), None, None, None, 0, H.shape[0], 1, 256,
                             32, 8, 5, 0.01, 1.0, float(fr.N0), 1.0, 0, 16, api.PREC["fp16"], None)
    assert code == 1   # DBP_ERR_INVALID
    torch.cuda.synchronize()


def test_output_buffers_validated_before_launch():
    """Output buffers of the wrong shape, dtype or device, a short P_cluster
    or a small workspace are refused on the host (ValueError / TypeError)
    before any kernel is queued."""
    say("[gpu] output buffer validation")
    fr = inputs.uplink_frame(inputs.frame_seed(16, 0, 10), 8, 64, 8, 4, 10.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    good_s = torch.empty((8, 1, 8), dtype=torch.complex64, device=DEV)
    good_h = torch.empty((8, 1, 8), dtype=torch.uint8, device=DEV)
    for bad in ((torch.empty((7, 1, 8), dtype=torch.complex64, device=DEV), good_h),
                (good_s, torch.empty((8, 1, 4), dtype=torch.uint8, device=DEV)),
                (good_s.to(torch.complex128), good_h),
                (good_s, good_h, torch.empty(3, dtype=torch.int32, device=DEV)),
                (good_s.cpu(), good_h)):
        with pytest.raises((ValueError, TypeError)):
            api.detect(H, y, fr.N0, 4, 1.0, 3, qam=4, out=bad)
    with pytest.raises(ValueError):
        api.detect(H, y, fr.N0, 4, 1.0, 3, qam=4, workspace=torch.empty(16, dtype=torch.uint8, device=DEV))
    dl = inputs.downlink_frame(inputs.frame_seed(16, 1, 0), 8, 64, 8, 16)
    with pytest.raises(ValueError):
        api.precode(to_dev(dl.H), to_dev(dl.s), 8, 1.0, 3, P_cluster=torch.ones(4, device=DEV))
    with pytest.raises(ValueError):
        api.precode(to_dev(dl.H), to_dev(dl.s), 8, 1.0, 3,
                    out=(torch.empty((8, 1, 32), dtype=torch.complex64, device=DEV),
                         torch.empty((8, 1), dtype=torch.float32, device=DEV)))
    # the good buffers still work
    s, h = api.detect(H, y, fr.N0, 4, 1.0, 3, qam=4, out=(good_s, good_h))
    torch.cuda.synchronize()
    assert rel_err(s.cpu().numpy(), O.admm_ul_frame(fr.H, fr.y, 4, 1.0, 3, fr.N0)) <= 1e-5


def test_reslice_recomputes_in_fp64():
    """A guard-band subcarrier is recomputed in FP64: planted receive vectors
    whose exact soft value sits on a decision threshold (y = H s with s a
    midpoint between two points, ZF, so that s_hat = s exactly in exact
    arithmetic) are flagged, and their soft outputs equal the FP64 oracle's
    rounded to FP32 while the others keep the FP32 path's result."""
    say("[gpu] re-slice of planted threshold values")
    B, U, C, n_sc = 128, 16, 4, 24       # T = 60 brings these within 6e-5 of the threshold (slicer units)
    fr = inputs.uplink_frame(inputs.frame_seed(17, 0, 20), n_sc, B, U, 16, 20.0)
    Hs = fr.H.astype(np.complex128)
    y = fr.y.copy()
    mid = 2.0 / math.sqrt(10.0)           # 16-QAM threshold between the two upper levels
    planted = [3, 11, 17]
    for k in planted:
        s = np.full(U, 0.3 + 0.3j)
        s[5] = mid + 0.1j
        y[k, 0] = (Hs[k] @ s).astype(np.complex64)
    s_hat, h, st = api.detect(to_dev(fr.H), to_dev(y), 0.0, C, 1.0, 60, reg="zf", qam=16, status=True)
    torch.cuda.synchronize()
    s_hat, h, st = s_hat.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    for k in planted:
        assert st[k] & STATUS_RESLICED, k
    ref = O.admm_ul_frame(fr.H, y, C, 1.0, 60, 0.0, reg="zf")
    for k in np.flatnonzero(st & STATUS_RESLICED):
        assert np.array_equal(s_hat[k], ref[k].astype(np.complex64)) or \
            np.abs(s_hat[k] - ref[k]).max() <= 2.0 ** -23 * np.abs(ref[k]).max()
    assert np.array_equal(h, O.slice_qam(ref, 16))


# -- budgeted step (P1): every x-update meets ||x_c||^2 <= P_c exactly
@pytest.mark.parametrize("B,U,C", [(256, 32, 16), (128, 16, 16), (64, 8, 8), (128, 16, 8), (256, 64, 8)])
def test_precode_per_cluster_budget(B, U, C):
    say(f"[gpu] precode budgeted P1 B={B} U={U} C={C}")
    S = B // C
    fr = inputs.downlink_frame(inputs.frame_seed(18, B + U, C), 23, B, U, 64)
    # budgets below the unconstrained per-cluster energy on most subcarriers
    free = O.admm_dl_frame(fr.H[:6], fr.s[:6], C, 1.0, 5)
    e = np.array([[np.sum(np.abs(free[k, 0, c * S:(c + 1) * S]) ** 2) for c in range(C)] for k in range(6)])
    Pc = [float(np.float32(0.5 * np.median(e) * (1.0 + 0.2 * (c % 3)))) for c in range(C)]
    P = torch.tensor(Pc, dtype=torch.float32, device=DEV)
    x, beta = api.precode(to_dev(fr.H), to_dev(fr.s), C, 1.0, 5, P_cluster=P, power="per_cluster")
    torch.cuda.synchronize()
    x, beta = x.cpu().numpy(), beta.cpu().numpy()
    ref = O.admm_dl_frame(fr.H, fr.s, C, 1.0, 5, P=Pc)
    err = rel_err(x, ref)
    en = np.array([[np.sum(np.abs(ref[k, 0, c * S:(c + 1) * S]) ** 2) for c in range(C)] for k in range(23)])
    active = np.mean(en >= np.array(Pc) * (1 - 1e-9))
    say(f"    rel_err={err:.2e}, budget active on {active:.0%} of (subcarrier, cluster) at the last step")
    assert active > 0.3
    assert err <= 1e-5
    assert per_vec_rel(x, ref) <= 1e-4
    assert np.all(beta == 1.0)
    for k in range(23):
        for c in range(C):
            assert np.sum(np.abs(x[k, 0, c * S:(c + 1) * S]) ** 2) <= Pc[c] * (1 + 1e-5)


def test_precode_budget_that_never_binds():
    """Budgets far above every cluster's energy: the budgeted form takes the
    unconstrained step everywhere (Algorithm 3)."""
    fr = inputs.downlink_frame(inputs.frame_seed(18, 1, 0), 17, 256, 32, 64)
    P = torch.full((16,), 1e6, dtype=torch.float32, device=DEV)
    x, _ = api.precode(to_dev(fr.H), to_dev(fr.s), 16, 1.0, 5, P_cluster=P, power="per_cluster")
    x0, _ = api.precode(to_dev(fr.H), to_dev(fr.s), 16, 1.0, 5)
    torch.cuda.synchronize()
    assert rel_err(x.cpu().numpy(), x0.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("B,U,C", [(256, 32, 16), (128, 16, 8), (256, 64, 8)])
def test_precode_downlink_layout(B, U, C):
    """H given as the downlink channel H^d [n_sc][U][B] (the transpose of the
    uplink layout, made contiguous) gives the same precoder output as the
    uplink layout read in place, with and without budgets."""
    say(f"[gpu] precode downlink-native layout B={B} U={U} C={C}")
    fr = inputs.downlink_frame(inputs.frame_seed(19, B + U, C), 13, B, U, 64)
    Hu = to_dev(fr.H)
    Hd = Hu.transpose(1, 2).contiguous()
    s = to_dev(fr.s)
    P = torch.full((C,), 0.01, dtype=torch.float32, device=DEV)
    for kw in ({}, {"P_cluster": P, "power": "per_cluster"}, {"eps": 0.3}):
        xu, _ = api.precode(Hu, s, C, 1.0, 5, **kw)
        xd, _ = api.precode(Hd, s, C, 1.0, 5, layout="downlink", **kw)
        torch.cuda.synchronize()
        assert rel_err(xd.cpu().numpy(), xu.cpu().numpy()) <= 1e-6
    ref = O.admm_dl_frame(fr.H, fr.s, C, 1.0, 5)
    xd, _ = api.precode(Hd, s, C, 1.0, 5, layout="downlink")
    torch.cuda.synchronize()
    assert rel_err(xd.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("kind", ["admm", "cg"])
def test_autotune_keeps_results(kind):
    """The autotuner picks a launch plan by timing; detection results are the
    same bits under every plan."""
    say(f"[gpu] autotune {kind}")
    fr = inputs.uplink_frame(inputs.frame_seed(20, 0, 10), 600, 128, 16, 16, 10.0)
    H, y = to_dev(fr.H), to_dev(fr.y)
    before, hb = api.detect(H, y, fr.N0, 8, 1.0, 5, algo=kind, qam=16)
    scratch = torch.empty_like(before)
    best = api.autotune(kind, H, y, scratch, 8, 5, reps=3)
    assert best in (1, 2, 4, 8) and api.autotune_get(kind, 16, 8) == best
    after, ha = api.detect(H, y, fr.N0, 8, 1.0, 5, algo=kind, qam=16)
    torch.cuda.synchronize()
    say(f"    chose {best} waves minimum")
    assert torch.equal(before, after) and torch.equal(hb, ha)


def test_detect_batch_uneven_frames():
    """Frames of one U with different B, C, subcarrier counts, symbols, T,
    QAM and regularisers in one launch: every output bit equals the
    single-frame call, and decisions equal the oracle's."""
    say("[gpu] uneven batch")
    specs = [(256, 32, 8, 300, 64, 25.0, 5, "mmse", 1), (128, 32, 4, 72, 16, 0.0, 5, "mmse", 1),
             (512, 32, 16, 600, 64, 10.0, 3, "zf", 2), (256, 32, 4, 1, 16, 5.0, 4, "box", 1),
             (64, 32, 2, 37, 4, 0.0, 5, "mmse", 1)]
    frames, refs = [], []
    for i, (B, U, C, n_sc, qam, snr, T, reg, n_sym) in enumerate(specs):
        fr = inputs.uplink_frame(inputs.frame_seed(60, i, int(snr)), n_sc, B, U, qam, snr, n_sym=n_sym)
        frames.append(dict(H=to_dev(fr.H), y=to_dev(fr.y), N0=fr.N0, C=C, T=T, qam=qam, reg=reg, status=True))
        refs.append(fr)
    out = api.detect_batch(frames)
    single = [api.detect(f["H"], f["y"], f["N0"], f["C"], 1.0, f["T"], qam=f["qam"], reg=f["reg"], status=True)
              for f in frames]
    torch.cuda.synchronize()
    for (s, h, st), (s1, h1, st1), f, fr in zip(out, single, frames, refs):
        assert torch.equal(s, s1) and torch.equal(h, h1) and torch.equal(st, st1)
        ref = O.admm_ul_frame(fr.H, fr.y, f["C"], 1.0, f["T"], n0_f32(fr.N0), reg=f["reg"],
                              box_r=O.box_radius(fr.qam))
        assert rel_err(s.cpu().numpy(), ref) <= 1e-5
        assert np.array_equal(h.cpu().numpy(), O.slice_qam(ref, fr.qam))
    with pytest.raises(ValueError):
        api.detect_batch([frames[0], dict(H=to_dev(inputs.uplink_frame(1, 4, 64, 16, 4, 10.0).H),
                                          y=to_dev(inputs.uplink_frame(1, 4, 64, 16, 4, 10.0).y), N0=0.1, C=4)])
