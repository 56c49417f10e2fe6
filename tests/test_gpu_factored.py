"""Resident factorisation (dbp_factor_admm + dbp_detect_admm_factored) on the
GPU: a static channel is factored once and several received frames are
detected against it; every result is checked against the FP64 oracle with the
FP32 bars of test_gpu_parity, and against the one-shot dbp_detect_admm."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import dbp_oracle as O  # noqa: E402
from paper_1702_04458_amd import inputs  # noqa: E402

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1702_04458_amd import api  # noqa: E402

from test_gpu_parity import check_hard, check_hard_low_precision, n0_f32, per_vec_rel, rel_err, to_dev  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


# (B, U, C, n_sc, qam, snr): the configurations' shapes, a ragged subcarrier
# count, C = 3 / 6 (padding cluster slots in the workgroup), and U = 32 with
# S = 36 and S = 45 antennas per cluster (row counts that end inside the
# Gram's prefetch chunks)
SHAPES = [(256, 32, 8, 40, 64, 25.0), (128, 16, 8, 75, 16, 10.0), (64, 8, 4, 16, 4, 10.0),
          (512, 64, 8, 9, 64, 25.0), (96, 16, 3, 37, 16, 15.0), (384, 32, 6, 11, 64, 20.0),
          (72, 32, 2, 5, 16, 15.0), (90, 32, 2, 4, 64, 20.0)]


@pytest.mark.parametrize("B,U,C,n_sc,qam,snr", SHAPES)
def test_factor_once_detect_many(B, U, C, n_sc, qam, snr):
    say(f"[gpu] factored B={B} U={U} C={C} n_sc={n_sc}")
    fr = inputs.uplink_frame(inputs.frame_seed(21, B + U + C, int(snr)), n_sc, B, U, qam, snr, n_sym=3)
    H = to_dev(fr.H)
    fac = api.factor(H, C, 1.0)
    ref = O.admm_ul_frame(fr.H, fr.y, C, 1.0, 5, n0_f32(fr.N0))
    # three frames received over the same channel, one call each
    for n in range(3):
        y = to_dev(fr.y[:, n:n + 1])
        s, h, st = api.detect_factored(H, fac, y, fr.N0, C, 1.0, 5, qam=qam, status=True)
        s1, h1 = api.detect(H, y, fr.N0, C, 1.0, 5, qam=qam)
        torch.cuda.synchronize()
        s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
        err = rel_err(s, ref[:, n:n + 1])
        say(f"    frame {n}: rel_err={err:.2e}")
        assert err <= 1e-5
        assert per_vec_rel(s, ref[:, n:n + 1]) <= 1e-4
        check_hard(s, h, ref[:, n:n + 1], qam, st)
        assert rel_err(s, s1.cpu().numpy()) <= 1e-5
        assert np.array_equal(h, h1.cpu().numpy())
    # and all three in one call (N_sym = 3)
    s3, h3, st3 = api.detect_factored(H, fac, to_dev(fr.y), fr.N0, C, 1.0, 5, qam=qam, status=True)
    torch.cuda.synchronize()
    assert rel_err(s3.cpu().numpy(), ref) <= 1e-5
    check_hard(s3.cpu().numpy(), h3.cpu().numpy(), ref, qam, st3.cpu().numpy())


@pytest.mark.parametrize("prec,factor", [("fp16", "fp32"), ("bf16", "fp32"), ("fp16", "fp64")])
def test_mixed_precision_factors(prec, factor):
    """Factors made by the mixed-precision preprocessing serve the same FP32
    iterations (headline shape, B=256, U=32, C=8)."""
    say(f"[gpu] factored mixed prec={prec} factor={factor}")
    fr = inputs.uplink_frame(inputs.frame_seed(22, 1, 25), 29, 256, 32, 64, 25.0)
    H = to_dev(fr.H)
    fac = api.factor(H, 8, 1.0, prec=prec, factor=factor)
    s, h, st = api.detect_factored(H, fac, to_dev(fr.y), fr.N0, 8, 1.0, 5, qam=64, status=True)
    torch.cuda.synchronize()
    ref = O.admm_ul_frame(fr.H, fr.y, 8, 1.0, 5, n0_f32(fr.N0))
    s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    err = rel_err(s, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= (1e-5 if prec == "fp16" else 1e-3)
    if prec == "fp16":
        check_hard(s, h, ref, 64, st)
    else:
        # decisions identical anyway (re-sliced subcarriers are FP64); the
        # BF16-Gram factors are a low-precision path for the FP32 outputs
        assert np.array_equal(h, O.slice_qam(ref, 64))


@pytest.mark.parametrize("B,U,C,n_sc", [(128, 16, 8, 6), (256, 32, 8, 3), (72, 32, 2, 3), (90, 32, 2, 3)])
def test_factors_match_oracle_inverse(B, U, C, n_sc):
    """The stored blocks are B_c^{-1} = (H_c^H H_c + rho I)^{-1}: the library's
    internal layout holds the upper triangle of block (k, c) column by column,
    entry (i, v) with i <= v at v (v + 1) / 2 + i."""
    say(f"[gpu] factors vs oracle inverse B={B} U={U} C={C} n_sc={n_sc}")
    fr = inputs.uplink_frame(inputs.frame_seed(23, B + U, C), n_sc, B, U, 16, 10.0)
    fac = api.factor(to_dev(fr.H), C, 0.7).cpu().numpy()          # [n_sc, C, U (U + 1) / 2] as stored
    assert fac.shape == (n_sc, C, U * (U + 1) // 2)
    S = B // C
    for k in range(n_sc):
        for c in range(C):
            Hc = fr.H[k, c * S:(c + 1) * S].astype(np.complex128)
            Binv = np.linalg.inv(Hc.conj().T @ Hc + 0.7 * np.eye(U))
            stored = np.zeros((U, U), dtype=np.complex128)
            for v in range(U):
                for i in range(v + 1):
                    stored[i, v] = fac[k, c, v * (v + 1) // 2 + i]
                    stored[v, i] = np.conj(fac[k, c, v * (v + 1) // 2 + i])
            assert np.linalg.norm(stored - Binv) <= 1e-5 * np.linalg.norm(Binv)


# -- mixed-precision resident channel: H packed as complex FP16 with one
# power-of-two scale per (subcarrier, cluster) tile, FP32 factors and FP32
# iterations (dbp_pack_channel_h16 + dbp_detect_admm_factored_h16).

def decode_h16(packed, n_sc, B, U, C):
    raw = packed.cpu().numpy()
    n = n_sc * B * U
    halves = raw[:4 * n].view(np.float16).astype(np.float64).reshape(n_sc, B, U, 2)   # real part in the low half
    scale = raw[4 * n:].view(np.float32).reshape(n_sc, C)
    return halves[..., 0] + 1j * halves[..., 1], scale


@pytest.mark.parametrize("B,U,C,n_sc", [(128, 16, 8, 7), (1024, 64, 8, 5)])
def test_pack_h16_format(B, U, C, n_sc):
    """Bit-exact against the definition: e = floor(log2 m) - 14 for the tile's
    largest |component| m (e = 0 for an all-zero tile), entries rounded to
    nearest even in binary16 after scaling by 2^-e; tiles spanning 1e-30 .. 1e20,
    held in registers (16 x 16 tiles) or read twice (128 x 64 tiles)."""
    say(f"[gpu] pack_h16 format B={B} U={U} C={C}")
    S = B // C
    fr = inputs.uplink_frame(inputs.frame_seed(24, 0, 10), n_sc, B, U, 16, 10.0)
    H = fr.H.astype(np.complex64)
    H[2, S:2 * S] *= np.float32(1e-30)
    H[3, 0:S] = 0
    H[4, 2 * S:3 * S] *= np.float32(1e20)
    packed = api.pack_channel_h16(to_dev(H), C)
    torch.cuda.synchronize()
    h16, scale = decode_h16(packed, n_sc, B, U, C)
    for k in range(n_sc):
        for c in range(C):
            tile = H[k, c * S:(c + 1) * S]
            m = float(max(np.abs(tile.real).max(), np.abs(tile.imag).max()))
            e = 0 if m == 0 else max(math.floor(math.log2(m)) - 14, -126)
            assert scale[k, c] == 2.0 ** e, (k, c, scale[k, c], e)
            want_re = np.ldexp(tile.real.astype(np.float64), -e).astype(np.float16)
            want_im = np.ldexp(tile.imag.astype(np.float64), -e).astype(np.float16)
            got = h16[k, c * S:(c + 1) * S]
            assert np.array_equal(got.real, want_re.astype(np.float64)), (k, c)
            assert np.array_equal(got.imag, want_im.astype(np.float64)), (k, c)


@pytest.mark.parametrize("B,U,C,n_sc", [(256, 32, 8, 12), (72, 32, 2, 5), (90, 32, 2, 4), (128, 16, 8, 6),
                                        (512, 64, 8, 3)])
def test_factor_h16_one_call(B, U, C, n_sc):
    """dbp_factor_admm_h16 gives the factors of dbp_factor_admm and the packed
    channel of dbp_pack_channel_h16 bit for bit (one launch at U = 32, the two
    calls in turn otherwise)."""
    say(f"[gpu] factor + pack in one call B={B} U={U} C={C} n_sc={n_sc}")
    fr = inputs.uplink_frame(inputs.frame_seed(25, B + U, C), n_sc, B, U, 16, 10.0)
    H = to_dev(fr.H)
    f1 = api.factor(H, C, 0.8)
    p1 = api.pack_channel_h16(H, C)
    f2, p2 = api.factor_h16(H, C, 0.8)
    torch.cuda.synchronize()
    assert np.array_equal(f1.cpu().numpy().view(np.uint32), f2.cpu().numpy().view(np.uint32))
    assert np.array_equal(p1.cpu().numpy(), p2.cpu().numpy())


def test_factor_h16_one_call_extreme_tiles():
    """The packed channel of the one-launch form at tiles spanning 1e-30 ..
    1e20 and an all-zero tile equals dbp_pack_channel_h16's, byte for byte."""
    say("[gpu] factor + pack in one call, extreme tiles")
    B, U, C, n_sc = 256, 32, 8, 6
    S = B // C
    fr = inputs.uplink_frame(inputs.frame_seed(26, 0, 10), n_sc, B, U, 16, 10.0)
    Hn = fr.H.astype(np.complex64)
    Hn[2, S:2 * S] *= np.float32(1e-30)
    Hn[3, 0:S] = 0
    Hn[4, 2 * S:3 * S] *= np.float32(1e20)
    H = to_dev(Hn)
    p1 = api.pack_channel_h16(H, C)
    _, p2 = api.factor_h16(H, C, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(p1.cpu().numpy(), p2.cpu().numpy())


@pytest.mark.parametrize("B,U,C,n_sc,qam,snr", SHAPES)
def test_factored_h16(B, U, C, n_sc, qam, snr):
    """Low-precision bar (frame error <= 1e-3 against the FP64 oracle) and the
    hard-decision rule of the low-precision paths (not re-sliced)."""
    say(f"[gpu] factored h16 B={B} U={U} C={C} n_sc={n_sc}")
    fr = inputs.uplink_frame(inputs.frame_seed(25, B + U + C, int(snr)), n_sc, B, U, qam, snr, n_sym=2)
    H = to_dev(fr.H)
    fac = api.factor(H, C, 1.0)
    packed = api.pack_channel_h16(H, C)
    s, h = api.detect_factored_h16(packed, fac, to_dev(fr.y), fr.N0, B, U, C, 1.0, 5, qam=qam)
    torch.cuda.synchronize()
    s, h = s.cpu().numpy(), h.cpu().numpy()
    ref = O.admm_ul_frame(fr.H, fr.y, C, 1.0, 5, fr.N0)
    err = rel_err(s, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-3
    check_hard_low_precision(s, h, ref, qam)


def test_factored_h16_headline_and_scaling():
    """B=256, U=32, C=8 at 25 dB: within 1e-3 of the oracle (about 2e-4
    expected from rounding H to 11 significant bits), and bit-identical under
    (H, y, N0, rho) -> (4H, 4y, 16N0, 16rho): the tile exponents absorb the
    factor 4 exactly."""
    say("[gpu] factored h16 headline shape")
    fr = inputs.uplink_frame(inputs.frame_seed(26, 1, 25), 41, 256, 32, 64, 25.0)
    outs = []
    for f in (1.0, 4.0):
        H = to_dev(fr.H) * f
        fac = api.factor(H, 8, f * f)
        packed = api.pack_channel_h16(H, 8)
        outs.append(api.detect_factored_h16(packed, fac, to_dev(fr.y) * f, fr.N0 * f * f, 256, 32, 8, f * f, 5,
                                            qam=64))
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    s, h = outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()
    ref = O.admm_ul_frame(fr.H, fr.y, 8, 1.0, 5, fr.N0)
    err = rel_err(s, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-3
    check_hard_low_precision(s, h, ref, 64)
