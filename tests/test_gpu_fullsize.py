"""Full-size launches as the benchmark times them, checked on sampled outputs
the FP64 oracle computes one by one, and hard decisions identical to the
oracle's on every symbol of whole frames (all five configuration-2 SNRs for
ADMM and CG, the headline shape, configuration 1)."""
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

from test_gpu_parity import STATUS_RESLICED, check_hard, n0_f32, rel_err, to_dev  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def device_frame(n_sc, B, U, qam, snr_db, seed):
    """Seeded frame generated on the device (same distribution as the input
    recipe: CN(0,1) channel, unit-energy QAM, N0 = U / SNR)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    L = inputs.qam_side(qam)
    kappa = inputs.qam_kappa(qam)
    sd = 0.5 ** 0.5
    H = torch.complex(torch.randn(n_sc, B, U, device="cuda", generator=g) * sd,
                      torch.randn(n_sc, B, U, device="cuda", generator=g) * sd)
    iI = torch.randint(0, L, (n_sc, U), device="cuda", generator=g)
    iQ = torch.randint(0, L, (n_sc, U), device="cuda", generator=g)
    s = torch.complex((2 * iI - (L - 1)).float() / kappa, (2 * iQ - (L - 1)).float() / kappa)
    N0 = U / 10.0 ** (snr_db / 10.0)
    nsd = (N0 / 2) ** 0.5
    n = torch.complex(torch.randn(n_sc, B, device="cuda", generator=g) * nsd,
                      torch.randn(n_sc, B, device="cuda", generator=g) * nsd)
    y = (torch.matmul(H, s.unsqueeze(-1)).squeeze(-1) + n).unsqueeze(1).contiguous()
    return H.contiguous(), y, N0


@pytest.mark.parametrize("algo,B,U,C,qam,snr", [("admm", 256, 32, 8, 64, 25.0), ("admm", 128, 16, 8, 16, 10.0),
                                                ("cg", 128, 16, 8, 16, 10.0), ("admm", 512, 64, 8, 64, 25.0)])
def test_bench_launch_sampled(algo, B, U, C, qam, snr):
    """38,400 subcarriers (32 frames of 1200) in one launch, the benchmark's
    step; 48 sampled subcarriers, including the first and the last, against
    the oracle."""
    say(f"[gpu] full-size launch {algo} B={B} U={U} C={C}")
    n_sc = 38400
    H, y, N0 = device_frame(n_sc, B, U, qam, snr, seed=77 + U)
    s, h, st = api.detect(H, y, N0, C, 1.0, 5, algo=algo, qam=qam, status=True)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    resliced = np.flatnonzero(st & STATUS_RESLICED)
    say(f"    re-sliced {len(resliced)} of {n_sc} subcarriers")
    rng = np.random.default_rng(U)
    # the sample includes re-sliced subcarriers (FP64 outputs) when there are any
    sel = np.unique(np.concatenate([[0, n_sc - 1], rng.choice(n_sc, 46, replace=False), resliced[:8]]))
    Hs = H[sel].cpu().numpy()
    ys = y[sel].cpu().numpy()
    if algo == "admm":
        ref = O.admm_ul_frame(Hs, ys, C, 1.0, 5, n0_f32(N0))
    else:
        ref = O.dcg_ul_frame(Hs, ys, C, 5, n0_f32(N0))
    ss, hs = s[sel].cpu().numpy(), h[sel].cpu().numpy()
    err = rel_err(ss, ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-5
    check_hard(ss, hs, ref, qam, st[sel])


def test_precode_bench_launch_sampled():
    """Downlink at B=256, U=32, C=16: 38,400 subcarriers in one launch, the
    benchmark's step, with per-cluster budgets; 48 sampled subcarriers
    against the oracle."""
    say("[gpu] full-size launch precode B=256 U=32 C=16")
    n_sc, B, U, C = 38400, 256, 32, 16
    g = torch.Generator(device="cuda")
    g.manual_seed(91)
    L, kappa = inputs.qam_side(64), inputs.qam_kappa(64)
    sd = 0.5 ** 0.5
    H = torch.complex(torch.randn(n_sc, B, U, device="cuda", generator=g) * sd,
                      torch.randn(n_sc, B, U, device="cuda", generator=g) * sd).contiguous()
    iI = torch.randint(0, L, (n_sc, 1, U), device="cuda", generator=g)
    iQ = torch.randint(0, L, (n_sc, 1, U), device="cuda", generator=g)
    s = torch.complex((2 * iI - (L - 1)).float() / kappa, (2 * iQ - (L - 1)).float() / kappa).contiguous()
    Pc = [0.007] * C
    x, beta = api.precode(H, s, C, 1.0, 5, P_cluster=torch.tensor(Pc, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    sel = np.unique(np.concatenate([[0, n_sc - 1], np.random.default_rng(5).choice(n_sc, 46, replace=False)]))
    Hs, ss = H[sel].cpu().numpy(), s[sel].cpu().numpy()
    ref = O.admm_dl_frame(Hs, ss, C, 1.0, 5)
    refb = np.zeros((len(sel), 1))
    for i in range(len(sel)):
        ref[i, 0], refb[i, 0] = O.power_scale(ref[i, 0], C, Pc)
    err = rel_err(x[sel].cpu().numpy(), ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-5
    assert np.abs(beta[sel].cpu().numpy() - refb).max() <= 1e-5


def test_precode_budget_bench_launch_sampled():
    """Configuration 3 with the budgeted step (P1): 38,400 subcarriers in one
    launch, 48 sampled subcarriers against the oracle."""
    say("[gpu] full-size launch budgeted precode B=256 U=32 C=16")
    n_sc, B, U, C = 38400, 256, 32, 16
    g = torch.Generator(device="cuda")
    g.manual_seed(92)
    L, kappa = inputs.qam_side(64), inputs.qam_kappa(64)
    sd = 0.5 ** 0.5
    H = torch.complex(torch.randn(n_sc, B, U, device="cuda", generator=g) * sd,
                      torch.randn(n_sc, B, U, device="cuda", generator=g) * sd).contiguous()
    iI = torch.randint(0, L, (n_sc, 1, U), device="cuda", generator=g)
    iQ = torch.randint(0, L, (n_sc, 1, U), device="cuda", generator=g)
    s = torch.complex((2 * iI - (L - 1)).float() / kappa, (2 * iQ - (L - 1)).float() / kappa).contiguous()
    Pc = [0.005] * C
    x, _ = api.precode(H, s, C, 1.0, 5, P_cluster=torch.tensor(Pc, dtype=torch.float32, device="cuda"),
                       power="per_cluster")
    torch.cuda.synchronize()
    sel = np.unique(np.concatenate([[0, n_sc - 1], np.random.default_rng(6).choice(n_sc, 46, replace=False)]))
    ref = O.admm_dl_frame(H[sel].cpu().numpy(), s[sel].cpu().numpy(), C, 1.0, 5, P=Pc)
    err = rel_err(x[sel].cpu().numpy(), ref)
    say(f"    rel_err={err:.2e}")
    assert err <= 1e-5


WHOLE_FRAMES = ([("admm", 128, 16, 8, 16, snr) for snr in (0.0, 5.0, 10.0, 15.0, 20.0)]
                + [("cg", 128, 16, 8, 16, snr) for snr in (0.0, 5.0, 10.0, 15.0, 20.0)]
                + [("admm", 256, 32, 8, 64, 25.0), ("admm", 256, 32, 8, 64, 15.0), ("admm", 64, 8, 4, 4, 10.0)])


@pytest.mark.parametrize("algo,B,U,C,qam,snr", WHOLE_FRAMES)
def test_hard_decisions_identical_on_whole_frames(algo, B, U, C, qam, snr):
    """Every symbol of a 1200-subcarrier frame equals the oracle's FP64
    decision; the number of subcarriers the FP64 re-slice recomputed is
    printed."""
    say(f"[gpu] whole-frame decisions {algo} B={B} U={U} C={C} snr={snr}")
    fr = inputs.uplink_frame(inputs.frame_seed(31, U, int(snr)), 1200, B, U, qam, snr)
    T = 5 if B > 64 else 3
    s, h, st = api.detect(to_dev(fr.H), to_dev(fr.y), fr.N0, C, 1.0, T, algo=algo, qam=qam, status=True)
    torch.cuda.synchronize()
    s, h, st = s.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    if algo == "admm":
        ref = O.admm_ul_frame(fr.H, fr.y, C, 1.0, T, n0_f32(fr.N0))
    else:
        ref = O.dcg_ul_frame(fr.H, fr.y, C, T, n0_f32(fr.N0))
    assert rel_err(s, ref) <= 1e-5
    n = check_hard(s, h, ref, qam, st)
    say(f"    0 of {h.size} decisions differ; {n} of 1200 subcarriers re-sliced in FP64")
