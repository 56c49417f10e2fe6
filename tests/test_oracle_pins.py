"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these compare the oracle with itself: each uses a hand-worked example,
an exact-arithmetic run, an independent formulation of the same steps (generic
least squares / projection), a closed-form limit, a library routine or brute
force.  They run on the CPU only.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import dbp_oracle as O
from oracle import ml as ML
from oracle import rational as R
from paper_1702_04458_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def cplx(rows):
    return np.array([complex(a, b) for a, b in rows])


# --------------------------------------------------------------------------
# Hand-worked examples (golden fixtures)
# --------------------------------------------------------------------------

def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_alg1_hand_examples():
    g = _load("hand_examples.json")
    for key in ("alg1_zf_two_clusters", "alg1_zf_equal_clusters"):
        ex = g[key]
        H = cplx(ex["H"]).reshape(-1, 1)
        y = cplx(ex["y"])
        for T, (num, den) in ex["s_by_T"].items():
            s = O.admm_ul(H, y, ex["C"], ex["rho"], int(T), ex["N0"], reg="zf")
            assert abs(s[0] - num / den) < 1e-15, (key, T)
            r = R.admm_ul(H.tolist(), y.tolist(), ex["C"], ex["rho"], int(T), ex["N0"])
            assert Fraction(r[0].real).limit_denominator(10**6) == Fraction(num, den)


def test_alg2_hand_example():
    ex = _load("hand_examples.json")["alg2_scalar"]
    H = cplx(ex["H"]).reshape(-1, 1)
    y = cplx(ex["y"])
    x = O.dcg_ul(H, y, ex["C"], 1, ex["N0"], reg="zf")
    assert abs(x[0] - 1.0) < 1e-15


def test_alg3_hand_example():
    ex = _load("hand_examples.json")["alg3_two_clusters"]
    Hu = cplx(ex["Hu"]).reshape(-1, 1)
    s = cplx(ex["s"])
    for T, vals in ex["x_by_T"].items():
        x = O.admm_dl(Hu, s, ex["C"], ex["rho"], int(T))
        want = np.array([n / d for n, d in vals])
        assert np.abs(x - want).max() < 1e-15, T


# --------------------------------------------------------------------------
# Constellation and slicer
# --------------------------------------------------------------------------

def test_qam_levels_textbook():
    g = _load("qam_textbook.json")
    for M in (4, 16, 64):
        lv = O.qam_levels(M)
        want = np.array(g[str(M)]["amplitudes"]) / math.sqrt(g[str(M)]["norm_sq"])
        assert np.abs(lv - want).max() < 1e-15
        pts = ML.alphabet(M)
        assert abs(np.mean(np.abs(pts) ** 2) - 1.0) < 1e-14        # Es = 1
        assert abs(O.box_radius(M) - lv[-1]) == 0.0


@pytest.mark.parametrize("M", [4, 16, 64])
def test_slicer_is_nearest_point(M):
    rng = np.random.default_rng(M)
    x = 1.6 * cn(rng, 5000)
    idx = O.slice_qam(x, M)
    pts = ML.alphabet(M)                                 # index a*L + b -> (lv[a], lv[b])
    L = int(math.sqrt(M))
    d = np.abs(x[:, None] - pts[None, :])
    near = np.argmin(d, axis=1)
    # ML.alphabet orders by (real index a, imag index b) -> a * L + b; slicer packs iI + L*iQ
    a, b = near // L, near % L
    assert np.array_equal(idx.astype(int), a + L * b)


def test_slicer_ties_and_clamp():
    # thresholds for 16-QAM are at 0 and +-2/sqrt(10); ties go to the upper level
    k = math.sqrt(10.0)
    x = np.array([0.0, 2 / k, -2 / k, 100.0, -100.0]) + 0j
    assert list(O.slice_qam(x, 16) % 4) == [2, 3, 1, 3, 0]
    assert list(O.slice_qam_f32(np.float32(x.real) + 0j, 16) % 4)[0] == 2
    # transmitted points slice to themselves (noiseless)
    rng = np.random.default_rng(3)
    for M in (4, 16, 64):
        L = int(math.sqrt(M))
        iI, iQ = rng.integers(0, L, 200), rng.integers(0, L, 200)
        pts = inputs.qam_points(iI, iQ, M)
        assert np.array_equal(O.slice_qam(pts, M).astype(int), iI + L * iQ)
        assert np.array_equal(O.slice_qam_f32(pts, M).astype(int), iI + L * iQ)


def test_slicer_f32_agrees_off_threshold():
    rng = np.random.default_rng(5)
    x = 1.5 * cn(rng, 20000)
    for M in (4, 16, 64):
        a, b = O.slice_qam(x, M), O.slice_qam_f32(x, M)
        L = int(math.sqrt(M))
        kappa = math.sqrt(2 * (M - 1) / 3)
        # distance of kappa*x to the nearest threshold (odd integers ... even: thresholds at 2i - L + 2)
        def gap(v):
            t = kappa * v + L
            return np.abs(t / 2 - np.round(t / 2))
        far = (gap(x.real) > 1e-5) & (gap(x.imag) > 1e-5)
        assert np.array_equal(a[far], b[far])


# --------------------------------------------------------------------------
# Exact rational arithmetic at finite T
# --------------------------------------------------------------------------

def _gauss_int(rng, *shape):
    return rng.integers(-3, 4, shape) + 1j * rng.integers(-3, 4, shape)


@pytest.mark.parametrize("B,U,C", [(4, 2, 2), (6, 2, 2), (4, 3, 2), (6, 3, 3)])
def test_rational_alg1(B, U, C):
    rng = np.random.default_rng(B * 10 + U)
    H, y = _gauss_int(rng, B, U), _gauss_int(rng, B)
    for mode in ("SS", "UU"):
        for T in (1, 2, 4):
            r = np.array(R.admm_ul(H.tolist(), y.tolist(), C, Fraction(3, 2), T, Fraction(1, 2), mode=mode))
            f = O.admm_ul(H, y, C, 1.5, T, 0.5, mode=mode)
            assert np.abs(r - f).max() <= 1e-13 * max(1.0, np.abs(r).max())


@pytest.mark.parametrize("B,U,C", [(4, 2, 2), (6, 3, 3)])
def test_rational_alg2(B, U, C):
    rng = np.random.default_rng(B + U)
    H, y = _gauss_int(rng, B, U), _gauss_int(rng, B)
    for T in (1, 2, 3):
        r = np.array(R.dcg_ul(H.tolist(), y.tolist(), C, T, Fraction(1, 4)))
        f = O.dcg_ul(H, y, C, T, 0.25)
        assert np.abs(r - f).max() <= 1e-13 * max(1.0, np.abs(r).max())


@pytest.mark.parametrize("B,U,C", [(4, 2, 2), (6, 2, 3), (4, 3, 2)])
def test_rational_alg3(B, U, C):
    rng = np.random.default_rng(B * U + C)
    Hu, s = _gauss_int(rng, B, U), _gauss_int(rng, U)
    for mode in ("SS", "UU"):
        for T in (1, 2, 4):
            r = np.array(R.admm_dl(Hu.tolist(), s.tolist(), C, Fraction(2), T, mode=mode))
            f = O.admm_dl(Hu, s, C, 2.0, T, mode=mode)
            assert np.abs(r - f).max() <= 1e-13 * max(1.0, np.abs(r).max())


# --------------------------------------------------------------------------
# Independent formulations: literal argmin steps, both solver branches
# --------------------------------------------------------------------------

@pytest.mark.parametrize("B,U,C", [(16, 4, 4), (32, 8, 4), (32, 8, 8), (24, 8, 3), (64, 8, 4)])
@pytest.mark.parametrize("reg", ["mmse", "zf"])
def test_alg1_equals_literal_steps(B, U, C, reg):
    rng = np.random.default_rng(B + U + C)
    H, y = cn(rng, B, U), cn(rng, B)
    for T in (1, 3, 5):
        a = O.admm_ul(H, y, C, 0.7, T, 0.3, reg=reg)
        b = O.admm_ul_literal(H, y, C, 0.7, T, 0.3, reg=reg)
        assert np.abs(a - b).max() < 1e-12


def test_alg1_box_equals_literal_steps():
    rng = np.random.default_rng(11)
    B, U, C = 16, 4, 4
    H = cn(rng, B, U)
    s = inputs.qam_points(rng.integers(0, 2, U), rng.integers(0, 2, U), 4)
    y = H @ s + 0.4 * cn(rng, B)
    r = O.box_radius(4)
    for T in (1, 2, 4):
        a = O.admm_ul(H, y, C, 1.0, T, 0.0, reg="box", box_r=r)
        b = O.admm_ul_literal(H, y, C, 1.0, T, 0.0, reg="box", box_r=r)
        assert np.abs(a - b).max() < 1e-6


@pytest.mark.parametrize("B,U,C", [(16, 4, 4), (32, 8, 8), (32, 4, 4), (64, 16, 8)])
def test_alg1_branches_agree(B, U, C):
    rng = np.random.default_rng(B * U)
    H, y = cn(rng, B, U), cn(rng, B)
    a = O.admm_ul(H, y, C, 1.0, 5, 0.2, mode="SS")
    b = O.admm_ul(H, y, C, 1.0, 5, 0.2, mode="UU")
    assert np.abs(a - b).max() < 1e-12


@pytest.mark.parametrize("B,U,C", [(16, 4, 4), (32, 8, 8), (16, 2, 2), (64, 16, 16)])
def test_alg3_equals_literal_and_branches(B, U, C):
    rng = np.random.default_rng(B + 7 * U)
    Hu, s = cn(rng, B, U), cn(rng, U)
    for T in (1, 2, 5):
        a = O.admm_dl(Hu, s, C, 1.0, T, mode="SS")
        b = O.admm_dl(Hu, s, C, 1.0, T, mode="UU")
        c = O.admm_dl_literal(Hu, s, C, 1.0, T)
        assert np.abs(a - b).max() < 1e-12
        assert np.abs(a - c).max() < 1e-12


# --------------------------------------------------------------------------
# Lemma 1 and Lemma 2 against generic solvers
# --------------------------------------------------------------------------

def test_lemma1_prox_is_the_minimiser():
    from scipy.optimize import minimize
    rng = np.random.default_rng(21)
    U, C, rho, N0, Es = 3, 4, 0.8, 0.5, 1.0
    wc = cn(rng, C, U)
    s = O.prox(wc.sum(axis=0), C, rho, N0, Es, "mmse")

    def f(v):
        sv = v[:U] + 1j * v[U:]
        val = N0 / (2 * Es) * np.sum(np.abs(sv) ** 2) + sum(rho / 2 * np.sum(np.abs(sv - w) ** 2) for w in wc)
        return val
    res = minimize(f, np.zeros(2 * U), method="BFGS", options={"gtol": 1e-12})
    assert np.abs(s - (res.x[:U] + 1j * res.x[U:])).max() < 1e-6


def test_lemma2_projection_eps0():
    # z_c = w_c + (s - sum w)/C is the projection of (w_c) onto {sum_c z_c = s}:
    # check against the KKT system of min 1/2||z - w||^2 s.t. D z = s
    rng = np.random.default_rng(22)
    U, C = 3, 4
    w = cn(rng, C * U)
    s = cn(rng, U)
    D = np.kron(np.ones((1, C)), np.eye(U))
    K = np.block([[np.eye(C * U), D.T], [D, np.zeros((U, U))]])
    sol = np.linalg.solve(K, np.concatenate([w, s]))
    wc = w.reshape(C, U)
    z = np.concatenate([wc[c] + (s - wc.sum(axis=0)) / C for c in range(C)])
    assert np.abs(z - sol[:C * U]).max() < 1e-13


def _lemma2_z(wc, s, eps):
    # the z-update of Lemma 2 as the oracle's Algorithm 3 applies it
    w = wc.sum(axis=0)
    f = O.lemma2_factor(s - w, eps)
    return np.concatenate([wc[c] + f * (s - w) / len(wc) for c in range(len(wc))])


@pytest.mark.parametrize("eps", [0.05, 0.4, 1.5, 50.0])
def test_lemma2_projection_eps_positive_kkt(eps):
    # the projection of w_all onto {z : ||s - D z|| <= eps}: z feasible, and
    # either z = w_all (constraint inactive) or ||s - D z|| = eps with
    # z - w_all = mu D^H (s - D z) for a real mu >= 0 (KKT, complementary slackness)
    rng = np.random.default_rng(int(eps * 100))
    U, C = 3, 4
    wc, s = cn(rng, C, U), cn(rng, U)
    D = np.kron(np.ones((1, C)), np.eye(U))
    wall = wc.reshape(-1)
    z = _lemma2_z(wc, s, eps)
    r = s - D @ z
    assert np.linalg.norm(r) <= eps * (1 + 1e-12)
    if np.linalg.norm(s - D @ wall) <= eps:
        assert np.abs(z - wall).max() == 0.0
    else:
        assert abs(np.linalg.norm(r) - eps) < 1e-12
        g = D.conj().T @ r
        mu = np.vdot(g, z - wall) / np.vdot(g, g)
        assert abs(mu.imag) < 1e-12 and mu.real > 0
        assert np.abs(z - wall - mu.real * g).max() < 1e-12


def test_lemma2_projection_eps_positive_generic_solver():
    # against a general constrained minimiser (SLSQP on real coordinates)
    from scipy.optimize import minimize
    rng = np.random.default_rng(23)
    U, C, eps = 2, 3, 0.3
    wc, s = cn(rng, C, U), cn(rng, U)
    wall = wc.reshape(-1)
    n = C * U

    def cz(v):
        return v[:n] + 1j * v[n:]

    def resid(v):
        return s - cz(v).reshape(C, U).sum(axis=0)

    cons = {"type": "ineq", "fun": lambda v: eps ** 2 - np.sum(np.abs(resid(v)) ** 2)}
    x0 = np.concatenate([wall.real, wall.imag])
    res = minimize(lambda v: 0.5 * np.sum(np.abs(cz(v) - wall) ** 2), x0, constraints=[cons],
                   method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
    assert np.linalg.norm(s - wall.reshape(C, U).sum(axis=0)) > eps     # the constraint is active
    assert np.abs(_lemma2_z(wc, s, eps) - cz(res.x)).max() < 1e-6


def test_lemma2_statement_denominator_is_infeasible():
    # The statement of Lemma 2 divides eps by ||s - v|| with v = w / C; with
    # that denominator the result leaves ||s - sum_c z_c|| above eps, while the
    # proof's ||s - w|| lands on eps exactly.
    rng = np.random.default_rng(24)
    U, C, eps = 4, 4, 0.3
    wc, s = cn(rng, C, U), cn(rng, U)
    w = wc.sum(axis=0)
    f_stmt = max(0.0, 1 - eps / np.linalg.norm(s - w / C))
    z_stmt = wc + f_stmt * (s - w) / C
    assert np.linalg.norm(s - z_stmt.sum(axis=0)) > eps * 1.01
    z = _lemma2_z(wc, s, eps).reshape(C, U)
    assert abs(np.linalg.norm(s - z.sum(axis=0)) - eps) < 1e-12


@pytest.mark.parametrize("B,U,C", [(16, 4, 4), (32, 8, 8), (64, 16, 16), (16, 8, 2)])
@pytest.mark.parametrize("eps", [0.02, 0.3, 1e6])
def test_alg3_eps_equals_literal_and_branches(B, U, C, eps):
    # Algorithm 3 with the Lemma 2 z-update against the steps (P1)-(P3) with
    # (P2) solved through its Lagrange multiplier
    rng = np.random.default_rng(B + 3 * U + C)
    Hu, s = cn(rng, B, U), cn(rng, U)
    for T in (1, 2, 5):
        a = O.admm_dl(Hu, s, C, 1.0, T, mode="SS", eps=eps)
        b = O.admm_dl(Hu, s, C, 1.0, T, mode="UU", eps=eps)
        c = O.admm_dl_literal(Hu, s, C, 1.0, T, eps=eps)
        assert np.abs(a - b).max() < 1e-12
        assert np.abs(a - c).max() < 1e-10


# --------------------------------------------------------------------------
# Convergence limits (centralized closed forms)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("C", [1, 2, 4])
def test_alg1_converges_to_mmse(C):
    rng = np.random.default_rng(30 + C)
    B, U = 16, 4
    H, y = cn(rng, B, U), cn(rng, B)
    s = O.admm_ul(H, y, C, 1.0, 3000, 0.3)
    assert np.abs(s - O.mmse_detect(H, y, 0.3)).max() < 1e-10


def test_alg1_converges_to_zf():
    rng = np.random.default_rng(41)
    B, U, C = 16, 4, 4
    H, y = cn(rng, B, U), cn(rng, B)
    s = O.admm_ul(H, y, C, 1.0, 3000, 0.0, reg="zf")
    assert np.abs(s - O.zf_detect(H, y)).max() < 1e-10


def test_dcg_reaches_direct_solve_in_U_steps():
    rng = np.random.default_rng(50)
    for B, U, C in [(16, 4, 4), (32, 8, 8), (64, 16, 8)]:
        H, y = cn(rng, B, U), cn(rng, B)
        x = O.dcg_ul(H, y, C, U, 0.25)
        assert np.abs(x - O.mmse_detect(H, y, 0.25)).max() < 1e-9
        xz = O.dcg_ul(H, y, C, U, 0.0, reg="zf")
        assert np.abs(xz - O.zf_detect(H, y)).max() < 1e-9


def test_dcg_independent_of_C():
    rng = np.random.default_rng(51)
    H, y = cn(rng, 32, 8), cn(rng, 32)
    xs = [O.dcg_ul(H, y, C, 3, 0.5) for C in (1, 2, 4, 8)]
    for x in xs[1:]:
        assert np.abs(x - xs[0]).max() < 1e-13


def test_dcg_stops_on_zero_residual():
    rng = np.random.default_rng(52)
    H = cn(rng, 8, 2)
    y = np.zeros(8, complex)
    x = O.dcg_ul(H, y, 2, 5, 0.1)
    assert np.all(x == 0)


@pytest.mark.parametrize("B,U,C,mode", [(64, 8, 16, "SS"), (16, 2, 4, "UU")])
def test_alg3_converges_to_zf_precoder(B, U, C, mode):
    rng = np.random.default_rng(60 + B)
    Hu, s = cn(rng, B, U), cn(rng, U)
    x = O.admm_dl(Hu, s, C, 1.0, 3000, mode=mode)
    assert np.abs(x - O.zf_precode(Hu.T, s)).max() < 1e-9
    assert np.abs(Hu.T @ x - s).max() < 1e-9


def test_eps_precode_is_the_p0_minimiser():
    # the closed form of problem P0 with eps > 0 against a generic constrained
    # minimiser, its residual on the boundary, and x = 0 once ||s|| <= eps
    from scipy.optimize import minimize
    rng = np.random.default_rng(61)
    U, B, eps = 2, 4, 0.4
    Hd, s = cn(rng, U, B), cn(rng, U)

    def cz(v):
        return v[:B] + 1j * v[B:]

    cons = {"type": "ineq", "fun": lambda v: eps ** 2 - np.sum(np.abs(s - Hd @ cz(v)) ** 2)}
    x0 = np.concatenate([O.zf_precode(Hd, s).real, O.zf_precode(Hd, s).imag])
    res = minimize(lambda v: 0.5 * np.sum(v ** 2), x0, constraints=[cons], method="SLSQP",
                   options={"ftol": 1e-14, "maxiter": 500})
    x = O.eps_precode(Hd, s, eps)
    assert abs(np.linalg.norm(s - Hd @ x) - eps) < 1e-12
    assert np.abs(x - cz(res.x)).max() < 1e-6
    assert np.all(O.eps_precode(Hd, s, 1.01 * np.linalg.norm(s)) == 0)


@pytest.mark.parametrize("eps", [0.1, 0.6])
def test_alg3_eps_converges_to_p0(eps):
    rng = np.random.default_rng(62)
    B, U, C = 16, 4, 4
    Hu, s = cn(rng, B, U), cn(rng, U)
    x = O.admm_dl(Hu, s, C, 1.0, 3000, eps=eps)
    assert np.abs(x - O.eps_precode(Hu.T, s, eps)).max() < 1e-9
    assert abs(np.linalg.norm(s - Hu.T @ x) - eps) < 1e-9


# --------------------------------------------------------------------------
# Invariances and metamorphic relations
# --------------------------------------------------------------------------

def test_power_of_two_scaling_invariance():
    rng = np.random.default_rng(70)
    B, U, C = 32, 8, 4
    H, y = cn(rng, B, U), cn(rng, B)
    for k in (-3, 2):
        a = 2.0 ** k
        s0 = O.admm_ul(H, y, C, 1.0, 5, 0.3)
        s1 = O.admm_ul(a * H, a * y, C, a * a, 5, a * a * 0.3)
        assert np.abs(s0 - s1).max() < 1e-14
        x0 = O.dcg_ul(H, y, C, 4, 0.3)
        x1 = O.dcg_ul(a * H, a * y, C, 4, a * a * 0.3)
        assert np.abs(x0 - x1).max() < 1e-14
    Hu, s = cn(rng, B, U), cn(rng, U)
    x0 = O.admm_dl(Hu, s, C, 1.0, 5)
    x1 = O.admm_dl(2.0 * Hu, s, C, 0.25, 5)
    assert np.abs(x0 / 2.0 - x1).max() < 1e-14


def test_unitary_user_rotation():
    rng = np.random.default_rng(71)
    B, U, C = 32, 8, 4
    H, y = cn(rng, B, U), cn(rng, B)
    Q, _ = np.linalg.qr(cn(rng, U, U))
    for T in (1, 4):
        s0 = O.admm_ul(H, y, C, 1.0, T, 0.3, mode="UU")
        s1 = O.admm_ul(H @ Q, y, C, 1.0, T, 0.3, mode="UU")
        assert np.abs(Q.conj().T @ s0 - s1).max() < 1e-12


def test_row_permutation_inside_cluster():
    rng = np.random.default_rng(72)
    B, U, C = 32, 4, 4
    H, y = cn(rng, B, U), cn(rng, B)
    perm = np.concatenate([c * 8 + rng.permutation(8) for c in range(C)])
    a = O.admm_ul(H, y, C, 1.0, 5, 0.3)
    b = O.admm_ul(H[perm], y[perm], C, 1.0, 5, 0.3)
    assert np.abs(a - b).max() < 1e-12


def test_noiseless_detection_recovers_symbols():
    rng = np.random.default_rng(73)
    for M in (4, 16, 64):
        B, U, C = 64, 8, 4
        L = int(math.sqrt(M))
        H = cn(rng, B, U)
        iI, iQ = rng.integers(0, L, U), rng.integers(0, L, U)
        s = inputs.qam_points(iI, iQ, M)
        y = H @ s
        for est in (O.admm_ul(H, y, C, 1.0, 400, 0.0, reg="zf"), O.dcg_ul(H, y, C, U, 0.0, reg="zf")):
            assert np.array_equal(O.slice_qam(est, M).astype(int), iI + L * iQ)


def test_box_vertex_certificate_equals_ml():
    # if the BOX-regularised equaliser lands on a vertex of the box (a QPSK
    # point), that point minimises ||y - Hs|| over the box and hence over O^U.
    # Received vectors are drawn with amplified symbols so that the box is active.
    rng = np.random.default_rng(74)
    r = O.box_radius(4)
    hits = 0
    for trial in range(40):
        B, U, C = 8, 3, 2
        H = cn(rng, B, U)
        s = inputs.qam_points(rng.integers(0, 2, U), rng.integers(0, 2, U), 4)
        y = H @ (1.8 * s) + 0.5 * cn(rng, B)
        est = O.admm_ul(H, y, C, 1.0, 600, 0.0, reg="box", box_r=r)
        on_vertex = np.all(np.abs(np.abs(est.real) - r) < 1e-9) and np.all(np.abs(np.abs(est.imag) - r) < 1e-9)
        if on_vertex:
            hits += 1
            ml = ML.ml_detect(H, y, 4)
            assert np.abs(est - ml).max() < 1e-8
    assert hits >= 10


def _power_scale_is_tight(x, C, P, xs, beta):
    """The common gain of the per-cluster budget reading is the LARGEST gain in
    (0, 1] under which every cluster meets its budget: with beta < 1 the
    cluster that sets it meets its budget with equality, and beta = 1 exactly
    when every cluster is within budget unscaled."""
    S = len(x) // C
    e = [float(np.real(np.vdot(x[c * S:(c + 1) * S], x[c * S:(c + 1) * S]))) for c in range(C)]
    es = [float(np.real(np.vdot(xs[c * S:(c + 1) * S], xs[c * S:(c + 1) * S]))) for c in range(C)]
    if not all(es[c] <= P[c] * (1 + 1e-12) for c in range(C)):
        return False
    if all(e[c] <= P[c] for c in range(C)):
        return beta == 1.0
    return beta < 1.0 and min(abs(es[c] - P[c]) / P[c] for c in range(C)) <= 1e-12


def test_power_scale_meets_budgets():
    rng = np.random.default_rng(75)
    B, U, C = 64, 8, 8
    Hu, s = cn(rng, B, U), cn(rng, U)
    x = O.admm_dl(Hu, s, C, 1.0, 5)
    P = [(B // C) / B * U * 0.05] * C
    xs, beta = O.power_scale(x, C, P)
    assert 0 < beta <= 1
    for c in range(C):
        seg = xs[c * 8:(c + 1) * 8]
        assert np.real(np.vdot(seg, seg)) <= P[c] * (1 + 1e-12)
    assert np.abs(Hu.T @ xs - beta * (Hu.T @ x)).max() < 1e-12


@pytest.mark.parametrize("budget", [0.02, 0.2, 1.0, 50.0])
def test_power_scale_is_tight(budget):
    # beta is pinned by two facts independent of its formula: no cluster may
    # exceed its budget, and no larger common gain would do.  Unequal budgets
    # make a different cluster bind than the one with the most energy.
    rng = np.random.default_rng(76)
    B, U, C = 64, 8, 8
    for trial in range(5):
        Hu, s = cn(rng, B, U), cn(rng, U)
        x = O.admm_dl(Hu, s, C, 1.0, 5)
        S = B // C
        emax = max(float(np.real(np.vdot(x[c * S:(c + 1) * S], x[c * S:(c + 1) * S]))) for c in range(C))
        P = [budget * emax * (1.0 + 0.5 * rng.random()) for _ in range(C)]
        xs, beta = O.power_scale(x, C, P)
        assert _power_scale_is_tight(x, C, P, xs, beta)


def test_power_scale_tightness_check_rejects_a_gain_without_square_root():
    # the tightness check above must catch the plausible mistake of a gain
    # min(1, P_c / ||x_c||^2) (energy scaled to P^2/e < P when the budget binds)
    rng = np.random.default_rng(77)
    B, U, C = 64, 8, 8
    Hu, s = cn(rng, B, U), cn(rng, U)
    x = O.admm_dl(Hu, s, C, 1.0, 5)
    S = B // C
    e = [float(np.real(np.vdot(x[c * S:(c + 1) * S], x[c * S:(c + 1) * S]))) for c in range(C)]
    P = [0.25 * min(e)] * C
    bad = min(1.0, min(P[c] / e[c] for c in range(C)))
    assert bad < 1.0
    assert not _power_scale_is_tight(x, C, P, bad * x, bad)
    xs, beta = O.power_scale(x, C, P)
    assert _power_scale_is_tight(x, C, P, xs, beta)


# -- Step (P1) under a per-cluster budget ||x_c||^2 <= P_c ----------------------

def _p1_kkt_ok(Hc, v, rho, P, x, tol=1e-9):
    """KKT conditions of min 1/2||x||^2 + rho/2||H x - v||^2 s.t. ||x||^2 <= P:
    primal feasibility, and a multiplier mu >= 0 with
    (1 + mu) x + rho H^H (H x - v) = 0 and mu (||x||^2 - P) = 0."""
    e = float(np.real(np.vdot(x, x)))
    if e > P * (1 + tol):
        return False
    g = rho * (Hc.conj().T @ (Hc @ x - v))          # = -(1 + mu) x
    if np.linalg.norm(x) == 0:
        return np.linalg.norm(g) <= tol
    one_mu = -float(np.real(np.vdot(x, g))) / e
    mu = one_mu - 1.0
    stat = np.linalg.norm(one_mu * x + g) / max(np.linalg.norm(g), 1e-300)
    if mu < -tol or stat > tol:
        return False
    return abs(mu * (e - P)) <= tol * max(1.0, P) * max(1.0, abs(mu))


@pytest.mark.parametrize("scale", [0.05, 0.5, 0.95, 2.0])
def test_p1_budget_kkt(scale):
    # budgets from far below to above the unconstrained step's energy
    rng = np.random.default_rng(80)
    for trial in range(6):
        U, S, rho = 6, 4, 0.7
        Hc, v = cn(rng, U, S), cn(rng, U)
        x0 = np.linalg.solve(Hc.conj().T @ Hc + np.eye(S) / rho, Hc.conj().T @ v)
        P = scale * float(np.real(np.vdot(x0, x0)))
        x, tau = O.p1_budget(Hc, v, rho, P)
        assert _p1_kkt_ok(Hc, v, rho, P, x)
        if scale >= 1.0:
            assert np.array_equal(x, x0) and tau == 1.0 / rho
        else:
            assert abs(float(np.real(np.vdot(x, x))) - P) <= 1e-12 * P and tau > 1.0 / rho


def test_p1_budget_kkt_check_rejects_a_rescaled_step():
    # the plausible shortcut of scaling the unconstrained step onto the ball
    # is feasible but not the minimiser: the KKT check must reject it
    rng = np.random.default_rng(81)
    U, S, rho = 6, 4, 1.0
    Hc, v = cn(rng, U, S), cn(rng, U)
    x0 = np.linalg.solve(Hc.conj().T @ Hc + np.eye(S) / rho, Hc.conj().T @ v)
    P = 0.3 * float(np.real(np.vdot(x0, x0)))
    assert not _p1_kkt_ok(Hc, v, rho, P, x0 * math.sqrt(P / float(np.real(np.vdot(x0, x0)))))
    assert _p1_kkt_ok(Hc, v, rho, P, O.p1_budget(Hc, v, rho, P)[0])


def test_p1_budget_equals_generic_solver():
    from scipy.optimize import minimize

    rng = np.random.default_rng(82)
    for trial in range(5):
        U, S, rho = 5, 3, 1.3
        Hc, v = cn(rng, U, S), cn(rng, U)
        P = 0.2
        x, _ = O.p1_budget(Hc, v, rho, P)

        def f(r):
            z = r[:S] + 1j * r[S:]
            e = Hc @ z - v
            return 0.5 * np.sum(np.abs(z) ** 2) + 0.5 * rho * np.sum(np.abs(e) ** 2)

        res = minimize(f, np.zeros(2 * S), constraints=[{"type": "ineq", "fun": lambda r: P - r @ r}],
                       method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
        assert np.abs(res.x[:S] + 1j * res.x[S:] - x).max() < 1e-6


def test_alg3_budget_equals_literal_steps():
    rng = np.random.default_rng(83)
    B, U, C = 16, 4, 2
    for T in (1, 3, 5):
        Hu, s = cn(rng, B, U), cn(rng, U)
        x = O.admm_dl(Hu, s, C, 1.0, T)
        S = B // C
        P = [0.6 * float(np.real(np.vdot(x[c * S:(c + 1) * S], x[c * S:(c + 1) * S]))) for c in range(C)]
        a = O.admm_dl(Hu, s, C, 1.0, T, P=P)
        b = O.admm_dl_literal(Hu, s, C, 1.0, T, P=P)
        assert np.abs(a - b).max() < 1e-7 * np.abs(a).max()
        for c in range(C):
            assert float(np.real(np.vdot(a[c * S:(c + 1) * S], a[c * S:(c + 1) * S]))) <= P[c] * (1 + 1e-12)


def test_alg3_budget_inactive_is_algorithm3():
    rng = np.random.default_rng(84)
    B, U, C = 32, 8, 4
    Hu, s = cn(rng, B, U), cn(rng, U)
    assert np.array_equal(O.admm_dl(Hu, s, C, 1.0, 5, P=[1e9] * C), O.admm_dl(Hu, s, C, 1.0, 5))


def test_alg3_budget_converges_to_the_constrained_p0():
    # T -> infinity: the minimum-energy x with H x = s and ||x_c||^2 <= P_c,
    # found independently by SLSQP on the centralized problem
    from scipy.optimize import minimize

    rng = np.random.default_rng(85)
    B, U, C = 12, 3, 3
    S = B // C
    Hu, s = cn(rng, B, U), cn(rng, U)
    Hd = Hu.T
    xzf = O.zf_precode(Hd, s)
    e = [float(np.real(np.vdot(xzf[c * S:(c + 1) * S], xzf[c * S:(c + 1) * S]))) for c in range(C)]
    cmax = int(np.argmax(e))
    P = [10.0 * max(e)] * C
    P[cmax] = 0.7 * e[cmax]                      # the ZF precoder violates this budget
    x = O.admm_dl(Hu, s, C, 1.0, 4000, P=P)

    def unpack(r):
        return r[:B] + 1j * r[B:]

    cons = [{"type": "eq", "fun": lambda r: np.concatenate([(Hd @ unpack(r) - s).real, (Hd @ unpack(r) - s).imag])}]
    for c in range(C):
        cons.append({"type": "ineq", "fun": lambda r, c=c: P[c] - np.sum(np.abs(unpack(r)[c * S:(c + 1) * S]) ** 2)})
    res = minimize(lambda r: 0.5 * r @ r, np.concatenate([xzf.real, xzf.imag]), constraints=cons, method="SLSQP",
                   options={"ftol": 1e-15, "maxiter": 2000})
    assert res.success
    ref = unpack(res.x)
    assert np.abs(Hd @ x - s).max() < 1e-6
    assert np.abs(x - ref).max() < 1e-5 * np.abs(ref).max()
