"""FP64 CPU oracle for decentralized baseband processing.

TEST INFRASTRUCTURE ONLY: this module is imported by the tests, by the smoke
check and by the bench's CPU-baseline leg, never by the product path.  It shares
no code with the HIP library.

It follows Li, Sharan, Chen, Goldstein, Cavallaro and Studer, "Decentralized
Baseband Processing for Massive MU-MIMO Systems" (arXiv:1702.04458):

* ``admm_ul``      -- Algorithm 1 (decentralized ADMM detection), both the S x S
                      branch (Woodbury form, eq. StepE1variant2) and the U x U
                      branch (eq. StepE1variant1), MMSE / ZF / BOX proximal steps
                      (Section III-C, Step E2, Lemma 1).
* ``admm_ul_literal`` -- the same method written as the three argmin steps
                      (E1), (E2), (E3) of Section III-B, each solved as a generic
                      least-squares problem; used to pin ``admm_ul``.
* ``dcg_ul``       -- Algorithm 2 (decentralized conjugate gradients,
                      Section III-D, eqs. CGiteration / CGdecentralization).
* ``admm_dl``      -- Algorithm 3 (decentralized ADMM beamforming, Section IV),
                      A_c (S x S) and B_c (U x U) branches; epsilon = 0 as in the
                      algorithm, or epsilon > 0 with the z-update of Lemma 2.
* ``p1_budget``    -- step (P1) under a per-cluster transmit-energy budget
                      ||x_c||^2 <= P_c (problem P0 with the budgets added;
                      the paper has none): the constrained least-squares
                      minimiser through its Lagrange multiplier.
* ``admm_dl_literal`` -- the steps (P1), (P2), (P3) of Section IV-B written as
                      argmin / projection problems (P2 for epsilon > 0 solved
                      through its Lagrange multiplier); used to pin ``admm_dl``.
* ``mmse_detect``, ``zf_detect``, ``zf_precode`` -- centralized closed forms
                      (Section III-A, problem E0; Section IV-A, problem P0 with
                      epsilon = 0) used as convergence pins.
* ``slice_qam``    -- nearest-point slicing to the square QAM alphabet.

Readings of points where the paper is silent or inconsistent:

* Algorithm 2's residual update uses e^(t) (the printed e^(t-1) is a typo: with
  it CG does not reach the direct solve after U steps); the consensus sum runs
  over c = 1..C.
* In Algorithm 2 ``rho`` is the MMSE regularizer N0/Es (0 for ZF); it is not the
  ADMM penalty.  ``alpha`` uses Re(p^H e) (p^H e is real for a Hermitian PD
  system).  When the residual norm reaches exactly zero the iteration stops
  (x is then exact) instead of dividing by zero.
* T counts x-estimates: Algorithm 1 returns s^(T) (T proximal steps, T
  consensus sums), Algorithm 2 performs T CG iterations (T + 1 sums with the
  MRC sum), Algorithm 3 performs T x-updates (T - 1 sums).
* At S = U Algorithms 1 and 3 take the S x S branch, as printed; the two
  branches are equal up to rounding (Woodbury identity) and the tests pin this.
* Constellations are unit-energy (Es = 1); the BOX radius is (L - 1) / kappa.
* Slicing: per dimension, index i = clamp(floor((kappa x + L) / 2), 0, L - 1);
  a value exactly on a decision threshold goes to the upper level.  The hard
  output is the QAM index iI + L * iQ.
* Downlink per-cluster power budget (not part of problem P0): after Algorithm 3,
  a common gain beta = min(1, min_c sqrt(P_c / ||x_c||^2)) is applied to the
  whole vector, so every cluster meets its budget and the users see beta * s.
* Lemma 2 (epsilon > 0): the statement divides epsilon by ||s - v|| with
  v = w / C, the proof by ||s - D w_all|| = ||s - w||.  Only the proof's form
  yields a z with ||s - sum_c z_c|| <= epsilon, so the oracle uses ||s - w||.
  When s = w the step adds nothing (factor 0).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "partition_rows", "admm_ul", "admm_ul_literal", "admm_ul_frame",
    "dcg_ul", "dcg_ul_frame", "admm_dl", "admm_dl_literal", "admm_dl_frame",
    "mmse_detect", "zf_detect", "zf_precode", "eps_precode", "lemma2_factor",
    "project_ball_constraint", "slice_qam", "slice_qam_f32", "p1_budget",
    "qam_levels", "box_radius", "power_scale", "prox",
]


# ---------------------------------------------------------------------------
# Partitioning (Section II-A2, eq. uplinkdecomposedmodel; Section II-B2)
# ---------------------------------------------------------------------------

def partition_rows(X: np.ndarray, C: int):
    """Split the B rows of X into C equal clusters of S = B / C rows each."""
    B = X.shape[0]
    if B % C:
        raise ValueError("B must be a multiple of C")
    S = B // C
    return [X[c * S:(c + 1) * S] for c in range(C)]


# ---------------------------------------------------------------------------
# Constellation helpers (Section III-A: slicing to the nearest point of O)
# ---------------------------------------------------------------------------

def qam_levels(M: int) -> np.ndarray:
    L = int(round(math.sqrt(M)))
    kappa = math.sqrt(2.0 * (M - 1) / 3.0)
    return (2.0 * np.arange(L) - (L - 1)) / kappa


def box_radius(M: int) -> float:
    """Radius of the square that is the convex hull of the unit-energy M-QAM alphabet."""
    return float(qam_levels(M)[-1])


def slice_qam(x: np.ndarray, M: int) -> np.ndarray:
    """Nearest-point slicing in FP64; returns uint8 index iI + L * iQ."""
    L = int(round(math.sqrt(M)))
    kappa = math.sqrt(2.0 * (M - 1) / 3.0)

    def dim(v):
        i = np.floor((kappa * v + L) / 2.0)
        return np.clip(i, 0, L - 1).astype(np.int64)

    x = np.asarray(x)
    return (dim(x.real) + L * dim(x.imag)).astype(np.uint8)


def slice_qam_f32(x: np.ndarray, M: int) -> np.ndarray:
    """The same decision taken in FP32 with the operation order
    t = round32(round32(kappa32 * v) + L); i = floor(t * 0.5), so that a single
    precision producer can be compared bit for bit."""
    L = int(round(math.sqrt(M)))
    kappa32 = np.float32(math.sqrt(2.0 * (M - 1) / 3.0))

    def dim(v):
        v = np.asarray(v, dtype=np.float32)
        t = (v * kappa32).astype(np.float32)
        t = (t + np.float32(L)).astype(np.float32)
        i = np.floor(t * np.float32(0.5))
        return np.clip(i, 0, L - 1).astype(np.int64)

    x = np.asarray(x).astype(np.complex64)
    return (dim(x.real) + L * dim(x.imag)).astype(np.uint8)


# ---------------------------------------------------------------------------
# Proximal step of (E2) after Lemma 1: s = argmin g(s) + (C rho / 2)||s - v||^2
# ---------------------------------------------------------------------------

def prox(w: np.ndarray, C: int, rho: float, N0: float, Es: float, reg: str,
         box_r: float | None = None) -> np.ndarray:
    """Consensus scaling of the summed vector w = sum_c w_c (v = w / C).

    (E2-MMSE): s = C rho Es / (N0 + C rho Es) v  = w / (N0 / (rho Es) + C)
    (E2-ZF):   s = v                              (the MMSE form with N0 = 0)
    (E2-BOX):  entrywise clip of Re and Im of v to [-r, r]
    """
    if reg in ("mmse", "zf"):
        n0 = N0 if reg == "mmse" else 0.0
        return w / (n0 / (rho * Es) + C)
    if reg == "box":
        v = w / C
        r = box_r
        return np.clip(v.real, -r, r) + 1j * np.clip(v.imag, -r, r)
    raise ValueError(reg)


# ---------------------------------------------------------------------------
# Algorithm 1: decentralized ADMM-based data detection
# ---------------------------------------------------------------------------

def admm_ul(H, y, C, rho, T, N0, Es=1.0, gamma=1.0, mode=None, reg="mmse",
            box_r=None):
    """Algorithm 1 for one received vector.  H: (B, U), y: (B,).  Returns s^(T).

    Preprocessing (per cluster c):
      S <= U:  A_c = H_c H_c^H + rho I_S,  y_c^reg = H_c^H A_c^{-1} y_c
      S >  U:  B_c = H_c^H H_c + rho I_U,  y_c^reg = B_c^{-1} H_c^H y_c
    Init: lambda_c = 0, z_c = y_c^reg, s = prox(sum_c z_c).
    For t = 2..T:
      lambda_c += gamma (z_c - s)
      z_c = y_c^reg + (I - H_c^H A_c^{-1} H_c)(s - lambda_c)       (S <= U)
      z_c = y_c^reg + rho B_c^{-1} (s - lambda_c)                  (S >  U)
      w_c = z_c + lambda_c;  w = sum_c w_c  (consensus);  s = prox(w)
    """
    H = np.asarray(H, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    B, U = H.shape
    S = B // C
    if T < 1:
        raise ValueError("T >= 1")
    if mode is None:
        mode = "SS" if S <= U else "UU"
    Hc = partition_rows(H, C)
    yc = partition_rows(y, C)
    yreg, K = [], []
    for c in range(C):
        Hk = Hc[c]
        if mode == "SS":
            A = Hk @ Hk.conj().T + rho * np.eye(S)
            yreg.append(Hk.conj().T @ np.linalg.solve(A, yc[c]))
            K.append(lambda q, Hk=Hk, A=A: q - Hk.conj().T @ np.linalg.solve(A, Hk @ q))
        elif mode == "UU":
            Bm = Hk.conj().T @ Hk + rho * np.eye(U)
            yreg.append(np.linalg.solve(Bm, Hk.conj().T @ yc[c]))
            K.append(lambda q, Bm=Bm: rho * np.linalg.solve(Bm, q))
        else:
            raise ValueError(mode)
    lam = [np.zeros(U, np.complex128) for _ in range(C)]
    z = [yreg[c].copy() for c in range(C)]
    w = np.zeros(U, np.complex128)
    for c in range(C):
        w = w + z[c]
    s = prox(w, C, rho, N0, Es, reg, box_r)
    for _t in range(2, T + 1):
        w = np.zeros(U, np.complex128)
        for c in range(C):
            lam[c] = lam[c] + gamma * (z[c] - s)
            z[c] = yreg[c] + K[c](s - lam[c])
            w = w + (z[c] + lam[c])
        s = prox(w, C, rho, N0, Es, reg, box_r)
    return s


def admm_ul_literal(H, y, C, rho, T, N0, Es=1.0, gamma=1.0, reg="mmse",
                    box_r=None):
    """Section III-B steps in their own order, each argmin solved generically.

    Start s = 0, lambda_c = 0 and repeat T times:
      (E1) z_c = argmin 1/2||y_c - H_c z||^2 + rho/2 ||s - z - lambda_c||^2,
           solved as the stacked least-squares problem
           [H_c; sqrt(rho) I] z ~ [y_c; sqrt(rho)(s - lambda_c)];
      (E2) s = argmin g(s) + sum_c rho/2 ||s - z_c - lambda_c||^2, solved for
           MMSE / ZF as a stacked least-squares problem over all clusters
           (g = N0/(2 Es)||s||^2 contributes the rows sqrt(N0/Es) I), and for
           BOX by projected gradient on the separable quadratic;
      (E3) lambda_c = lambda_c - gamma (s - z_c).
    Returns s after T rounds, which the paper states equals Algorithm 1's
    output (the reordering E3, E1, E2 does not change the result).
    """
    H = np.asarray(H, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    B, U = H.shape
    S = B // C
    Hc = partition_rows(H, C)
    yc = partition_rows(y, C)
    s = np.zeros(U, np.complex128)
    lam = [np.zeros(U, np.complex128) for _ in range(C)]
    z = [None] * C
    sq = math.sqrt(rho)
    for _t in range(T):
        for c in range(C):
            Amat = np.vstack([Hc[c], sq * np.eye(U)])
            bvec = np.concatenate([yc[c], sq * (s - lam[c])])
            z[c] = np.linalg.lstsq(Amat, bvec, rcond=None)[0]
        if reg in ("mmse", "zf"):
            rows, rhs = [], []
            if reg == "mmse" and N0 > 0:
                rows.append(math.sqrt(N0 / Es) * np.eye(U))
                rhs.append(np.zeros(U, np.complex128))
            for c in range(C):
                rows.append(sq * np.eye(U))
                rhs.append(sq * (z[c] + lam[c]))
            s = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0]
        elif reg == "box":
            # minimise sum_c rho/2 ||s - w_c||^2 over the box |Re|, |Im| <= r with a
            # generic bound-constrained solver on the 2U real unknowns
            from scipy.optimize import minimize
            wv = np.array([z[c] + lam[c] for c in range(C)])
            W = np.concatenate([wv.real, wv.imag], axis=1)          # C x 2U

            def f(v):
                d = v[None, :] - W
                return 0.5 * rho * float(np.sum(d * d)), rho * np.sum(d, axis=0)

            res = minimize(f, np.zeros(2 * U), jac=True, method="L-BFGS-B",
                           bounds=[(-box_r, box_r)] * (2 * U),
                           options={"ftol": 1e-15, "gtol": 1e-13, "maxiter": 1000})
            s = res.x[:U] + 1j * res.x[U:]
        else:
            raise ValueError(reg)
        for c in range(C):
            lam[c] = lam[c] - gamma * (s - z[c])
    return s


def admm_ul_frame(H, y, C, rho, T, N0, Es=1.0, gamma=1.0, mode=None, reg="mmse",
                  box_r=None):
    """Algorithm 1 over a frame: H [n_sc][B][U], y [n_sc][n_sym][B] -> [n_sc][n_sym][U]."""
    n_sc, B, U = H.shape
    n_sym = y.shape[1]
    out = np.zeros((n_sc, n_sym, U), np.complex128)
    for k in range(n_sc):
        for n in range(n_sym):
            out[k, n] = admm_ul(H[k], y[k, n], C, rho, T, N0, Es, gamma, mode, reg, box_r)
    return out


# ---------------------------------------------------------------------------
# Algorithm 2: decentralized CG-based data detection
# ---------------------------------------------------------------------------

def dcg_ul(H, y, C, T, N0, Es=1.0, reg="mmse"):
    """Algorithm 2 for one received vector.

    Preprocessing: y^MRC = sum_c H_c^H y_c.  r = p = y^MRC, x = 0, and for
    t = 1..T:  w = sum_c H_c^H (H_c p);  e = rho p + w;
               alpha = ||r||^2 / Re(p^H e);  x += alpha p;  r' = r - alpha e;
               beta = ||r'||^2 / ||r||^2;  p = r' + beta p;  r = r'
    with rho = N0 / Es (MMSE) or 0 (ZF).
    """
    H = np.asarray(H, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    B, U = H.shape
    rho = (N0 / Es) if reg == "mmse" else 0.0
    Hc = partition_rows(H, C)
    yc = partition_rows(y, C)
    ymrc = np.zeros(U, np.complex128)
    for c in range(C):
        ymrc = ymrc + Hc[c].conj().T @ yc[c]
    r = ymrc.copy()
    p = r.copy()
    x = np.zeros(U, np.complex128)
    rr = float(np.real(np.vdot(r, r)))
    for _t in range(T):
        if rr == 0.0:
            break
        w = np.zeros(U, np.complex128)
        for c in range(C):
            w = w + Hc[c].conj().T @ (Hc[c] @ p)
        e = rho * p + w
        alpha = rr / float(np.real(np.vdot(p, e)))
        x = x + alpha * p
        r = r - alpha * e
        rr_new = float(np.real(np.vdot(r, r)))
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return x


def dcg_ul_frame(H, y, C, T, N0, Es=1.0, reg="mmse"):
    n_sc, B, U = H.shape
    n_sym = y.shape[1]
    out = np.zeros((n_sc, n_sym, U), np.complex128)
    for k in range(n_sc):
        for n in range(n_sym):
            out[k, n] = dcg_ul(H[k], y[k, n], C, T, N0, Es, reg)
    return out


# ---------------------------------------------------------------------------
# Algorithm 3: decentralized ADMM-based beamforming
# ---------------------------------------------------------------------------

def lemma2_factor(d, eps):
    """Scale max{0, 1 - eps / ||d||} of Lemma 2 for d = s - w (1 at eps = 0)."""
    if eps == 0.0:
        return 1.0
    nd = float(np.linalg.norm(d))
    return max(0.0, 1.0 - eps / nd) if nd > 0.0 else 0.0


def p1_budget(Hc, v, rho, P):
    """Step (P1) of Section IV-B with a per-cluster transmit-energy budget:

        x_c = argmin_x 1/2||x||^2 + rho/2||H_c x - v||^2  subject to ||x||^2 <= P

    (v = z_c + lambda_c, H_c the U x S downlink block).  Without the budget
    the minimiser is x(1/rho) with x(tau) = (H_c^H H_c + tau I)^{-1} H_c^H v.
    When ||x(1/rho)||^2 > P the budget is active: stationarity of the
    Lagrangian 1/2||x||^2 + rho/2||H_c x - v||^2 + mu/2 (||x||^2 - P) gives
    x = x(tau) with tau = (1 + mu) / rho > 1/rho, and tau solves
    ||x(tau)||^2 = P.  With H_c^H H_c = V diag(sig) V^H and b = V^H H_c^H v,
    ||x(tau)||^2 = sum_i |b_i|^2 / (sig_i + tau)^2 decreases strictly in tau,
    so the root is unique; it is found by a bracketing root search.
    Returns (x, tau)."""
    from scipy.optimize import brentq

    Hc = np.asarray(Hc, dtype=np.complex128)
    v = np.asarray(v, dtype=np.complex128)
    S = Hc.shape[1]
    G = Hc.conj().T @ Hc
    h = Hc.conj().T @ v
    tau0 = 1.0 / rho
    x0 = np.linalg.solve(G + tau0 * np.eye(S), h)
    if float(np.real(np.vdot(x0, x0))) <= P:
        return x0, tau0
    sig, V = np.linalg.eigh(G)
    b2 = np.abs(V.conj().T @ h) ** 2

    def f(tau):
        return float(np.sum(b2 / (sig + tau) ** 2)) - P

    hi = 2.0 * tau0
    while f(hi) > 0.0:
        hi *= 2.0
    tau = brentq(f, tau0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
    return np.linalg.solve(G + tau * np.eye(S), h), tau


def admm_dl(Hu, s, C, rho, T, gamma=1.0, mode=None, eps=0.0, P=None):
    """Algorithm 3 for one target vector s (U,).

    ``Hu`` is the uplink channel (B, U); by reciprocity the downlink channel is
    H^d = Hu^T, and cluster c owns the column block H_c = (Hu_c)^T (U x S).
    Preprocessing:  S <= U: A_c = H_c^H H_c + rho^-1 I_S,  x_c = A_c^{-1} H_c^H v
                    S >  U: B_c = H_c H_c^H + rho^-1 I_U,  x_c = H_c^H B_c^{-1} v
    Init: z_c = max(U/B, 1/C) s, lambda_c = 0, x_c = apply(z_c).
    For t = 2..T:  m_c = H_c x_c;  w_c = m_c - lambda_c;  w = sum_c w_c;
                   z_c = w_c + f (s - w)/C;  lambda_c -= gamma (m_c - z_c);
                   x_c = apply(z_c + lambda_c).
    f = 1 for eps = 0 (Algorithm 3); f = max{0, 1 - eps/||s - w||} for
    eps > 0 (Lemma 2, the z-update of problem P0 with ||s - H x|| <= eps).
    With per-cluster budgets P (length C) every x-update is the budgeted
    step (P1) of ``p1_budget`` instead (the constraint ||x_c||^2 <= P_c added
    to problem P0 and kept inside the cluster's own step).
    Returns x = [x_1; ...; x_C] (B,).
    """
    Hu = np.asarray(Hu, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    B, U = Hu.shape
    S = B // C
    if mode is None:
        mode = "SS" if S <= U else "UU"
    Hd = [blk.T for blk in partition_rows(Hu, C)]          # U x S each
    apply = []
    for c in range(C):
        Hk = Hd[c]
        if mode == "SS":
            A = Hk.conj().T @ Hk + (1.0 / rho) * np.eye(S)
            apply.append(lambda v, Hk=Hk, A=A: np.linalg.solve(A, Hk.conj().T @ v))
        elif mode == "UU":
            Bm = Hk @ Hk.conj().T + (1.0 / rho) * np.eye(U)
            apply.append(lambda v, Hk=Hk, Bm=Bm: Hk.conj().T @ np.linalg.solve(Bm, v))
        else:
            raise ValueError(mode)
    if P is not None:
        apply = [lambda v, c=c: p1_budget(Hd[c], v, rho, P[c])[0] for c in range(C)]
    z0 = max(U / B, 1.0 / C) * s
    z = [z0.copy() for _ in range(C)]
    lam = [np.zeros(U, np.complex128) for _ in range(C)]
    x = [apply[c](z[c]) for c in range(C)]
    for _t in range(2, T + 1):
        m = [Hd[c] @ x[c] for c in range(C)]
        wc = [m[c] - lam[c] for c in range(C)]
        w = np.zeros(U, np.complex128)
        for c in range(C):
            w = w + wc[c]
        f = lemma2_factor(s - w, eps)
        for c in range(C):
            z[c] = wc[c] + f * (s - w) / C
            lam[c] = lam[c] - gamma * (m[c] - z[c])
            x[c] = apply[c](z[c] + lam[c])
    return np.concatenate(x)


def project_ball_constraint(wall, s, D, eps):
    """argmin_z 1/2||wall - z||^2 subject to ||s - D z|| <= eps, without Lemma 2.

    If wall is feasible it is the answer.  Otherwise the constraint is active
    and the KKT conditions give z(mu) = (I + mu D^H D)^{-1} (wall + mu D^H s)
    for a multiplier mu > 0 with ||s - D z(mu)|| = eps; the residual falls
    monotonically in mu, so mu is found by a bracketing root search.
    """
    from scipy.optimize import brentq

    if np.linalg.norm(s - D @ wall) <= eps:
        return wall.copy()
    n = wall.size
    DhD = D.conj().T @ D
    Dhs = D.conj().T @ s

    def z_of(mu):
        return np.linalg.solve(np.eye(n) + mu * DhD, wall + mu * Dhs)

    def g(mu):
        return np.linalg.norm(s - D @ z_of(mu)) - eps

    hi = 1.0
    while g(hi) > 0.0:
        hi *= 4.0
    mu = brentq(g, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
    return z_of(mu)


def admm_dl_literal(Hu, s, C, rho, T, gamma=1.0, eps=0.0, P=None):
    """Section IV-B steps written as argmin / projection problems.

    Start z_c = max(U/B, 1/C) s, lambda_c = 0, then
      (P1) x_c = argmin 1/2||x||^2 + rho/2||H_c x - z_c - lambda_c||^2, as the
           stacked least-squares [sqrt(rho) H_c; I] x ~ [sqrt(rho)(z_c+lambda_c); 0];
    and T - 1 times
      (P2) z = orthogonal projection of (H_c x_c - lambda_c)_c onto
           {z : ||s - sum_c z_c|| <= eps}, with D = 1_{1 x C} kron I_U: for
           eps = 0 the affine projection z = w_all + pinv(D) (s - D w_all), for
           eps > 0 ``project_ball_constraint``;
      (P3) lambda_c = lambda_c - gamma (H_c x_c - z_c);
      (P1) as above.
    With per-cluster budgets P, (P1) is the same objective minimised over
    ||x||^2 <= P_c by a generic constrained solver (SLSQP on the real and
    imaginary parts), without the closed form of ``p1_budget``.
    """
    Hu = np.asarray(Hu, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    B, U = Hu.shape
    S = B // C
    Hd = [blk.T for blk in partition_rows(Hu, C)]
    sq = math.sqrt(rho)
    D = np.kron(np.ones((1, C)), np.eye(U))
    Dp = np.linalg.pinv(D)
    z = [max(U / B, 1.0 / C) * s for _ in range(C)]
    lam = [np.zeros(U, np.complex128) for _ in range(C)]

    def p1(c):
        Amat = np.vstack([sq * Hd[c], np.eye(S)])
        bvec = np.concatenate([sq * (z[c] + lam[c]), np.zeros(S)])
        x = np.linalg.lstsq(Amat, bvec, rcond=None)[0]
        if P is None or float(np.real(np.vdot(x, x))) <= P[c]:
            return x
        return _slsqp_budget_p1(Hd[c], z[c] + lam[c], rho, P[c], x)

    x = [p1(c) for c in range(C)]
    for _t in range(T - 1):
        wall = np.concatenate([Hd[c] @ x[c] - lam[c] for c in range(C)])
        if eps == 0.0:
            zall = wall + Dp @ (s - D @ wall)
        else:
            zall = project_ball_constraint(wall, s, D, eps)
        z = [zall[c * U:(c + 1) * U] for c in range(C)]
        lam = [lam[c] - gamma * (Hd[c] @ x[c] - z[c]) for c in range(C)]
        x = [p1(c) for c in range(C)]
    return np.concatenate(x)


def _slsqp_budget_p1(Hc, v, rho, P, x_start):
    """1/2||x||^2 + rho/2||H_c x - v||^2 over ||x||^2 <= P by SLSQP on the
    stacked real vector [Re x; Im x] (a generic solver, for pinning only)."""
    from scipy.optimize import minimize

    S = Hc.shape[1]

    def unpack(r):
        return r[:S] + 1j * r[S:]

    def obj(r):
        x = unpack(r)
        e = Hc @ x - v
        return 0.5 * float(np.real(np.vdot(x, x))) + 0.5 * rho * float(np.real(np.vdot(e, e)))

    def grad(r):
        x = unpack(r)
        g = x + rho * (Hc.conj().T @ (Hc @ x - v))
        return np.concatenate([g.real, g.imag])

    x0 = x_start * math.sqrt(P / float(np.real(np.vdot(x_start, x_start))))
    cons = {"type": "ineq", "fun": lambda r: P - float(r @ r), "jac": lambda r: -2.0 * r}
    res = minimize(obj, np.concatenate([x0.real, x0.imag]), jac=grad, constraints=[cons], method="SLSQP",
                   options={"ftol": 1e-15, "maxiter": 1000})
    return unpack(res.x)


def admm_dl_frame(Hu, s, C, rho, T, gamma=1.0, mode=None, eps=0.0, P=None):
    """Algorithm 3 over a frame: Hu [n_sc][B][U], s [n_sc][n_sym][U] -> x [n_sc][n_sym][B]
    (optional per-cluster budgets P, the budgeted step (P1))."""
    n_sc, B, U = Hu.shape
    n_sym = s.shape[1]
    out = np.zeros((n_sc, n_sym, B), np.complex128)
    for k in range(n_sc):
        for n in range(n_sym):
            out[k, n] = admm_dl(Hu[k], s[k, n], C, rho, T, gamma, mode, eps, P)
    return out


def power_scale(x, C, P):
    """Common gain beta = min(1, min_c sqrt(P_c / ||x_c||^2)) for one vector x (B,).

    Returns (beta * x, beta).  P is a length-C sequence of per-cluster budgets."""
    x = np.asarray(x, dtype=np.complex128)
    xs = partition_rows(x, C)
    beta = 1.0
    for c in range(C):
        e = float(np.real(np.vdot(xs[c], xs[c])))
        if e > 0.0:
            beta = min(beta, math.sqrt(P[c] / e))
    return beta * x, beta


# ---------------------------------------------------------------------------
# Centralized references (problem E0 with ZF / MMSE regularizers; problem P0
# with epsilon = 0, the ZF beamformer)
# ---------------------------------------------------------------------------

def mmse_detect(H, y, N0, Es=1.0):
    H = np.asarray(H, dtype=np.complex128)
    U = H.shape[1]
    return np.linalg.solve(H.conj().T @ H + (N0 / Es) * np.eye(U), H.conj().T @ y)


def zf_detect(H, y):
    return np.linalg.lstsq(np.asarray(H, dtype=np.complex128), y, rcond=None)[0]


def zf_precode(Hd, s):
    """Minimum-norm x with Hd x = s: x = Hd^H (Hd Hd^H)^{-1} s."""
    return np.linalg.pinv(np.asarray(Hd, dtype=np.complex128)) @ s


def eps_precode(Hd, s, eps):
    """Problem P0 for eps > 0: the minimum-norm x with ||s - Hd x|| <= eps.

    x = 0 if ||s|| <= eps.  Otherwise the constraint is active and stationarity
    of 1/2||x||^2 + nu/2 (||s - Hd x||^2 - eps^2) gives
    x = Hd^H (Hd Hd^H + t I)^{-1} s with t = 1/nu > 0.  With Hd = Q diag(sig) V^H
    and c = Q^H s the residual is ||s - Hd x||^2 = sum_i (t/(sig_i^2+t))^2 |c_i|^2
    (Hd of full row rank), increasing in t; t is found by a bracketing root
    search.
    """
    from scipy.optimize import brentq

    Hd = np.asarray(Hd, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    if np.linalg.norm(s) <= eps:
        return np.zeros(Hd.shape[1], np.complex128)
    Q, sig, Vh = np.linalg.svd(Hd, full_matrices=False)
    c = Q.conj().T @ s

    def g(t):
        return math.sqrt(float(np.sum((t / (sig ** 2 + t)) ** 2 * np.abs(c) ** 2))) - eps

    hi = 1.0
    while g(hi) < 0.0:
        hi *= 4.0
    t = brentq(g, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
    return Vh.conj().T @ (sig / (sig ** 2 + t) * c)
