"""Exact rational arithmetic versions of Algorithms 1, 2 and 3 for tiny instances.

TEST INFRASTRUCTURE ONLY (imported by the oracle's own tests).

Every step of Algorithms 1-3 uses only +, -, x and division, so with
Gaussian-integer inputs and rational parameters the iterates are exact complex
rationals.  This module carries them as pairs of ``fractions.Fraction`` in plain
Python loops (matrices as lists of rows, linear systems by Gaussian elimination),
so that the FP64 oracle can be checked against an exact result at finite T.
It is written independently of ``dbp_oracle`` and does not import it.
"""
from __future__ import annotations

from fractions import Fraction as F


class Q:
    """Exact complex rational a + i b."""
    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = F(re)
        self.im = F(im)

    def __add__(self, o):
        o = _q(o)
        return Q(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _q(o)
        return Q(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _q(o) - self

    def __neg__(self):
        return Q(-self.re, -self.im)

    def __mul__(self, o):
        o = _q(o)
        return Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def conj(self):
        return Q(self.re, -self.im)

    def abs2(self):
        return self.re * self.re + self.im * self.im

    def __truediv__(self, o):
        o = _q(o)
        d = o.abs2()
        n = self * o.conj()
        return Q(n.re / d, n.im / d)

    def __complex__(self):
        return complex(float(self.re), float(self.im))


def _q(x):
    if isinstance(x, Q):
        return x
    if isinstance(x, complex):
        return Q(F(x.real), F(x.imag))
    return Q(F(x), 0)


def mat(rows):
    return [[_q(v) for v in r] for r in rows]


def vec(v):
    return [_q(x) for x in v]


def hermitian(A):
    return [[A[i][j].conj() for i in range(len(A))] for j in range(len(A[0]))]


def transpose(A):
    return [[A[i][j] for i in range(len(A))] for j in range(len(A[0]))]


def matmul(A, Bm):
    n, k, m = len(A), len(Bm), len(Bm[0])
    return [[sum((A[i][t] * Bm[t][j] for t in range(k)), Q()) for j in range(m)]
            for i in range(n)]


def matvec(A, x):
    return [sum((A[i][t] * x[t] for t in range(len(x))), Q()) for i in range(len(A))]


def add_diag(A, d):
    return [[A[i][j] + (d if i == j else 0) for j in range(len(A))] for i in range(len(A))]


def solve(A, b):
    """Gaussian elimination with exact arithmetic (first nonzero pivot)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col].abs2() != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col].abs2() != 0:
                f = M[r][col] / M[col][col]
                M[r] = [M[r][j] - f * M[col][j] for j in range(n + 1)]
    return [M[i][n] / M[i][i] for i in range(n)]


def vadd(a, b):
    return [x + y for x, y in zip(a, b)]


def vsub(a, b):
    return [x - y for x, y in zip(a, b)]


def vscale(a, f):
    return [x * f for x in a]


def dot(a, b):
    """a^H b"""
    return sum((x.conj() * y for x, y in zip(a, b)), Q())


def clusters(rows, C):
    S = len(rows) // C
    return [rows[c * S:(c + 1) * S] for c in range(C)]


def admm_ul(H, y, C, rho, T, N0, Es=1, gamma=1, mode=None):
    """Algorithm 1 (MMSE proximal step) in exact arithmetic."""
    H, y = mat(H), vec(y)
    rho, N0, Es, gamma = F(rho), F(N0), F(Es), F(gamma)
    B, U = len(H), len(H[0])
    S = B // C
    if mode is None:
        mode = "SS" if S <= U else "UU"
    Hc, yc = clusters(H, C), clusters(y, C)
    yreg, K = [], []
    for c in range(C):
        Hk = Hc[c]
        HkH = hermitian(Hk)
        if mode == "SS":
            A = add_diag(matmul(Hk, HkH), rho)
            yreg.append(matvec(HkH, solve(A, yc[c])))
            K.append(lambda q, Hk=Hk, HkH=HkH, A=A: vsub(q, matvec(HkH, solve(A, matvec(Hk, q)))))
        else:
            Bm = add_diag(matmul(HkH, Hk), rho)
            yreg.append(solve(Bm, matvec(HkH, yc[c])))
            K.append(lambda q, Bm=Bm: vscale(solve(Bm, q), rho))
    scale = 1 / (N0 / (rho * Es) + C)
    lam = [[Q() for _ in range(U)] for _ in range(C)]
    z = [list(v) for v in yreg]
    w = [Q() for _ in range(U)]
    for c in range(C):
        w = vadd(w, z[c])
    s = vscale(w, scale)
    for _ in range(2, T + 1):
        w = [Q() for _ in range(U)]
        for c in range(C):
            lam[c] = vadd(lam[c], vscale(vsub(z[c], s), gamma))
            z[c] = vadd(yreg[c], K[c](vsub(s, lam[c])))
            w = vadd(w, vadd(z[c], lam[c]))
        s = vscale(w, scale)
    return [complex(v) for v in s]


def dcg_ul(H, y, C, T, N0, Es=1):
    """Algorithm 2 (MMSE, rho = N0/Es) in exact arithmetic."""
    H, y = mat(H), vec(y)
    rho = F(N0) / F(Es)
    U = len(H[0])
    Hc, yc = clusters(H, C), clusters(y, C)
    r = [Q() for _ in range(U)]
    for c in range(C):
        r = vadd(r, matvec(hermitian(Hc[c]), yc[c]))
    p = list(r)
    x = [Q() for _ in range(U)]
    rr = dot(r, r).re
    for _ in range(T):
        if rr == 0:
            break
        w = [Q() for _ in range(U)]
        for c in range(C):
            w = vadd(w, matvec(hermitian(Hc[c]), matvec(Hc[c], p)))
        e = vadd(vscale(p, rho), w)
        alpha = rr / dot(p, e).re
        x = vadd(x, vscale(p, alpha))
        r = vsub(r, vscale(e, alpha))
        rr_new = dot(r, r).re
        beta = rr_new / rr
        p = vadd(r, vscale(p, beta))
        rr = rr_new
    return [complex(v) for v in x]


def admm_dl(Hu, s, C, rho, T, gamma=1, mode=None):
    """Algorithm 3 (epsilon = 0) in exact arithmetic; Hu is the uplink channel."""
    Hu, s = mat(Hu), vec(s)
    rho, gamma = F(rho), F(gamma)
    B, U = len(Hu), len(Hu[0])
    S = B // C
    if mode is None:
        mode = "SS" if S <= U else "UU"
    Hd = [transpose(blk) for blk in clusters(Hu, C)]        # U x S
    apply = []
    for c in range(C):
        Hk = Hd[c]
        HkH = hermitian(Hk)
        if mode == "SS":
            A = add_diag(matmul(HkH, Hk), 1 / rho)
            apply.append(lambda v, A=A, HkH=HkH: solve(A, matvec(HkH, v)))
        else:
            Bm = add_diag(matmul(Hk, HkH), 1 / rho)
            apply.append(lambda v, Bm=Bm, HkH=HkH: matvec(HkH, solve(Bm, v)))
    f0 = max(F(U, B), F(1, C))
    z = [vscale(s, f0) for _ in range(C)]
    lam = [[Q() for _ in range(U)] for _ in range(C)]
    x = [apply[c](z[c]) for c in range(C)]
    for _ in range(2, T + 1):
        m = [matvec(Hd[c], x[c]) for c in range(C)]
        wc = [vsub(m[c], lam[c]) for c in range(C)]
        w = [Q() for _ in range(U)]
        for c in range(C):
            w = vadd(w, wc[c])
        for c in range(C):
            z[c] = vadd(wc[c], vscale(vsub(s, w), F(1, C)))
            lam[c] = vsub(lam[c], vscale(vsub(m[c], z[c]), gamma))
            x[c] = apply[c](vadd(z[c], lam[c]))
    out = []
    for c in range(C):
        out.extend(complex(v) for v in x[c])
    return out
