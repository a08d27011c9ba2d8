"""Analytic test fields and closed-form right-hand sides (test helpers; no product code).

The exact RHS is derived symbolically from the continuous compressible NS equations in
total-energy flux form (Sec. 2, Eqs. cont, mome, ie, with an ideal gas, mu = mu_ref (T/T_ref)^n
and k = mu c_p / Pr), so it shares nothing with either the oracle or the GPU library.
"""
from __future__ import annotations

import functools
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def grid(n):
    """Coordinates x, y, z of an (nz, ny, nx) grid on [0, 2 pi)^3, index order [z][y][x]."""
    nx, ny, nz = n
    x = np.arange(nx) * TWO_PI / nx
    y = np.arange(ny) * TWO_PI / ny
    z = np.arange(nz) * TWO_PI / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def conservative(rho, u, v, w, T, gamma=1.4, gas_r=1.0):
    cv = gas_r / (gamma - 1.0)
    return np.stack([rho, rho * u, rho * v, rho * w, rho * (cv * T + 0.5 * (u * u + v * v + w * w))])


@functools.lru_cache(maxsize=None)
def _symbolic(gamma, gas_r, prandtl, mu_ref, t_ref, mu_exp_num, mu_exp_den):
    import sympy as sp
    x, y, z, t = sp.symbols("x y z t", real=True)
    rho = 1 + sp.Rational(1, 10) * sp.sin(y + z + 3 * t) + sp.Rational(1, 20) * sp.cos(x - t)
    u = sp.Rational(3, 10) * sp.sin(x + 2 * t) * sp.cos(y) + sp.Rational(1, 10) * sp.cos(z - t)
    v = -sp.Rational(1, 5) * sp.cos(x) * sp.sin(y + t) + sp.Rational(1, 10) * sp.sin(z)
    w = sp.Rational(1, 10) * sp.sin(x + y - t) + sp.Rational(1, 20) * sp.cos(2 * z)
    T = 1 + sp.Rational(1, 10) * sp.cos(x - 2 * z + t)
    g = sp.nsimplify(gamma)
    R = sp.nsimplify(gas_r)
    cv = R / (g - 1)
    cp = g * R / (g - 1)
    mu = sp.nsimplify(mu_ref) * (T / sp.nsimplify(t_ref)) ** sp.Rational(mu_exp_num, mu_exp_den)
    kap = mu * cp / sp.nsimplify(prandtl)
    vel = [u, v, w]
    X = [x, y, z]
    p = rho * R * T
    E = rho * (cv * T + (u * u + v * v + w * w) / 2)
    Gm = [[sp.diff(vel[i], X[j]) for j in range(3)] for i in range(3)]
    th = Gm[0][0] + Gm[1][1] + Gm[2][2]
    sig = [[mu * (Gm[i][j] + Gm[j][i]) - (sp.Rational(2, 3) * mu * th if i == j else 0)
            for j in range(3)] for i in range(3)]
    q = [rho, rho * u, rho * v, rho * w, E]
    rhs = []
    for c in range(5):
        div = 0
        for j in range(3):
            if c == 0:
                F = rho * vel[j]
            elif c <= 3:
                i = c - 1
                F = rho * vel[i] * vel[j] + (p if i == j else 0) - sig[i][j]
            else:
                F = (E + p) * vel[j] - sum(vel[i] * sig[i][j] for i in range(3)) - kap * sp.diff(T, X[j])
            div += sp.diff(F, X[j])
        rhs.append(-div)
    fq = sp.lambdify((x, y, z, t), q, "numpy")
    fr = sp.lambdify((x, y, z, t), rhs, "numpy")
    return fq, fr


@functools.lru_cache(maxsize=None)
def _symbolic_paper(gamma, gas_r, prandtl, mu_ref, t_ref, law, law_num, law_den):
    """The same analytic fields in the paper's variables (rho, rho u_i, rho e), e = c_v T, and the
    exact right-hand side of Sec. 2, Eqs. cont, mome, ie (internal-energy form) with the power law
    (law = "power", exponent law_num / law_den) or Sutherland's law (law = "sutherland", constant
    S = law_num / law_den)."""
    import sympy as sp
    x, y, z, t = sp.symbols("x y z t", real=True)
    rho = 1 + sp.Rational(1, 10) * sp.sin(y + z + 3 * t) + sp.Rational(1, 20) * sp.cos(x - t)
    u = sp.Rational(3, 10) * sp.sin(x + 2 * t) * sp.cos(y) + sp.Rational(1, 10) * sp.cos(z - t)
    v = -sp.Rational(1, 5) * sp.cos(x) * sp.sin(y + t) + sp.Rational(1, 10) * sp.sin(z)
    w = sp.Rational(1, 10) * sp.sin(x + y - t) + sp.Rational(1, 20) * sp.cos(2 * z)
    T = 1 + sp.Rational(1, 10) * sp.cos(x - 2 * z + t)
    g = sp.nsimplify(gamma)
    R = sp.nsimplify(gas_r)
    cv = R / (g - 1)
    cp = g * R / (g - 1)
    Tr = sp.nsimplify(t_ref)
    if law == "power":
        mu = sp.nsimplify(mu_ref) * (T / Tr) ** sp.Rational(law_num, law_den)
    else:
        S = sp.Rational(law_num, law_den)
        mu = sp.nsimplify(mu_ref) * (T / Tr) ** sp.Rational(3, 2) * (Tr + S) / (T + S)
    kap = mu * cp / sp.nsimplify(prandtl)
    vel = [u, v, w]
    X = [x, y, z]
    p = rho * R * T
    re = rho * cv * T
    Gm = [[sp.diff(vel[i], X[j]) for j in range(3)] for i in range(3)]
    th = Gm[0][0] + Gm[1][1] + Gm[2][2]
    sig = [[mu * (Gm[i][j] + Gm[j][i]) - (sp.Rational(2, 3) * mu * th if i == j else 0)
            for j in range(3)] for i in range(3)]
    q = [rho, rho * u, rho * v, rho * w, re]
    rhs = [-sum(sp.diff(rho * vel[j], X[j]) for j in range(3))]
    for i in range(3):
        rhs.append(-sum(sp.diff(rho * vel[i] * vel[j], X[j]) for j in range(3)) - sp.diff(p, X[i])
                   + sum(sp.diff(sig[i][j], X[j]) for j in range(3)))
    diss = sum(sig[i][j] * (Gm[i][j] + Gm[j][i]) / 2 for i in range(3) for j in range(3))
    rhs.append(-sum(sp.diff(re * vel[j], X[j]) for j in range(3)) - p * th
               + sum(sp.diff(kap * sp.diff(T, X[j]), X[j]) for j in range(3)) + diss)
    fq = sp.lambdify((x, y, z, t), q, "numpy")
    fr = sp.lambdify((x, y, z, t), rhs, "numpy")
    return fq, fr


def analytic_paper(n, t, law="power", law_param=(19, 25), gamma=1.4, gas_r=1.0, prandtl=0.7, mu_ref=0.05,
                   t_ref=1.0):
    """(state, exact RHS) of the paper's internal-energy form on an (nz, ny, nx) grid at time t."""
    fq, fr = _symbolic_paper(gamma, gas_r, prandtl, mu_ref, t_ref, law, law_param[0], law_param[1])
    X, Y, Z = grid(n)
    st = np.stack([np.broadcast_to(np.asarray(a, dtype=np.float64), X.shape) for a in fq(X, Y, Z, t)])
    rh = np.stack([np.broadcast_to(np.asarray(a, dtype=np.float64), X.shape) for a in fr(X, Y, Z, t)])
    return st, rh


def analytic_state(n, t, gamma=1.4, gas_r=1.0, prandtl=0.7, mu_ref=0.05, t_ref=1.0, mu_exp=(19, 25)):
    fq, _ = _symbolic(gamma, gas_r, prandtl, mu_ref, t_ref, mu_exp[0], mu_exp[1])
    X, Y, Z = grid(n)
    return np.stack([np.broadcast_to(np.asarray(a, dtype=np.float64), X.shape) for a in fq(X, Y, Z, t)])


def analytic_rhs(n, t, gamma=1.4, gas_r=1.0, prandtl=0.7, mu_ref=0.05, t_ref=1.0, mu_exp=(19, 25)):
    _, fr = _symbolic(gamma, gas_r, prandtl, mu_ref, t_ref, mu_exp[0], mu_exp[1])
    X, Y, Z = grid(n)
    return np.stack([np.broadcast_to(np.asarray(a, dtype=np.float64), X.shape) for a in fr(X, Y, Z, t)])


def modified_wavenumber(m, h):
    """k'_m of the 4th-order central first derivative: D sin(m x) = k'_m cos(m x)."""
    return (8.0 * math.sin(m * h) - math.sin(2.0 * m * h)) / (6.0 * h)


def rk3_amplification(z):
    """Stability polynomial of any 3-stage, third-order explicit Runge-Kutta method."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0


def read_appb(path):
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, stencil, side, div = [s.strip() for s in line.split("|")]
        hs = head.split()
        # w: the coefficients of the weight polynomial in k, highest power first
        rows.append(dict(side=hs[0], l=int(hs[1]), w=tuple(float(v) for v in hs[2:]),
                         a=[float(v) for v in stencil.split()], delayed=side, div=float(div)))
    return rows
