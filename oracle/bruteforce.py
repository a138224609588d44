"""Brute-force time step for tiny lattices (e.g. 3x3), written independently of
``lbm_oracle.c`` to pin it.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Everything is pure Python over nodes and velocity indices with the equations taken as
printed: the force sums of Eq. 6 run over alpha = 0..8 (the rest velocity adds zero), the
Guo term (Eq. 23 / Eq. 31) is an explicit i, j tensor contraction, the moment matrix is the
numeric Lallemand-Luo table and its inverse comes from numpy.linalg.inv, and streaming is
written in the gather form f_a(x, t+1) = f*_a(x - e_a, t), equivalent to Eq. 36.
Same readings as the C stepper (see its header).
"""
from __future__ import annotations

import math

import numpy as np

E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
CS2 = 1 / 3

# Lallemand-Luo moment matrix for the velocity order E, rows (rho, e, eps, jx, qx, jy, qy,
# pxx, pxy) as in Eq. 35.
M_TABLE = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=float)


def w_of_e2(e):
    """w(|e|^2): 1/3 for |e|^2 = 1, 1/12 for |e|^2 = 2 (Eq. 4); 0 for the rest velocity."""
    e2 = e[0] ** 2 + e[1] ** 2
    return {0: 0.0, 1: 1 / 3, 2: 1 / 12}[e2]


def pressure(rho, T, a, b, R, K):
    eta = b * rho / 4
    return K * (rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2)


def feq(rho, u):
    out = []
    for a in range(9):
        eu = E[a][0] * u[0] + E[a][1] * u[1]
        uu = u[0] ** 2 + u[1] ** 2
        out.append(W[a] * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2)))
    return out


def guo_term(F, V):
    """w_a [F_i e_ai / cs^2 + (F_i V_j + V_i F_j)(e_ai e_aj - cs^2 delta_ij) / (2 cs^4)]."""
    out = []
    for a in range(9):
        e = E[a]
        s = sum(F[i] * e[i] for i in range(2)) / CS2
        for i in range(2):
            for j in range(2):
                s += (F[i] * V[j] + V[i] * F[j]) * (e[i] * e[j] - CS2 * (i == j)) / (2 * CS2 ** 2)
        out.append(W[a] * s)
    return out


def step(f, nx, ny, T, tau, scheme, collision, a=1.0, b=4.0, R=1.0, K=1.0, G=-1.0, A=0.0,
         sigma=0.0, s=(1.0,) * 9, ss_eps=None):
    """One time step; f is indexed f[alpha][y][x] (nested lists or an array).
    scheme: 'EDM', 'GUO', 'GUO_LI', 'SC'; collision: 'BGK' or 'MRT'.
    ss_eps: None for psi from the EOS (Eq. 7), else the exponent of Eq. 33's psi."""
    nodes = [(x, y) for y in range(ny) for x in range(nx)]
    rho = {n: sum(f[al][n[1]][n[0]] for al in range(9)) for n in nodes}
    psi = {}
    for n in nodes:
        if ss_eps is None:
            U = pressure(rho[n], T, a, b, R, K) - CS2 * rho[n]  # Eq. 7
            psi[n] = math.sqrt(2 * U / G)
        elif ss_eps == 0:
            psi[n] = math.exp(-1.0 / rho[n])                      # Eq. 33, eps = 0
        else:
            psi[n] = (rho[n] / (1.0 + rho[n])) ** (1.0 / ss_eps)   # Eq. 33
    F = {}
    for (x, y) in nodes:
        Fx = Fy = 0.0
        for al in range(9):
            ex, ey = E[al]
            nb = ((x + ex) % nx, (y + ey) % ny)
            Unb = G * psi[nb] ** 2 / 2
            term = -A * w_of_e2(E[al]) * Unb - (1 - A) * G * psi[(x, y)] * w_of_e2(E[al]) * psi[nb]
            Fx += term * ex
            Fy += term * ey
        F[(x, y)] = (Fx, Fy)
    Minv = np.linalg.inv(M_TABLE)
    post = {}
    for n in nodes:
        fn = [f[al][n[1]][n[0]] for al in range(9)]
        r = rho[n]
        u = (sum(fn[al] * E[al][0] for al in range(9)) / r,
             sum(fn[al] * E[al][1] for al in range(9)) / r)
        Fn = F[n]
        v = (u[0] + Fn[0] / (2 * r), u[1] + Fn[1] / (2 * r))
        if collision == "BGK":
            if scheme == "SC":
                fe = feq(r, (u[0] + tau * Fn[0] / r, u[1] + tau * Fn[1] / r))
                post[n] = [fn[al] - (fn[al] - fe[al]) / tau for al in range(9)]
            elif scheme == "EDM":
                fe = feq(r, u)
                fs = feq(r, (u[0] + Fn[0] / r, u[1] + Fn[1] / r))
                post[n] = [fn[al] - (fn[al] - fe[al]) / tau + fs[al] - fe[al] for al in range(9)]
            else:
                vb = v
                if scheme == "GUO_LI":
                    c = sigma / ((tau - 0.5) * psi[n] ** 2)
                    vb = (v[0] + c * Fn[0], v[1] + c * Fn[1])
                fe = feq(r, v)
                g = guo_term(Fn, vb)
                post[n] = [fn[al] - (fn[al] - fe[al]) / tau + (1 - 1 / (2 * tau)) * g[al]
                           for al in range(9)]
        else:
            m = M_TABLE @ np.array(fn)
            meq = M_TABLE @ np.array(feq(r, v))
            S = M_TABLE @ np.array(guo_term(Fn, v))
            if scheme == "GUO_LI":
                X = np.array([[Fn[i] * Fn[j] for j in range(2)] for i in range(2)])
                X *= 2 * sigma / psi[n] ** 2
                S[1] += 3 * np.trace(X) / (1 / s[1] - 0.5)
                S[2] -= 3 * np.trace(X) / (1 / s[2] - 0.5)
                S[7] += (X[0, 0] - X[1, 1]) / (1 / s[7] - 0.5)
                S[8] += X[0, 1] / (1 / s[8] - 0.5)
            Lam = np.diag(s)
            mstar = m - Lam @ (m - meq) + (np.eye(9) - Lam / 2) @ S
            post[n] = list(Minv @ mstar)
    out = np.zeros((9, ny, nx))
    for al in range(9):
        for (x, y) in nodes:
            src = ((x - E[al][0]) % nx, (y - E[al][1]) % ny)
            out[al, y, x] = post[src][al]
    return out
