"""Brute-force and closed-form references used to pin the oracle.

Nothing here calls the oracle's arithmetic: the dense operators below are
assembled in numpy from the mesh geometry arrays (vector areas, face-cell
adjacency, volumes) and solved with ``numpy.linalg.solve``; graph facts are
computed by exhaustive reachability; the pure-absorber closed form is
evaluated in mpmath."""
from __future__ import annotations

import math

import numpy as np


def face_dots(S, omega, dim):
    """Omega . S for every (direction, face), evaluated left to right."""
    om = np.asarray(omega)
    d = om[:, None, 0] * S[None, :, 0] + om[:, None, 1] * S[None, :, 1]
    if dim == 3:
        d = d + om[:, None, 2] * S[None, :, 2]
    return d


def edges_for_direction(S, fcell, omega_m, dim):
    """Interior sweep edges (u, v): v needs u's outgoing flux."""
    d = face_dots(S, omega_m[None, :], dim)[0]
    out = []
    for f in range(len(fcell)):
        K, L = fcell[f]
        if L < 0 or d[f] == 0.0:
            continue
        out.append((K, L) if d[f] > 0 else (L, K))
    return out


def reachability(n, edges):
    R = np.zeros((n, n), dtype=bool)
    for u, v in edges:
        R[u, v] = True
    for k in range(n):  # Warshall
        R |= R[:, k:k + 1] & R[k:k + 1, :]
    return R


def lag_rule_bruteforce(n, edges):
    """Edges u -> v with u > v whose endpoints lie on a common cycle."""
    R = reachability(n, edges)
    lag = set()
    for u, v in edges:
        if R[u, v] and R[v, u] and u > v:
            lag.add((u, v))
    return lag


def longest_path_levels(n, edges):
    """level(v) = 0 without predecessors else 1 + max predecessor level,
    by memoised depth-first search (the graph must be acyclic)."""
    preds = [[] for _ in range(n)]
    for u, v in edges:
        preds[v].append(u)
    memo = [-1] * n
    import sys
    sys.setrecursionlimit(max(10000, 4 * n))

    def lev(v):
        if memo[v] < 0:
            memo[v] = 0 if not preds[v] else 1 + max(lev(u) for u in preds[v])
        return memo[v]

    return np.array([lev(v) for v in range(n)], dtype=np.int64)


def cell_face_terms(S, fcell, cface, K, j):
    """Outward vector area of local face j of cell K and the neighbour."""
    f = cface[K, j]
    if fcell[f, 0] == K:
        return S[f], fcell[f, 1]
    return -S[f], fcell[f, 0]


def dense_direction_operator(S, fcell, cface, vol, sigma_t, omega_m, dim, lagged=frozenset()):
    """Matrix L_m (V-weighted balance) and the boundary-inflow indicator.
    Row K: (sigma_t V + sum_out a) psi_K - sum_in a psi_up (non-lagged).
    Returns (L, bnd_in, lag_terms) with bnd_in[K] = sum of a over inflow
    boundary faces and lag_terms a list (K, up, a) of lagged inflows."""
    n = len(vol)
    L = np.zeros((n, n))
    bnd = np.zeros(n)
    lag_terms = []
    om = np.asarray(omega_m)
    for K in range(n):
        L[K, K] = sigma_t[K] * vol[K]
        for j in range(cface.shape[1]):
            s, nb = cell_face_terms(S, fcell, cface, K, j)
            d = om[0] * s[0] + om[1] * s[1] + (om[2] * s[2] if dim == 3 else 0.0)
            if d > 0:
                L[K, K] += d
            elif d < 0:
                if nb < 0:
                    bnd[K] += -d
                elif (nb, K) in lagged:
                    lag_terms.append((K, nb, -d))
                else:
                    L[K, nb] -= -d
    return L, bnd, lag_terms


def dense_si_solution(S, fcell, cface, vol, sigma_t, sigma_s, q, omega, weight, dim, psi_b=0.0):
    """Solve the full discrete system (un-lagged streaming + isotropic
    scattering) densely: returns psi [nd, n]."""
    n, nd = len(vol), len(weight)
    A = np.zeros((n * nd, n * nd))
    b = np.zeros(n * nd)
    for m in range(nd):
        L, bnd, _ = dense_direction_operator(S, fcell, cface, vol, sigma_t, omega[m], dim)
        A[m * n:(m + 1) * n, m * n:(m + 1) * n] += L
        b[m * n:(m + 1) * n] = vol * q + bnd * psi_b
        for mp in range(nd):
            A[m * n:(m + 1) * n, mp * n:(mp + 1) * n] -= np.diag(sigma_s * vol * weight[mp])
    return np.linalg.solve(A, b).reshape(nd, n)


def dense_mg_solution(S, fcell, cface, vol, sigma_t, sigma_s, q, omega, weight, dim, psi_b=0.0):
    """Dense solve of the multigroup system: unknowns psi[g, m, K]; block
    (g, m) holds the un-lagged streaming operator with sigma_t,g, and every
    (g', m') couples into (g, m) through -sigma_s[g', g] V w_m'.  Returns
    psi [G, nd, n]."""
    G, n, nd = sigma_t.shape[0], len(vol), len(weight)
    M = G * nd * n
    A = np.zeros((M, M))
    b = np.zeros(M)
    blk = lambda g, m: slice((g * nd + m) * n, (g * nd + m + 1) * n)  # noqa: E731
    for g in range(G):
        for m in range(nd):
            L, bnd, _ = dense_direction_operator(S, fcell, cface, vol, sigma_t[g], omega[m], dim)
            A[blk(g, m), blk(g, m)] += L
            b[blk(g, m)] = vol * q[g] + bnd * psi_b
            for gp in range(G):
                for mp in range(nd):
                    A[blk(g, m), blk(gp, mp)] -= np.diag(sigma_s[gp, g] * vol * weight[mp])
    return np.linalg.solve(A, b).reshape(G, nd, n)


def closed_form_absorber(n, h, sigma_t, q, omega, digits=50):
    """Pure absorber on an undeformed n^3 hexahedral lattice with vacuum
    boundaries: the step recursion psi = g + a psi_x + b psi_y + c psi_z
    unrolled over lattice paths, in mpmath.  Returns psi[i, j, k] indexed
    by lattice position (0-based, physical orientation)."""
    import mpmath as mp

    mp.mp.dps = digits
    mu, eta, xi = (mp.mpf(abs(float(x))) for x in omega)
    D = mp.mpf(sigma_t) * mp.mpf(h) + mu + eta + xi
    a, b, c, g = mu / D, eta / D, xi / D, mp.mpf(q) * mp.mpf(h) / D
    fact = [mp.factorial(k) for k in range(3 * n + 1)]
    out = np.zeros((n, n, n))
    for I in range(1, n + 1):
        for J in range(1, n + 1):
            for K in range(1, n + 1):
                s = mp.mpf(0)
                for p in range(I):
                    for r in range(J):
                        for t in range(K):
                            s += fact[p + r + t] / (fact[p] * fact[r] * fact[t]) * a ** p * b ** r * c ** t
                # map inflow-corner indices to physical lattice positions
                i = I - 1 if omega[0] > 0 else n - I
                j = J - 1 if omega[1] > 0 else n - J
                k = K - 1 if omega[2] > 0 else n - K
                out[i, j, k] = float(g * s)
    return out
