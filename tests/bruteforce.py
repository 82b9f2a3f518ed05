"""Brute-force triplet / quadruplet counting on tiny grids: pins for the oracle.

These functions share nothing with the oracle: their own offset enumeration
(integer bin edges, so the (e_b, e_{b+1}] test is an integer comparison),
their own angular functions (Legendre polynomials for the 3PCF via the
addition theorem, an explicit associated-Legendre Y_lm and sympy's 3j symbols
for the 4PCF, cos/sin of the polar angle for the projected forms), and sums
over explicit pairs / triples of offsets about every cell.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import lpmv


def int_offsets(shape, edges_int):
    """All offsets r with e_b^2 < |r|^2 <= e_{b+1}^2 (integer edges), r != 0."""
    nd = len(shape)
    emax = int(edges_int[-1])
    rng = range(-emax, emax + 1)
    offs, bins = [], []
    for r in np.ndindex(*([2 * emax + 1] * nd)):
        v = tuple(int(t) - emax for t in r)
        n = sum(t * t for t in v)
        if n == 0:
            continue
        # keep only offsets that are distinct cells of the periodic grid
        ok = all((2 * t < s and -2 * t <= s) for t, s in zip(v, shape))
        if not ok:
            continue
        for b in range(len(edges_int) - 1):
            if edges_int[b] ** 2 < n <= edges_int[b + 1] ** 2:
                offs.append(v)
                bins.append(b)
                break
    del rng
    return np.array(offs, dtype=np.int64), np.array(bins, dtype=np.int64)


def neighbour_matrix(delta, offs):
    """V[x, o] = delta((x + r_o) mod N) for every cell x (flat) and offset o."""
    nd = delta.ndim
    idx = np.indices(delta.shape).reshape(nd, -1).T
    V = np.empty((idx.shape[0], offs.shape[0]))
    for o, r in enumerate(offs):
        j = (idx + r) % np.array(delta.shape)
        V[:, o] = delta[tuple(j.T)]
    return V


def zeta3_legendre(delta, edges_int, lmax):
    """sum_x delta(x) sum_{r1 in b1, r2 in b2} delta(x+r1) delta(x+r2) (2l+1)/(4 pi) L_l(r1^.r2^).

    By the addition theorem this equals sum_x delta sum_m a^b1_lm conj(a^b2_lm)
    with a^b_lm = sum_{r in b} conj(Y_lm(r^)) delta(x+r)."""
    offs, bins = int_offsets(delta.shape, edges_int)
    V = neighbour_matrix(delta, offs)
    M = (V * delta.reshape(-1)[:, None]).T @ V
    u = offs / np.linalg.norm(offs, axis=1)[:, None]
    C = np.clip(u @ u.T, -1.0, 1.0)
    nb = len(edges_int) - 1
    out = np.zeros((lmax + 1, nb, nb))
    for l in range(lmax + 1):
        coef = np.zeros(l + 1)
        coef[l] = 1.0
        P = npleg.legval(C, coef) * (2 * l + 1) / (4 * math.pi)
        MP = M * P
        for b1 in range(nb):
            for b2 in range(nb):
                out[l, b1, b2] = MP[np.ix_(bins == b1, bins == b2)].sum()
    return out


def ylm_explicit(l, m, u):
    """Y_lm(u^) = N_lm P_l^m(cos theta) e^{i m phi}, Condon-Shortley phase included
    in scipy's lpmv; negative m from Y_{l,-m} = (-1)^m conj(Y_lm)."""
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    mm = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - mm) / math.factorial(l + mm))
    val = norm * lpmv(mm, l, z) * np.exp(1j * mm * np.arctan2(y, x))
    if m < 0:
        val = (-1) ** mm * np.conj(val)
    return val


def zeta4_quadruplets(delta, edges_int, lam):
    """sum_x delta(x) sum_{r1,r2,r3} delta(x+r1) delta(x+r2) delta(x+r3) F(r1^, r2^, r3^)
    with F = sum_M 3j(Lambda; M) conj(Y_l1m1(r1^) Y_l2m2(r2^) Y_l3m3(r3^)) tabulated over
    every offset triple, for one Lambda.  Returns (nb, nb, nb) complex."""
    from sympy.physics.wigner import wigner_3j
    l1, l2, l3 = lam
    offs, bins = int_offsets(delta.shape, edges_int)
    u = offs / np.linalg.norm(offs, axis=1)[:, None]
    n = offs.shape[0]
    F = np.zeros((n, n, n), dtype=np.complex128)
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            m3 = -m1 - m2
            if abs(m3) > l3:
                continue
            w = float(wigner_3j(l1, l2, l3, m1, m2, m3))
            if w == 0.0:
                continue
            A = np.conj(ylm_explicit(l1, m1, u))
            B = np.conj(ylm_explicit(l2, m2, u))
            C = np.conj(ylm_explicit(l3, m3, u))
            F += w * A[:, None, None] * B[None, :, None] * C[None, None, :]
    V = neighbour_matrix(delta, offs)
    d = delta.reshape(-1)
    nb = len(edges_int) - 1
    out = np.zeros((nb, nb, nb), dtype=np.complex128)
    # T[x, o1, o2] = sum_o3 F[o1,o2,o3] V[x,o3]  per bin of o3
    for b3 in range(nb):
        s3 = bins == b3
        T = np.einsum("ijk,xk->xij", F[:, :, s3], V[:, s3])
        for b2 in range(nb):
            s2 = bins == b2
            U = np.einsum("xij,xj->xi", T[:, :, s2], V[:, s2])
            for b1 in range(nb):
                s1 = bins == b1
                out[b1, b2, b3] = np.sum(d * np.einsum("xi,xi->x", U[:, s1], V[:, s1]))
    return out


def zeta4_0ll_legendre(delta, edges_int, l):
    """Lambda = (0, l, l): sum_M 3j Y Y Y reduces to (-1)^l sqrt(2l+1) / (4 pi)^{3/2} L_l(r2^.r3^),
    so the 4PCF is a pair-angle sum weighted by the bin-b1 neighbour total."""
    offs, bins = int_offsets(delta.shape, edges_int)
    V = neighbour_matrix(delta, offs)
    d = delta.reshape(-1)
    u = offs / np.linalg.norm(offs, axis=1)[:, None]
    C = np.clip(u @ u.T, -1.0, 1.0)
    coef = np.zeros(l + 1)
    coef[l] = 1.0
    P = npleg.legval(C, coef) * (-1) ** l * math.sqrt(2 * l + 1) / (4 * math.pi) ** 1.5
    nb = len(edges_int) - 1
    out = np.zeros((nb, nb, nb))
    for b1 in range(nb):
        s1 = V[:, bins == b1].sum(axis=1)
        w = d * s1
        M = (V * w[:, None]).T @ V
        MP = M * P
        for b2 in range(nb):
            for b3 in range(nb):
                out[b1, b2, b3] = MP[np.ix_(bins == b2, bins == b3)].sum()
    return out


def zeta3_proj_pairs(delta, edges_int, mmax):
    """sum_x delta sum_{rho1 in b1, rho2 in b2} delta delta e^{-i m (phi1 - phi2)}, m = 0..mmax."""
    offs, bins = int_offsets(delta.shape, edges_int)
    V = neighbour_matrix(delta, offs)
    M = (V * delta.reshape(-1)[:, None]).T @ V
    phi = np.arctan2(offs[:, 1].astype(float), offs[:, 0].astype(float))
    nb = len(edges_int) - 1
    out = np.zeros((mmax + 1, nb, nb), dtype=np.complex128)
    for m in range(mmax + 1):
        # cos/sin form of the phase, not a complex exponential
        dphi = phi[:, None] - phi[None, :]
        ph = np.cos(m * dphi) - 1j * np.sin(m * dphi)
        MP = M * ph
        for b1 in range(nb):
            for b2 in range(nb):
                out[m, b1, b2] = MP[np.ix_(bins == b1, bins == b2)].sum()
    return out


def zeta4_proj_triples(delta, edges_int, m1, m2):
    """sum_x delta sum_{rho1,rho2,rho3} delta delta delta e^{-i (m1 phi1 + m2 phi2 + m3 phi3)}, m3 = -(m1+m2)."""
    m3 = -(m1 + m2)
    offs, bins = int_offsets(delta.shape, edges_int)
    V = neighbour_matrix(delta, offs)
    d = delta.reshape(-1)
    phi = np.arctan2(offs[:, 1].astype(float), offs[:, 0].astype(float))
    nb = len(edges_int) - 1
    out = np.zeros((nb, nb, nb), dtype=np.complex128)
    e = lambda m: np.cos(m * phi) - 1j * np.sin(m * phi)  # noqa: E731
    W1 = V * e(m1)[None, :]
    W2 = V * e(m2)[None, :]
    W3 = V * e(m3)[None, :]
    for b1 in range(nb):
        s1 = W1[:, bins == b1].sum(axis=1)
        for b2 in range(nb):
            s2 = W2[:, bins == b2].sum(axis=1)
            for b3 in range(nb):
                s3 = W3[:, bins == b3].sum(axis=1)
                out[b1, b2, b3] = np.sum(d * s1 * s2 * s3)
    return out
