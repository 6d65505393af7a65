"""Oracle of the double-layer operator K(s) and the direct Dirichlet solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 (eq. wavebio) defines the double-layer operator with the normal
derivative of the fundamental solution taken at the source point y; in the
Laplace domain (eq. fundsol) its kernel is

    d/dn_y  exp(-s r) / (4 pi r) = (1 + s r) exp(-s r) (x - y).n_y / (4 pi r^3),

r = |x - y|, n_y the unit normal of the source triangle (outward for the
meshes used here: the triangle's vertex order).  For a pure Dirichlet
boundary (Gamma_D = Gamma, g_N absent) the Galerkin formulation of Section
2.2 (eq. wavegalform) reduces to the direct equation

    < w, V q >  =  < w, (-1/2 I + K) g_D >

for the Neumann datum q; Section 3.2 turns it, frequency by frequency, into
V_l q_l = (-1/2 I + K_l) g_l.

Reading taken here (the paper represents g_D in the piecewise-linear space
S_h^1): the Dirichlet datum is represented in S_h^0, by its L2 projection
onto piecewise constants (coefficients c_i = int_tau_i g_D / |tau_i|, the
right-hand side b of the single-layer solve divided by the areas), so K_l is
the square piecewise-constant Galerkin matrix

    K_l[i, j] = int_tau_i int_tau_j d/dn_y G(x - y, s_l) dS(y) dS(x)

and I is the piecewise-constant mass matrix diag(|tau_i|).

Quadrature (the same pair classes as the single layer): pairs sharing no
vertex use the 6-point rule on both triangles; pairs sharing a vertex split
the kernel into the static Laplace part (x - y).n_y / (4 pi r^3) and the
bounded remainder (exp(-s r)(1 + s r) - 1)(x - y).n_y / (4 pi r^3), the
latter by the 6-point rule.  The static part vanishes for identical (flat)
triangles; for edge and vertex pairs it is integrated in the Duffy
coordinates of the single layer's rules, where the radial variable again
integrates in closed form.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .cqm import (classify_pairs, forward_dft, frequencies, gauss_legendre01, inverse_dft,
                  near_pairs, near_static, num_frequencies_half, rhs, triangle_quadrature,
                  assemble_V)

__all__ = ["normals", "static_K_edge", "static_K_vertex", "near_static_K", "remainder_K",
           "near_dynamic_K", "far_entries_K", "assemble_K", "solve_direct", "static_Kp_edge",
           "static_Kp_vertex", "near_static_Kp", "assemble_Kp"]

FOUR_PI = 4.0 * math.pi


def normals(V, T):
    """Unit normals of the triangles, oriented by their vertex order."""
    P = V[T]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def static_K_edge(A, B, C, D, nj, q):
    """Integral of (x - y).n_j / (4 pi |x - y|^3) over tau x t, tau = (A,B,C)
    (target), t = (A,B,D) (source, unit normal nj).

    The coordinates of the single layer's edge rule: x - y = delta e + alpha c
    - beta d = rho E omega, with the free edge coordinate integrated to
    1 - rho (h(omega) = 1 on the four pieces).  n_j is orthogonal to e and d,
    so (x - y).n_j = rho alpha (c.n_j), and the kernel is
    alpha (c.n_j) / (4 pi rho^2 |E omega|^3); with the radial measure
    rho^2 (1 - rho) the radial integral is 1/2, leaving
        K = |tau||t| / (2 pi) * sum_pieces int int jac alpha (c.n_j) / |E omega|^3.
    """
    e, c, d = B - A, C - A, D - A
    at = 0.5 * np.linalg.norm(np.cross(e, c), axis=-1)
    bt = 0.5 * np.linalg.norm(np.cross(e, d), axis=-1)
    cn = np.sum(c * nj, axis=-1)
    x, w = gauss_legendre01(q)
    acc = np.zeros(at.shape)
    for p, wp in zip(x, w):
        for r, wr in zip(x, w):
            pieces = [
                ((1 - p), p, r, 1.0),
                (p * (1 - r), p * r, 1.0, p),
                (-p * (1 - r), 1.0, p * r, p),
                (-p, r, 1 - p, 1.0),
            ]
            for dl, al, be, jac in pieces:
                v = dl * e + al * c - be * d
                nv = np.linalg.norm(v, axis=-1)
                acc += wp * wr * jac * al / (nv * nv * nv)
    return at * bt / (2.0 * math.pi) * cn * acc


def static_K_vertex(P, A1, A2, B1, B2, nj, q):
    """Integral of (x - y).n_j / (4 pi |x - y|^3) over tau x t sharing only the
    vertex P, tau = (P,A1,A2) (target), t = (P,B1,B2) (source, normal nj).

    The Duffy coordinates of the single layer's vertex rule, x = P + xi a(eta),
    y = P + zeta b(theta), split at zeta = w xi and xi = w zeta.  b lies in
    the source plane, so (x - y).n_j = xi a.n_j (first half) or zeta w a.n_j
    (second half); the radial variable integrates to 1/2 in both:
        K = |tau||t| / (2 pi) int_[0,1]^3 ( w a.n_j / |a - w b|^3
                                            + w^2 a.n_j / |w a - b|^3 ).
    """
    a1, a2, b1, b2 = A1 - P, A2 - P, B1 - P, B2 - P
    at = 0.5 * np.linalg.norm(np.cross(a1, a2), axis=-1)
    bt = 0.5 * np.linalg.norm(np.cross(b1, b2), axis=-1)
    x, w = gauss_legendre01(q)
    acc = np.zeros(at.shape)
    for eta, we in zip(x, w):
        a = a1 + eta * (a2 - a1)
        an = np.sum(a * nj, axis=-1)
        for th, wt in zip(x, w):
            b = b1 + th * (b2 - b1)
            for u, wu in zip(x, w):
                d1 = np.linalg.norm(a - u * b, axis=-1)
                d2 = np.linalg.norm(u * a - b, axis=-1)
                acc += we * wt * wu * an * (u / (d1 * d1 * d1) + u * u / (d2 * d2 * d2))
    return at * bt / (2.0 * math.pi) * acc


def near_static_K(V, T, pairs, q=5):
    """Static (Laplace) part of K for every near pair: zero for identical flat
    triangles, the two rules above for edge and vertex pairs."""
    n = normals(V, T)
    out = np.zeros(len(pairs))
    ident, edge, vert = classify_pairs(T, pairs)
    pj = np.asarray([p[1] for p in pairs])
    if len(edge):
        k = edge[:, 0]
        out[k] = static_K_edge(V[edge[:, 1]], V[edge[:, 2]], V[edge[:, 3]], V[edge[:, 4]],
                               n[pj[k]], q)
    if len(vert):
        k = vert[:, 0]
        out[k] = static_K_vertex(V[vert[:, 1]], V[vert[:, 2]], V[vert[:, 3]], V[vert[:, 4]],
                                 V[vert[:, 5]], n[pj[k]], q)
    return out


def remainder_K(z):
    """exp(-z)(1 + z) - 1 without cancellation: the series
    -sum_{k>=2} (k-1) (-z)^k / k! for |z| < 0.5 (40 terms), else direct."""
    z = np.asarray(z, dtype=np.complex128)
    direct = np.exp(-z) * (1.0 + z) - 1.0
    small = np.abs(z) < 0.5
    acc = np.zeros_like(z)
    term = np.ones_like(z)  # (-z)^k / k!
    for k in range(1, 41):
        term = term * (-z) / k
        if k >= 2:
            acc = acc - (k - 1) * term
    return np.where(small, acc, direct)


def near_dynamic_K(Xi, Wi, Xj, Wj, nj, s):
    """sum_ab W_ia W_jb (exp(-s r)(1 + s r) - 1)(x_a - y_b).n_j / (4 pi r^3); the
    remainder is O(r^2), so the summand tends to 0 with r (coincident points
    of identical triangles give 0).  Xi (...,6,3), Wi (...,6), nj (...,3)."""
    d = Xi[..., :, None, :] - Xj[..., None, :, :]
    r = np.linalg.norm(d, axis=-1)
    dn = np.einsum("...abk,...k->...ab", d, nj)
    safe = np.where(r > 0.0, r, 1.0)
    val = np.where(r > 0.0, remainder_K(s * safe) * dn / (FOUR_PI * safe ** 3), 0.0)
    return np.einsum("...a,...ab,...b->...", Wi, val, Wj)


def far_entries_K(Xi, Wi, Xj, Wj, nj, s):
    """sum_ab W_ia W_jb (1 + s r) exp(-s r)(x_a - y_b).n_j / (4 pi r^3) for blocks
    of triangles: Xi (m,6,3), Xj (n,6,3), nj (n,3) -> (m,n)."""
    d = Xi[:, :, None, None, :] - Xj[None, None, :, :, :]
    r = np.linalg.norm(d, axis=-1)
    dn = np.einsum("iajbk,jk->iajb", d, nj)
    safe = np.where(r > 0.0, r, 1.0)
    k = np.where(r > 0.0, (1.0 + s * safe) * np.exp(-s * safe) * dn / (FOUR_PI * safe ** 3), 0.0)
    return np.einsum("ia,iajb,jb->ij", Wi, k, Wj)


def assemble_K(V, T, s, q=5, pairs=None, static=None, rows=None):
    """Dense piecewise-constant Galerkin matrix K(s)[i,j] for one frequency."""
    X, W, _ = triangle_quadrature(V, T)
    n = normals(V, T)
    M = len(T)
    rows = np.arange(M) if rows is None else np.asarray(rows)
    if pairs is None:
        pairs = near_pairs(T)
    if static is None:
        static = near_static_K(V, T, pairs, q)
    out = np.empty((len(rows), M), dtype=np.complex128)
    chunk = 32
    for c0 in range(0, len(rows), chunk):
        rr = rows[c0:c0 + chunk]
        out[c0:c0 + chunk] = far_entries_K(X[rr], W[rr], X, W, n, s)
    pos = np.full(M, -1)
    pos[rows] = np.arange(len(rows))
    pi = np.asarray([p[0] for p in pairs])
    pj = np.asarray([p[1] for p in pairs])
    sel = pos[pi] >= 0
    pi, pj, sv = pi[sel], pj[sel], np.asarray(static)[sel]
    out[pos[pi], pj] = sv + near_dynamic_K(X[pi], W[pi], X[pj], W[pj], n[pj], s)
    return out


def solve_direct(V, T, N, Tend, rho=None, q=5, direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5,
                 amplitude=1.0, samples=None, return_all=False):
    """All-at-once CQM solve of the direct Dirichlet equation
    V q = (-1/2 I + K) g_D (Section 2.2 with Gamma_D = Gamma, Section 3.2 per
    frequency); returns the Neumann datum q (N+1, M) real."""
    s, rho, dt = frequencies(N, Tend, rho)
    F = N + 1
    H = num_frequencies_half(F)
    _, _, area = triangle_quadrature(V, T)
    b = rhs(V, T, N, Tend, direction, sigma, t0, amplitude, samples)
    bhat = forward_dft(b, rho, H)
    pairs = near_pairs(T)
    sv = near_static(V, T, pairs, q)
    sk = near_static_K(V, T, pairs, q)
    xhat = np.empty((H, len(T)), dtype=np.complex128)
    ghat = np.empty_like(xhat)
    for l in range(H):
        K = assemble_K(V, T, s[l], q, pairs, sk)
        ghat[l] = -0.5 * bhat[l] + K @ (bhat[l] / area)
        A = assemble_V(V, T, s[l], q, pairs, sv)
        xhat[l] = sla.lu_solve(sla.lu_factor(A), ghat[l])
    qn, im_ratio = inverse_dft(xhat, rho, F, conjugate_fill=True)
    if return_all:
        return dict(q=qn, s=s, rho=rho, dt=dt, b=b, bhat=bhat, ghat=ghat, xhat=xhat,
                    im_ratio=im_ratio)
    return qn


def static_Kp_edge(A, B, C, D, ni, q):
    """Integral of -(x - y).n_i / (4 pi |x - y|^3) over tau x t, tau = (A,B,C)
    (target, unit normal ni), t = (A,B,D) (source): the adjoint double
    layer's kernel d/dn_x 1/(4 pi r).  n_i is orthogonal to e and c, so
    -(x - y).n_i = beta (d.n_i), and the radial integral is 1/2 as for K."""
    e, c, d = B - A, C - A, D - A
    at = 0.5 * np.linalg.norm(np.cross(e, c), axis=-1)
    bt = 0.5 * np.linalg.norm(np.cross(e, d), axis=-1)
    dn = np.sum(d * ni, axis=-1)
    x, w = gauss_legendre01(q)
    acc = np.zeros(at.shape)
    for p, wp in zip(x, w):
        for r, wr in zip(x, w):
            pieces = [
                ((1 - p), p, r, 1.0),
                (p * (1 - r), p * r, 1.0, p),
                (-p * (1 - r), 1.0, p * r, p),
                (-p, r, 1 - p, 1.0),
            ]
            for dl, al, be, jac in pieces:
                v = dl * e + al * c - be * d
                nv = np.linalg.norm(v, axis=-1)
                acc += wp * wr * jac * be / (nv * nv * nv)
    return at * bt / (2.0 * math.pi) * dn * acc


def static_Kp_vertex(P, A1, A2, B1, B2, ni, q):
    """The adjoint double layer for a vertex pair, tau = (P,A1,A2) (target,
    normal ni), t = (P,B1,B2): a lies in the target plane, so
    -(x - y).n_i = zeta b.n_i, with zeta = w xi in the first half and the
    radial variable zeta in the second; the radial integral is 1/2 in both:
        K' = |tau||t| / (2 pi) int_[0,1]^3 ( w^2 b.n_i / |a - w b|^3
                                             + w b.n_i / |w a - b|^3 )."""
    a1, a2, b1, b2 = A1 - P, A2 - P, B1 - P, B2 - P
    at = 0.5 * np.linalg.norm(np.cross(a1, a2), axis=-1)
    bt = 0.5 * np.linalg.norm(np.cross(b1, b2), axis=-1)
    x, w = gauss_legendre01(q)
    acc = np.zeros(at.shape)
    for th, wt in zip(x, w):
        b = b1 + th * (b2 - b1)
        bn = np.sum(b * ni, axis=-1)
        for eta, we in zip(x, w):
            a = a1 + eta * (a2 - a1)
            for u, wu in zip(x, w):
                d1 = np.linalg.norm(a - u * b, axis=-1)
                d2 = np.linalg.norm(u * a - b, axis=-1)
                acc += we * wt * wu * bn * (u * u / (d1 * d1 * d1) + u / (d2 * d2 * d2))
    return at * bt / (2.0 * math.pi) * acc


def near_static_Kp(V, T, pairs, q=5):
    """Static part of the adjoint double layer K' (normal derivative at the
    target, eq. wavebio) for every near pair."""
    n = normals(V, T)
    out = np.zeros(len(pairs))
    ident, edge, vert = classify_pairs(T, pairs)
    pi = np.asarray([p[0] for p in pairs])
    if len(edge):
        k = edge[:, 0]
        out[k] = static_Kp_edge(V[edge[:, 1]], V[edge[:, 2]], V[edge[:, 3]], V[edge[:, 4]],
                                n[pi[k]], q)
    if len(vert):
        k = vert[:, 0]
        out[k] = static_Kp_vertex(V[vert[:, 1]], V[vert[:, 2]], V[vert[:, 3]], V[vert[:, 4]],
                                  V[vert[:, 5]], n[pi[k]], q)
    return out


def assemble_Kp(V, T, s, q=5, pairs=None, static=None):
    """Dense piecewise-constant Galerkin matrix of the adjoint double layer,
    K'(s)[i,j] = int_tau_i int_tau_j d/dn_x G(x - y, s), kernel
    -(1 + s r) exp(-s r)(x - y).n_x / (4 pi r^3) with n_x the target's normal."""
    X, W, _ = triangle_quadrature(V, T)
    n = normals(V, T)
    M = len(T)
    if pairs is None:
        pairs = near_pairs(T)
    if static is None:
        static = near_static_Kp(V, T, pairs, q)
    d = X[:, :, None, None, :] - X[None, None, :, :, :]
    r = np.linalg.norm(d, axis=-1)
    dn = np.einsum("iajbk,ik->iajb", d, n)
    safe = np.where(r > 0.0, r, 1.0)
    kf = np.where(r > 0.0, -(1.0 + s * safe) * np.exp(-s * safe) * dn / (FOUR_PI * safe ** 3), 0.0)
    out = np.einsum("ia,iajb,jb->ij", W, kf, W).astype(np.complex128)
    for k, (i, j, _) in enumerate(pairs):
        dd = X[i][:, None, :] - X[j][None, :, :]
        rr = np.linalg.norm(dd, axis=-1)
        dni = dd @ n[i]
        sr = np.where(rr > 0.0, rr, 1.0)
        val = np.where(rr > 0.0, -remainder_K(s * sr) * dni / (FOUR_PI * sr ** 3), 0.0)
        out[i, j] = static[k] + W[i] @ val @ W[j]
    return out
