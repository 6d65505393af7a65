"""Independent reference for the static near-field integrals (test helper).

The inner integral of 1/|x-y| over a flat triangle is evaluated in closed form
(the analytic potential of a uniform triangle, Wilton et al., IEEE TAP 1984);
the outer integral over the other triangle is taken by adaptive subdivision
with a Gauss product rule.  No Duffy transform is involved, so agreement with
the oracle's Duffy rules pins those rules.
"""
import math

import numpy as np


def triangle_potential(P, A, B, C):
    """int_T dy / |P - y| for points P (n,3), triangle T = (A,B,C)."""
    P = np.atleast_2d(P)
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    w = (P - A) @ n
    Pp = P - w[:, None] * n
    aw = np.abs(w)
    tot = np.zeros(len(P))
    for l0, l1 in ((A, B), (B, C), (C, A)):
        s = (l1 - l0) / np.linalg.norm(l1 - l0)
        m = np.cross(s, n)
        lp = (l1 - Pp) @ s
        lm = (l0 - Pp) @ s
        p0 = (l0 - Pp) @ m
        Rp = np.linalg.norm(P - l1, axis=1)
        Rm = np.linalg.norm(P - l0, axis=1)
        R0sq = p0 * p0 + w * w
        ok = np.abs(p0) > 1e-14
        num = np.where(ok, Rp + lp, 1.0)
        den = np.where(ok, Rm + lm, 1.0)
        tot += np.where(ok, p0 * np.log(num / den), 0.0)
        tot -= aw * (np.arctan2(p0 * lp, R0sq + aw * Rp) - np.arctan2(p0 * lm, R0sq + aw * Rm))
    return tot


def _tri_rule(n):
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1), 0.5 * w
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    return np.stack([u.ravel(), (v * (1 - u)).ravel()], 1), (wu * wv * (1 - u)).ravel()


_RULE = _tri_rule(7)


def _est(f, a, b, c):
    pts, wts = _RULE
    ar = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    X = a[None] + pts[:, :1] * (b - a)[None] + pts[:, 1:] * (c - a)[None]
    return 2.0 * ar * np.dot(wts, f(X))


def _adapt(f, a, b, c, whole, tol, depth):
    ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
    kids = ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca))
    parts = [_est(f, *k) for k in kids]
    tot = sum(parts)
    if abs(tot - whole) < tol or depth >= 12:
        return tot
    return sum(_adapt(f, *k, p, tol / 2, depth + 1) for k, p in zip(kids, parts))


def static_reference(Ti, Tj, rtol=1e-11):
    """int_{Ti} int_{Tj} 1/(4 pi |x-y|)."""
    f = lambda X: triangle_potential(X, *Tj)
    whole = _est(f, *Ti)
    return _adapt(f, *Ti, whole, rtol * abs(whole), 0) / (4.0 * math.pi)


def solid_angle(P, A, B, C):
    """Signed solid angle int_T (y - P).n / |y - P|^3 dS(y) of the flat triangle
    T = (A,B,C) (n = (B-A) x (C-A) normalised) seen from points P (n,3): the
    closed form of Van Oosterom and Strackee (IEEE TBME 1983)."""
    P = np.atleast_2d(P)
    R1, R2, R3 = A[None] - P, B[None] - P, C[None] - P
    r1, r2, r3 = (np.linalg.norm(R, axis=1) for R in (R1, R2, R3))
    num = np.einsum("ij,ij->i", R1, np.cross(R2, R3))
    den = (r1 * r2 * r3 + np.einsum("ij,ij->i", R1, R2) * r3 + np.einsum("ij,ij->i", R1, R3) * r2
           + np.einsum("ij,ij->i", R2, R3) * r1)
    return 2.0 * np.arctan2(num, den)


def double_layer_reference(Ti, Tj, rtol=1e-11):
    """int_{Ti} int_{Tj} (x - y).n_j / (4 pi |x - y|^3) = int_{Ti} -Omega_j(x) / (4 pi):
    the solid angle of Tj in closed form, the outer integral adaptive."""
    f = lambda X: solid_angle(X, *Tj)
    whole = _est(f, *Ti)
    return -_adapt(f, *Ti, whole, rtol * max(abs(whole), 1e-300), 0) / (4.0 * math.pi)


def _barycentric_gradient(T, b):
    """lambda_b(y) = 1 + g . (y - T[b]) on the flat triangle T: g = n x e_b / (2|T|),
    e_b the edge opposite vertex b taken in the vertex order."""
    A, B, C = T
    c = np.cross(B - A, C - A)
    n = c / np.linalg.norm(c)
    e = T[(b + 2) % 3] - T[(b + 1) % 3]
    return np.cross(n, e) / np.linalg.norm(c), n


def weighted_triangle_potential(P, T, b):
    """int_T lambda_b(y) dy / |P - y| for points P (n,3): lambda_b is linear, so
    lambda_b(y) = lambda_b(P') + g.(y - P') with P' the projection of P on the
    plane; the first part is the uniform potential, and the in-plane moment
    int_T (y - P')/|P - y| dy is the surface gradient of |P - y| integrated,
    i.e. by the divergence theorem the boundary integral of |P - y| times the
    outward edge normal, each edge in closed form."""
    P = np.atleast_2d(P)
    g, n = _barycentric_gradient(T, b)
    w = (P - T[0]) @ n
    Pp = P - w[:, None] * n
    lam = 1.0 + (Pp - T[b]) @ g
    mom = np.zeros(len(P))
    for k in range(3):
        Q1, Q2 = T[k], T[(k + 1) % 3]
        L = np.linalg.norm(Q2 - Q1)
        u = (Q2 - Q1) / L
        nu = np.cross(u, n)  # outward in-plane normal for the vertex order
        t0 = (P - Q1) @ u
        rho2 = np.maximum(np.sum((P - Q1) ** 2, axis=1) - t0 * t0, 0.0)
        rho = np.sqrt(rho2)

        def F(tau):
            sq = np.sqrt(tau * tau + rho2)
            safe = np.where(rho > 0.0, rho, 1.0)
            return 0.5 * (tau * sq + np.where(rho > 0.0, rho2 * np.arcsinh(tau / safe), 0.0))

        mom += (F(L - t0) - F(-t0)) * (nu @ g)
    return lam * triangle_potential(P, *T) + mom


def weighted_static_reference(Ti, Tj, a, b, rtol=1e-11):
    """int_{Ti} int_{Tj} lambda_a(x) lambda_b(y) / (4 pi |x-y|), lambda the
    barycentric coordinates of vertex a of Ti and vertex b of Tj."""
    Ti = [np.asarray(v, float) for v in Ti]
    Tj = [np.asarray(v, float) for v in Tj]
    ga, _ = _barycentric_gradient(Ti, a)
    f = lambda X: (1.0 + (X - Ti[a]) @ ga) * weighted_triangle_potential(X, Tj, b)
    whole = _est(f, *Ti)
    return _adapt(f, *Ti, whole, rtol * abs(whole), 0) / (4.0 * math.pi)
