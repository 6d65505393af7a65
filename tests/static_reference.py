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
