"""Oracle of the hypersingular operator D(s) on the piecewise-linear space S_h^1.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 (eq. wavebio) defines D by the kernel gamma_{1,x} gamma_{1,y} u*;
Section 3.2 turns it, frequency by frequency, into the Galerkin matrix
D_l[p, j] = < phi_p^1, D_l phi_j^1 > over the continuous piecewise-linear hat
functions phi^1 of the mesh vertices (the space S_h^1 of Section 3.2).

Reading taken here (the paper gives no formula for the entries): the
hypersingular kernel is not integrable, so the entries are formed by the
classical integration by parts on a closed surface (the identity of Maue and
Nedelec for the Helmholtz operator, here with wavenumber i s):

    D_l[p, j] = int int G(x - y, s_l) [ curl phi_j(y) . curl phi_p(x)
                                        + s_l^2 (n_x . n_y) phi_j(y) phi_p(x) ] dS(y) dS(x),

G = exp(-s r)/(4 pi r), curl the surface curl n x grad_Gamma.  Of the two
signs that the trace conventions allow, this is the one with which D_l is
elliptic, as Section 3.1 states for Im s_l != 0 (at s = 0 it is the positive
semi-definite Laplace form that vanishes on constants).  On a flat triangle
tau with vertices (P_0, P_1, P_2) the barycentric coordinate lambda_a has the
constant curl -e_a / (2 |tau|), e_a = P_{a+2} - P_{a+1} (indices mod 3), so
the first term is the piecewise-constant single-layer matrix of
oracle.cqm.assemble_V with the edge-vector products e_a . e_b / (4 |tau||t|)
as weights.  The second term needs the weighted single-layer integrals

    W[tau, a; t, b](s) = int_tau int_t G(x - y, s) lambda_a(x) lambda_b(y),

by the same pair classes as the single layer: pairs sharing no vertex by the
6-point rule on both triangles; pairs sharing a vertex split G into the static
part 1/(4 pi r), integrated by the Sauter-Schwab transformations (Sauter and
Schwab, Boundary Element Methods, Section 5.2: identical triangles, a common
edge, a common vertex, each mapped to the unit 4-cube where the integrand is
smooth, with a q-point Gauss-Legendre rule per axis), and the bounded
remainder (exp(-s r) - 1)/(4 pi r), by the 6-point rule.
"""
from __future__ import annotations

import math

import numpy as np

from .cqm import (assemble_V, classify_pairs, dunavant6, expm1_complex, gauss_legendre01,
                  near_pairs, triangle_quadrature)

__all__ = ["edge_vectors", "unit_normals", "ss_static_weighted", "near_static_weighted",
           "weighted_single_layer", "assemble_D", "mass_P1", "apply_D"]

FOUR_PI = 4.0 * math.pi


def edge_vectors(V, T):
    """e[m, a] = P_{a+2} - P_{a+1} of triangle m (the edge opposite vertex a)."""
    P = V[T]
    return np.stack([P[:, 2] - P[:, 1], P[:, 0] - P[:, 2], P[:, 1] - P[:, 0]], axis=1)


def unit_normals(V, T):
    P = V[T]
    c = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def _bary(xi1, xi2):
    """Barycentric weights of the point chi(xi1, xi2) = P0 + xi1 (P1 - P0) +
    xi2 (P2 - P1), 0 <= xi2 <= xi1 <= 1, in the order (P0, P1, P2)."""
    return np.stack([1.0 - xi1, xi1 - xi2, xi2], axis=-1)


def _ss_nodes(kind, q):
    """Sauter-Schwab transformations: lists of (x_hat, y_hat, jacobian) over
    the Gauss-Legendre tensor grid of [0,1]^4 in (xi, eta1, eta2, eta3); each
    x_hat, y_hat is a pair of arrays in the reference coordinates above."""
    t, w = gauss_legendre01(q)
    xi, e1, e2, e3 = np.meshgrid(t, t, t, t, indexing="ij")
    wt = np.einsum("i,j,k,l->ijkl", w, w, w, w)
    xi, e1, e2, e3, wt = (a.ravel() for a in (xi, e1, e2, e3, wt))
    out = []
    if kind == "identical":
        jac = wt * xi ** 3 * e1 ** 2 * e2
        maps = [
            ((xi, xi * (1 - e1 + e1 * e2)), (xi * (1 - e1 * e2 * e3), xi * (1 - e1))),
            ((xi * (1 - e1 * e2 * e3), xi * (1 - e1)), (xi, xi * (1 - e1 + e1 * e2))),
            ((xi, xi * e1 * (1 - e2 + e2 * e3)), (xi * (1 - e1 * e2), xi * e1 * (1 - e2))),
            ((xi * (1 - e1 * e2), xi * e1 * (1 - e2)), (xi, xi * e1 * (1 - e2 + e2 * e3))),
            ((xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), (xi, xi * e1 * (1 - e2))),
            ((xi, xi * e1 * (1 - e2)), (xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3))),
        ]
        out = [(x, y, jac) for x, y in maps]
    elif kind == "edge":
        j1 = wt * xi ** 3 * e1 ** 2
        j2 = j1 * e2
        out = [
            ((xi, xi * e1 * e3), (xi * (1 - e1 * e2), xi * e1 * (1 - e2)), j1),
            ((xi, xi * e1), (xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)), j2),
            ((xi * (1 - e1 * e2), xi * e1 * (1 - e2)), (xi, xi * e1 * e2 * e3), j2),
            ((xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)), (xi, xi * e1), j2),
            ((xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)), (xi, xi * e1 * e2), j2),
        ]
    elif kind == "vertex":
        jac = wt * xi ** 3 * e2
        out = [
            ((xi, xi * e1), (xi * e2, xi * e2 * e3), jac),
            ((xi * e2, xi * e2 * e3), (xi, xi * e1), jac),
        ]
    else:
        raise ValueError(kind)
    return out


def ss_static_weighted(kind, X, Y, q, chunk=256):
    """Static weighted integrals int_tau int_t lambda_a(x) lambda_b(y) / (4 pi r)
    for pairs of triangles X = (P0, P1, P2) (target), Y = (Q0, Q1, Q2)
    (source), arrays (n, 3, 3), vertex order as the transformations need it:
    identical P = Q; edge P0 = Q0, P1 = Q1; vertex P0 = Q0.  Returns (n, 3, 3)
    indexed [a, b] in these vertex orders."""
    X, Y = np.asarray(X, float), np.asarray(Y, float)
    n = len(X)
    out = np.zeros((n, 3, 3))
    if n == 0:
        return out
    ax = 0.5 * np.linalg.norm(np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), axis=1)
    ay = 0.5 * np.linalg.norm(np.cross(Y[:, 1] - Y[:, 0], Y[:, 2] - Y[:, 0]), axis=1)
    for (x1, x2), (y1, y2), jac in _ss_nodes(kind, q):
        bx, by = _bary(x1, x2), _bary(y1, y2)  # (K, 3)
        for c0 in range(0, n, chunk):
            Xc, Yc = X[c0:c0 + chunk], Y[c0:c0 + chunk]
            px = np.einsum("ka,nad->nkd", bx, Xc)
            py = np.einsum("kb,nbd->nkd", by, Yc)
            r = np.linalg.norm(px - py, axis=-1)  # (n, K)
            f = jac[None, :] / r
            out[c0:c0 + chunk] += np.einsum("nk,ka,kb->nab", f, bx, by)
    # surface elements: the reference triangle has area 1/2
    return out * (4.0 * ax * ay / FOUR_PI)[:, None, None]


def near_static_weighted(V, T, pairs, q=5):
    """(len(pairs), 3, 3) static weighted integrals of every near pair (i, j),
    indexed [a, b] by the local vertex numbers of T[i] and T[j]."""
    out = np.full((len(pairs), 3, 3), np.nan)
    ident, edge, vert = classify_pairs(T, pairs)

    def local(rows, verts):  # local index in triangle rows of each global vertex
        return np.array([[list(T[r]).index(v) for v in vs] for r, vs in zip(rows, verts)])

    pi = np.array([p[0] for p in pairs])
    pj = np.array([p[1] for p in pairs])
    for kind, arr, xv, yv in (("identical", ident, (1, 2, 3), (1, 2, 3)),
                              ("edge", edge, (1, 2, 3), (1, 2, 4)),
                              ("vertex", vert, (1, 2, 3), (1, 4, 5))):
        if not len(arr):
            continue
        k = arr[:, 0]
        gx, gy = arr[:, list(xv)], arr[:, list(yv)]
        val = ss_static_weighted(kind, V[gx], V[gy], q)
        la, lb = local(pi[k], gx), local(pj[k], gy)
        res = np.zeros((len(k), 3, 3))
        for a in range(3):
            for b in range(3):
                res[np.arange(len(k)), la[:, a], lb[:, b]] = val[:, a, b]
        out[k] = res
    return out


def weighted_single_layer(V, T, s, q=5, pairs=None, wstatic=None, rows=None):
    """W[(i, a), (j, b)](s) for target triangles `rows` (default all): array
    (len(rows), 3, M, 3) complex."""
    X, Wq, _ = triangle_quadrature(V, T)
    bary, _ = dunavant6()  # (6, 3): lambda_a at the rule's points
    M = len(T)
    rows = np.arange(M) if rows is None else np.asarray(rows)
    if pairs is None:
        pairs = near_pairs(T)
    if wstatic is None:
        wstatic = near_static_weighted(V, T, pairs, q)
    WL = Wq[:, :, None] * bary[None, :, :]  # (M, 6, 3): weight times lambda
    out = np.empty((len(rows), 3, M, 3), dtype=np.complex128)
    chunk = 16
    for c0 in range(0, len(rows), chunk):
        rr = rows[c0:c0 + chunk]
        r = np.linalg.norm(X[rr][:, :, None, None, :] - X[None, None, :, :, :], axis=-1)
        safe = np.where(r > 0.0, r, 1.0)
        g = np.where(r > 0.0, np.exp(-s * safe) / (FOUR_PI * safe), 0.0)
        out[c0:c0 + chunk] = np.einsum("iva,ivjw,jwb->iajb", WL[rr], g, WL)
    pos = np.full(M, -1)
    pos[rows] = np.arange(len(rows))
    pi = np.array([p[0] for p in pairs])
    pj = np.array([p[1] for p in pairs])
    sel = pos[pi] >= 0
    for k in np.nonzero(sel)[0]:
        i, j = pi[k], pj[k]
        r = np.linalg.norm(X[i][:, None, :] - X[j][None, :, :], axis=-1)
        safe = np.where(r > 0.0, r, 1.0)
        rem = np.where(r > 0.0, expm1_complex(-s * safe) / (FOUR_PI * safe), -s / FOUR_PI)
        out[pos[i], :, j, :] = wstatic[k] + np.einsum("va,vw,wb->ab", WL[i], rem, WL[j])
    return out


def assemble_D(V, T, s, q=5, rows=None, pairs=None, wstatic=None, vstatic=None):
    """Dense D(s)[p, j] over the mesh vertices (rows: a subset of vertex ids,
    default all): the sum over triangle pairs of the curl term with the
    single-layer entries and the s^2 n.n term with the weighted entries,
    scattered from local vertex numbers (triangle, a) to vertex ids."""
    V = np.asarray(V, float)
    T = np.asarray(T)
    M, Nv = len(T), len(V)
    rows = np.arange(Nv) if rows is None else np.asarray(rows)
    if pairs is None:
        pairs = near_pairs(T)
    # target triangles incident to a requested vertex
    want = np.zeros(Nv, bool)
    want[rows] = True
    tri = np.nonzero(want[T].any(axis=1))[0]
    Vs = assemble_V(V, T, s, q, pairs=pairs, static=vstatic, rows=tri)  # (nt, M)
    Ws = weighted_single_layer(V, T, s, q, pairs=pairs, wstatic=wstatic, rows=tri)
    area = 0.5 * np.linalg.norm(np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]]), axis=1)
    curl = edge_vectors(V, T) / (2.0 * area)[:, None, None]  # (M, 3, 3); sign irrelevant
    n = unit_normals(V, T)
    cc = np.einsum("iad,jbd->iajb", curl[tri], curl)  # (nt, 3, M, 3)
    nn = n[tri] @ n.T  # (nt, M)
    loc = cc * Vs[:, None, :, None] + (s * s) * nn[:, None, :, None] * Ws
    # columns: scatter (j, b) -> T[j, b]
    colsum = np.zeros((len(tri), 3, Nv), dtype=np.complex128)
    for b in range(3):
        np.add.at(colsum, (slice(None), slice(None), T[:, b]), loc[:, :, :, b])
    pos = np.full(Nv, -1)
    pos[rows] = np.arange(len(rows))
    out = np.zeros((len(rows), Nv), dtype=np.complex128)
    for a in range(3):
        vid = T[tri, a]
        sel = pos[vid] >= 0
        np.add.at(out, pos[vid[sel]], colsum[sel, a, :])
    return out


def mass_P1(V, T):
    """P1 mass matrix int phi_p phi_j (exact: |tau|/12 (1 + delta_ab))."""
    V, T = np.asarray(V, float), np.asarray(T)
    area = 0.5 * np.linalg.norm(np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]]), axis=1)
    Mm = np.zeros((len(V), len(V)))
    loc = (np.ones((3, 3)) + np.eye(3)) / 12.0
    for a in range(3):
        for b in range(3):
            np.add.at(Mm, (T[:, a], T[:, b]), area * loc[a, b])
    return Mm


def apply_D(V, T, s_list, x, q=5, rows=None):
    """y_l = D(s_l) x_l for each frequency of s_list; x (nl, Nv) complex."""
    pairs = near_pairs(np.asarray(T))
    from .cqm import near_static
    vst = near_static(np.asarray(V, float), np.asarray(T), pairs, q)
    wst = near_static_weighted(np.asarray(V, float), np.asarray(T), pairs, q)
    out = []
    for s, xl in zip(s_list, np.asarray(x)):
        Dm = assemble_D(V, T, s, q, rows=rows, pairs=pairs, wstatic=wst, vstatic=vst)
        out.append(Dm @ xl)
    return np.asarray(out)
