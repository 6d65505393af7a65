"""Oracle of the compressed operator: H2 in space x MACA in frequency.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's Sections 4-6:
  * cluster tree by geometric bisection of the support boxes (Section 4.1),
    split at the midpoint of the longest box axis while #r > n_min; a split
    with an empty side falls back to the median (so no cluster has one son);
  * block cluster tree with the box admissibility max(diam B_r, diam B_c) <=
    eta dist(B_r, B_c) (eq. qadm); inadmissible leaf pairs form the near field;
  * tensor Chebyshev interpolation on the boxes (eq. degexp): leaf matrices
    U_r[i, mu] = int L_r,mu phi_i (6-point rule), transfer matrices
    E_r',r[lambda, mu] = L_r,mu(xi_r',lambda) (Section 4.2, Algorithm 1);
  * MACA (Section 5.1, Algorithm 2) on every block tensor: the coupling tensor
    S_b[mu, nu, k] = g(xi_r,mu, xi_c,nu, s_k) of a far block and the Galerkin
    block V[r, c, k] of a near block, combined as in Algorithm 3 / eq. lrfinal.

The oracle works on explicit tensors (entries are formed up front; the MACA
steps only ever read one slice and one fibre per rank, as on-demand access
would).  Readings of the MACA listing: the first slice is frequency 0, the
spatial pivot is the largest residual entry (first in row-major order on
ties), the next frequency pivot the largest |d_l[k]| over frequencies not
used before, the last update is kept, an exactly zero pivot ends the loop.
"""
from __future__ import annotations

import math

import numpy as np

from .cqm import FOUR_PI, triangle_quadrature

__all__ = ["cluster_tree", "block_tree", "cheb_nodes", "lagrange_1d", "cluster_basis",
           "transfer_matrix", "maca", "maca_norm2", "build_compressed", "compressed_matvec",
           "dense_tensor", "block_tensor", "compressed_dense", "solve_compressed"]


def cluster_tree(V, T, n_min):
    """Clusters as dicts (idx, lo, hi, sons, level, parent); clusters[0] = root."""
    P = V[T]
    cen = P.mean(axis=1)
    lo_t, hi_t = P.min(axis=1), P.max(axis=1)
    clusters = []

    def rec(idx, level, parent):
        cid = len(clusters)
        c = dict(idx=np.asarray(idx), lo=lo_t[idx].min(0), hi=hi_t[idx].max(0), sons=[],
                 level=level, parent=parent)
        clusters.append(c)
        if len(idx) > n_min:
            ax = int(np.argmax(c["hi"] - c["lo"]))
            mid = 0.5 * (c["lo"][ax] + c["hi"][ax])
            left = [t for t in idx if cen[t, ax] <= mid]
            right = [t for t in idx if cen[t, ax] > mid]
            if not left or not right:
                order = sorted(idx, key=lambda t: cen[t, ax])
                left, right = order[: len(order) // 2], order[len(order) // 2:]
            s0 = rec(left, level + 1, cid)
            s1 = rec(right, level + 1, cid)
            c["sons"] = [s0, s1]
        return cid

    rec(list(range(len(T))), 0, -1)
    return clusters


def _diam(c):
    return float(np.linalg.norm(c["hi"] - c["lo"]))


def _dist(a, b):
    gap = np.maximum(0.0, np.maximum(a["lo"] - b["hi"], b["lo"] - a["hi"]))
    return float(np.linalg.norm(gap))


def block_tree(clusters, eta):
    """Leaves of the block cluster tree: (far, near) lists of (r, c)."""
    far, near = [], []

    def rec(r, c):
        R, C = clusters[r], clusters[c]
        if max(_diam(R), _diam(C)) <= eta * _dist(R, C):
            far.append((r, c))
            return
        if not R["sons"] and not C["sons"]:
            near.append((r, c))
            return
        for a in (R["sons"] or [r]):
            for b in (C["sons"] or [c]):
                rec(a, b)

    rec(0, 0)
    return far, near


def cheb_nodes(c, m):
    """First-kind Chebyshev nodes on each axis of the box (3 x m); a flat axis
    is given a tiny extent."""
    ctr = 0.5 * (c["lo"] + c["hi"])
    half = np.maximum(0.5 * (c["hi"] - c["lo"]), 0.5e-12 * _diam(c))
    k = np.arange(m)
    return ctr[:, None] + half[:, None] * np.cos((2 * k + 1) * np.pi / (2 * m))[None, :]


def lagrange_1d(nodes, t):
    """L_k(t) for the Lagrange polynomials on `nodes`: array (len(t), m)."""
    t = np.atleast_1d(t)
    m = len(nodes)
    out = np.ones((len(t), m))
    for k in range(m):
        for j in range(m):
            if j != k:
                out[:, k] *= (t - nodes[j]) / (nodes[k] - nodes[j])
    return out


def _lagrange_3d(nodes, X):
    """L_mu(x) for mu = (a0 m + a1) m + a2: array (len(X), m^3)."""
    m = nodes.shape[1]
    lx, ly, lz = (lagrange_1d(nodes[d], X[:, d]) for d in range(3))
    return (lx[:, :, None, None] * ly[:, None, :, None] * lz[:, None, None, :]).reshape(len(X), m ** 3)


def cluster_basis(V, T, c, nodes):
    """U_c[i, mu] = sum_a W_ia L_c,mu(x_ia) for the triangles of c (#c x p)."""
    X, W, _ = triangle_quadrature(V, T)
    idx = c["idx"]
    L = _lagrange_3d(nodes, X[idx].reshape(-1, 3)).reshape(len(idx), 6, -1)
    return np.einsum("ia,iam->im", W[idx], L)


def transfer_matrix(child_nodes, parent_nodes):
    """E[lambda, mu] = L_parent,mu(xi_child,lambda)."""
    m = child_nodes.shape[1]
    g = np.stack(np.meshgrid(*child_nodes, indexing="ij"), axis=-1).reshape(m ** 3, 3)
    return _lagrange_3d(parent_nodes, g)


def maca_norm2(C, d):
    """||sum_l C_l (x)_3 d_l||_F^2 formed explicitly (for checks)."""
    G = np.einsum("lij,lk->ijk", np.asarray(C), np.asarray(d))
    return float(np.sum(np.abs(G) ** 2))


def maca(G, eps, rcap=None):
    """Algorithm 2 on an explicit tensor G (m x n x p).  Returns (C, d, info)
    with G ~ sum_l C[l] (x)_3 d[l]."""
    G = np.asarray(G, dtype=np.complex128)
    m, n, p = G.shape
    rcap = p if rcap is None else min(rcap, p)
    C, D = [], []
    used = np.zeros(p, dtype=bool)
    k = 0
    norm2 = 0.0
    pivots = []
    for l in range(rcap):
        Cl = G[:, :, k] - sum(C[t] * D[t][k] for t in range(l)) if l else G[:, :, k].copy()
        flat = (Cl.real ** 2 + Cl.imag ** 2).ravel()
        e = int(np.argmax(flat))  # first maximal entry in row-major order
        if flat[e] == 0.0:
            break
        i, j = divmod(e, n)
        piv = Cl[i, j]
        dl = (G[i, j, :] - sum(C[t][i, j] * D[t] for t in range(l))) / piv
        # Gram identity for ||G^(l)||_F^2
        cross = sum(np.vdot(C[t], Cl) * np.vdot(D[t], dl) for t in range(l))
        nc2, nd2 = float(np.sum(np.abs(Cl) ** 2)), float(np.sum(np.abs(dl) ** 2))
        norm2 += nc2 * nd2 + 2.0 * float(np.real(cross))
        C.append(Cl)
        D.append(dl)
        pivots.append((k, i, j))
        used[k] = True
        if math.sqrt(nc2 * nd2) <= eps * math.sqrt(max(norm2, 0.0)):
            break
        cand = np.where(~used, dl.real ** 2 + dl.imag ** 2, -1.0)
        if cand.max() < 0:
            break
        k = int(np.argmax(cand))
    return C, D, dict(rank=len(C), norm2=norm2, pivots=pivots)


def dense_tensor(V, T, s_list, q=5):
    """Dense Galerkin tensor V[i, j, k] = V(s_k)[i, j] (eq. tensor)."""
    from .cqm import assemble_V, near_pairs, near_static
    pairs = near_pairs(T)
    static = near_static(V, T, pairs, q)
    return np.stack([assemble_V(V, T, s, q, pairs, static) for s in s_list], axis=-1)


def block_tensor(V, T, ir, ic, s_list, near, q=5):
    """Galerkin block tensor V[ir, ic, k] = V(s_k)[ir, ic] (eq. tensor) with its
    entries formed on demand, as Algorithm 3 reads the entries of the block it
    compresses: pairs sharing no vertex by the 6-point rule on both triangles,
    pairs sharing a vertex by the static Duffy part plus the 6 x 6 rule of the
    bounded remainder (Section 3.2).  `near` maps (i, j) to the static value of
    every pair sharing a vertex."""
    from .cqm import far_entries, near_dynamic
    X, W, _ = triangle_quadrature(V, T)
    ir, ic = np.asarray(ir), np.asarray(ic)
    out = np.stack([far_entries(X[ir], W[ir], X[ic], W[ic], s) for s in s_list], axis=-1)
    pos_c = {int(j): b for b, j in enumerate(ic)}
    cols = set(pos_c)
    ia, jb, gi, gj, st = [], [], [], [], []
    for a, i in enumerate(ir):
        for j in sorted(cols & near["by_row"][int(i)]):
            ia.append(a)
            jb.append(pos_c[j])
            gi.append(int(i))
            gj.append(j)
            st.append(near["static"][(int(i), j)])
    if ia:
        gi, gj, st = np.asarray(gi), np.asarray(gj), np.asarray(st)
        for k, s in enumerate(s_list):
            out[ia, jb, k] = st + near_dynamic(X[gi], W[gi], X[gj], W[gj], s)
    return out


def _near_lookup(V, T, q=5):
    from .cqm import near_pairs, near_static
    pairs = near_pairs(T)
    static = near_static(V, T, pairs, q)
    by_row = [set() for _ in range(len(T))]
    for i, j, _ in pairs:
        by_row[i].add(j)
    return dict(by_row=by_row, static={(i, j): v for (i, j, _), v in zip(pairs, static)})


def build_compressed(V, T, s_list, n_min, eta, m, eps, dense=None, rcap=None, rows=None):
    """Algorithm 3: partition, bases, MACA of every block.  The near-field
    block tensors are taken from `dense` (M x M x F) when it is given, else
    their entries are formed on demand (block_tensor), block by block.  With
    `rows` only the blocks whose row cluster holds one of those triangles are
    compressed: the operator's rows `rows` are then complete (the others
    are not), which reaches sampled rows of meshes whose whole compressed
    operator would take hours here."""
    clusters = cluster_tree(V, T, n_min)
    far, near = block_tree(clusters, eta)
    nodes = [cheb_nodes(c, m) for c in clusters]
    lookup = _near_lookup(V, T) if dense is None else None
    s_list = np.asarray(s_list)
    rowset = None if rows is None else set(int(i) for i in rows)

    def kept(r):
        return rowset is None or not rowset.isdisjoint(clusters[r]["idx"].tolist())

    blocks = []
    for (r, c) in far:
        if not kept(r):
            continue
        gr = np.stack(np.meshgrid(*nodes[r], indexing="ij"), -1).reshape(-1, 3)
        gc = np.stack(np.meshgrid(*nodes[c], indexing="ij"), -1).reshape(-1, 3)
        dist = np.linalg.norm(gr[:, None, :] - gc[None, :, :], axis=-1)
        S = np.exp(-s_list[None, None, :] * dist[:, :, None]) / (FOUR_PI * dist[:, :, None])
        Cs, Ds, info = maca(S, eps, rcap)
        blocks.append(dict(kind="far", r=r, c=c, C=Cs, d=Ds, rank=info["rank"]))
    for (r, c) in near:
        if not kept(r):
            continue
        ir, ic = clusters[r]["idx"], clusters[c]["idx"]
        G = dense[np.ix_(ir, ic)] if dense is not None else block_tensor(V, T, ir, ic, s_list, lookup)
        Cs, Ds, info = maca(G, eps, rcap)
        blocks.append(dict(kind="near", r=r, c=c, C=Cs, d=Ds, rank=info["rank"]))
    U = {}
    for b in blocks:
        if b["kind"] == "far":
            for cid in (b["r"], b["c"]):
                if cid not in U:
                    U[cid] = cluster_basis(V, T, clusters[cid], nodes[cid])
    return dict(clusters=clusters, far=far, near=near, nodes=nodes, blocks=blocks, U=U,
                F=len(s_list), rows=rows)


def compressed_matvec(op, x):
    """y[l] = (eq. lrfinal operator at frequency l) x[l]; x is (F, M)."""
    cl = op["clusters"]
    y = np.zeros_like(x, dtype=np.complex128)
    for b in op["blocks"]:
        ir, ic = cl[b["r"]]["idx"], cl[b["c"]]["idx"]
        if not b["C"]:
            continue
        Cs, Ds = np.asarray(b["C"]), np.asarray(b["d"])  # (r, a, b), (r, F)
        for l in range(x.shape[0]):
            S = np.tensordot(Ds[:, l], Cs, axes=1)
            if b["kind"] == "near":
                y[l, ir] += S @ x[l, ic]
            else:
                y[l, ir] += op["U"][b["r"]] @ (S @ (op["U"][b["c"]].T @ x[l, ic]))
    return y


def compressed_dense(op, M):
    """The compressed operator written out as an M x M x F tensor."""
    cl = op["clusters"]
    out = np.zeros((M, M, op["F"]), dtype=np.complex128)
    for b in op["blocks"]:
        if not b["C"]:
            continue
        ir, ic = cl[b["r"]]["idx"], cl[b["c"]]["idx"]
        Cs, Ds = np.asarray(b["C"]), np.asarray(b["d"])
        if b["kind"] == "far":
            Cs = np.einsum("im,lmn,jn->lij", op["U"][b["r"]], Cs, op["U"][b["c"]])
        out[np.ix_(ir, ic)] += np.einsum("lij,lk->ijk", Cs, Ds)
    return out


def solve_compressed(V, T, N, Tend, n_min, eta, m, eps, rho=None, **wave):
    """All-at-once solve (as cqm.solve) with the compressed operator of every
    one of the N+1 frequencies (full band: MACA approximants are not
    conjugate-symmetric)."""
    import scipy.linalg as sla

    from .cqm import forward_dft, frequencies, inverse_dft, rhs
    s, rho, dt = frequencies(N, Tend, rho)
    F = N + 1
    b = rhs(V, T, N, Tend, **wave)
    ghat = forward_dft(b, rho, F)
    op = build_compressed(V, T, s, n_min, eta, m, eps)
    A = compressed_dense(op, len(T))
    xhat = np.stack([sla.lu_solve(sla.lu_factor(A[:, :, l]), ghat[l]) for l in range(F)])
    q, im = inverse_dft(xhat, rho, F, conjugate_fill=False)
    return q, im, op
