"""FP64 oracle: dense Galerkin assembly of V(s_l), LU per frequency, scaled DFTs.

TEST INFRASTRUCTURE ONLY (see the package docstring). Not part of the product.

What is computed (all-at-once convolution quadrature for the indirect
single-layer equation V * phi = g_D on a closed triangulated surface):

1. Frequencies (Section 3.1, eq. cqm_freq with the BDF2 characteristic
   function): s_l = delta(rho * zeta^-l) / dt, delta(xi) = 3/2 - 2 xi + xi^2/2,
   zeta = exp(2 pi i / F), F = N + 1, l = 0..N.
2. Piecewise-constant Galerkin matrices V_l[i,j] = <phi_i, V(s_l) phi_j>
   (Section 3.2) with the Laplace-domain kernel exp(-s r)/(4 pi r)
   (eq. fundsol).  Pairs of triangles that share no vertex use the 6-point
   Dunavant rule on both triangles; pairs sharing a vertex (including i = j)
   use a Duffy-type rule for the static part 1/(4 pi r) plus the 6-point rule
   for the bounded remainder (exp(-s r) - 1)/(4 pi r).
3. Right-hand side b_n[i] = integral over triangle i of g_D(., t_n) (the L2
   projection onto piecewise constants, Section 3.2) by the 6-point rule.
4. Forward scaled DFT  ghat_l = sum_n rho^n b_n zeta^(-(n l mod F)).
5. Per frequency, the dense system V_l xhat_l = ghat_l is solved by LU with
   partial pivoting (the all-at-once alternative in the remark closing
   Section 6.2: N+1 independent Helmholtz-type systems).
6. Inverse scaled DFT q_n = Re[rho^-n / F sum_l xhat_l zeta^(n l mod F)]
   (eq. vhat / eq. dft structure), n = 0..N.

Readings taken where the paper is silent or inconsistent are listed in the
design document of the repository; the ones that change numbers are: F = N+1
points, BDF2, rho^N = 1e-8 by default, forward kernel zeta^-nl and inverse
zeta^+nl, g_D = -u_inc (sound-soft), triangles are "near" when they share a
vertex index.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

__all__ = [
    "frequencies", "twiddles", "dunavant6", "gauss_legendre01", "triangle_quadrature",
    "incident_dirichlet", "rhs", "forward_dft", "inverse_dft", "near_pairs",
    "static_identical", "static_edge", "static_vertex", "classify_pairs", "near_static",
    "near_dynamic", "expm1_complex", "far_entries", "assemble_V", "solve",
    "rel_error", "step_errors", "num_frequencies_half",
]

FOUR_PI = 4.0 * math.pi


# ---------------------------------------------------------------- frequencies

def frequencies(N: int, T: float, rho: float | None = None):
    """BDF2 convolution-quadrature frequencies (Section 3.1, eq. cqm_freq).

    Returns (s, rho, dt) with s complex128 of length F = N+1.  The paper's
    radius parameter R is called rho here; by default rho^N = 1e-8.
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    dt = T / N
    if rho is None or rho == 0.0:
        rho = 10.0 ** (-8.0 / N)
    F = N + 1
    l = np.arange(F)
    # zeta^-l evaluated from the reduced angle 2 pi l / F
    xi = rho * (np.cos(2.0 * np.pi * l / F) - 1j * np.sin(2.0 * np.pi * l / F))
    s = (1.5 - 2.0 * xi + 0.5 * xi * xi) / dt
    return s, rho, dt


def num_frequencies_half(F: int) -> int:
    """Number of frequencies l = 0..floor(F/2); the rest are conjugates."""
    return F // 2 + 1


def twiddles(F: int, sign: int):
    """Table zeta^(sign*k) = exp(sign * 2 pi i k / F), k = 0..F-1, in FP64.

    Indices n*l are reduced modulo F before lookup so no large angle is formed.
    """
    k = np.arange(F)
    return np.cos(2.0 * np.pi * k / F) + 1j * sign * np.sin(2.0 * np.pi * k / F)


# ---------------------------------------------------------------- quadrature

def dunavant6():
    """Dunavant's degree-4, 6-point rule on a triangle (barycentric points,
    weights normalised to sum 1)."""
    a, b = 0.445948490915965, 0.091576213509771
    wa, wb = 0.223381589678011, 0.109951743655322
    bary = np.array([
        [1 - 2 * a, a, a], [a, 1 - 2 * a, a], [a, a, 1 - 2 * a],
        [1 - 2 * b, b, b], [b, 1 - 2 * b, b], [b, b, 1 - 2 * b],
    ])
    w = np.array([wa, wa, wa, wb, wb, wb])
    return bary, w


def gauss_legendre01(q: int):
    """Gauss-Legendre nodes and weights mapped to [0, 1], correctly rounded to
    FP64: Newton's method on the Legendre polynomial P_q in 40-digit decimal
    arithmetic (three-term recurrence; P_q'(t) = q (t P_q - P_{q-1})/(t^2 - 1)),
    weights 2 / ((1 - t^2) P_q'(t)^2), both halved onto [0, 1].  (The FP64
    routine of NumPy leaves weights off by up to about 1e-15 relative, which
    the rho^-N amplification of the time-domain solution turns into 1e-8.)"""
    from decimal import Decimal, localcontext
    t0, _ = np.polynomial.legendre.leggauss(q)  # starting points only
    xs, ws = [], []
    with localcontext() as ctx:
        ctx.prec = 40
        one, two = Decimal(1), Decimal(2)
        for guess in t0:
            t = Decimal(float(guess))
            for _ in range(100):
                p0, p1 = one, t
                for k in range(2, q + 1):
                    p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
                dp = q * (t * p1 - p0) / (t * t - one)
                step = p1 / dp
                t -= step
                if abs(step) < Decimal("1e-35"):
                    break
            p0, p1 = one, t
            for k in range(2, q + 1):
                p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
            dp = q * (t * p1 - p0) / (t * t - one)
            xs.append(float((t + one) / two))
            ws.append(float(one / ((one - t * t) * dp * dp)))
    order = np.argsort(xs)
    return np.asarray(xs)[order], np.asarray(ws)[order]


def triangle_quadrature(V, T):
    """Quadrature points X (M,6,3), weights W (M,6) = area * w_a, areas (M,)."""
    P = V[T]  # (M,3,3)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    bary, w = dunavant6()
    X = np.einsum("ak,mkd->mad", bary, P)
    W = area[:, None] * w[None, :]
    return X, W, area


# ---------------------------------------------------------------- data

def incident_dirichlet(X, t, direction, sigma, t0, amplitude=1.0):
    """Sound-soft Dirichlet data g_D = -u_inc for the Gaussian plane wave
    u_inc(x,t) = A exp(-((t - x.d - t0)/sigma)^2)."""
    d = np.asarray(direction, dtype=np.float64)
    arg = (t - X @ d - t0) / sigma
    return -amplitude * np.exp(-arg * arg)


def rhs(V, T, N, Tend, direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5, amplitude=1.0,
        samples=None):
    """b[n, i] = sum_a W_ia g_D(x_ia, t_n), n = 0..N (Section 3.2, L2 projection
    onto piecewise constants with the 6-point rule).

    If `samples` (shape (N+1, M, 6)) is given it replaces g_D at the points.
    """
    X, W, _ = triangle_quadrature(V, T)
    dt = Tend / N
    out = np.empty((N + 1, len(T)))
    for n in range(N + 1):
        if samples is None:
            g = incident_dirichlet(X, n * dt, direction, sigma, t0, amplitude)
        else:
            g = samples[n]
        out[n] = np.sum(W * g, axis=1)
    return out


# ---------------------------------------------------------------- transforms

def forward_dft(b, rho, nfreq=None):
    """ghat[l] = sum_n rho^n b[n] zeta^-(n l mod F), l = 0..nfreq-1 (F = rows of b)."""
    F = b.shape[0]
    nfreq = F if nfreq is None else nfreq
    tw = twiddles(F, -1)
    out = np.zeros((nfreq,) + b.shape[1:], dtype=np.complex128)
    for l in range(nfreq):
        for n in range(F):
            out[l] += (rho ** n) * b[n] * tw[(n * l) % F]
    return out


def inverse_dft(xhat, rho, F, conjugate_fill=True):
    """q[n] = rho^-n / F sum_{l<F} xhat[l] zeta^(n l mod F), n = 0..F-1.

    With conjugate_fill, xhat holds l = 0..floor(F/2) and the remaining
    frequencies are taken as xhat[F-l] = conj(xhat[l]).  Returns (Re q, |Im q|
    relative to |Re q|) -- the imaginary part is the conjugate-symmetry check.
    """
    if conjugate_fill:
        full = np.empty((F,) + xhat.shape[1:], dtype=np.complex128)
        H = num_frequencies_half(F)
        full[:H] = xhat[:H]
        for l in range(H, F):
            full[l] = np.conj(xhat[F - l])
    else:
        full = np.asarray(xhat, dtype=np.complex128)
    tw = twiddles(F, +1)
    q = np.zeros((F,) + full.shape[1:], dtype=np.complex128)
    for n in range(F):
        acc = np.zeros(full.shape[1:], dtype=np.complex128)
        for l in range(F):
            acc += full[l] * tw[(n * l) % F]
        q[n] = acc * (rho ** (-n)) / F
    re = q.real
    im_ratio = np.linalg.norm(q.imag) / max(np.linalg.norm(re), 1e-300)
    return re, im_ratio


# ---------------------------------------------------------------- near pairs

def near_pairs(T):
    """All ordered pairs (i, j) of triangles that share at least one vertex
    index, including i == j.  Returns a list of (i, j, nshared)."""
    M = len(T)
    by_vertex = {}
    for i in range(M):
        for v in T[i]:
            by_vertex.setdefault(int(v), []).append(i)
    out = []
    for i in range(M):
        cand = set()
        for v in T[i]:
            cand.update(by_vertex[int(v)])
        for j in sorted(cand):
            ns = len(set(T[i].tolist()) & set(T[j].tolist()))
            out.append((i, j, ns))
    return out


def static_identical(A, B, C, q):
    """Integral of 1/(4 pi |x-y|) over tau x tau, tau = (A,B,C); arrays (...,3).

    Duffy-type rule: with y - x = rho * v on the six sectors of the difference
    hexagon of the reference triangle, the sector Jacobian rho cancels the
    kernel singularity; the remaining (1-rho)^2 factor and the inner point
    integral are integrated exactly, leaving one Gauss-Legendre dimension per
    sector.  Opposite sectors coincide, so three segments are summed twice:
        S = |tau|^2 / (3 pi) * sum_{3 segments a->b} int_0^1 dt / |a + t(b-a)|
    with segments (B-A -> C-A), (C-A -> C-B), (C-B -> A-B).
    """
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=-1)
    t, w = gauss_legendre01(q)
    segs = [(B - A, C - A), (C - A, C - B), (C - B, A - B)]
    acc = np.zeros(area.shape)
    for a, b in segs:
        for tk, wk in zip(t, w):
            acc += wk / np.linalg.norm(a + tk * (b - a), axis=-1)
    return area * area / (3.0 * math.pi) * acc


def static_edge(A, B, C, D, q):
    """Integral of 1/(4 pi |x-y|) over tau x t with tau = (A,B,C), t = (A,B,D).

    With x = A + u e + alpha c, y = A + v e + beta d (e = B-A, c = C-A, d = D-A),
    x - y depends only on (delta, alpha, beta), delta = u - v; the free edge
    coordinate integrates to 1 - h with h = max(0,delta) + max(alpha, beta-delta)
    a gauge.  Radial coordinates (delta,alpha,beta) = rho*omega, h(omega) = 1,
    give rho^2 (1-rho) / (rho |E omega|); integrating rho exactly leaves four
    planar pieces of {h = 1}, each a unit square in (p, r):
        P1: ( 1-p,     p,      r   ) jac 1
        P2: ( p(1-r),  p r,    1   ) jac p
        P3: (-p(1-r),  1,      p r ) jac p
        P4: (-p,       r,      1-p ) jac 1
        S = |tau||t| / (6 pi) * sum_pieces int int jac / |delta e + alpha c - beta d|
    """
    e, c, d = B - A, C - A, D - A
    at = 0.5 * np.linalg.norm(np.cross(e, c), axis=-1)
    bt = 0.5 * np.linalg.norm(np.cross(e, d), axis=-1)
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
                acc += wp * wr * jac / np.linalg.norm(v, axis=-1)
    return at * bt / (6.0 * math.pi) * acc


def static_vertex(P, A1, A2, B1, B2, q):
    """Integral of 1/(4 pi |x-y|) over tau x t sharing only the vertex P,
    tau = (P,A1,A2), t = (P,B1,B2).

    Duffy coordinates from the shared vertex, x = P + xi a(eta),
    y = P + zeta b(theta) (a, b interpolate the opposite edges), split at
    zeta = xi; in each half the radial variable integrates exactly (xi^2 -> 1/3):
        S = |tau||t| / (3 pi) * int_[0,1]^3 w ( 1/|a - w b| + 1/|w a - b| )
    """
    a1, a2, b1, b2 = A1 - P, A2 - P, B1 - P, B2 - P
    at = 0.5 * np.linalg.norm(np.cross(a1, a2), axis=-1)
    bt = 0.5 * np.linalg.norm(np.cross(b1, b2), axis=-1)
    x, w = gauss_legendre01(q)
    acc = np.zeros(at.shape)
    for eta, we in zip(x, w):
        a = a1 + eta * (a2 - a1)
        for th, wt in zip(x, w):
            b = b1 + th * (b2 - b1)
            for u, wu in zip(x, w):
                f = 1.0 / np.linalg.norm(a - u * b, axis=-1) + 1.0 / np.linalg.norm(u * a - b, axis=-1)
                acc += we * wt * wu * u * f
    return at * bt / (3.0 * math.pi) * acc


def classify_pairs(T, pairs):
    """Vertex correspondence for each near pair.

    Returns per-kind index arrays: identical -> (k, A, B, C); edge -> (k, A, B,
    C, D) with A < B the shared vertices and C in tau_i, D in tau_j; vertex ->
    (k, P, A1, A2, B1, B2) with P shared.  Entries are vertex indices into V.
    """
    ident, edge, vert = [], [], []
    for k, (i, j, ns) in enumerate(pairs):
        ti, tj = [int(v) for v in T[i]], [int(v) for v in T[j]]
        if i == j:
            ident.append((k, ti[0], ti[1], ti[2]))
        elif ns == 2:
            # shared edge oriented by increasing vertex index, so the rule for
            # (j, i) is the mirror image of the rule for (i, j)
            sh = sorted(v for v in ti if v in tj)
            c = [v for v in ti if v not in sh][0]
            d = [v for v in tj if v not in sh][0]
            edge.append((k, sh[0], sh[1], c, d))
        elif ns == 1:
            p = [v for v in ti if v in tj][0]
            a = [v for v in ti if v != p]
            b = [v for v in tj if v != p]
            vert.append((k, p, a[0], a[1], b[0], b[1]))
        else:
            raise ValueError("pair shares no vertex")
    f = lambda L, n: np.asarray(L, dtype=np.int64).reshape(-1, n)
    return f(ident, 4), f(edge, 5), f(vert, 6)


def near_static(V, T, pairs, q=5):
    """Static singular part S_ij for every near pair, by the three rules above
    (evaluated for all pairs of one kind at once)."""
    out = np.full(len(pairs), np.nan)
    ident, edge, vert = classify_pairs(T, pairs)
    if len(ident):
        out[ident[:, 0]] = static_identical(V[ident[:, 1]], V[ident[:, 2]], V[ident[:, 3]], q)
    if len(edge):
        out[edge[:, 0]] = static_edge(V[edge[:, 1]], V[edge[:, 2]], V[edge[:, 3]], V[edge[:, 4]], q)
    if len(vert):
        out[vert[:, 0]] = static_vertex(V[vert[:, 1]], V[vert[:, 2]], V[vert[:, 3]],
                                        V[vert[:, 4]], V[vert[:, 5]], q)
    return out


def expm1_complex(z):
    """exp(z) - 1 for complex z without cancellation:
    Re = expm1(x) cos y - 2 sin^2(y/2), Im = exp(x) sin y."""
    x, y = z.real, z.imag
    sh = np.sin(0.5 * y)
    return (np.expm1(x) * np.cos(y) - 2.0 * sh * sh) + 1j * (np.exp(x) * np.sin(y))


def near_dynamic(Xi, Wi, Xj, Wj, s):
    """D_ij(s) = sum_ab W_ia W_jb (exp(-s r_ab) - 1)/(4 pi r_ab), with the
    r = 0 value -s/(4 pi).  Xi (...,6,3), Wi (...,6)."""
    r = np.linalg.norm(Xi[..., :, None, :] - Xj[..., None, :, :], axis=-1)
    safe = np.where(r > 0.0, r, 1.0)
    val = np.where(r > 0.0, expm1_complex(-s * safe) / (FOUR_PI * safe), -s / FOUR_PI)
    return np.einsum("...a,...ab,...b->...", Wi, val, Wj)


def far_entries(Xi, Wi, Xj, Wj, s):
    """sum_ab W_ia W_jb exp(-s r_ab)/(4 pi r_ab) for blocks of triangles:
    Xi (m,6,3), Xj (n,6,3) -> (m,n).  Coincident points are not allowed."""
    r = np.linalg.norm(Xi[:, :, None, None, :] - Xj[None, None, :, :, :], axis=-1)
    safe = np.where(r > 0.0, r, 1.0)
    k = np.where(r > 0.0, np.exp(-s * safe) / (FOUR_PI * safe), 0.0)
    return np.einsum("ia,iajb,jb->ij", Wi, k, Wj)


def assemble_V(V, T, s, q=5, pairs=None, static=None, rows=None):
    """Dense Galerkin matrix V(s)[i,j] (Section 3.2) for one complex frequency.

    Far pairs: 6x6 Dunavant rule of exp(-s r)/(4 pi r).  Near pairs (sharing a
    vertex): Duffy static part + 6x6 rule of (exp(-s r) - 1)/(4 pi r).
    `rows` restricts the output to a subset of rows (for sampled checks).
    """
    X, W, _ = triangle_quadrature(V, T)
    M = len(T)
    rows = np.arange(M) if rows is None else np.asarray(rows)
    if pairs is None:
        pairs = near_pairs(T)
    if static is None:
        static = near_static(V, T, pairs, q)
    out = np.empty((len(rows), M), dtype=np.complex128)
    chunk = 32
    for c0 in range(0, len(rows), chunk):
        rr = rows[c0:c0 + chunk]
        out[c0:c0 + chunk] = far_entries(X[rr], W[rr], X, W, s)
    pos = np.full(M, -1)
    pos[rows] = np.arange(len(rows))
    pi = np.asarray([p[0] for p in pairs])
    pj = np.asarray([p[1] for p in pairs])
    sel = pos[pi] >= 0
    pi, pj, sv = pi[sel], pj[sel], np.asarray(static)[sel]
    out[pos[pi], pj] = sv + near_dynamic(X[pi], W[pi], X[pj], W[pj], s)
    return out


# ---------------------------------------------------------------- solve

def solve(V, T, N, Tend, rho=None, q=5, direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5,
          amplitude=1.0, samples=None, return_all=False):
    """All-at-once CQM solve of V * phi = g_D; returns q (N+1, M) real."""
    s, rho, dt = frequencies(N, Tend, rho)
    F = N + 1
    H = num_frequencies_half(F)
    b = rhs(V, T, N, Tend, direction, sigma, t0, amplitude, samples)
    ghat = forward_dft(b, rho, H)
    pairs = near_pairs(T)
    static = near_static(V, T, pairs, q)
    xhat = np.empty((H, len(T)), dtype=np.complex128)
    for l in range(H):
        A = assemble_V(V, T, s[l], q, pairs, static)
        xhat[l] = sla.lu_solve(sla.lu_factor(A), ghat[l])
    qn, im_ratio = inverse_dft(xhat, rho, F, conjugate_fill=True)
    if return_all:
        return dict(q=qn, s=s, rho=rho, dt=dt, b=b, ghat=ghat, xhat=xhat,
                    im_ratio=im_ratio, pairs=pairs, static=static)
    return qn


def rel_error(q, q_ref, area):
    """Area-weighted relative Frobenius error over all (n, i)."""
    num = np.sqrt(np.sum(area[None, :] * (q - q_ref) ** 2))
    den = np.sqrt(np.sum(area[None, :] * q_ref ** 2))
    return num / den


def step_errors(q, q_ref, area):
    """Per-step relative L2(Gamma) error (one value per time step)."""
    num = np.sqrt(np.sum(area[None, :] * (q - q_ref) ** 2, axis=1))
    den = np.sqrt(np.sum(area[None, :] * q_ref ** 2, axis=1))
    return num / np.maximum(den, 1e-300)
