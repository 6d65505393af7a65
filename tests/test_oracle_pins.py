"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks one oracle function against something other than itself:
closed forms, exact polynomial integration, an independent quadrature,
brute-force contour sums, invariants of the operator and of the transforms.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import cqm_workloads as W
import oracle as O
from static_reference import static_reference


# ------------------------------------------------------------------ A1

def test_frequencies_closed_form_and_symmetry():
    for N, T in ((8, 2.0), (32, 4.0), (64, 4.0), (128, 6.0)):
        s, rho, dt = O.frequencies(N, T)
        F = N + 1
        assert abs(rho ** N - 1e-8) < 1e-20
        # BDF2: delta(xi) = (1 - xi)(3 - xi)/2, xi = rho exp(-2 pi i l / F)
        xi = rho * np.exp(-2j * np.pi * np.arange(F) / F)
        assert np.allclose(s * dt, (1 - xi) * (3 - xi) / 2, rtol=1e-14, atol=1e-14)
        assert np.all(s.real > 0)
        for l in range(1, F):
            assert abs(s[F - l] - np.conj(s[l])) < 1e-12 * abs(s[l])
        assert abs(s[0].imag) < 1e-15 and abs(s[0] * dt - (1 - rho) * (3 - rho) / 2) < 1e-14


# ------------------------------------------------------------------ quadrature

def test_dunavant_exact_for_degree_4():
    bary, w = O.dunavant6()
    assert abs(w.sum() - 1) < 1e-14
    # reference triangle (0,0),(1,0),(0,1): int x^a y^b = a! b! / (a+b+2)!
    x, y = bary[:, 1], bary[:, 2]
    for a in range(5):
        for b in range(5 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(0.5 * np.dot(w, x ** a * y ** b) - exact) < 1e-14
    # and it is not exact at degree 5 (so the test above is meaningful)
    assert abs(0.5 * np.dot(w, x ** 5) - 1 / 42) > 1e-6


# ------------------------------------------------------------------ transforms (A3, A8)

def aliased_weights_inverse_s(N, T, rho):
    """F-point weights of K(s) = 1/s for BDF2, exact in closed form:
    dt [1/(1-rho^F) - 3^-(n+1)/(1-(rho/3)^F)]."""
    F, dt = N + 1, T / N
    n = np.arange(F)
    return dt * (1 / (1 - rho ** F) - 3.0 ** (-(n + 1)) / (1 - (rho / 3) ** F))


@pytest.mark.parametrize("N,T", [(16, 2.0), (32, 4.0), (64, 4.0)])
def test_inverse_transform_weights_of_inverse_s(N, T):
    s, rho, dt = O.frequencies(N, T)
    F = N + 1
    exact = aliased_weights_inverse_s(N, T, rho)
    H = O.num_frequencies_half(F)
    w_half, im_half = O.inverse_dft((1 / s[:H])[:, None], rho, F, conjugate_fill=True)
    w_full, im_full = O.inverse_dft((1 / s)[:, None], rho, F, conjugate_fill=False)
    for w in (w_half[:, 0], w_full[:, 0]):
        # rounding of the DFT is amplified by rho^-n (at most 1e8)
        err = np.abs(w - exact) / (rho ** -np.arange(F) * 1e-15 * dt + 1e-15 * dt)
        assert np.max(np.abs(w - exact) / dt) < 5e-8
        assert np.max(err) < 50
    # the unaliased weights dt (1 - 3^-(n+1)) agree to O(rho^F)
    n = np.arange(F)
    assert np.max(np.abs(w_half[:, 0] - dt * (1 - 3.0 ** (-(n + 1))))) < 3 * rho ** F * dt


def test_inverse_transform_polynomial_symbols():
    N, T = 24, 3.0
    s, rho, dt = O.frequencies(N, T)
    F = N + 1
    H = O.num_frequencies_half(F)
    one, _ = O.inverse_dft(np.ones((H, 1), dtype=complex), rho, F)
    e0 = np.zeros(F)
    e0[0] = 1.0
    assert np.max(np.abs(one[:, 0] - e0) * rho ** np.arange(F)) < 1e-14
    der, _ = O.inverse_dft(s[:H, None], rho, F)
    ref = np.zeros(F)
    ref[:3] = np.array([1.5, -2.0, 0.5]) / dt
    assert np.max(np.abs(der[:, 0] - ref) * rho ** np.arange(F)) < 1e-13 / dt


def test_all_at_once_equals_discrete_convolution():
    """forward DFT -> multiply by K(s_l) -> inverse DFT is the causal CQM
    convolution with the aliased weights, plus a rho^F-damped wrap-around."""
    N, T = 20, 2.5
    s, rho, dt = O.frequencies(N, T)
    F = N + 1
    rng = np.random.default_rng(3)
    g = rng.standard_normal((F, 4))
    ghat = O.forward_dft(g, rho, F)
    q, _ = O.inverse_dft(ghat / s[:, None], rho, F, conjugate_fill=False)
    w = aliased_weights_inverse_s(N, T, rho)
    ref = np.zeros_like(g)
    for n in range(F):
        for k in range(F):
            if k <= n:
                ref[n] += w[n - k] * g[k]
            else:
                ref[n] += rho ** F * w[F + n - k] * g[k]
    assert np.max(np.abs(q - ref)) < 1e-7 * np.max(np.abs(ref))
    # half band + conjugate fill gives the same sequence
    H = O.num_frequencies_half(F)
    ghalf = O.forward_dft(g, rho, H)
    q2, im = O.inverse_dft(ghalf / s[:H, None], rho, F)
    assert np.max(np.abs(q2 - ref)) < 1e-7 * np.max(np.abs(ref))


def test_weights_of_laplace_kernel_match_brute_force_contour():
    """CQM weights of K(s) = exp(-s r)/(4 pi r): F-point scaled DFT against a
    J-point contour sum at another radius (aliasing r_c^J negligible)."""
    N, T, r = 16, 2.0, 0.7
    s, rho, dt = O.frequencies(N, T)
    F = N + 1
    K = lambda z: np.exp(-z * r) / (4 * np.pi * r)
    w_f, _ = O.inverse_dft(K(s)[:, None], rho, F, conjugate_fill=False)
    J, rc = 4096, 0.8
    j = np.arange(J)
    xi = rc * np.exp(2j * np.pi * j / J)
    vals = K((1.5 - 2 * xi + 0.5 * xi ** 2) / dt)
    w_b = np.array([(rc ** -n / J) * np.sum(vals * np.exp(-2j * np.pi * j * n / J)) for n in range(F)]).real
    assert np.max(np.abs(w_f[:, 0] - w_b)) < 1e-8 * np.max(np.abs(w_b))


# ------------------------------------------------------------------ A4 static near part

def test_static_identical_closed_form():
    # int_T int_T 1/|x-y| over a triangle = (4|T|^2/3) sum_edges (1/|e|) ln(...)
    rng = np.random.default_rng(5)
    for _ in range(5):
        A, B, C = rng.standard_normal((3, 3))
        area = 0.5 * np.linalg.norm(np.cross(B - A, C - A))
        tot = 0.0
        for a, b in ((B - A, C - A), (C - A, C - B), (C - B, A - B)):
            d = b - a
            nd = np.linalg.norm(d)
            tot += math.log((nd * np.linalg.norm(a + d) + a @ d + nd * nd) / (nd * np.linalg.norm(a) + a @ d)) / nd
        exact = area * area / (3 * math.pi) * tot
        assert abs(O.static_identical(A, B, C, 24) - exact) < 1e-12 * exact
    # equilateral unit triangle: 3 ln 3 / (16 pi)
    A, B, C = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0.5, math.sqrt(3) / 2, 0])
    assert abs(O.static_identical(A, B, C, 12) - 3 * math.log(3) / (16 * math.pi)) < 1e-15


def _mesh_pair(kind):
    V, T = W.icosphere(1)
    pairs = O.near_pairs(T)
    ident, edge, vert = O.classify_pairs(T, pairs)
    if kind == "edge":
        k, a, b, c, d = edge[0]
        return (V[a], V[b], V[c]), (V[a], V[b], V[d]), lambda q: O.static_edge(V[a], V[b], V[c], V[d], q)
    k, p, a1, a2, b1, b2 = vert[0]
    return (V[p], V[a1], V[a2]), (V[p], V[b1], V[b2]), lambda q: O.static_vertex(V[p], V[a1], V[a2], V[b1], V[b2], q)


@pytest.mark.parametrize("kind", ["edge", "vertex"])
def test_static_adjacent_against_analytic_inner_integral(kind):
    Ti, Tj, rule = _mesh_pair(kind)
    ref = static_reference(Ti, Tj, rtol=1e-10)
    assert abs(rule(14) - ref) < 1e-9 * ref
    assert abs(rule(5) - ref) < 1e-5 * ref  # default order q = 5


def test_static_folded_pairs_against_analytic_inner_integral():
    A, B, C = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0.4, 0.9, 0.0])
    D = np.array([0.5, 0.0, 0.8])  # 90 degree fold across AB
    assert abs(O.static_edge(A, B, C, D, 12) - static_reference((A, B, C), (A, B, D))) < 1e-12
    B1, B2 = np.array([-0.8, 0.1, 0.2]), np.array([-0.3, -0.9, 0.1])
    assert abs(O.static_vertex(A, B, C, B1, B2, 12) - static_reference((A, B, C), (A, B1, B2))) < 1e-12


def test_static_rules_symmetric_and_convergent_in_q():
    V, T = W.icosphere(2)
    pairs = O.near_pairs(T)
    S5 = O.near_static(V, T, pairs, 5)
    S10 = O.near_static(V, T, pairs, 10)
    assert np.max(np.abs(S5 - S10) / S10) < 2e-6
    idx = {(i, j): k for k, (i, j, _) in enumerate(pairs)}
    # the q = 5 rule itself is symmetric in (i, j), not only the exact integral
    for S in (S5, S10):
        for (i, j, _), v in zip(pairs, S):
            assert abs(v - S[idx[(j, i)]]) < 1e-14 * v


# ------------------------------------------------------------------ A5 dynamic part

def test_expm1_complex_against_extended_precision():
    mpmath.mp.dps = 40
    for z in (1e-9 + 2e-9j, -3e-5 + 1e-4j, 0.3 - 0.2j, -2.0 + 5.0j, 1e-3j):
        ref = complex(mpmath.expm1(mpmath.mpc(z.real, z.imag)))
        assert abs(O.expm1_complex(np.complex128(z)) - ref) < 2e-16 * abs(ref) + 1e-300


def test_near_dynamic_limit_and_symmetry():
    V, T = W.icosphere(1)
    X, Wt, _ = O.triangle_quadrature(V, T)
    s = 3.0 + 2.0j
    # coincident points use the limit -s/(4 pi): compare with tiny offset
    d0 = O.near_dynamic(X[0], Wt[0], X[0], Wt[0], s)
    Xs = X[0] + 1e-9
    d1 = O.near_dynamic(X[0], Wt[0], Xs, Wt[0], s)
    assert abs(d0 - d1) < 1e-8 * abs(d0)
    assert abs(O.near_dynamic(X[0], Wt[0], X[1], Wt[1], s) - O.near_dynamic(X[1], Wt[1], X[0], Wt[0], s)) < 1e-16


# ------------------------------------------------------------------ A6 operator

def test_operator_symmetric_and_conjugate():
    V, T = W.icosphere(1)
    s = 2.0 + 3.0j
    A = O.assemble_V(V, T, s)
    assert np.max(np.abs(A - A.T)) < 1e-15 * np.max(np.abs(A))
    Ac = O.assemble_V(V, T, np.conj(s))
    assert np.max(np.abs(Ac - np.conj(A))) < 1e-15 * np.max(np.abs(A))
    rows = O.assemble_V(V, T, s, rows=[3, 17, 40])
    assert np.array_equal(rows, A[[3, 17, 40]])


@pytest.mark.parametrize("s", [1.0, 2.0 + 3.0j])
def test_sphere_row_sums_converge_to_closed_form(s):
    """V(s)1 = (1 - exp(-2s))/(2s) on the unit sphere; Galerkin row sums over
    |tau_i| converge at O(h^2)."""
    exact = (1 - np.exp(-2 * s)) / (2 * s)
    errs = []
    for level in (1, 2, 3):
        V, T = W.icosphere(level)
        _, _, area = O.triangle_quadrature(V, T)
        A = O.assemble_V(V, T, s)
        errs.append(np.sqrt(np.sum(area * np.abs(A.sum(1) / area - exact) ** 2) / np.sum(area)) / abs(exact))
    assert errs[2] < 0.01
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_far_entries_against_refined_quadrature():
    """A far-pair entry from the 6x6 rule agrees with the same double integral
    taken by a much finer rule to the rule's expected accuracy."""
    V, T = W.icosphere(2)
    X, Wt, area = O.triangle_quadrature(V, T)
    i, j, s = 0, 200, 2.0 + 5.0j
    v6 = O.far_entries(X[i:i + 1], Wt[i:i + 1], X[j:j + 1], Wt[j:j + 1], s)[0, 0]
    x, w = np.polynomial.legendre.leggauss(12)
    x, w = 0.5 * (x + 1), 0.5 * w
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    pts = np.stack([u.ravel(), (v * (1 - u)).ravel()], 1)
    wts = (wu * wv * (1 - u)).ravel() * 2

    def fine(tri):
        P = V[T[tri]]
        return P[0] + pts[:, :1] * (P[1] - P[0]) + pts[:, 1:] * (P[2] - P[0]), wts * area[tri]
    Xa, wa = fine(i)
    Xb, wb = fine(j)
    r = np.linalg.norm(Xa[:, None] - Xb[None], axis=-1)
    ref = np.einsum("a,ab,b->", wa, np.exp(-s * r) / (4 * np.pi * r), wb)
    assert abs(v6 - ref) < 1e-4 * abs(ref)


# ------------------------------------------------------------------ pipeline

def test_step_zero_is_a_single_real_solve():
    """omega_0 = K(delta(0)/dt) = K(3/(2 dt)) for BDF2, so q_0 solves
    V(3/(2 dt)) q_0 = b_0 up to O(rho^F) aliasing."""
    wl = W.C0_TINY
    V, T = wl.mesh()
    r = O.solve(V, T, wl.N, wl.T, return_all=True)
    A0 = O.assemble_V(V, T, 1.5 / r["dt"], pairs=r["pairs"], static=r["static"])
    q0 = np.linalg.solve(A0.real, r["b"][0])
    assert np.abs(A0.imag).max() == 0.0
    assert np.linalg.norm(r["q"][0] - q0) < 1e-6 * np.linalg.norm(q0)
    assert r["im_ratio"] < 1e-9


def test_causality_and_linearity():
    wl = W.C0_TINY
    V, T = wl.mesh()
    X, Wt, _ = O.triangle_quadrature(V, T)
    rng = np.random.default_rng(9)
    g = rng.standard_normal((wl.N + 1, len(T), 6))
    q1 = O.solve(V, T, wl.N, wl.T, samples=g)
    g2 = g.copy()
    g2[5:] += rng.standard_normal(g2[5:].shape)
    q2 = O.solve(V, T, wl.N, wl.T, samples=g2)
    scale = np.abs(q1).max()
    assert np.max(np.abs(q1[:5] - q2[:5])) < 1e-6 * scale
    assert np.max(np.abs(q1[5:] - q2[5:])) > 1e-2 * scale
    q3 = O.solve(V, T, wl.N, wl.T, samples=2.0 * g)
    assert np.max(np.abs(q3 - 2 * q1)) < 1e-9 * scale


def _profile(t, ts=0.3):
    z = t - ts
    return np.where(z > -0.2, np.cos(5 * z + 1) - 1, 0.0)


def test_radial_data_gives_sphere_transfer_function():
    """Uniform Dirichlet data gamma(t) on the unit sphere: the density is
    constant with Laplace transform gamma_hat * 2s/(1 - exp(-2s)); the mesh
    solution's area mean approaches this scalar CQM solution at O(h^2)."""
    N, T = 16, 4.0
    s, rho, dt = O.frequencies(N, T)
    F = N + 1
    gam = _profile(np.arange(F) * dt)
    ghat = O.forward_dft(gam[:, None], rho, F)
    lam = (1 - np.exp(-2 * s)) / (2 * s)
    scalar, _ = O.inverse_dft(ghat / lam[:, None], rho, F, conjugate_fill=False)
    errs = []
    for level in (1, 2):
        V, Tr = W.icosphere(level)
        _, _, area = O.triangle_quadrature(V, Tr)
        samples = np.broadcast_to(gam[:, None, None], (F, len(Tr), 6)).copy()
        q = O.solve(V, Tr, N, T, samples=samples)
        mean = (q * area).sum(1) / area.sum()
        spread = np.max(np.abs(q - mean[:, None]))
        assert spread < 0.05 * np.abs(mean).max()
        errs.append(np.linalg.norm(mean - scalar[:, 0]) / np.linalg.norm(scalar))
    assert errs[1] < 0.02 and errs[0] / errs[1] > 3.0
